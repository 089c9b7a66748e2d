"""FP64 reference of the learned rank / d0 predictor (oracle).

TEST INFRASTRUCTURE ONLY.  A plain multilayer perceptron
    h_1 = relu(W_1 x + b_1), h_2 = relu(W_2 h_1 + b_2),
    h_3 = relu(W_3 h_2 + b_3), y = W_4 h_3 + b_4,
trained on the masked mean squared error
    L = sum_{s,o} mask[s,o] (y[s,o] - t[s,o])^2 / max(1, sum mask)
with Adam (Kingma & Ba, 2015: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
p <- p - lr * mhat / (sqrt(vhat) + eps), mhat = m/(1-b1^k), vhat = v/(1-b2^k)).
Weights are stored row-major, W_l of shape (out, in).  Backward is the
chain rule written out layer by layer; the tests pin it by finite
differences.  The network is not part of the paper: it is the learned
predictor the HIP library adds on top of the paper's adaptive method, which
still decides every node.
"""
from __future__ import annotations

import numpy as np


def init_params(sizes, seed):
    """He-uniform weights, zero biases: [(W_1, b_1), ..., (W_L, b_L)]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(len(sizes) - 1):
        fan_in, fan_out = sizes[i], sizes[i + 1]
        lim = np.sqrt(6.0 / fan_in)
        out.append((rng.uniform(-lim, lim, (fan_out, fan_in)), np.zeros(fan_out)))
    return out


def forward(params, X):
    """Activations [x, h_1, ..., h_{L-1}, y] for a batch X (B x in)."""
    acts = [np.asarray(X, dtype=np.float64)]
    for i, (W, b) in enumerate(params):
        z = acts[-1] @ W.T + b
        acts.append(z if i == len(params) - 1 else np.maximum(z, 0.0))
    return acts


def loss(params, X, T, M):
    y = forward(params, X)[-1]
    return float((M * (y - T) ** 2).sum() / max(1.0, float(M.sum())))


def gradients(params, X, T, M):
    """dL/dW_l, dL/db_l for every layer (chain rule, layer by layer)."""
    acts = forward(params, X)
    y = acts[-1]
    delta = 2.0 * M * (y - T) / max(1.0, float(M.sum()))   # dL/dy
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        grads[i] = (delta.T @ acts[i], delta.sum(axis=0))
        if i > 0:
            delta = (delta @ W) * (acts[i] > 0.0)
    return grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; state = {'k': steps, 'm': [...], 'v': [...]}."""
    if not state:
        state.update(k=0, m=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params],
                     v=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params])
    state["k"] += 1
    k = state["k"]
    new = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m = b1 * state["m"][i][j] + (1 - b1) * g
            v = b2 * state["v"][i][j] + (1 - b2) * g * g
            state["m"][i] = tuple(m if jj == j else state["m"][i][jj] for jj in range(2))
            state["v"][i] = tuple(v if jj == j else state["v"][i][jj] for jj in range(2))
            mh = m / (1 - b1 ** k)
            vh = v / (1 - b2 ** k)
            out.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append((out[0], out[1]))
    return new
