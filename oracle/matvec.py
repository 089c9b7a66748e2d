"""HSS matrix-vector product and reconstruction error (oracle).

The product follows the HSS format of Sec. 2.1: D_tau on the leaves,
sibling blocks A(I_nu1, I_nu2) ~= U^big_nu1 B_12 (V^big_nu2)^T, and the
nested bases of eq. (nestedUV), U^big_tau = diag(U^big_nu1, U^big_nu2) U_tau.
With x_hat_tau = (V^big_tau)^T x(I_tau) (upward pass) the contribution of
every sibling pair is U^big_nu1 B_12 x_hat_nu2, accumulated top-down.

`dense_from_generators` rebuilds H block by block from the explicit big
bases instead; the two routes share nothing but the stored generators and
pin each other.  All vectors are in the permuted order of the tree.
"""
from __future__ import annotations

import numpy as np


def hss_matvec(h, X: np.ndarray) -> np.ndarray:
    T, nodes = h.tree, h.nodes
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    nn = T.num_nodes
    xh = [None] * nn
    order = sorted(range(nn), key=lambda t: -int(T.level[t]))   # deepest first
    for t in order:
        if T.parent[t] < 0:
            continue
        nd = nodes[t]
        if T.is_leaf(t):
            xin = X[T.lo[t]:T.hi[t]]
        else:
            xin = np.vstack([xh[T.left[t]], xh[T.right[t]]])
        xh[t] = nd.idc.basis(xin.shape[0]).T @ xin          # V_tau^T
    yh = [None] * nn
    Y = np.zeros_like(X)
    for t in sorted(range(nn), key=lambda t: int(T.level[t])):   # root first
        nd = nodes[t]
        if T.is_leaf(t):
            if T.parent[t] < 0:
                Y[:] = nd.D @ X
                continue
            y = nd.idr.basis(T.size(t)) @ yh[t]              # U_tau
            Y[T.lo[t]:T.hi[t]] = y + nd.D @ X[T.lo[t]:T.hi[t]]
            continue
        l, r = T.left[t], T.right[t]
        rl = nodes[l].rank_r
        if T.parent[t] < 0:
            z = np.zeros((rl + nodes[r].rank_r, X.shape[1]))
        else:
            z = nd.idr.basis(rl + nodes[r].rank_r) @ yh[t]
        yh[l] = z[:rl] + nd.B12 @ xh[r]
        yh[r] = z[rl:] + nd.B21 @ xh[l]
    return Y[:, 0] if vec else Y


def big_bases(h):
    """Explicit U^big_tau, V^big_tau for every non-root node (eq. nestedUV)."""
    T, nodes = h.tree, h.nodes
    Ub, Vb = {}, {}
    for t in sorted(range(T.num_nodes), key=lambda t: -int(T.level[t])):
        if T.parent[t] < 0:
            continue
        nd = nodes[t]
        if T.is_leaf(t):
            Ub[t] = nd.idr.basis(T.size(t))
            Vb[t] = nd.idc.basis(T.size(t))
        else:
            l, r = T.left[t], T.right[t]
            bl_u = np.zeros((T.size(t), Ub[l].shape[1] + Ub[r].shape[1]))
            bl_u[:T.size(l), :Ub[l].shape[1]] = Ub[l]
            bl_u[T.size(l):, Ub[l].shape[1]:] = Ub[r]
            bl_v = np.zeros((T.size(t), Vb[l].shape[1] + Vb[r].shape[1]))
            bl_v[:T.size(l), :Vb[l].shape[1]] = Vb[l]
            bl_v[T.size(l):, Vb[l].shape[1]:] = Vb[r]
            Ub[t] = bl_u @ nd.idr.basis(bl_u.shape[1])
            Vb[t] = bl_v @ nd.idc.basis(bl_v.shape[1])
    return Ub, Vb


def dense_from_generators(h) -> np.ndarray:
    """H assembled block by block (eq. HSSexamplematrix)."""
    T, nodes = h.tree, h.nodes
    Ub, Vb = big_bases(h)
    H = np.zeros((T.n, T.n))
    for t in range(T.num_nodes):
        lo, hi = T.lo[t], T.hi[t]
        if T.is_leaf(t):
            H[lo:hi, lo:hi] = nodes[t].D
            continue
        l, r = T.left[t], T.right[t]
        H[T.lo[l]:T.hi[l], T.lo[r]:T.hi[r]] = Ub[l] @ nodes[t].B12 @ Vb[r].T
        H[T.lo[r]:T.hi[r], T.lo[l]:T.hi[l]] = Ub[r] @ nodes[t].B21 @ Vb[l].T
    return H


def rel_error(h, op, block: int = 512) -> float:
    """||A_hat - H||_F / ||A_hat||_F, exact, by column blocks of H."""
    n = h.tree.n
    num = 0.0
    den = 0.0
    rows = np.arange(n)
    for j0 in range(0, n, block):
        cols = np.arange(j0, min(n, j0 + block))
        E = np.zeros((n, len(cols)))
        E[cols, np.arange(len(cols))] = 1.0
        Hc = hss_matvec(h, E)
        Ac = op.extract(rows, cols)
        num += float(((Ac - Hc) ** 2).sum())
        den += float((Ac ** 2).sum())
    return float(np.sqrt(num / den))
