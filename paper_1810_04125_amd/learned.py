"""Learned d0 / rank predictor for the adaptive HSS compression.

The adaptive driver (Alg. 3) with the incrementing strategy (Alg. 5) adds
delta_d sample columns per round until every node passes its stopping test.
Each round repeats sampling, local samples, stopping tests and IDs over the
whole tree, so a compression that starts at d0 and ends at d_final costs
1 + (d_final - d0) / delta_d tree passes.  This module predicts d_final
from what is known before sampling, so d0 can start close to it:

  features (8, all known before any sampling):
    one-hot family (Toeplitz, Laplace, Gaussian); log2 of the kernel
    parameter (Toeplitz h, Gaussian sigma; 0 for Laplace); log2 n; tree
    level; log2 of the mean node size at that level; -log10 rtol
  targets (2, masked):
    level >= 1 rows: log2(1 + largest node rank at that level);
    level 0 (root) row: log2(d_final) of an incrementing run started at
    d0 = 128, the start of the workloads it serves (a run's end depends on
    its start: a wider first block can pass where a narrower one grows)
  network: 8 -> 128 -> 128 -> 128 -> 2, ReLU, FP32 (hss_mlp_* kernels)

The compression's stopping tests still decide every node: a low
prediction costs extra rounds, a high one extra sample columns, neither
changes the accuracy guarantee.

    python -m paper_1810_04125_amd.learned generate --count 1536 --out FILE
    python -m paper_1810_04125_amd.learned train --data FILE --out WEIGHTS
    python -m paper_1810_04125_amd.learned curve --data FILE
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import hss, inputs

SIZES = [8, 128, 128, 128, 2]
FAMILIES = ("toeplitz", "laplace", "gauss")
_PKG = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(_PKG, "data", "d0_predictor.npz")
TRAIN_DATA = os.path.join(_PKG, "data", "d0_train.npz")
TREE_METHOD = {"toeplitz": "bisect", "laplace": "rcb", "gauss": "kd"}


def features(family, param, n, level, node_size, rtol) -> np.ndarray:
    f = np.zeros(8, np.float32)
    f[FAMILIES.index(family)] = 1.0
    f[3] = 0.5 * math.log2(param) if family != "laplace" else 0.0
    f[4] = (math.log2(n) - 14.0) / 3.0
    f[5] = level / 8.0
    f[6] = (math.log2(max(1.0, node_size)) - 10.0) / 4.0
    f[7] = (-math.log10(rtol) - 6.0) / 2.0
    return f


def level_sizes(tree):
    """Mean node size of each tree level (level 0 = root)."""
    sizes = tree.hi - tree.lo
    L = int(tree.level.max())
    return [float(sizes[tree.level == l].mean()) for l in range(L + 1)]


def param_of(spec):
    return spec.get("h") if spec["family"] == "toeplitz" else spec.get("sigma", 1.0)


def make_problem(spec):
    """(generator, tree) on the device for a spec dict (see inputs.learned_problems)."""
    import torch
    fam, n = spec["family"], spec["n"]
    if fam == "toeplitz":
        return hss.toeplitz(n, spec["h"]), hss.Tree(n, spec["leaf"])
    if fam == "laplace":
        pts = inputs.sphere_points(n, spec["points_seed"])
        return hss.laplace(torch.from_numpy(pts).cuda()), hss.Tree(n, spec["leaf"], pts, "rcb")
    pts = inputs.cube_points(n, spec["points_seed"])
    return (hss.gauss(torch.from_numpy(pts).cuda(), spec["sigma"], 1e-2),
            hss.Tree(n, spec["leaf"], pts, "kd"))


def rows_of(spec, tree, level_rank, d_final):
    """Training rows of one compressed problem, one per tree level."""
    X, T, M = [], [], []
    for lvl, size in enumerate(level_sizes(tree)):
        X.append(features(spec["family"], param_of(spec), spec["n"], lvl, size, spec["rtol"]))
        if lvl == 0:
            T.append([0.0, math.log2(d_final)])
            M.append([0.0, 1.0])
        else:
            T.append([math.log2(1.0 + level_rank[lvl]), 0.0])
            M.append([1.0, 0.0])
    return X, T, M


def generate(count, seed, chunk=48, delta_d=64, eta=0.05, d_max=4096, log=print, n_lo=1024, n_hi=32768,
             d0=128):
    """Compress `count` random problems on the GPU (incrementing strategy
    from `d0` in steps of delta_d, R drawn by the library from the seed) and
    return the training set as a dict of arrays."""
    specs = inputs.learned_problems(count, seed, n_lo, n_hi)
    X, T, M = [], [], []
    dropped = 0
    meta = {k: [] for k in ("family", "n", "leaf", "param", "rtol", "d_final", "rounds", "status", "max_rank")}
    t0 = time.time()
    for c0 in range(0, count, chunk):
        part = specs[c0:c0 + chunk]
        probs = [make_problem(s) for s in part]
        Hs, _ = hss.compress_batched([p[0] for p in probs], [p[1] for p in probs], None,
                                     rtol=[s["rtol"] for s in part], atol=1e-12, eta=eta,
                                     strategy="inc_fnorm", d0=d0, delta_d=delta_d,
                                     d_max=[min(d_max, s["n"]) for s in part], seed=seed + 1)
        for s, (gen, tree), H in zip(part, probs, Hs):
            info = H.info()
            if info["status"] == hss.NOT_CONVERGED:   # d_final capped at d_max: no label
                dropped += 1
                continue
            lr = np.zeros(int(tree.level.max()) + 1)
            for node in range(tree.num_nodes):
                ni = H.node_info(node)
                lv = tree.level[node]
                lr[lv] = max(lr[lv], ni["rank_r"], ni["rank_c"])
            x, t, m = rows_of(s, tree, lr, info["d_final"])
            X += x
            T += t
            M += m
            for k, v in (("family", FAMILIES.index(s["family"])), ("n", s["n"]), ("leaf", s["leaf"]),
                         ("param", param_of(s) or 0.0), ("rtol", s["rtol"]), ("d_final", info["d_final"]),
                         ("rounds", info["rounds"]), ("status", info["status"]), ("max_rank", lr.max())):
                meta[k].append(v)
        del Hs, probs
        log("generate: %d / %d problems (%d not converged, left out), %.1f s"
            % (min(count, c0 + chunk), count, dropped, time.time() - t0))
    out = {"X": np.array(X, np.float32), "T": np.array(T, np.float32), "M": np.array(M, np.float32)}
    out.update({"p_" + k: np.array(v) for k, v in meta.items()})
    out["p_eta"] = np.array([eta])
    out["p_d0"] = np.array([d0])
    return out


def merge(a, b, every):
    """Training sets a and b as one, b's problems placed after every
    `every` problems of a (rows stay grouped per problem, root row first)."""
    def groups(d):
        st = list(np.flatnonzero(d["X"][:, 5] == 0.0)) + [len(d["X"])]
        return [(st[i], st[i + 1]) for i in range(len(st) - 1)]
    ga, gb = groups(a), groups(b)
    order, ib = [], 0   # (set, problem index)
    for i in range(len(ga)):
        order.append((0, i))
        if (i + 1) % every == 0 and ib < len(gb):
            order.append((1, ib))
            ib += 1
    order += [(1, j) for j in range(ib, len(gb))]
    src, grp = (a, b), (ga, gb)
    out = {k: np.concatenate([src[w][k][grp[w][i][0]:grp[w][i][1]] for w, i in order]) for k in ("X", "T", "M")}
    for k in a:
        if k.startswith("p_") and k not in ("p_eta", "p_d0") and k in b:
            out[k] = np.array([src[w][k][i] for w, i in order])
    out["p_eta"] = a.get("p_eta", np.array([0.05]))
    if "p_d0" in a:
        if "p_d0" in b and int(b["p_d0"][0]) != int(a["p_d0"][0]):
            raise ValueError("the two sets were labelled from different starts d0")
        out["p_d0"] = a["p_d0"]
    return out


def _split(data, holdout):
    """(training rows, held-out rows, problem starts, number held out): whole
    problems are held out (rows are grouped per problem, root row first)."""
    starts = np.flatnonzero(data["X"][:, 5] == 0.0)
    nprob = len(starts)
    nhold = int(round(holdout * nprob))
    cut = starts[nprob - nhold] if nhold else len(data["X"])
    return ({k: data[k][:cut] for k in ("X", "T", "M")}, {k: data[k][cut:] for k in ("X", "T", "M")},
            starts, nhold)


def holdout_error(params, ho):
    """Mean absolute error on held-out rows: log2(1 + rank) and log2 d_final."""
    import torch
    Y = hss.mlp_forward(SIZES, torch.from_numpy(params).cuda(), torch.from_numpy(ho["X"]).cuda()).cpu().numpy()
    err = np.abs(Y - ho["T"]) * ho["M"]
    return (float(err[:, 0].sum() / max(1.0, ho["M"][:, 0].sum())),
            float(err[:, 1].sum() / max(1.0, ho["M"][:, 1].sum())))


def train(data, epochs=400, batch=256, lr=1e-3, seed=0, init_seed=1):
    """Train the predictor on the device; returns (flat float32 params, per-epoch losses)."""
    import torch
    dev = torch.device("cuda")
    X = torch.from_numpy(np.ascontiguousarray(data["X"], np.float32)).to(dev)
    T = torch.from_numpy(np.ascontiguousarray(data["T"], np.float32)).to(dev)
    M = torch.from_numpy(np.ascontiguousarray(data["M"], np.float32)).to(dev)
    p = torch.from_numpy(inputs.mlp_params(SIZES, init_seed)).to(dev)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    losses, _ = hss.mlp_train(SIZES, p, m, v, 0, X, T, M, batch=batch, epochs=epochs, lr=lr, seed=seed)
    return p.cpu().numpy(), losses


def save(params, path=WEIGHTS, **meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=np.asarray(params, np.float32), sizes=np.array(SIZES, np.int32),
             meta=np.array(json.dumps(meta)))


class D0Predictor:
    """Predicted d_final and per-level ranks from the trained network (FP32 HIP forward)."""

    def __init__(self, path=WEIGHTS, params=None):
        import torch
        if params is None:
            with np.load(path, allow_pickle=False) as z:
                if list(z["sizes"]) != SIZES:
                    raise ValueError("weights are for a network of sizes %s" % list(z["sizes"]))
                params = z["params"]
        self.params = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()

    def handle(self):
        """The network as an hss_predictor for hss_compress (options.predictor),
        which then computes the same features and d0 itself."""
        return hss.Predictor(SIZES, self.params)

    def predict(self, family, param, n, tree, rtol):
        """{'d_final': predicted final d, 'level_rank': [largest rank per level 1..L]}."""
        import torch
        sizes = level_sizes(tree)
        X = np.stack([features(family, param, n, l, s, rtol) for l, s in enumerate(sizes)])
        Y = hss.mlp_forward(SIZES, self.params, torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
        return {"d_final": float(2.0 ** Y[0, 1]), "level_rank": [float(2.0 ** y - 1.0) for y in Y[1:, 0]]}

    def d0(self, family, param, n, tree, rtol, delta_d=64, d_max=None, margin=0.0):
        """Initial sample count: the predicted d_final, shrunk by `margin`,
        rounded to the nearest multiple of delta_d, at least delta_d (a
        prediction a little low would cost a whole round, one a little
        high some sample columns)."""
        d = self.predict(family, param, n, tree, rtol)["d_final"] * (1.0 - margin)
        d0 = max(delta_d, delta_d * int(math.floor(d / delta_d + 0.5)))
        return min(d0, d_max) if d_max else d0


def _main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--count", type=int, default=1536)
    g.add_argument("--seed", type=int, default=10000)
    g.add_argument("--out", default=TRAIN_DATA)
    g.add_argument("--eta", type=float, default=0.05)
    g.add_argument("--n-lo", type=int, default=1024)
    g.add_argument("--n-hi", type=int, default=32768)
    g.add_argument("--d-max", type=int, default=4096)
    g.add_argument("--d0", type=int, default=128, help="start of the labelling runs")
    g.add_argument("--merge-into", default=None,
                   help="an existing set: write it with the new problems interleaved (one after every k-th)")
    g.add_argument("--every", type=int, default=4)
    g.add_argument("--chunk", type=int, default=48, help="problems per batched compression")
    c = sub.add_parser("curve", help="held-out error against the number of training problems")
    c.add_argument("--data", default=TRAIN_DATA)
    c.add_argument("--sizes", default="256,512,1024,2048,0")
    c.add_argument("--steps", type=int, default=0, help="optimizer steps per run (0: those of 400 epochs on all)")
    c.add_argument("--batch", type=int, default=256)
    c.add_argument("--holdout", type=float, default=0.1)
    t = sub.add_parser("train")
    t.add_argument("--data", default=TRAIN_DATA)
    t.add_argument("--out", default=WEIGHTS)
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--holdout", type=float, default=0.1)
    a = ap.parse_args()
    log = lambda m: print(m, flush=True)
    if a.cmd == "generate":
        d = generate(a.count, a.seed, chunk=a.chunk, eta=a.eta, log=log, n_lo=a.n_lo, n_hi=a.n_hi,
                     d_max=a.d_max, d0=a.d0)
        if a.merge_into:
            with np.load(a.merge_into, allow_pickle=False) as z:
                d = merge({k: z[k] for k in z.files}, d, a.every)
        np.savez_compressed(a.out, **d)
        log("wrote %s: %d rows from %d problems" % (a.out, len(d["X"]), len(d["p_n"])))
        return
    with np.load(a.data, allow_pickle=False) as z:
        data = {k: z[k] for k in z.files}
    tr, ho, starts, nhold = _split(data, a.holdout)
    nprob = len(starts)
    if a.cmd == "curve":
        ntr = nprob - nhold
        steps = a.steps or 400 * math.ceil(len(tr["X"]) / a.batch)
        for size in [int(x) for x in a.sizes.split(",")]:
            size = ntr if size <= 0 or size > ntr else size
            rows = starts[size] if size < ntr else len(tr["X"])
            sub_tr = {k: v[:rows] for k, v in tr.items()}
            epochs = max(1, round(steps / math.ceil(rows / a.batch)))
            t0 = time.time()
            params, losses = train(sub_tr, epochs=epochs, batch=a.batch)
            e_rank, e_d = holdout_error(params, ho)
            log(json.dumps({"train_problems": size, "train_rows": int(rows), "epochs": epochs,
                            "seconds": round(time.time() - t0, 1), "loss_last": float(losses[-1]),
                            "holdout_problems": nhold, "holdout_mae_log2_rank": round(e_rank, 4),
                            "holdout_mae_log2_dfinal": round(e_d, 4)}))
        return
    t0 = time.time()
    params, losses = train(tr, epochs=a.epochs, batch=a.batch, lr=a.lr)
    el = time.time() - t0
    res = {"epochs": a.epochs, "train_seconds": round(el, 2), "loss_first": float(losses[0]),
           "loss_last": float(losses[-1]), "train_problems": nprob - nhold, "holdout_problems": nhold}
    if nhold:
        res["holdout_mae_log2_rank"], res["holdout_mae_log2_dfinal"] = holdout_error(params, ho)
    save(params, a.out, **res)
    log(json.dumps(res))


if __name__ == "__main__":
    sys.exit(_main())
