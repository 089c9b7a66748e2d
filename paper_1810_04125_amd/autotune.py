"""Autotuner of the launch-shape tunables (hss_tunables).

For one workload (family, n, sampling precision, strategy), times the
compression with the built-in tunables and with candidate values, one
tunable at a time (coordinate descent over a small grid), and keeps a
candidate only when it is faster and its result stays within the parity
bar against the built-in run (same rounds and final d, every node's ranks
within 2, error at or below rtol).  The best values go into a tunables
table keyed by (device architecture, family, precision, n range of the
power-of-two bucket of n), which hss_load_tunables reads.

    python -m paper_1810_04125_amd.autotune --family laplace --n 32768 --out TABLE
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import tempfile
import time

import numpy as np

from . import hss, inputs

GRID = {"sample_wg": (1024, 2048, 4096), "gemm_wg": (1024, 2048, 4096), "gemm_max_split": (16, 32, 64),
        "qrcp_wg": (640, 1280, 2560)}


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def bucket(n: int):
    lo = 1 << int(math.floor(math.log2(n)))
    return lo, 2 * lo


def problem(family, n, leaf, seed, h=0.1, sigma=0.5):
    import torch
    if family == "toeplitz":
        return hss.toeplitz(n, h), hss.Tree(n, leaf)
    if family == "laplace":
        pts = inputs.sphere_points(n, seed)
        return hss.laplace(torch.from_numpy(pts).cuda()), hss.Tree(n, leaf, pts, "rcb")
    pts = inputs.cube_points(n, seed)
    return hss.gauss(torch.from_numpy(pts).cuda(), sigma, 1e-2), hss.Tree(n, leaf, pts, "kd")


def table_line(arch, family, precision, n, t):
    lo, hi = bucket(n)
    return "%s %d %d %d %d %d %d %d %d" % (arch, hss.FAMILY[family], hss.PRECISION[precision], lo, hi, t["gemm_wg"],
                                           t["gemm_max_split"], t["sample_wg"], t["qrcp_wg"])


def _with(arch, family, precision, n, t, fn):
    """Run fn() with a one-line table holding t for this key."""
    fd, path = tempfile.mkstemp(suffix=".tune")
    try:
        with os.fdopen(fd, "w") as f:
            f.write(table_line(arch, family, precision, n, t) + "\n")
        hss.load_tunables(path)
        return fn()
    finally:
        hss.load_tunables(None)
        os.unlink(path)


def tune(family, n, leaf=128, precision="fp64", rtol=1e-6, eta=0.05, strategy="inc_fnorm", d0=128, delta_d=64,
         d_max=4096, steps=2, seed=1, log=print):
    import torch
    arch = device_arch()
    gen, T = problem(family, n, leaf, seed)
    kw = dict(rtol=rtol, atol=1e-12, eta=eta, strategy=strategy, d0=d0, delta_d=delta_d, d_max=min(d_max, n),
              precision=precision, seed=0)

    def run():
        hss.compress(gen, T, None, **kw)   # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            H, st = hss.compress(gen, T, None, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, H, st

    def summary(H):
        i = H.info()
        ranks = np.array([[H.node_info(v)["rank_r"], H.node_info(v)["rank_c"]] for v in range(1, T.num_nodes)])
        return i["rounds"], i["d_final"], ranks

    best = hss.default_tunables()
    t_best, H0, st0 = _with(arch, family, precision, n, best, run)
    ref = summary(H0)
    err0 = H0.rel_error() if n <= 8192 else None
    del H0
    log("autotune: %s n=%d %s: built-in %s %.2f ms" % (family, n, precision, best, 1e3 * t_best))
    for name, values in GRID.items():
        for v in values:
            if v == best[name]:
                continue
            cand = dict(best, **{name: v})
            t, H, st = _with(arch, family, precision, n, cand, run)
            rounds, dfin, ranks = summary(H)
            ok = st == st0 and rounds == ref[0] and dfin == ref[1] and np.abs(ranks - ref[2]).max() <= 2
            if ok and err0 is not None:
                ok = H.rel_error() <= max(rtol, 2 * err0)
            del H
            log("autotune:   %s=%d: %.2f ms%s" % (name, v, 1e3 * t, "" if ok else " (outside the parity bar)"))
            if ok and t < 0.98 * t_best:
                best, t_best = cand, t
    log("autotune: best %s %.2f ms" % (best, 1e3 * t_best))
    return arch, best, t_best


def merge_table(path, line):
    """Write `line` into the table at `path`, replacing a line with the same key."""
    key = line.split()[:5]
    lines = []
    if os.path.exists(path):
        with open(path) as f:
            lines = [l.rstrip("\n") for l in f if l.strip() and l.split()[:5] != key]
    lines.append(line)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--family", choices=("toeplitz", "laplace", "gauss"), required=True)
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--leaf", type=int, default=128)
    ap.add_argument("--precision", default="fp64", choices=sorted(hss.PRECISION))
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--strategy", default="inc_fnorm")
    ap.add_argument("--d0", type=int, default=128)
    ap.add_argument("--delta-d", type=int, default=64)
    ap.add_argument("--d-max", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    arch, best, _ = tune(a.family, a.n, a.leaf, a.precision, a.rtol, 0.05, a.strategy, a.d0, a.delta_d, a.d_max,
                         a.steps, a.seed, log=lambda m: print(m, flush=True))
    merge_table(a.out, table_line(arch, a.family, a.precision, a.n, best))
    print("autotune: wrote", a.out, flush=True)


if __name__ == "__main__":
    sys.exit(_main())
