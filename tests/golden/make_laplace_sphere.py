"""Writes the oracle's reference results for the sphere-Laplace workload.

    python tests/golden/make_laplace_sphere.py [--n 32768] [--out FILE]

Workload: n points uniform on the unit sphere (inputs.sphere_points, seed
1), recursive coordinate bisection with leaf 128, A_ij = 1/(4 pi |x_i - x_j|)
for i != j and A_ii = 1; incrementing strategy (Alg. 5) with d0 = 128 and
delta_d = 64, rtol 1e-6, atol 1e-12, per-node safety factor eta = 0.05,
d_max = 4096; R from the counter-based generator with seed 0.

Calls only the oracle (and the seeded point drawer); nothing here touches
the HIP library.  The output holds every node's ranks, the round count,
the final sample count and the exact relative Frobenius error of the
oracle's compression.  At n = 32768 this takes on the order of an hour of
CPU time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import philox  # noqa: E402
from oracle.hss import compress  # noqa: E402
from oracle.matvec import rel_error  # noqa: E402
from oracle.operators import Laplace, PermutedOperator  # noqa: E402
from oracle.tree import build_tree  # noqa: E402
from paper_1810_04125_amd import inputs  # noqa: E402

CONFIG = dict(points_seed=1, leaf=128, tree="rcb", strategy="inc_fnorm", d0=128, delta_d=64,
              rtol=1e-6, atol=1e-12, eta=0.05, d_max=4096, r_seed=0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    n = a.n
    c = CONFIG
    out = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "laplace_sphere_%d.json" % n)
    t0 = time.time()
    pts = inputs.sphere_points(n, c["points_seed"])
    tree = build_tree(n, c["leaf"], pts, c["tree"])
    op = PermutedOperator(Laplace(pts, 1.0), tree.perm)
    d_max = min(c["d_max"], n)
    R = philox.gaussian_matrix(n, d_max, c["r_seed"])
    print("golden: n=%d tree and R ready (%.0f s)" % (n, time.time() - t0), flush=True)
    h = compress(op, tree, R, rtol=c["rtol"], atol=c["atol"], strategy=c["strategy"], d0=c["d0"],
                 delta_d=c["delta_d"], d_max=d_max, eta=c["eta"])
    print("golden: compressed, rounds %d, d %d, rank %d (%.0f s)" % (h.rounds, h.d, h.hss_rank(),
                                                                       time.time() - t0), flush=True)
    err = rel_error(h, op)
    print("golden: exact rel err %.6e (%.0f s)" % (err, time.time() - t0), flush=True)
    res = dict(config=dict(c, n=n, d_max=d_max), rounds=h.rounds, d_final=h.d, schedule=h.d_schedule,
               converged=h.converged, hss_rank=h.hss_rank(), rel_err=err,
               rank_r=[int(x.rank_r) for x in h.nodes], rank_c=[int(x.rank_c) for x in h.nodes],
               seconds=round(time.time() - t0, 1))
    with open(out, "w") as f:
        json.dump(res, f, indent=0)
    print("golden: wrote", out, flush=True)


if __name__ == "__main__":
    main()
