"""The sphere-Laplace workload at full size (n = 32768, leaf 128, RCB
tree, incrementing strategy with d0 = 128 and delta_d = 64, rtol 1e-6,
eta = 0.05, R from the counter-based generator) against the oracle's
stored results in tests/golden/laplace_sphere_32768.json.  That file is
written by tests/golden/make_laplace_sphere.py, which calls the oracle
only; both sides draw the same R from the seed with their own generators.

Bar: the same round count and final sample count, every node's ranks
within 2 of the oracle's, and an exact relative Frobenius error at or
below rtol and within twice the oracle's."""
import json
import os

import pytest

from paper_1810_04125_amd import hss, inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "laplace_sphere_32768.json")


def test_laplace_sphere_32768_matches_the_oracle():
    import torch
    with open(GOLDEN) as f:
        g = json.load(f)
    c = g["config"]
    n = c["n"]
    print("golden laplace sphere n=%d" % n, flush=True)
    pts = inputs.sphere_points(n, c["points_seed"])
    T = hss.Tree(n, c["leaf"], pts, c["tree"])
    gen = hss.laplace(torch.from_numpy(pts).cuda())
    H, st = hss.compress(gen, T, None, rtol=c["rtol"], atol=c["atol"], eta=c["eta"], strategy=c["strategy"],
                         d0=c["d0"], delta_d=c["delta_d"], d_max=c["d_max"], seed=c["r_seed"])
    info = H.info()
    print("library", info, "oracle rounds %d d %d rank %d" % (g["rounds"], g["d_final"], g["hss_rank"]), flush=True)
    assert st == hss.OK and g["converged"]
    assert info["rounds"] == g["rounds"] and info["d_final"] == g["d_final"]
    worst = 0
    for t in range(1, T.num_nodes):
        ni = H.node_info(t)
        worst = max(worst, abs(ni["rank_r"] - g["rank_r"][t]), abs(ni["rank_c"] - g["rank_c"][t]))
    assert worst <= 2, worst
    err = H.rel_error()
    print("rel err %.3e (oracle %.3e), worst node rank difference %d" % (err, g["rel_err"], worst), flush=True)
    assert err <= c["rtol"] and err <= 2.0 * g["rel_err"]
