"""Stopping test of eq. HMT_IQQH (strategy inc_hmt, Sec. 3.1 with Lemma 4.1
of Halko, Martinsson and Tropp) on the GPU against the FP64 oracle: rounds,
final sample count, node ranks and the compression error on the same
operator and R."""
import numpy as np
import pytest

from oracle.hss import compress as ocompress
from oracle.matvec import rel_error as orel
from paper_1810_04125_amd import hss, inputs
from tests.gpu_util import dev_colmajor, problem

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _check(H, oh, ot, atol_bound):
    for t in range(1, ot.num_nodes):
        ni = H.node_info(t)
        assert ni["state"] == 2
        assert abs(ni["rank_r"] - oh.nodes[t].rank_r) <= 2, t
        assert abs(ni["rank_c"] - oh.nodes[t].rank_c) <= 2, t
    assert H.info()["rounds"] == oh.rounds
    assert H.info()["d_final"] == oh.d
    err = H.rel_error()
    assert err <= atol_bound and err <= 2 * max(orel(oh, _op_of(oh)), 1e-15), err
    return err


_OPS = {}


def _op_of(oh):
    return _OPS[id(oh)]


def _run(family, n, leaf, atol, d0, dd, seed=0, alpha=10.0, dense=None, symmetric=True, rtol=1e-6):
    gen, T, ot, op = problem(family, n, leaf, seed=seed, dense=dense, symmetric=symmetric)
    R = inputs.gaussian_matrix(n, 1024, seed + 1)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=rtol, atol=atol, strategy="inc_hmt", d0=d0,
                         delta_d=dd, hmt_alpha=alpha)
    oh = ocompress(op, ot, R, rtol, atol, "inc_hmt", d0=d0, delta_d=dd, alpha=alpha)
    _OPS[id(oh)] = op
    return H, st, oh, ot, op


@pytest.mark.parametrize("family,n,leaf,atol,d0,dd", [("toeplitz", 1024, 64, 1e-8, 32, 32),
                                                     ("laplace", 2048, 128, 1e-7, 128, 64)])
def test_inc_hmt_matches_oracle(family, n, leaf, atol, d0, dd):
    _log("inc_hmt %s %d atol %g" % (family, n, atol))
    H, st, oh, ot, op = _run(family, n, leaf, atol, d0, dd, seed=1)
    assert st == hss.OK and oh.rounds > 1
    _check(H, oh, ot, 1e-3)


def test_inc_hmt_planted_rank():
    """I + U V^T (dense in HBM): ranks exactly r; the block that completes the
    range fails the test and the next one passes (oracle's round count)."""
    _log("inc_hmt planted rank")
    n, r = 512, 20
    U = inputs.orthonormal_columns(n, r, 40)
    V = inputs.orthonormal_columns(n, r, 41)
    A = np.eye(n) + U @ V.T
    H, st, oh, ot, op = _run("dense", n, 64, 1e-10, 8, 8, seed=9, dense=A, symmetric=False)
    for t in range(1, ot.num_nodes):
        ni = H.node_info(t)
        assert ni["rank_r"] == r and ni["rank_c"] == r, t
    assert H.info()["rounds"] == oh.rounds == 4
    assert H.rel_error() < 1e-12


def test_inc_hmt_ignores_rtol_and_alpha_orders_rounds():
    _log("inc_hmt rtol / alpha")
    n, leaf = 1024, 64
    gen, T, ot, op = problem("toeplitz", n, leaf)
    R = dev_colmajor(inputs.gaussian_matrix(n, 1024, 3))
    kw = dict(atol=1e-8, strategy="inc_hmt", d0=16, delta_d=16)
    a, _ = hss.compress(gen, T, R, rtol=1e-2, **kw)
    b, _ = hss.compress(gen, T, R, rtol=1e-12, **kw)
    assert a.info()["rounds"] == b.info()["rounds"]
    for t in range(1, T.num_nodes):
        assert np.array_equal(a.node(t, "JR"), b.node(t, "JR"))
    lo, _ = hss.compress(gen, T, R, rtol=0.0, hmt_alpha=1.0, **kw)
    hi, _ = hss.compress(gen, T, R, rtol=0.0, hmt_alpha=100.0, **kw)
    assert hi.info()["d_final"] >= lo.info()["d_final"]
    Rn = inputs.gaussian_matrix(n, 1024, 3)
    for alpha, H in ((1.0, lo), (100.0, hi)):
        oh = ocompress(op, ot, Rn, 0.0, 1e-8, "inc_hmt", d0=16, delta_d=16, alpha=alpha)
        assert H.info()["rounds"] == oh.rounds and H.info()["d_final"] == oh.d


def test_inc_hmt_nonsymmetric_both_sides():
    _log("inc_hmt nonsymmetric dense 400")
    n = 400
    pts = inputs.cube_points(n, 8)
    from oracle.operators import Laplace
    A = Laplace(pts).entries(np.arange(n), np.arange(n)) * (1.0 + 0.3 * pts[:, 0])[:, None]
    H, st, oh, ot, op = _run("dense", n, 50, 1e-9, 16, 16, seed=2, dense=A, symmetric=False)
    _check(H, oh, ot, 1e-6)


def test_inc_hmt_batched_equals_single():
    """A batch of two problems under the HMT-lemma test: each result has the
    rounds, ranks and skeleton rows of its own compression."""
    _log("inc_hmt batched")
    n, leaf = 1024, 64
    gens = [hss.toeplitz(n, 0.1), hss.toeplitz(n, 0.3)]
    trees = [hss.Tree(n, leaf), hss.Tree(n, leaf)]
    Rs = [dev_colmajor(inputs.gaussian_matrix(n, 1024, 7)), dev_colmajor(inputs.gaussian_matrix(n, 1024, 8))]
    kw = dict(rtol=0.0, atol=1e-9, strategy="inc_hmt", d0=32, delta_d=32)
    Hb, st = hss.compress_batched(gens, trees, Rs, **kw)
    for k in range(2):
        Hs, _ = hss.compress(gens[k], trees[k], Rs[k], **kw)
        assert Hb[k].info()["rounds"] == Hs.info()["rounds"]
        for t in range(1, trees[k].num_nodes):
            assert Hb[k].node_info(t)["rank_r"] == Hs.node_info(t)["rank_r"]
            assert np.array_equal(Hb[k].node(t, "JR"), Hs.node(t, "JR"))
        assert Hb[k].rel_error() <= 1e-6
