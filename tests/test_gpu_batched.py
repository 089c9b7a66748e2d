"""Batched compression (hss_compress_batched): many independent problems of
uneven size in one job, every level launch covering all of them.  Each
problem must come out exactly as when compressed alone (the oracle pins the
single-problem path), within tolerance."""
import numpy as np
import pytest

from oracle.hss import compress as ocompress
from paper_1810_04125_amd import hss, inputs
from tests.gpu_util import dev, dev_colmajor, problem

pytestmark = pytest.mark.gpu


def _batch(seed, count, n_lo, n_hi):
    specs = inputs.batch_problems(count, seed, n_lo, n_hi)
    out = []
    for sp in specs:
        if sp["family"] == "toeplitz":
            gen, T, ot, op = problem("toeplitz", sp["n"], 128, h=sp["h"])
        else:
            gen, T, ot, op = problem("laplace", sp["n"], 128, seed=sp["points_seed"])
        R = inputs.gaussian_matrix(sp["n"], min(sp["n"], 1024), 3)
        out.append((gen, T, ot, op, R))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_matches_individual(prec):
    print("batched", prec, flush=True)
    probs = _batch(3, 8, 600, 3000)
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.1, strategy="dbl_fnorm", d0=64, precision=prec)
    Rs = [dev_colmajor(p[4]) for p in probs]
    Hb, st = hss.compress_batched([p[0] for p in probs], [p[1] for p in probs], Rs, **kw)
    # The work partition of the GEMMs (K slices) and of the pivot steps
    # depends on the whole batch, so a problem's sums may be taken in another
    # order than when it runs alone: same decisions, E equal to rounding.
    for (gen, T, ot, op, R), Rd, hb in zip(probs, Rs, Hb):
        hi, _ = hss.compress(gen, T, Rd, **kw)
        assert hb.info()["rounds"] == hi.info()["rounds"]
        for t in range(1, T.num_nodes):
            assert hb.node_info(t) == hi.node_info(t)
            assert np.array_equal(hb.node(t, "JR"), hi.node(t, "JR"))
            Eb, Ei = hb.node(t, "ER"), hi.node(t, "ER")
            if Ei.size:
                assert np.abs(Eb - Ei).max() <= 1e-7 * max(1.0, np.abs(Ei).max())
        e, ei = hb.rel_error(), hi.rel_error()
        assert e <= (1e-6 if prec == "fp64" else 2e-5), e
        assert abs(e - ei) <= 1e-3 * ei


def test_batched_fp64_against_oracle():
    probs = _batch(5, 4, 500, 1500)
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.1, strategy="dbl_fnorm", d0=64)
    Hb, st = hss.compress_batched([p[0] for p in probs], [p[1] for p in probs],
                                  [dev_colmajor(p[4]) for p in probs], **kw)
    for (gen, T, ot, op, R), hb in zip(probs, Hb):
        oh = ocompress(op, ot, R, 1e-6, 1e-12, "dbl_fnorm", d0=64, eta=0.1)
        for t in range(1, ot.num_nodes):
            assert abs(hb.node_info(t)["rank_r"] - oh.nodes[t].rank_r) <= 2
        assert hb.rel_error() <= 1e-6
