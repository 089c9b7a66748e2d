"""The library's Gaussian R (hss_random_normal / hss_random_words and
compressions that draw R themselves) against the oracle's generator."""
import numpy as np
import pytest

from oracle import philox
from oracle.hss import compress as ocompress
from oracle.matvec import rel_error as orel
from paper_1810_04125_amd import hss
from tests.gpu_util import problem

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("n,c0,ncols,seed", [(1003, 5, 7, 2 ** 63 + 12345), (4, 0, 1, 0), (1, 3, 2, 1),
                                              (65536, 1000, 3, 7)])
def test_raw_words_bit_exact(n, c0, ncols, seed):
    _log("words n=%d c0=%d ncols=%d" % (n, c0, ncols))
    W = hss.random_words(n, c0, ncols, seed).cpu().numpy().view(np.uint64)
    q = np.arange((n + 3) // 4, dtype=np.uint64)
    for t in range(ncols):
        w = philox.philox4x64((q, np.uint64(c0 + t), np.uint64(0), np.uint64(0)), (seed, 0))
        ref = np.empty(4 * len(q), dtype=np.uint64)
        for u in range(4):
            ref[u::4] = w[u]
        assert np.array_equal(W[:, t], ref[:n]), t


@pytest.mark.parametrize("n,c0,ncols,seed", [(1003, 0, 9, 11), (32768, 64, 4, 0), (7, 2, 3, 5)])
def test_normals_within_4_ulp(n, c0, ncols, seed):
    _log("normals n=%d c0=%d ncols=%d" % (n, c0, ncols))
    R = hss.random_normal(n, c0, ncols, seed).cpu().numpy()
    ref = philox.gaussian_columns(n, c0, c0 + ncols, seed)
    ulp = np.abs(R - ref) / np.spacing(np.abs(ref))
    assert ulp.max() <= 4.0, ulp.max()


def test_compression_with_library_r_matches_oracle():
    """Toeplitz n = 1024 (doubling, d0 = 64, rtol 1e-6): R drawn by the
    library from the seed; the oracle draws the same R with its own
    generator.  Ranks within 2, the same rounds, error at or below rtol and
    within 2x the oracle's."""
    n, seed = 1024, 0
    gen, T, ot, op = problem("toeplitz", n, 64)
    H, st = hss.compress(gen, T, None, rtol=1e-6, atol=1e-12, eta=0.05, strategy="dbl_fnorm", d0=64,
                         d_max=512, seed=seed)
    oh = ocompress(op, ot, philox.gaussian_matrix(n, 512, seed), 1e-6, 1e-12, "dbl_fnorm", d0=64, d_max=512,
                   eta=0.05)
    info = H.info()
    assert st == 0 and info["rounds"] == oh.rounds and info["d_final"] == oh.d
    for t in range(1, ot.num_nodes):
        assert abs(H.node_info(t)["rank_r"] - oh.nodes[t].rank_r) <= 2, t
    err, oerr = H.rel_error(), orel(oh, op)
    assert err <= 1e-6 and err <= 2 * oerr, (err, oerr)


def test_library_r_equals_the_same_r_passed_in():
    """Drawing R inside the compression and passing hss_random_normal's R
    give bitwise-equal generators (the sampled columns are the same)."""
    n, seed = 2048, 42
    gen, T, ot, op = problem("laplace", n, 64, seed=3)
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.05, strategy="inc_fnorm", d0=64, delta_d=32, d_max=1024)
    H1, _ = hss.compress(gen, T, None, seed=seed, **kw)
    R = hss.random_normal(n, 0, 1024, seed)
    H2, _ = hss.compress(gen, T, R, **kw)
    i1, i2 = H1.info(), H2.info()
    assert (i1["rounds"], i1["d_final"], i1["hss_rank"]) == (i2["rounds"], i2["d_final"], i2["hss_rank"])
    for t in range(1, T.num_nodes):
        assert H1.node_info(t) == H2.node_info(t)
        assert np.array_equal(H1.node(t, "JR"), H2.node(t, "JR"))
        assert np.array_equal(H1.node(t, "ER"), H2.node(t, "ER"))
