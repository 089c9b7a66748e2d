"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle."""
import numpy as np
import pytest

from oracle.hss import compress as ocompress, interpolative
from oracle.matvec import hss_matvec as omatvec, rel_error as orel
from oracle.operators import PermutedOperator, Toeplitz
from paper_1810_04125_amd import hss, inputs
from tests.gpu_util import dev, dev_colmajor, problem

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("family,n,leaf,ncols", [("toeplitz", 1000, 64, 70), ("laplace", 777, 50, 64),
                                                 ("gauss", 1500, 100, 130), ("toeplitz", 3, 2, 1),
                                                 ("toeplitz", 1000, 64, 128), ("toeplitz", 1000, 64, 200)])
def test_sampling_matches_dense_product(family, n, leaf, ncols):
    _log("sample %s n=%d ncols=%d" % (family, n, ncols))
    gen, T, ot, op = problem(family, n, leaf, seed=3)
    R = inputs.gaussian_matrix(n, ncols, 5)
    S = hss.sample(gen, dev(T.perm), dev_colmajor(R)).cpu().numpy()
    ref = op.dense() @ R
    err = np.linalg.norm(S - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("n,ncols", [(1000, 70), (3000, 128)])
def test_sampling_toeplitz_any_permutation(n, ncols):
    """Toeplitz sampling under the index-bisection tree takes its entries
    from an LDS window of t(|i - j|), which needs the identity permutation;
    under any other permutation the kernel reads the table by permuted
    index.  Both must give the oracle's product (a random permutation, and
    the identity again, on the same inputs)."""
    _log("sample toeplitz perms n=%d ncols=%d" % (n, ncols))
    gen = hss.toeplitz(n, 0.1)
    R = inputs.gaussian_matrix(n, ncols, 5)
    for perm in (np.random.default_rng(11).permutation(n).astype(np.int64), np.arange(n, dtype=np.int64)):
        ref = PermutedOperator(Toeplitz(n, 0.1), perm).dense() @ R
        S = hss.sample(gen, dev(perm), dev_colmajor(R)).cpu().numpy()
        err = np.linalg.norm(S - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= 1e-12


@pytest.mark.parametrize("family,n,leaf", [("toeplitz", 80000, 128), ("gauss", 40000, 256)])
@pytest.mark.parametrize("ncols", [128, 200, 192])
def test_sampling_wide_tiles_split_k(family, n, leaf, ncols):
    """Sizes where the Toeplitz and Gaussian kernels take their 128-column
    tiles (128 and 200 columns; 192 runs as three narrow tiles), with the K
    dimension split over workgroups and ragged rows and columns: sampled
    rows against the oracle's entries, in both orientations (both
    operators are symmetric)."""
    _log("sample %s wide n=%d ncols=%d" % (family, n, ncols))
    gen, T, ot, op = problem(family, n, leaf, seed=6)
    R = inputs.gaussian_matrix(n, ncols, 9)
    rows = np.unique(np.concatenate([[0, 63, 64, 127, 128, n - 1], np.random.default_rng(4).integers(0, n, 12)]))
    ref = op.extract(rows, np.arange(n)) @ R
    for tr in (False, True):
        S = hss.sample(gen, dev(T.perm), dev_colmajor(R), transpose=tr).cpu().numpy()
        err = np.linalg.norm(S[rows] - ref, axis=1) / np.linalg.norm(ref, axis=1)
        assert err.max() <= 1e-12, (tr, err.max())


def test_sampling_transpose_nonsymmetric_dense():
    n = 600
    A = inputs.gaussian_matrix(n, n, 7)
    gen, T, ot, op = problem("dense", n, 64, dense=A, symmetric=False)
    R = inputs.gaussian_matrix(n, 33, 8)
    Ah = op.dense()
    for tr, ref in ((False, Ah @ R), (True, Ah.T @ R)):
        S = hss.sample(gen, dev(T.perm), dev_colmajor(R), transpose=tr).cpu().numpy()
        assert np.linalg.norm(S - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,ncols", [(700, 45), (1000, 640), (130, 1), (8000, 4096)])
def test_dense_sampling_random_permutation(n, ncols):
    """Dense matrices sample as a row scatter of R, one GEMM and a row gather:
    a random permutation (not a tree's); one workspace chunk, two chunks
    (n = 8000, 4096 columns: columns on both sides of the boundary are
    checked), and no workspace at all (n = 130: the entry kernel)."""
    _log("dense sample perm n=%d ncols=%d" % (n, ncols))
    A = inputs.gaussian_matrix(n, n, 21)
    gen = hss.dense(dev(A), symmetric=False)
    perm = np.random.default_rng(n).permutation(n).astype(np.int64)
    Ah = A[np.ix_(perm, perm)]
    R = inputs.gaussian_matrix(n, ncols, 22)
    cols = sorted({0, ncols // 2 - 1 if ncols > 1 else 0, ncols // 2, ncols - 1} | set(range(0, ncols, 97)))
    for tr in (False, True):
        S = hss.sample(gen, dev(perm), dev_colmajor(R), transpose=tr).cpu().numpy()
        ref = (Ah.T if tr else Ah) @ R[:, cols]
        err = np.linalg.norm(S[:, cols] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= 1e-13, (tr, err.max())


@pytest.mark.parametrize("family", ["toeplitz", "laplace", "gauss"])
def test_extraction_matches_entries(family):
    n = 900
    gen, T, ot, op = problem(family, n, 64, seed=4)
    rng = np.random.default_rng(1)
    I = rng.integers(0, n, 37)
    J = rng.integers(0, n, 53)
    out = hss.extract(gen, dev(T.perm), dev(I), dev(J)).cpu().numpy()
    ref = op.extract(I, J)
    if family == "toeplitz":
        assert np.array_equal(out, ref)
    else:
        assert np.allclose(out, ref, rtol=1e-14, atol=0)


def test_batched_id_matches_oracle():
    rng = np.random.default_rng(2)
    mats = []
    for m, d, r in ((40, 25, 25), (64, 100, 12), (200, 150, 90), (7, 3, 3), (0, 5, 0), (30, 30, 0)):
        if r == 0:
            mats.append(np.zeros((m, d)))
        else:
            mats.append(rng.standard_normal((m, r)) @ np.diag(0.8 ** np.arange(r)) @ rng.standard_normal((r, d)))
    out = hss.interpolative_batched(mats, 1e-7, 1e-300)
    for S, (r, piv, E) in zip(mats, out):
        o = interpolative(S, 1e-7, 1e-300)
        assert r == o.rank
        assert np.array_equal(piv[:r], o.J)
        assert np.array_equal(piv[r:], o.rest)
        if r and S.shape[0] > r:
            assert np.allclose(E, o.E, rtol=1e-9, atol=1e-9 * np.abs(o.E).max())


def _compare(H, oh, ot, gen, op, T, rtol, rank_tol=2):
    assert np.array_equal(T.perm, ot.perm) and np.array_equal(T.lo, ot.lo) and np.array_equal(T.hi, ot.hi)
    diffs = []
    for t in range(1, ot.num_nodes):
        ni = H.node_info(t)
        assert ni["state"] == 2
        diffs.append(abs(ni["rank_r"] - oh.nodes[t].rank_r))
        diffs.append(abs(ni["rank_c"] - oh.nodes[t].rank_c))
    assert max(diffs) <= rank_tol, diffs
    err = H.rel_error()
    oerr = orel(oh, op)
    assert err <= rtol and err <= 2 * max(oerr, 1e-15), (err, oerr)
    return err, oerr


@pytest.mark.parametrize("strategy", ["dbl_fnorm", "inc_fnorm", "dbl_hmt"])
def test_compress_toeplitz_config0(strategy):
    _log("compress toeplitz 1024 " + strategy)
    n, leaf = 1024, 64
    gen, T, ot, op = problem("toeplitz", n, leaf)
    R = inputs.gaussian_matrix(n, 512, 0)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-6, atol=1e-12, strategy=strategy, d0=64, delta_d=64)
    oh = ocompress(op, ot, R, 1e-6, 1e-12, strategy, d0=64, delta_d=64)
    _compare(H, oh, ot, gen, op, T, 1e-6)
    assert H.info()["rounds"] == oh.rounds
    # leaf D is bit-exact (Toeplitz entries are a table lookup)
    for t in range(ot.num_nodes):
        if ot.left[t] < 0:
            assert np.array_equal(H.node(t, "D"), oh.nodes[t].D)
    # matvec in original ordering
    x = np.random.default_rng(3).standard_normal((n, 3))
    y = H.matvec(dev_colmajor(x)).cpu().numpy()
    inv = np.empty(n, np.int64)
    inv[ot.perm] = np.arange(n)
    yo = omatvec(oh, x[ot.perm])[inv]
    assert np.linalg.norm(y - yo) <= 1e-6 * np.linalg.norm(yo)


def test_compress_laplace_sphere_inc():
    _log("compress laplace 2048 inc")
    n = 2048
    gen, T, ot, op = problem("laplace", n, 128, seed=1)
    R = inputs.gaussian_matrix(n, 1024, 0)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm",
                         d0=128, delta_d=64)
    oh = ocompress(op, ot, R, 1e-6, 1e-12, "inc_fnorm", d0=128, delta_d=64, eta=0.1)
    _compare(H, oh, ot, gen, op, T, 1e-6)


def test_compress_gauss_kd():
    _log("compress gauss 2048 inc")
    n = 2048
    gen, T, ot, op = problem("gauss", n, 256, seed=2)
    R = inputs.gaussian_matrix(n, 512, 0)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm",
                         d0=128, delta_d=64)
    oh = ocompress(op, ot, R, 1e-6, 1e-12, "inc_fnorm", d0=128, delta_d=64, eta=0.1)
    _compare(H, oh, ot, gen, op, T, 1e-6)


@pytest.mark.parametrize("strategy,r,d0,dd", [("inc_fnorm", 20, 8, 8), ("dbl_fnorm", 20, 8, 0),
                                              ("dbl_hmt", 20, 8, 0)])
def test_planted_rank(strategy, r, d0, dd):
    _log("planted rank %s r=%d" % (strategy, r))
    n = 512
    U = inputs.orthonormal_columns(n, r, 40)
    V = inputs.orthonormal_columns(n, r, 41)
    A = np.eye(n) + U @ V.T
    gen, T, ot, op = problem("dense", n, 64, dense=A, symmetric=False)
    R = inputs.gaussian_matrix(n, 256, 9)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-8, atol=1e-14, strategy=strategy, d0=d0, delta_d=dd)
    oh = ocompress(op, ot, R, 1e-8, 1e-14, strategy, d0=d0, delta_d=dd)
    for t in range(1, ot.num_nodes):
        ni = H.node_info(t)
        assert ni["rank_r"] == r and ni["rank_c"] == r, (t, ni)
    assert H.info()["rounds"] == oh.rounds
    assert H.rel_error() < 1e-12


def test_block_diagonal_rank_zero():
    n, leaf = 256, 32
    A = np.zeros((n, n))
    rng = np.random.default_rng(3)
    for k in range(n // leaf):
        A[k * leaf:(k + 1) * leaf, k * leaf:(k + 1) * leaf] = rng.standard_normal((leaf, leaf))
    gen, T, ot, op = problem("dense", n, leaf, dense=A, symmetric=False)
    H, st = hss.compress(gen, T, dev_colmajor(inputs.gaussian_matrix(n, 64, 1)), strategy="inc_fnorm",
                         d0=16, delta_d=16)
    assert H.info()["rounds"] == 1 and H.info()["hss_rank"] == 0
    assert H.rel_error() == 0.0


def test_nonsymmetric_dense_both_sides():
    from paper_1810_04125_amd import inputs as inp
    from oracle.operators import Laplace
    n = 400
    pts = inp.cube_points(n, 8)
    lap = Laplace(pts).entries(np.arange(n), np.arange(n))
    A = lap * (1.0 + 0.3 * pts[:, 0])[:, None]
    gen, T, ot, op = problem("dense", n, 50, dense=A, symmetric=False)
    R = inputs.gaussian_matrix(n, 400, 2)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-7, atol=1e-14, strategy="inc_fnorm", d0=32,
                         delta_d=16)
    oh = ocompress(op, ot, R, 1e-7, 1e-14, "inc_fnorm", d0=32, delta_d=16)
    _compare(H, oh, ot, gen, op, T, 1e-6)


def test_dmax_warning():
    n = 512
    U = inputs.orthonormal_columns(n, 60, 2)
    A = np.eye(n) + U @ inputs.orthonormal_columns(n, 60, 3).T
    gen, T, ot, op = problem("dense", n, 64, dense=A, symmetric=False)
    H, st = hss.compress(gen, T, dev_colmajor(inputs.gaussian_matrix(n, 32, 9)), rtol=1e-8, atol=1e-14,
                         strategy="inc_fnorm", d0=16, delta_d=16, d_max=32)
    assert st == hss.NOT_CONVERGED
    assert H.info()["d_final"] == 32


def test_deterministic():
    n = 2048
    gen, T, ot, op = problem("laplace", n, 128, seed=1)
    R = dev_colmajor(inputs.gaussian_matrix(n, 512, 0))
    outs = []
    for _ in range(2):
        H, _ = hss.compress(gen, T, R, rtol=1e-6, eta=0.1, strategy="inc_fnorm", d0=128, delta_d=64)
        outs.append([(H.node(t, "JR").tobytes(), H.node(t, "ER").tobytes()) for t in range(1, T.num_nodes)])
    assert outs[0] == outs[1]


def test_full_size_bench_workload_properties():
    """Sphere-Laplace n=32768 as in bench.py: exact ||A-H||_F/||A||_F <= rtol,
    U(J,:) = I structure via the stored pivots, skeleton indices inside the
    node, and sampled rows of S = A R against the oracle's rows."""
    from oracle.operators import Laplace
    n = 32768
    _log("full size laplace %d" % n)
    pts = inputs.sphere_points(n, 1)
    T = hss.Tree(n, 128, pts, "rcb")
    from oracle.tree import build_tree
    ot = build_tree(n, 128, pts, "rcb")
    assert np.array_equal(T.perm, ot.perm) and np.array_equal(T.lo, ot.lo)
    gen = hss.laplace(dev(pts))
    Rh = inputs.gaussian_matrix(n, 4096, 0)
    R = dev_colmajor(Rh)
    H, st = hss.compress(gen, T, R, rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm", d0=128, delta_d=64)
    assert st == hss.OK
    err = H.rel_error()
    _log("full size rel err %.3e" % err)
    assert err <= 1e-6
    for t in (1, 2, 5, 100, 300, 510):
        ni = H.node_info(t)
        J = H.node(t, "JR")
        assert sorted(J.tolist()) == list(range(ni["m_r"]))
        I = H.node(t, "IR")
        assert np.all((I >= ni["lo"]) & (I < ni["hi"]))
    # rows of S = A_hat R for the first 128 columns, oracle row by row
    rows = np.array([0, 7, 4096, 20000, n - 1])
    S = hss.sample(gen, dev(T.perm), dev_colmajor(Rh[:, :128])).cpu().numpy()
    lap = Laplace(pts)
    ref = lap.entries(ot.perm[rows], ot.perm) @ Rh[:, :128]
    assert np.linalg.norm(S[rows] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("family,n,leaf,dd", [("gauss", 2048, 256, 32), ("laplace", 2048, 128, 16)])
def test_compress_inc_narrow_blocks_rounds(family, n, leaf, dd):
    """Narrow increments: the stopping test's blocks run through the
    Cholesky-QR decision (well-conditioned, clearly failing or passing) or
    the Householder QR (near the threshold); the outcome must match the
    oracle's Householder-only test round for round."""
    _log("compress %s %d inc dd=%d" % (family, n, dd))
    gen, T, ot, op = problem(family, n, leaf, seed=2 if family == "gauss" else 1)
    R = inputs.gaussian_matrix(n, 1024, 0)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm",
                         d0=dd, delta_d=dd)
    oh = ocompress(op, ot, R, 1e-6, 1e-12, "inc_fnorm", d0=dd, delta_d=dd, eta=0.1)
    _compare(H, oh, ot, gen, op, T, 1e-6)
    assert H.info()["rounds"] == oh.rounds
    assert H.info()["d_final"] == oh.d


def test_release_cache_between_compressions():
    _log("release cache")
    n = 2048
    gen, T, ot, op = problem("laplace", n, 128, seed=1)
    R = dev_colmajor(inputs.gaussian_matrix(n, 1024, 0))
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm", d0=128, delta_d=64)
    H1, _ = hss.compress(gen, T, R, **kw)
    hss.release_cache()
    H2, _ = hss.compress(gen, T, R, **kw)
    H3, _ = hss.compress(gen, T, R, **kw)    # reuses the kept block
    for H in (H2, H3):
        assert H.info()["rounds"] == H1.info()["rounds"]
        for t in (1, 2, T.num_nodes - 1):
            assert np.array_equal(H.node(t, "ER"), H1.node(t, "ER"))


@pytest.mark.parametrize("strategy", ["inc_fnorm", "dbl_fnorm"])
def test_compress_large_first_block_tall_panels(strategy):
    """A first block of 1024 columns: the IDs of the lower levels factor
    tall panels (d >= 2 m) with the block-pivoted ID; ranks, rounds and the
    error must match the oracle's QRCP."""
    _log("compress laplace 4096 d0=1024 " + strategy)
    n = 4096
    gen, T, ot, op = problem("laplace", n, 128, seed=3)
    R = inputs.gaussian_matrix(n, 2048, 0)
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.1, strategy=strategy, d0=1024, delta_d=64)
    H, st = hss.compress(gen, T, dev_colmajor(R), **kw)
    oh = ocompress(op, ot, R, 1e-6, 1e-12, strategy, d0=1024, delta_d=64, eta=0.1)
    _compare(H, oh, ot, gen, op, T, 1e-6)
    assert H.info()["rounds"] == oh.rounds


@pytest.mark.parametrize("family,n,leaf,dd", [("laplace", 2048, 128, 100), ("gauss", 2048, 256, 200)])
def test_compress_inc_wide_ragged_blocks_rounds(family, n, leaf, dd):
    """Test blocks wider than 64 columns and not a multiple of 64: the
    triangular solve for Q_k (Sec. 3.2) runs in 64-row diagonal blocks with
    the updates on the matrix cores and a ragged last block; the rounds and
    the compressed nodes must match the oracle's."""
    _log("compress %s %d inc dd=%d" % (family, n, dd))
    gen, T, ot, op = problem(family, n, leaf, seed=3)
    R = inputs.gaussian_matrix(n, 1200, 1)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm",
                         d0=dd, delta_d=dd)
    oh = ocompress(op, ot, R, 1e-6, 1e-12, "inc_fnorm", d0=dd, delta_d=dd, eta=0.1)
    _compare(H, oh, ot, gen, op, T, 1e-6)
    assert H.info()["rounds"] == oh.rounds
    assert H.info()["d_final"] == oh.d
