"""HSS factorization and solve on the GPU (hss_factor / hss_solve).

Up to 16 right-hand sides the solve runs fused per-level substitutions,
above that one launch per block step; both paths are checked.

The expected solutions come from the oracle's side only: a dense solve of
the operator's entries (oracle/operators.py), which the solve of the
compressed matrix must match within kappa(A) times the compression
tolerance, and the factorization's own exactness, the residual against the
compressed H through hss_matvec (itself held to the oracle's matvec in
test_gpu_parity.py).  The oracle's factorization (oracle/ulv.py) is pinned
against dense solves in test_oracle_ulv.py.
"""
import numpy as np
import pytest

from paper_1810_04125_amd import hss, inputs
from tests.gpu_util import dev_colmajor, problem

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _dense_solve(op, perm, B):
    X = np.empty_like(B)
    X[perm] = np.linalg.solve(op.dense(), B[perm])
    return X


@pytest.mark.parametrize("family,n,leaf", [("laplace", 1536, 64), ("gauss", 1536, 64), ("toeplitz", 2048, 64)])
def test_solve_matches_dense_solve(family, n, leaf):
    _log("ulv %s n=%d" % (family, n))
    gen, T, ot, op = problem(family, n, leaf, seed=5)
    rtol = 1e-10
    H, st = hss.compress(gen, T, rtol=rtol, atol=1e-300, eta=0.05, strategy="dbl_fnorm", d0=64, seed=1)
    H.factor()
    B = inputs.gaussian_matrix(n, 3, 11)
    Bd = dev_colmajor(B)
    X = H.solve(Bd)
    # exact for H: the residual through the compressed matrix
    R = (H.matvec(X) - Bd).cpu().numpy()
    assert np.linalg.norm(R) <= 1e-10 * np.linalg.norm(B), np.linalg.norm(R) / np.linalg.norm(B)
    # and for A within kappa(A) times the compression error
    Xh = X.cpu().numpy()
    Xd = _dense_solve(op, np.asarray(T.perm), B)
    kappa = np.linalg.cond(op.dense())
    rel = np.linalg.norm(Xh - Xd) / np.linalg.norm(Xd)
    _log("  kappa %.2e  rel %.2e" % (kappa, rel))
    assert rel <= max(1e-12, 20.0 * kappa * rtol)
    # more right-hand sides than the fused substitutions take: the block-step
    # GEMM path, the same solution column by column
    B20 = inputs.gaussian_matrix(n, 20, 12)
    B20[:, :3] = B
    X20 = H.solve(dev_colmajor(B20))
    R20 = (H.matvec(X20) - dev_colmajor(B20)).cpu().numpy()
    assert np.linalg.norm(R20) <= 1e-10 * np.linalg.norm(B20)
    assert np.allclose(X20.cpu().numpy()[:, :3], Xh, rtol=0, atol=1e-11 * np.abs(Xh).max())


def test_root_leaf_single_rhs_and_call_order():
    n = 100   # the root is a leaf: the whole matrix is one dense block
    gen, T, ot, op = problem("laplace", n, 128, seed=2)
    H, st = hss.compress(gen, T, rtol=1e-6, atol=1e-12, strategy="dbl_fnorm", d0=64, seed=1)
    b = inputs.gaussian_matrix(n, 1, 3)[:, 0]
    with pytest.raises(hss.HSSError, match="not factored"):
        H.solve(dev_colmajor(b[:, None]))
    H.factor()
    H.factor()   # a second call keeps the factor
    x = H.solve(dev_colmajor(b[:, None])[:, 0]).cpu().numpy()
    xd = _dense_solve(op, np.asarray(T.perm), b[:, None])[:, 0]
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd) * np.linalg.cond(op.dense())


def test_full_size_bench_workload_residuals():
    # sphere-Laplace n = 32768 at the bench's settings: the residual through
    # H, and sampled rows of A (entries from the oracle's operator)
    n = 32768
    _log("ulv laplace n=%d" % n)
    gen, T, ot, op = problem("laplace", n, 128, seed=0)
    H, st = hss.compress(gen, T, rtol=1e-6, atol=1e-12, eta=0.05, strategy="inc_fnorm", d0=128, delta_d=64,
                         d_max=4096, seed=0)
    H.factor()
    B = inputs.gaussian_matrix(n, 2, 13)
    Bd = dev_colmajor(B)
    X = H.solve(Bd)
    R = (H.matvec(X) - Bd).cpu().numpy()
    _log("  residual through H %.2e" % (np.linalg.norm(R) / np.linalg.norm(B)))
    assert np.linalg.norm(R) <= 1e-8 * np.linalg.norm(B)
    Xh = X.cpu().numpy()
    perm = np.asarray(T.perm)
    rows = np.random.default_rng(3).integers(0, n, 12)
    Arows = op.extract(rows, np.arange(n))           # permuted rows of A
    res = Arows @ Xh[perm] - B[perm][rows]
    scale = np.linalg.norm(Arows, axis=1)[:, None] * np.linalg.norm(Xh, axis=0)[None, :]
    _log("  sampled rows of A x - b: %.2e" % (np.abs(res) / scale).max())
    assert (np.abs(res) / scale).max() <= 1e-5
