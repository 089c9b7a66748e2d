"""Pins of the oracle's cluster tree and operator families (CPU only)."""
import math
import os

import numpy as np
import pytest
from scipy.linalg import matmul_toeplitz

from oracle.operators import Dense, Gauss, Laplace, PermutedOperator, Toeplitz
from oracle.tree import build_tree
from paper_1810_04125_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_tree_matches_paper_figure():
    """BFS numbering of the 4-level example tree (Sec. 2.1, tree figure)."""
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLDEN, "fig_hss_tree.txt"))
            if l.strip() and not l.startswith("#")]
    leaf = 16
    T = build_tree(8 * leaf, leaf)
    assert T.num_nodes == len(rows)
    for node, parent, left, right, level in rows:
        assert (T.parent[node], T.left[node], T.right[node], T.level[node]) == (parent, left, right, level)
    # leaves 7..14 own consecutive blocks top to bottom
    for k, t in enumerate(range(7, 15)):
        assert (T.lo[t], T.hi[t]) == (k * leaf, (k + 1) * leaf)
    assert np.array_equal(T.perm, np.arange(8 * leaf))


@pytest.mark.parametrize("method,n,leaf", [("bisect", 1000, 64), ("rcb", 777, 50), ("kd", 1024, 128),
                                           ("rcb", 257, 128)])
def test_tree_invariants(method, n, leaf):
    pts = inputs.sphere_points(n, 5) if method != "kd" else inputs.cube_points(n, 6)
    T = build_tree(n, leaf, None if method == "bisect" else pts, method)
    assert sorted(T.perm.tolist()) == list(range(n))
    assert (T.lo[0], T.hi[0]) == (0, n)
    for t in range(T.num_nodes):
        m = T.hi[t] - T.lo[t]
        if T.left[t] < 0:
            assert 1 <= m <= leaf
            seg = T.perm[T.lo[t]:T.hi[t]]
            assert np.all(np.diff(seg) > 0), "leaf members sorted by original index"
            continue
        l, r = T.left[t], T.right[t]
        assert m > leaf
        assert T.lo[l] == T.lo[t] and T.hi[l] == T.lo[r] and T.hi[r] == T.hi[t]
        assert T.hi[l] - T.lo[l] == m // 2
        assert T.parent[l] == t and T.parent[r] == t
        assert T.level[l] == T.level[t] + 1
        if method != "bisect":
            idx = T.perm[T.lo[t]:T.hi[t]]
            sub = pts[idx]
            if method == "rcb":
                ext = sub.max(axis=0) - sub.min(axis=0)
                axis = int(np.argmax(ext))
            else:
                axis = int(T.level[t]) % 3
            a = pts[T.perm[T.lo[l]:T.hi[l]], axis]
            b = pts[T.perm[T.lo[r]:T.hi[r]], axis]
            assert a.max() <= b.min()
    # BFS numbering: levels non-decreasing with the node number
    assert np.all(np.diff(T.level) >= 0)


def test_toeplitz_entries_and_norm():
    """t(0)=pi^2/(6h^2), t(k)=(-1)^k/(k^2 h^2); ||A||_F^2 closed form."""
    n, h = 1024, 0.1
    op = Toeplitz(n, h)
    A = op.entries(np.arange(n), np.arange(n))
    assert A[0, 0] == pytest.approx(math.pi ** 2 / 6 / h ** 2, rel=1e-15)
    assert A[3, 5] == pytest.approx(1 / (4 * h * h), rel=1e-15)
    assert A[7, 4] == pytest.approx(-1 / (9 * h * h), rel=1e-15)
    t0 = math.pi ** 2 / (6 * h * h)
    fro2 = n * t0 ** 2 + 2 * sum((n - k) / (k ** 4 * h ** 4) for k in range(1, n))
    assert np.linalg.norm(A) ** 2 == pytest.approx(fro2, rel=1e-12)
    assert math.sqrt(fro2) == pytest.approx(7060.41, abs=0.01)
    # symbol theta^2/(2h^2): SPD with spectrum inside (0, pi^2/(2h^2))
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0 and ev.max() < math.pi ** 2 / (2 * h * h)


def test_toeplitz_sampling_matches_fft_product():
    n, h = 1500, 0.2
    T = build_tree(n, 64)
    op = PermutedOperator(Toeplitz(n, h), T.perm, block=256)
    R = inputs.gaussian_matrix(n, 7, 3)
    Sr, Sc = op.sample(R)
    t = Toeplitz(n, h).t
    ref = matmul_toeplitz((t, t), R)
    assert np.linalg.norm(Sr - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.array_equal(Sr, Sc)


def test_kernel_entries_brute_force():
    pts = inputs.sphere_points(20, 9)
    lap = Laplace(pts)
    gau = Gauss(pts, sigma=0.5, diag=1e-2)
    I = np.array([0, 3, 7, 19])
    J = np.array([3, 2, 19, 11, 0])
    L, G = lap.entries(I, J), gau.entries(I, J)
    for a, i in enumerate(I):
        for b, j in enumerate(J):
            dx = [pts[i][k] - pts[j][k] for k in range(3)]
            r = math.sqrt(sum(x * x for x in dx))
            lv = 1.0 if i == j else 1.0 / (4 * math.pi * r)
            gv = math.exp(-r * r / 0.5) + (1e-2 if i == j else 0.0)
            assert L[a, b] == pytest.approx(lv, rel=1e-14)
            assert G[a, b] == pytest.approx(gv, rel=1e-14)


def test_permuted_operator_and_transpose_sampling():
    n = 300
    pts = inputs.cube_points(n, 4)
    T = build_tree(n, 40, pts, "kd")
    a = inputs.gaussian_matrix(n, n, 12)        # non-symmetric dense operator
    op = PermutedOperator(Dense(a), T.perm, block=64)
    Ahat = a[np.ix_(T.perm, T.perm)]
    assert np.array_equal(op.dense(), Ahat)
    R = inputs.gaussian_matrix(n, 5, 13)
    Sr, Sc = op.sample(R)
    assert np.allclose(Sr, Ahat @ R, rtol=0, atol=1e-12)
    assert np.allclose(Sc, Ahat.T @ R, rtol=0, atol=1e-12)


def test_frobenius_estimator_identity():
    """E ||A R||_F^2 / d = ||A||_F^2 (Sec. 3.4); check the sample mean."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 30)) @ np.diag(0.7 ** np.arange(30)) @ rng.standard_normal((30, 50))
    fro2 = np.linalg.norm(A) ** 2
    d, trials = 8, 2000
    vals = []
    for s in range(trials):
        R = inputs.gaussian_matrix(50, d, 100 + s)
        vals.append(np.linalg.norm(A @ R) ** 2 / d)
    vals = np.array(vals)
    # Var(||Ax||^2) = 2 sum sigma^4; the mean of `trials` averages has sd below
    sig = np.linalg.svd(A, compute_uv=False)
    sd = math.sqrt(2 * (sig ** 4).sum() / d / trials)
    assert abs(vals.mean() - fro2) < 5 * sd
