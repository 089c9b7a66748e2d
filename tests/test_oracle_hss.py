"""Pins of the oracle's ID, stopping test, adaptive driver and matvec (CPU only)."""
import math

import numpy as np
import pytest
from scipy.linalg import qr

from oracle.hss import (COMPRESSED, FnormSide, compress, compress_fixed, fnorm_test,
                        hmt_factor, hmt_lemma_test, interpolative)
from oracle.matvec import dense_from_generators, hss_matvec, rel_error
from oracle.operators import Dense, Laplace, PermutedOperator, Toeplitz
from oracle.tree import build_tree
from paper_1810_04125_amd import inputs


# --------------------------------------------------------------------- ID
def _lowrank(m, d, r, seed, decay=None):
    rng = np.random.default_rng(seed)
    s = np.ones(r) if decay is None else decay ** np.arange(r)
    return rng.standard_normal((m, r)) @ np.diag(s) @ rng.standard_normal((r, d))


def test_id_structure_and_pivots_match_lapack():
    S = np.random.default_rng(1).standard_normal((40, 25))
    res = interpolative(S, 0.0, 0.0)
    assert res.rank == 25
    # same pivot order as LAPACK dgeqp3 on S^T (exact norms; generic matrix, no ties)
    _, _, P = qr(S.T, pivoting=True)
    assert np.array_equal(res.J, P[:25])
    U = res.basis(40)
    assert np.array_equal(U[res.J], np.eye(25))
    assert np.all(np.diff(res.pivot_norms) <= 1e-12 * res.pivot_norms[0])
    assert np.linalg.norm(S - U @ S[res.J]) <= 1e-10 * np.linalg.norm(S)


@pytest.mark.parametrize("r", [0, 1, 7, 19])
def test_id_recovers_exact_rank(r):
    S = _lowrank(60, 45, r, 7) if r else np.zeros((60, 45))
    res = interpolative(S, 1e-10, 1e-300)
    assert res.rank == r
    U = res.basis(60)
    scale = max(np.linalg.norm(S), 1.0)
    assert np.linalg.norm(S - U @ S[res.J]) <= 1e-9 * scale


def test_id_threshold_is_relative_to_first_pivot():
    S = _lowrank(50, 50, 50, 3, decay=0.5)
    for eps in (1e-2, 1e-4, 1e-6):
        res = interpolative(S, eps, 0.0)
        nu = res.pivot_norms
        assert nu[-1] > eps * nu[0]
        # the next pivot would have been below the threshold
        nxt = interpolative(S, 0.0, 0.0).pivot_norms[res.rank]
        assert nxt <= eps * nu[0]
        # absolute threshold alone
        resa = interpolative(S, 0.0, eps * nu[0])
        assert resa.rank == res.rank


def test_hmt_factor():
    # f_k = 1 + 4 sqrt(d)/(d-k-1) sqrt(min(m,n)) (eq. RRQRHMTstop)
    assert hmt_factor(74, 1, 64, 960) == pytest.approx(1 + 4 * math.sqrt(74) / 72 * 8)
    assert hmt_factor(10, 9, 5, 5) == math.inf
    assert hmt_factor(10, 8, 5, 5) == pytest.approx(1 + 4 * math.sqrt(10) * math.sqrt(5))
    S = _lowrank(64, 74, 74, 11, decay=0.7)
    plain = interpolative(S, 1e-6, 0.0)
    hmt = interpolative(S, 1e-6, 0.0, hmt_dims=(64, 960))
    assert hmt.rank >= plain.rank


# --------------------------------------------------------------------- Alg. 5 test
def test_fnorm_test_projection_and_rank_deficiency():
    rng = np.random.default_rng(4)
    F = _lowrank(80, 200, 12, 5)                   # Hankel block of rank 12
    st = FnormSide()
    S1 = F @ rng.standard_normal((200, 8))
    assert not fnorm_test(st, S1, 8, 1e-8, 0.0)    # 8 < 12: range not captured
    assert st.Q.shape == (80, 8)
    assert np.allclose(st.Q.T @ st.Q, np.eye(8), atol=1e-13)
    S2 = F @ rng.standard_normal((200, 8))
    assert fnorm_test(st, S2, 16, 1e-8, 0.0)       # 16 > 12: new block is rank deficient
    assert st.passed
    # wide samples pass at once (d >= m)
    assert fnorm_test(FnormSide(), rng.standard_normal((10, 4)), 10, 1e-8, 0.0)
    # a zero block passes
    assert fnorm_test(FnormSide(), np.zeros((30, 4)), 4, 1e-8, 0.0)


def test_hmt_lemma_test_by_hand():
    """eq. HMT_IQQH on a 4 x 2 block with Q = e1: the projected columns are
    0.1 e2 and 0.2 e3, so the statistic is alpha sqrt(2/pi) * 0.2 (the
    F-norm of the block, 0.2236, or its unprojected column norm, 1.005,
    would decide differently)."""
    e1 = np.array([[1.0], [0.0], [0.0], [0.0]])
    S = np.array([[1.0, 0.0], [0.1, 0.0], [0.0, 0.2], [0.0, 0.0]])
    c = math.sqrt(2.0 / math.pi) * 0.2
    for alpha in (1.0, 10.0):
        assert hmt_lemma_test(FnormSide(Q=e1.copy()), S, 3, alpha * c * (1 + 1e-12), alpha)
        assert hmt_lemma_test(FnormSide(Q=e1.copy()), S, 3, alpha * c, alpha)   # the bound is <=
        st = FnormSide(Q=e1.copy())
        assert not hmt_lemma_test(st, S, 3, alpha * c * (1 - 1e-9), alpha)
        # failing appends an orthonormal basis of the projected block
        assert st.Q.shape == (4, 3)
        assert np.allclose(st.Q.T @ st.Q, np.eye(3), atol=1e-14)
        assert np.allclose(np.abs(st.Q[:, 1:]), np.array([[0, 0], [1, 0], [0, 1], [0, 0]]), atol=1e-14)
    # the shortcut d >= m and an exactly rank-deficient projected block pass
    assert hmt_lemma_test(FnormSide(), S, 4, 0.0, 10.0)
    assert hmt_lemma_test(FnormSide(Q=e1.copy()), np.array([[0.0, 0.0], [0.3, 0.6], [0.0, 0.0], [0.0, 0.0]]),
                          3, 0.0, 10.0)


@pytest.mark.parametrize("seed", range(6))
def test_hmt_lemma_pass_bounds_the_spectral_error(seed):
    """Lemma 4.1: when the test passes, ||(I - QQ^T) F||_2 <= eps (failure
    probability alpha^-p = 1e-8 here); exact spectral norms by SVD."""
    rng = np.random.default_rng(100 + seed)
    m, n = 90, 300
    F = _lowrank(m, n, 40, 200 + seed, decay=0.6)
    st = FnormSide()
    eps = 1e-5 * np.linalg.norm(F, 2)
    d, passed = 0, False
    while not passed and d < m:
        S = F @ rng.standard_normal((n, 8))
        d += 8
        Q0 = st.Q
        passed = hmt_lemma_test(st, S, d, eps, 10.0)
    assert passed and d < m
    Q = Q0 if Q0 is not None else np.zeros((m, 0))
    err = np.linalg.norm(F - Q @ (Q.T @ F), 2)
    assert err <= eps
    assert Q.shape[1] >= 8   # blocks failed before the pass: the bound was exercised


# --------------------------------------------------------------------- full driver
def _toeplitz_problem(n=1024, leaf=64, h=0.1):
    T = build_tree(n, leaf)
    return T, PermutedOperator(Toeplitz(n, h), T.perm)


@pytest.mark.parametrize("strategy", ["dbl_fnorm", "inc_fnorm", "dbl_hmt"])
def test_toeplitz_reconstruction(strategy):
    T, op = _toeplitz_problem()
    R = inputs.gaussian_matrix(T.n, 512, 0)
    h = compress(op, T, R, 1e-6, 1e-12, strategy, d0=64, delta_d=64)
    assert h.converged
    err = rel_error(h, op)
    assert err <= 1e-6
    A = op.dense()
    H = dense_from_generators(h)
    assert np.linalg.norm(A - H) / np.linalg.norm(A) == pytest.approx(err, rel=1e-6)
    # symmetric operator: both sides identical
    for t, nd in enumerate(h.nodes):
        if t == 0:
            continue
        assert np.array_equal(nd.idr.J, nd.idc.J) and np.array_equal(nd.idr.E, nd.idc.E)
        if T.left[t] >= 0:
            assert np.array_equal(nd.B21, nd.B12.T)
    x = np.random.default_rng(2).standard_normal(T.n)
    assert np.linalg.norm(hss_matvec(h, x) - A @ x) <= 1e-6 * np.linalg.norm(A) * np.linalg.norm(x)


def test_hmt_overresolves_relative_to_fnorm():
    """The HMT bound gives larger ranks at the same tolerance (Table HMT)."""
    T, op = _toeplitz_problem()
    R = inputs.gaussian_matrix(T.n, 512, 0)
    a = compress(op, T, R, 1e-6, 1e-12, "dbl_fnorm", d0=64)
    b = compress(op, T, R, 1e-6, 1e-12, "dbl_hmt", d0=64)
    assert b.hss_rank() > a.hss_rank()
    assert rel_error(b, op) < rel_error(a, op)


def _planted(n, r, seed):
    U = inputs.orthonormal_columns(n, r, seed)
    V = inputs.orthonormal_columns(n, r, seed + 1)
    return np.eye(n) + U @ V.T


@pytest.mark.parametrize("strategy,r,d0,dd", [("inc_fnorm", 20, 8, 8), ("inc_fnorm", 5, 16, 16),
                                              ("dbl_fnorm", 20, 8, 0), ("dbl_hmt", 20, 8, 0),
                                              ("inc_hmt", 20, 8, 8)])
def test_planted_rank(strategy, r, d0, dd):
    """I + U V^T: every Hankel block has rank exactly r; rounds are predictable."""
    n, leaf = 512, 64
    T = build_tree(n, leaf)
    A = _planted(n, r, 40)
    op = PermutedOperator(Dense(A), T.perm)
    R = inputs.gaussian_matrix(n, 256, 9)
    # the HMT-lemma test is absolute only: rounding of the projected block
    # (about 1e-15 of its norm) must stay below atol
    atol = 1e-10 if strategy == "inc_hmt" else 1e-14
    h = compress(op, T, R, 1e-8, atol, strategy, d0=d0, delta_d=dd)
    for t in range(1, T.num_nodes):
        assert h.nodes[t].rank_r == r and h.nodes[t].rank_c == r, t
    if strategy == "inc_fnorm":
        k = 0
        while d0 + k * dd <= r:
            k += 1
        assert h.rounds == k + 1
    elif strategy == "inc_hmt":
        # no R-diagonal test: the block that completes the range still fails
        # (its projection is not small); the next one lies in the span
        k = 1
        while d0 + (k - 1) * dd < r:
            k += 1
        assert h.rounds == k + 1
    elif strategy == "dbl_fnorm":
        k = 0
        while d0 * 2 ** k <= r:
            k += 1
        assert h.rounds == k + 1
    else:
        k = 0
        while not r < d0 * 2 ** k - 10:
            k += 1
        assert h.rounds == k + 1
    assert rel_error(h, op) < 1e-12


def test_inc_hmt_ignores_rtol_and_alpha_is_monotone():
    """The HMT-lemma test has an absolute tolerance only; a larger alpha
    asks for more samples, so it never gives smaller ranks (Table HMT's
    HMT row: ranks above the F-norm test's at equal atol)."""
    T, op = _toeplitz_problem(512, 64)
    R = inputs.gaussian_matrix(T.n, 512, 3)
    kw = dict(strategy="inc_hmt", d0=16, delta_d=16)
    a = compress(op, T, R, 1e-2, 1e-8, **kw)
    b = compress(op, T, R, 1e-12, 1e-8, **kw)
    assert a.ranks() == b.ranks() and a.rounds == b.rounds
    for t in range(1, T.num_nodes):
        assert np.array_equal(a.nodes[t].idr.J, b.nodes[t].idr.J)
    lo = compress(op, T, R, 0.0, 1e-8, alpha=1.0, **kw)
    hi = compress(op, T, R, 0.0, 1e-8, alpha=100.0, **kw)
    assert hi.rounds >= lo.rounds and hi.d >= lo.d
    assert rel_error(hi, op) <= rel_error(lo, op) * (1 + 1e-9) or hi.hss_rank() >= lo.hss_rank()
    f = compress(op, T, R, 0.0, 1e-8, strategy="inc_fnorm", d0=16, delta_d=16)
    assert b.d >= f.d


def test_block_diagonal_gives_rank_zero():
    n, leaf = 256, 32
    T = build_tree(n, leaf)
    A = np.zeros((n, n))
    rng = np.random.default_rng(3)
    for t in range(T.num_nodes):
        if T.left[t] < 0:
            A[T.lo[t]:T.hi[t], T.lo[t]:T.hi[t]] = rng.standard_normal((leaf, leaf))
    op = PermutedOperator(Dense(A), T.perm)
    h = compress(op, T, inputs.gaussian_matrix(n, 64, 1), 1e-6, 1e-12, "inc_fnorm", d0=16, delta_d=16)
    assert h.rounds == 1
    assert all(a == 0 and b == 0 for a, b in h.ranks())
    assert np.array_equal(dense_from_generators(h), A)


def test_nonsymmetric_operator():
    n = 400
    pts = inputs.cube_points(n, 8)
    T = build_tree(n, 50, pts, "kd")
    lap = Laplace(pts).entries(np.arange(n), np.arange(n))
    A = lap * (1.0 + 0.3 * pts[:, 0])[:, None]       # row scaling breaks symmetry
    op = PermutedOperator(Dense(A), T.perm)
    R = inputs.gaussian_matrix(n, 400, 2)
    h = compress(op, T, R, 1e-7, 1e-14, "inc_fnorm", d0=32, delta_d=16)
    assert rel_error(h, op) <= 1e-6
    Ahat = op.dense()
    x = np.random.default_rng(5).standard_normal((n, 3))
    assert np.linalg.norm(hss_matvec(h, x) - Ahat @ x) <= 1e-5 * np.linalg.norm(Ahat @ x)
    assert np.allclose(dense_from_generators(h), hss_matvec(h, np.eye(n)), atol=1e-12)


def test_node_ranks_bracket_svd_ranks():
    """Each ID rank lies between the SVD eps-ranks of its Hankel block."""
    T, op = _toeplitz_problem(n=512, leaf=32)
    A = op.dense()
    h = compress(op, T, inputs.gaussian_matrix(T.n, 256, 0), 1e-6, 1e-14, "dbl_fnorm", d0=64)
    for t in range(1, T.num_nodes):
        lo, hi = T.lo[t], T.hi[t]
        F = np.hstack([A[lo:hi, :lo], A[lo:hi, hi:]])
        s = np.linalg.svd(F, compute_uv=False)
        eps = 1e-6 / T.level[t]
        lower = int((s > eps * s[0] * 10).sum())
        upper = int((s > eps * s[0] / 100).sum())
        assert lower <= h.nodes[t].rank_r <= upper, (t, lower, h.nodes[t].rank_r, upper)


def test_scale_invariance():
    """A(h) = A(1)/h^2: with atol off, ranks and relative error do not depend on h."""
    n = 512
    T = build_tree(n, 64)
    R = inputs.gaussian_matrix(n, 256, 0)
    out = []
    for hstep in (1.0, 0.05):
        op = PermutedOperator(Toeplitz(n, hstep), T.perm)
        hh = compress(op, T, R, 1e-6, 0.0, "dbl_fnorm", d0=64)
        out.append((hh.ranks(), rel_error(hh, op)))
    assert out[0][0] == out[1][0]
    assert out[0][1] == pytest.approx(out[1][1], rel=1e-6)


def test_dmax_forces_acceptance():
    n = 512
    T = build_tree(n, 64)
    A = _planted(n, 60, 2)
    op = PermutedOperator(Dense(A), T.perm)
    h = compress(op, T, inputs.gaussian_matrix(n, 256, 9), 1e-8, 1e-14, "inc_fnorm", d0=16,
                 delta_d=16, d_max=32)
    assert not h.converged and h.d == 32
    assert all(nd.state == COMPRESSED for nd in h.nodes)


def test_fixed_rank_compression_alg1():
    n, r = 512, 20
    T = build_tree(n, 64)
    op = PermutedOperator(Dense(_planted(n, r, 3)), T.perm)
    h = compress_fixed(op, T, inputs.gaussian_matrix(n, 64, 1), 40, 1e-8, 1e-14)
    assert h.rounds == 1 and rel_error(h, op) < 1e-12


def test_hmt_threshold_uses_the_hankel_block_sizes_hand_values():
    """Eq. RRQRHMTstop with the Hankel block sizes (#I_tau, N - #I_tau).

    S has orthogonal rows of norms 1, 0.1, 0.01, 1.7e-4, 1e-6 (m = 5 rows
    of a 20 x 30 sample, the other rows zero), so the pivot norms are exactly
    these values.  With rtol 1e-3, atol 0, d = 30 the threshold at step k is
    1e-3 / (1 + 4 sqrt(30) sqrt(min) / (29 - k)).  At k = 4:
      min = 64 (a node of 64 rows in N = 1024): 1e-3 / (1 + 175.27/25) = 1.248e-4
      min = 20 (the local sample's own 20 x 30):  1e-3 / (1 + 97.98/25)  = 2.033e-4
    so the fourth pivot (1.7e-4) is kept with the Hankel sizes (rank 4) and
    rejected with the sample sizes (rank 3); the fifth (1e-6) is below both."""
    S = np.zeros((20, 30))
    for i, s in enumerate((1.0, 0.1, 0.01, 1.7e-4, 1e-6)):
        S[3 * i, 2 * i + 1] = s
    assert interpolative(S, 1e-3, 0.0, hmt_dims=(64, 1024 - 64)).rank == 4
    assert interpolative(S, 1e-3, 0.0, hmt_dims=(20, 30)).rank == 3
    assert hmt_factor(30, 4, 64, 960) == pytest.approx(1.0 + 4.0 * math.sqrt(30.0) * 8.0 / 25.0)
    assert 1e-3 / hmt_factor(30, 4, 64, 960) == pytest.approx(1.248e-4, rel=1e-3)
    assert 1e-3 / hmt_factor(30, 4, 20, 30) == pytest.approx(2.033e-4, rel=1e-3)


def test_doubling_hmt_driver_passes_hankel_block_sizes(monkeypatch):
    """The doubling HMT strategy (Alg. 4) factors every non-root node with
    the sizes of its Hankel block A(I_tau, I \\ I_tau), not those of its
    local sample (whose rows are r1 + r2 above the leaves)."""
    import oracle.hss as H
    seen = []
    real = H.interpolative

    def spy(S, er, ea, hmt_dims=None):
        seen.append((S.shape, hmt_dims))
        return real(S, er, ea, hmt_dims=hmt_dims)

    monkeypatch.setattr(H, "interpolative", spy)
    n, leaf = 512, 64
    ot = build_tree(n, leaf)
    op = PermutedOperator(Toeplitz(n, 0.1), ot.perm)
    R = inputs.gaussian_matrix(n, 512, 3)
    H.compress(op, ot, R, 1e-6, 1e-12, "dbl_hmt", d0=64)
    assert seen
    sizes = {int(ot.hi[t] - ot.lo[t]) for t in range(1, ot.num_nodes)}
    for shape, dims in seen:
        assert dims is not None and dims[0] in sizes and dims[0] + dims[1] == n
    # above the leaves the local sample has fewer rows than the node
    assert any(shape[0] < dims[0] for shape, dims in seen)


def test_fnorm_absolute_test_divides_by_sqrt_of_the_block_width():
    """eq. stopping_criteria, absolute part: ||S_hat||_F / sqrt(b) < eps_a with
    b the width of the block under test (Sec. 3.4: E||S||_F^2 = b ||A||_F^2).
    S = [I_4; 0] (m = 16, b = 4, d = 8): ||S_hat||_F = 2, ||S_hat||_F/sqrt(b) = 1,
    every R diagonal entry 1, eps_r = 0.  Dividing by sqrt(d) (0.707) would
    pass at eps_a = 0.9; not dividing (2) would fail at eps_a = 1.5."""
    S = np.vstack([np.eye(4), np.zeros((12, 4))])
    assert fnorm_test(FnormSide(), S, 8, 0.0, 1.5)
    st = FnormSide()
    assert not fnorm_test(st, S, 8, 0.0, 0.9)
    assert st.Q.shape == (16, 4)        # a failed block joins the basis


def test_fnorm_relative_diagonal_test_uses_the_first_blocks_r11():
    """rho = |R11| of the first block QR'd on the side (the Alg. 5 choice):
    block 1 (R diagonal 10, 9) fails and sets rho = 10; block 2, orthogonal
    to it (R diagonal 1, 0.5), passes min|R_ii| = 0.5 < eps_r rho = 1.0 with
    eps_r = 0.1, where its own R11 (1) would give 0.5 < 0.1 and fail."""
    m = 12
    E = np.eye(m)
    st = FnormSide()
    S1 = np.column_stack([10.0 * E[:, 0], 9.0 * E[:, 1]])
    assert not fnorm_test(st, S1, 2, 0.1, 0.0)
    assert st.rho == pytest.approx(10.0)
    S2 = np.column_stack([1.0 * E[:, 2], 0.5 * E[:, 3]])
    assert fnorm_test(st, S2, 4, 0.1, 0.0)
    # the same block as a first block fails: its own R11 would be rho
    assert not fnorm_test(FnormSide(), S2, 2, 0.1, 0.0)


def test_fnorm_zero_diagonal_passes_with_zero_tolerances():
    """A projected block whose QR has an exactly zero diagonal entry passes
    (the block completes the range), even with eps_r = eps_a = 0; without
    the zero it fails."""
    E = np.eye(10)
    assert fnorm_test(FnormSide(), np.column_stack([E[:, 0], np.zeros(10)]), 2, 0.0, 0.0)
    assert not fnorm_test(FnormSide(), np.column_stack([E[:, 0], 1e-300 * E[:, 1]]), 2, 0.0, 0.0)


def test_first_test_replays_the_sampled_blocks_in_order(monkeypatch):
    """Reading 3: a node tested for the first time while several blocks are
    sampled runs Alg. 5 over them in sampling order, block by block with
    the schedule's widths (d = the cumulative count), and stops at the
    first pass, as if it had been tested every round.  The other reading
    (all d columns as one block) would make one call of width d."""
    import oracle.hss as H
    calls = []
    real_test, real_node = H.fnorm_test, H._Compressor.node_test_and_id
    visit = [0]

    def spy(st, S_new, d, er, ea):
        out = real_test(st, S_new, d, er, ea)
        calls.append((visit[0], id(st), S_new.shape[1], d, out))
        return out

    def node_spy(self, t, cols):
        visit[0] += 1
        return real_node(self, t, cols)

    monkeypatch.setattr(H, "fnorm_test", spy)
    monkeypatch.setattr(H._Compressor, "node_test_and_id", node_spy)
    n, leaf = 1024, 64
    ot = build_tree(n, leaf)
    op = PermutedOperator(Toeplitz(n, 0.1), ot.perm)
    R = inputs.gaussian_matrix(n, 512, 6)
    h = H.compress(op, ot, R, 1e-10, 1e-14, "inc_fnorm", d0=16, delta_d=16, d_max=512)
    sched = h.d_schedule
    widths = {c1: c1 - c0 for c0, c1 in zip([0] + sched, sched)}
    per_visit = {}
    for v, sid, b, d, out in calls:
        per_visit.setdefault((v, sid), []).append((b, d, out))
    replays = 0
    for seq in per_visit.values():
        ds = [d for _, d, _ in seq]
        assert ds == sorted(ds)                         # sampling order
        assert all(widths[d] == b for b, d, _ in seq)   # one sampled block per call
        assert all(not out for _, _, out in seq[:-1])   # nothing after a pass
        if len(seq) > 1:
            assert ds[0] == sched[0]                    # a replay starts at the first block
            replays += 1
    assert replays > 0
