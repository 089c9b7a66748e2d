"""Adaptive randomized HSS compression (oracle, FP64 numpy/scipy).

Written from arXiv 1810.04125:
  * Sec. 2.2 eqs. (sample_off_diag) .. (definition_of_tauSr): Hankel-block
    samples, the interpolative decomposition (ID) via QR with column
    pivoting, nested samples tau.S and reduced random matrices tau.R;
  * Alg. 1 (non-adaptive compression) and Alg. 2 (ComputeLocalSamples /
    ReduceLocalSamples);
  * Alg. 3 (HSSCompressAdaptive / CompressNodeAdaptive) with the node
    states UNTOUCHED / PARTIALLY_COMPRESSED / COMPRESSED;
  * Alg. 4 (doubling + RRQR_HMT, eq. RRQRHMTstop) and Alg. 5
    (incrementing + block Gram-Schmidt, eq. stopping_criteria).

Readings of points the paper leaves open (the HIP path uses the same):
  * tolerances are scaled per node as eta*eps/level(tau) (Sec. 2.2 text
    after the compression-stages figure; Alg. 1 and 3); eta is a global
    safety factor, 1 = the paper's literal rule;
  * new columns are the b most recently appended; an UNTOUCHED node
    computes all d columns (Alg. 3 column ranges);
  * a node that meets the stopping test for the first time, with several
    sampled blocks already available, runs Alg. 5 over those blocks in the
    order they were sampled (block widths = the sampling schedule) and
    stops at the first pass, as if it had been tested since the first
    round; an already tested node tests only the newest block;
  * the absolute F-norm test divides by sqrt(b), b = width of the new
    block (E||S||_F^2 = b ||A||_F^2, Sec. 3.4);
  * a side whose local sample has m <= d rows passes (the samples span
    its whole local range with probability one);
  * rho = |Rbar_11| of the first QR'd block (Alg. 5);
  * a zero new block (||S_new||_F = 0) passes, and so does a projected
    block whose QR has an exactly zero diagonal entry;
  * the doubling strategy grows the sample by b = d (Alg. 3 "double"),
    the HMT test accepts iff r < d - p or r = m (Alg. 4, p counted
    inside d), with min(m,n) taken from the Hankel block sizes
    #I_tau and N - #I_tau;
  * pivot ties go to the lowest row index; residual norms are recomputed
    exactly at every step (no downdating);
  * ID stops at the first pivot with norm <= threshold (eq. RRQRHMTstop
    uses <=); the F-norm tests use strict < (eq. stopping_criteria);
  * the HMT-lemma test (eq. HMT_IQQH, strategy inc_hmt) takes the columns
    of the block under test as the Gaussian vectors omega_i (p = block
    width) and the projection (I - QQ^T) of Alg. 5 with the basis Q of the
    blocks tested before; it passes iff alpha sqrt(2/pi) max_i ||.||_2 <=
    eps_a (the paper's <=).  It has no relative tolerance: eps_r = 0 in
    the test and in the ID.  A projected block whose QR has an exactly
    zero diagonal entry passes, as in the F-norm test.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

UNTOUCHED, PARTIALLY_COMPRESSED, COMPRESSED = 0, 1, 2

STRATEGIES = ("dbl_fnorm", "inc_fnorm", "dbl_hmt", "inc_hmt")


# ---------------------------------------------------------------------------
# Interpolative decomposition by QR with column pivoting (eqs. ID, QRCPSr)
# ---------------------------------------------------------------------------

@dataclass
class IDResult:
    rank: int
    J: np.ndarray        # selected rows of S, in pivot order
    rest: np.ndarray     # the other rows, ascending
    E: np.ndarray        # rank x (m - rank): S(rest,:) ~= E^T S(J,:)
    pivot_norms: np.ndarray  # |R_kk| of the accepted pivots

    def basis(self, m: int) -> np.ndarray:
        """U with U(J,:) = I, U(rest,:) = E^T (Sec. 2.2, definition of U_tau)."""
        U = np.zeros((m, self.rank))
        U[self.J, np.arange(self.rank)] = 1.0
        if len(self.rest):
            U[self.rest, :] = self.E.T
        return U


def hmt_factor(d: int, k: int, m_block: int, n_block: int) -> float:
    """Deviation factor of eq. (RRQRHMTstop) at (1-based) step k with d columns."""
    over = d - k - 1
    if over <= 0:
        return math.inf
    return 1.0 + 4.0 * math.sqrt(d) / over * math.sqrt(min(m_block, n_block))


def interpolative(S: np.ndarray, eps_r: float, eps_a: float,
                  hmt_dims: tuple[int, int] | None = None) -> IDResult:
    """ID of the rows of S (m x d): QRCP of S^T with threshold stopping.

    Step k selects the remaining column of S^T (row of S) with the largest
    residual norm nu_k = |R_kk|; it stops before accepting it when
    nu_k <= max(eps_a, eps_r * nu_1) (divided by the HMT factor when
    hmt_dims = (#I_tau, N - #I_tau) is given, Alg. 4).
    """
    m, d = S.shape
    A = np.array(S.T, dtype=np.float64, copy=True)   # d x m, columns = rows of S
    remaining = list(range(m))
    piv: list[int] = []
    norms: list[float] = []
    nu1 = None
    Rcols = {}
    for k in range(min(m, d)):
        res = np.linalg.norm(A[k:, remaining], axis=0)
        pos = int(np.argmax(res))          # first maximum = lowest row index
        nu = float(res[pos])
        if nu1 is None:
            nu1 = nu
        thr = max(eps_a, eps_r * nu1)
        if hmt_dims is not None:
            thr = thr / hmt_factor(d, k + 1, hmt_dims[0], hmt_dims[1])
        if nu <= thr:
            break
        p = remaining.pop(pos)
        # Householder reflector mapping A[k:, p] to alpha e_1
        x = A[k:, p].copy()
        alpha = -math.copysign(nu, x[0]) if x[0] != 0 else -nu
        v = x
        v[0] -= alpha
        vtv = float(v @ v)
        A[k:, p] = 0.0
        A[k, p] = alpha
        if vtv > 0 and remaining:
            W = A[k:, remaining]
            A[k:, remaining] = W - np.outer(v, (2.0 / vtv) * (v @ W))
        piv.append(p)
        norms.append(nu)
        Rcols[p] = A[:k + 1, p].copy()
    r = len(piv)
    rest = np.array(sorted(remaining), dtype=np.int64)
    J = np.array(piv, dtype=np.int64)
    if r == 0:
        E = np.zeros((0, len(rest)))
    else:
        R1 = np.zeros((r, r))
        for k, p in enumerate(piv):
            R1[:k + 1, k] = Rcols[p]
        R2 = A[:r, rest] if len(rest) else np.zeros((r, 0))
        E = solve_triangular(R1, R2, lower=False) if len(rest) else np.zeros((r, 0))
    return IDResult(r, J, rest, E, np.array(norms))


# ---------------------------------------------------------------------------
# Node stopping test, incrementing/doubling with block Gram-Schmidt
# (Alg. 5, eq. stopping_criteria)
# ---------------------------------------------------------------------------

@dataclass
class FnormSide:
    Q: np.ndarray | None = None   # orthonormal basis grown block by block
    rho: float | None = None
    passed: bool = False


def fnorm_test(st: FnormSide, S_new: np.ndarray, d: int, eps_r: float, eps_a: float) -> bool:
    if st.passed:
        return True
    m, b = S_new.shape
    if d >= m:
        st.passed = True
        return True
    Q = st.Q if st.Q is not None else np.zeros((m, 0))
    Sh = S_new - Q @ (Q.T @ S_new)          # block Gram-Schmidt, twice
    Sh = Sh - Q @ (Q.T @ Sh)
    nS = float(np.linalg.norm(S_new))
    nSh = float(np.linalg.norm(Sh))
    if nS == 0.0 or nSh < eps_r * nS or nSh / math.sqrt(b) < eps_a:
        st.passed = True
        return True
    Qk, Rk = np.linalg.qr(Sh, mode="reduced")
    dg = np.abs(np.diag(Rk))
    if st.rho is None:
        st.rho = float(dg[0])
    mn = float(dg.min())
    if mn == 0.0 or mn < eps_a or mn < eps_r * st.rho:
        st.passed = True
        return True
    st.Q = np.hstack([Q, Qk])
    return False


def hmt_lemma_test(st: FnormSide, S_new: np.ndarray, d: int, eps_a: float, alpha: float) -> bool:
    """Stopping test of eq. HMT_IQQH: by Lemma 4.1 of Halko, Martinsson and
    Tropp, ||(I - QQ^T) F||_2 <= alpha sqrt(2/pi) max_i ||(I - QQ^T) F w_i||_2
    except with probability alpha^-p.  The columns of S_new are the samples
    F w_i of the block's p = b Gaussian vectors; Q is the orthonormal basis
    of the blocks tested before (Alg. 5 bookkeeping)."""
    if st.passed:
        return True
    m, b = S_new.shape
    if d >= m:
        st.passed = True
        return True
    Q = st.Q if st.Q is not None else np.zeros((m, 0))
    Sh = S_new - Q @ (Q.T @ S_new)          # block Gram-Schmidt, twice
    Sh = Sh - Q @ (Q.T @ Sh)
    worst = float(np.max(np.linalg.norm(Sh, axis=0))) if b > 0 else 0.0
    if alpha * math.sqrt(2.0 / math.pi) * worst <= eps_a:
        st.passed = True
        return True
    Qk, Rk = np.linalg.qr(Sh, mode="reduced")
    if float(np.abs(np.diag(Rk)).min()) == 0.0:
        st.passed = True
        return True
    # Columns of S_hat at rounding level (the block is numerically rank
    # deficient) give directions of Qk that are not orthogonal to Q after
    # normalisation; Gram-Schmidt against Q twice more and a second QR keep
    # [Q Qk] orthonormal (such directions are then arbitrary but harmless).
    Qk = Qk - Q @ (Q.T @ Qk)
    Qk = Qk - Q @ (Q.T @ Qk)
    Qk, _ = np.linalg.qr(Qk, mode="reduced")
    st.Q = np.hstack([Q, Qk])
    return False


# ---------------------------------------------------------------------------
# HSS node payload and the adaptive driver (Alg. 2, Alg. 3)
# ---------------------------------------------------------------------------

@dataclass
class Node:
    state: int = UNTOUCHED
    D: np.ndarray | None = None
    B12: np.ndarray | None = None
    B21: np.ndarray | None = None
    Sr: np.ndarray | None = None   # local samples, m_r x d
    Sc: np.ndarray | None = None
    Rr: np.ndarray | None = None   # reduced random matrices V^T R(I_tau) (nested)
    Rc: np.ndarray | None = None   # U^T R(I_tau) (nested)
    idr: IDResult | None = None
    idc: IDResult | None = None
    Ir: np.ndarray | None = None   # skeleton row indices (permuted, global)
    Ic: np.ndarray | None = None
    tr: FnormSide = field(default_factory=FnormSide)
    tc: FnormSide = field(default_factory=FnormSide)

    @property
    def rank_r(self) -> int:
        return self.idr.rank if self.idr is not None else 0

    @property
    def rank_c(self) -> int:
        return self.idc.rank if self.idc is not None else 0


@dataclass
class HSS:
    tree: object
    nodes: list
    d: int
    rounds: int
    d_schedule: list
    converged: bool
    eta: float
    strategy: str

    def ranks(self):
        return [(n.rank_r, n.rank_c) for n in self.nodes]

    def hss_rank(self) -> int:
        return max(max(a, b) for a, b in self.ranks())


class _Compressor:
    def __init__(self, op, tree, R, rtol, atol, strategy, d0, delta_d, p, d_max, eta, alpha=10.0):
        if strategy not in STRATEGIES:
            raise ValueError("strategy must be one of %s" % (STRATEGIES,))
        self.op, self.tree, self.Rall = op, tree, R
        self.rtol, self.atol, self.strategy = rtol, atol, strategy
        self.d0, self.delta_d, self.p, self.eta = d0, delta_d, p, eta
        self.alpha = alpha
        self.N = tree.n
        self.d_max = min(d_max if d_max is not None else self.N, R.shape[1])
        self.nodes = [Node() for _ in range(tree.num_nodes)]
        self.force = False
        self.sched = []   # d after every sampling step (the block edges)

    # -- global samples --------------------------------------------------
    def append_columns(self, b: int):
        Rnew = np.asarray(self.Rall[:, self.d:self.d + b], dtype=np.float64)
        Sr, Sc = self.op.sample(Rnew)
        self.R = np.hstack([self.R, Rnew])
        self.Sr = np.hstack([self.Sr, Sr])
        self.Sc = np.hstack([self.Sc, Sc])
        self.d += b
        self.sched.append(self.d)

    def eps(self, t: int):
        lev = int(self.tree.level[t])
        er = 0.0 if self.strategy == "inc_hmt" else self.eta * self.rtol / lev   # absolute only
        return er, self.eta * self.atol / lev

    # -- Alg. 2 ComputeLocalSamples -------------------------------------
    def local_samples(self, t: int, cols: np.ndarray):
        T, nd = self.tree, self.nodes[t]
        if T.is_leaf(t):
            I = np.arange(T.lo[t], T.hi[t])
            Rl = self.R[np.ix_(I, cols)]
            sr = self.Sr[np.ix_(I, cols)] - nd.D @ Rl
            sc = self.Sc[np.ix_(I, cols)] - nd.D.T @ Rl
        else:
            a, b = self.nodes[T.left[t]], self.nodes[T.right[t]]
            sr = np.vstack([a.Sr[np.ix_(a.idr.J, cols)] - nd.B12 @ b.Rr[:, cols],
                            b.Sr[np.ix_(b.idr.J, cols)] - nd.B21 @ a.Rr[:, cols]])
            sc = np.vstack([a.Sc[np.ix_(a.idc.J, cols)] - nd.B21.T @ b.Rc[:, cols],
                            b.Sc[np.ix_(b.idc.J, cols)] - nd.B12.T @ a.Rc[:, cols]])
        if nd.Sr is None:
            nd.Sr, nd.Sc = sr, sc
        else:
            nd.Sr = np.hstack([nd.Sr, sr])
            nd.Sc = np.hstack([nd.Sc, sc])

    # -- Alg. 2 ReduceLocalSamples --------------------------------------
    @staticmethod
    def _apply_basis_t(idres: IDResult, X: np.ndarray) -> np.ndarray:
        """U^T X = X(J,:) + E X(rest,:) for U = Pi [I; E^T]."""
        out = X[idres.J, :].copy()
        if len(idres.rest) and idres.rank:
            out += idres.E @ X[idres.rest, :]
        return out

    def reduce(self, t: int, cols: np.ndarray):
        T, nd = self.tree, self.nodes[t]
        if T.is_leaf(t):
            I = np.arange(T.lo[t], T.hi[t])
            X = self.R[np.ix_(I, cols)]
            rr = self._apply_basis_t(nd.idc, X)
            rc = self._apply_basis_t(nd.idr, X)
            if nd.Ir is None:
                nd.Ic = I[nd.idc.J]
                nd.Ir = I[nd.idr.J]
        else:
            a, b = self.nodes[T.left[t]], self.nodes[T.right[t]]
            rr = self._apply_basis_t(nd.idc, np.vstack([a.Rr[:, cols], b.Rr[:, cols]]))
            rc = self._apply_basis_t(nd.idr, np.vstack([a.Rc[:, cols], b.Rc[:, cols]]))
            if nd.Ir is None:
                nd.Ir = np.concatenate([a.Ir, b.Ir])[nd.idr.J]
                nd.Ic = np.concatenate([a.Ic, b.Ic])[nd.idc.J]
        if nd.Rr is None:
            nd.Rr, nd.Rc = rr, rc
        else:
            nd.Rr = np.hstack([nd.Rr, rr])
            nd.Rc = np.hstack([nd.Rc, rc])

    # -- node test ---------------------------------------------------------
    def node_test_and_id(self, t: int, cols: np.ndarray) -> bool:
        nd = self.nodes[t]
        er, ea = self.eps(t)
        if self.strategy == "dbl_hmt":
            size = self.tree.size(t)
            dims = (size, self.N - size)
            idr = interpolative(nd.Sr, er, ea, hmt_dims=dims)
            idc = interpolative(nd.Sc, er, ea, hmt_dims=dims)
            ok = all(res.rank < self.d - self.p or res.rank == S.shape[0]
                     for res, S in ((idr, nd.Sr), (idc, nd.Sc)))
            if ok or self.force:
                nd.idr, nd.idc = idr, idc
                return True
            return False
        if nd.state == UNTOUCHED:
            edges = [0] + self.sched
            blocks = [(edges[i], edges[i + 1]) for i in range(len(self.sched))]
        else:
            blocks = [(self.d - len(cols), self.d)]
        ok = []
        for S, st in ((nd.Sr, nd.tr), (nd.Sc, nd.tc)):
            passed = st.passed
            for c0, c1 in blocks:
                if passed or c1 <= c0:
                    break
                if self.strategy == "inc_hmt":
                    passed = hmt_lemma_test(st, S[:, c0:c1], c1, ea, self.alpha)
                else:
                    passed = fnorm_test(st, S[:, c0:c1], c1, er, ea)
            ok.append(passed)
        if all(ok) or self.force:
            nd.idr = interpolative(nd.Sr, er, ea)
            nd.idc = interpolative(nd.Sc, er, ea)
            return True
        return False

    # -- Alg. 3 CompressNodeAdaptive ---------------------------------------
    def compress_node(self, t: int, b: int):
        T, nd = self.tree, self.nodes[t]
        if T.is_leaf(t):
            if nd.state == UNTOUCHED:
                I = np.arange(T.lo[t], T.hi[t])
                nd.D = self.op.extract(I, I)
        else:
            l, r = T.left[t], T.right[t]
            self.compress_node(l, b)
            self.compress_node(r, b)
            a, c = self.nodes[l], self.nodes[r]
            if a.state != COMPRESSED or c.state != COMPRESSED:
                return
            if nd.state == UNTOUCHED:
                nd.B12 = self.op.extract(a.Ir, c.Ic)
                nd.B21 = self.op.extract(c.Ir, a.Ic)
        if T.parent[t] < 0:
            nd.state = COMPRESSED
            return
        if nd.state == UNTOUCHED:
            cols = np.arange(0, self.d)
        else:
            cols = np.arange(self.d - b, self.d)
        self.local_samples(t, cols)
        if nd.state != COMPRESSED:
            if self.node_test_and_id(t, cols):
                nd.state = COMPRESSED
                self.reduce(t, np.arange(0, self.d))
            else:
                nd.state = PARTIALLY_COMPRESSED
        else:
            self.reduce(t, cols)

    # -- Alg. 3 HSSCompressAdaptive ----------------------------------------
    def run(self) -> HSS:
        self.d = 0
        self.R = np.zeros((self.N, 0))
        self.Sr = np.zeros((self.N, 0))
        self.Sc = np.zeros((self.N, 0))
        d0 = min(self.d0, self.d_max)
        self.append_columns(d0)
        b = d0
        rounds = 0
        root = 0
        while True:
            rounds += 1
            self.compress_node(root, b)
            if self.nodes[root].state == COMPRESSED:
                break
            if self.d >= self.d_max:
                if self.force:
                    raise RuntimeError("forced round did not compress the root")
                self.force = True
                b = 0
                continue
            b = self.d if self.strategy.startswith("dbl") else self.delta_d
            b = min(b, self.d_max - self.d)
            self.append_columns(b)
        return HSS(self.tree, self.nodes, self.d, rounds, list(self.sched),
                   not self.force, self.eta, self.strategy)


def compress(op, tree, R, rtol=1e-6, atol=1e-12, strategy="dbl_fnorm", d0=64,
             delta_d=64, p=10, d_max=None, eta=1.0, alpha=10.0) -> HSS:
    """Adaptive HSS compression of the permuted operator `op` (Alg. 3).

    R is the N x d_cap Gaussian matrix (rows in permuted order); its
    columns are consumed in order, so d never exceeds d_cap.  `alpha` is
    the factor of the HMT-lemma test (strategy inc_hmt).
    """
    return _Compressor(op, tree, np.asarray(R), rtol, atol, strategy, d0,
                       delta_d, p, d_max, eta, alpha).run()


def compress_fixed(op, tree, R, d, rtol=1e-6, atol=1e-12, eta=1.0) -> HSS:
    """Non-adaptive compression at a fixed sample count d (Alg. 1)."""
    return _Compressor(op, tree, np.asarray(R), rtol, atol, "dbl_fnorm", d, d,
                       10, d, eta)._run_fixed()


def _run_fixed(self) -> HSS:
    self.d = 0
    self.R = np.zeros((self.N, 0))
    self.Sr = np.zeros((self.N, 0))
    self.Sc = np.zeros((self.N, 0))
    self.append_columns(self.d0)
    self.force = True   # Alg. 1 has no test: every node is compressed at once
    self.compress_node(0, self.d)
    return HSS(self.tree, self.nodes, self.d, 1, [self.d], True, self.eta, "fixed")


_Compressor._run_fixed = _run_fixed
