"""Direct factorization and solve of a compressed HSS matrix (oracle).

Test infrastructure: only the tests, the package's smoke check and the
bench's CPU baseline use this module.

The paper reports ULV factorization and solve times of its compressed
matrices (table sixdrivers) without giving the algorithm; this is the
factorization that the interpolative bases of Sec. 2.2 lead to directly.
Every non-root node tau has a row basis U_tau = Pi_r [I; E_r^T] and a
column basis V_tau = Pi_c [I; E_c^T] (skeleton rows get I, the other rows
E^T).  In the order [redundant R; skeleton S] of tau's local rows
(columns),

    T_r = [[I, -E_r^T], [0, I]]   maps   U_tau  to  [0; I],

and T_c likewise maps V_tau, so after T_r on the rows and T_c^T on the
columns the redundant rows and columns of tau couple only to tau's own
local block.  With D' the local block in those orders (the leaf's D, or
above the leaves the children's skeleton Schur complements joined by B12
and B21, eq. HSSexamplematrix),

    Dhat = T_r D' T_c^T:  Dhat_RR = D'_RR - E_r^T D'_SR - D'_RS E_c + E_r^T D'_SS E_c
                          Dhat_RS = D'_RS - E_r^T D'_SS,  Dhat_SR = D'_SR - D'_SS E_c
                          Dhat_SS = D'_SS,

and eliminating the redundant unknowns leaves on the skeleton the Schur
complement S_tau = Dhat_SS - Dhat_SR Dhat_RR^{-1} Dhat_RS, which is the
parent's diagonal block for tau's skeleton (the parent's local block is
[[S_nu1, B12], [B21, S_nu2]]).  The root's local block is factored whole.
Dhat_RR must be square: every node needs equal row and column ranks.  It
is factored by LU with partial pivoting (the sphere-Laplace matrices are
symmetric but indefinite).

The solve runs the row transforms on the right-hand side bottom-up (the
skeleton part of each node's reduced right-hand side goes to its parent),
solves at the root, and recovers the redundant unknowns top-down:
x_R = Dhat_RR^{-1}(bhat_R - Dhat_RS x_S), then x = T_c^T xhat.

Pins (tests/test_oracle_ulv.py): the solution equals a dense solve of H
rebuilt from the generators by `matvec.dense_from_generators`, and
T U = [0; I] on every node.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import lu_factor, lu_solve


def _order(idr):
    """Local rows in [redundant; skeleton] order and the number redundant."""
    return np.concatenate([idr.rest, idr.J]).astype(np.int64), len(idr.rest)


def transform(ids, m: int) -> np.ndarray:
    """T in [R; S] order (rows R <- R - E^T S) for one side's ID."""
    k = len(ids.rest)
    T = np.eye(m)
    T[:k, k:] = -ids.E.T
    return T


def _check_ranks(h):
    for t, nd in enumerate(h.nodes):
        if h.tree.parent[t] >= 0 and nd.idr.rank != nd.idc.rank:
            raise ValueError("node %d: row rank %d, column rank %d; the factorization needs equal ranks"
                             % (t, nd.idr.rank, nd.idc.rank))


def factor(h):
    """Per node: the [R;S] row and column orders, E_r, E_c, the LU of
    Dhat_RR, Dhat_SR, Dhat_RS and S_tau (the root: the LU of its whole
    local block)."""
    _check_ranks(h)
    T, nodes = h.tree, h.nodes
    fac = [None] * T.num_nodes
    for t in sorted(range(T.num_nodes), key=lambda v: -int(T.level[v])):   # deepest first
        nd = nodes[t]
        if T.is_leaf(t):
            D = nd.D
        else:
            l, r = T.left[t], T.right[t]
            D = np.block([[fac[l]["S"], nd.B12], [nd.B21, fac[r]["S"]]])
        if T.parent[t] < 0:
            fac[t] = {"root": True, "lu": lu_factor(D)}
            continue
        orow, k = _order(nd.idr)
        ocol, _ = _order(nd.idc)
        Er, Ec = nd.idr.E, nd.idc.E
        Dp = D[np.ix_(orow, ocol)]
        DRR, DRS, DSR, DSS = Dp[:k, :k], Dp[:k, k:], Dp[k:, :k], Dp[k:, k:]
        DhSR = DSR - DSS @ Ec
        DhRS = DRS - Er.T @ DSS
        DhRR = DRR - Er.T @ DSR - DRS @ Ec + Er.T @ DSS @ Ec
        lu = lu_factor(DhRR) if k else None
        S = DSS - DhSR @ lu_solve(lu, DhRS) if k else DSS.copy()
        fac[t] = {"root": False, "orow": orow, "ocol": ocol, "k": k, "Er": Er, "Ec": Ec, "lu": lu,
                  "DhSR": DhSR, "DhRS": DhRS, "S": S}
    return fac


def solve(h, fac, B: np.ndarray) -> np.ndarray:
    """X = H^{-1} B in the permuted order of the tree (B: n or n x nrhs)."""
    T = h.tree
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    if vec:
        B = B[:, None]
    nn = T.num_nodes
    rhs = [None] * nn   # reduced skeleton right-hand side passed to the parent
    yR = [None] * nn
    for t in sorted(range(nn), key=lambda v: -int(T.level[v])):
        b = B[T.lo[t]:T.hi[t]] if T.is_leaf(t) else np.vstack([rhs[T.left[t]], rhs[T.right[t]]])
        f = fac[t]
        if f["root"]:
            rhs[t] = b
            continue
        bp = b[f["orow"]]
        k = f["k"]
        bR = bp[:k] - f["Er"].T @ bp[k:]
        y = lu_solve(f["lu"], bR) if k else np.zeros((0, B.shape[1]))
        yR[t] = y
        rhs[t] = bp[k:] - f["DhSR"] @ y
    X = np.zeros_like(B)
    xs = [None] * nn   # each node's skeleton unknowns (transformed), from its parent
    for t in sorted(range(nn), key=lambda v: int(T.level[v])):   # root first
        f = fac[t]
        if f["root"]:
            xloc = lu_solve(f["lu"], rhs[t])
        else:
            k = f["k"]
            xS = xs[t]
            xR = yR[t] - lu_solve(f["lu"], f["DhRS"] @ xS) if k else np.zeros((0, B.shape[1]))
            xp = np.vstack([xR, xS - f["Ec"] @ xR])
            xloc = np.zeros_like(xp)
            xloc[f["ocol"]] = xp
        if T.is_leaf(t):
            X[T.lo[t]:T.hi[t]] = xloc
        else:
            rl = fac[T.left[t]]["S"].shape[1]   # the left child's column skeleton
            xs[T.left[t]] = xloc[:rl]
            xs[T.right[t]] = xloc[rl:]
    return X[:, 0] if vec else X
