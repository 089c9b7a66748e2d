"""Pins of the oracle's HSS factorization and solve (oracle/ulv.py).

The solve is held to a dense solve of H rebuilt block by block from the
generators (oracle/matvec.py dense_from_generators, code the factorization
shares nothing with), and the node transform to the identity it rests on:
T U = [0; I] for every basis.
"""
import dataclasses

import numpy as np
import pytest

from oracle import ulv
from oracle.hss import compress
from oracle.matvec import dense_from_generators
from oracle.operators import Dense, Gauss, Laplace, PermutedOperator, Toeplitz
from oracle.tree import build_tree
from paper_1810_04125_amd import inputs


def _problem(family, n, leaf, rtol=1e-6, strategy="dbl_fnorm"):
    if family == "toeplitz":
        T = build_tree(n, leaf)
        op = PermutedOperator(Toeplitz(n, 0.1), T.perm)
    elif family == "laplace":
        pts = inputs.sphere_points(n, 1)
        T = build_tree(n, leaf, pts, "rcb")
        op = PermutedOperator(Laplace(pts), T.perm)
    else:
        pts = inputs.cube_points(n, 2)
        T = build_tree(n, leaf, pts, "kd")
        op = PermutedOperator(Gauss(pts, 0.5, 1e-2), T.perm)
    R = inputs.gaussian_matrix(n, n, 3)
    h = compress(op, T, R, rtol=rtol, atol=1e-12 if rtol > 1e-12 else 1e-300, strategy=strategy, d0=64,
                 delta_d=32, eta=0.05 if rtol > 1e-12 else 1.0)
    return h


@pytest.mark.parametrize("family,n,strategy", [("laplace", 768, "inc_fnorm"), ("gauss", 768, "dbl_fnorm"),
                                               ("toeplitz", 1024, "dbl_fnorm")])
def test_solve_equals_dense_solve_of_h(family, n, strategy):
    h = _problem(family, n, 64, strategy=strategy)
    fac = ulv.factor(h)
    B = inputs.gaussian_matrix(n, 3, 4)
    X = ulv.solve(h, fac, B)
    H = dense_from_generators(h)
    Xd = np.linalg.solve(H, B)
    # both solves are backward stable; kappa(H) <= 1e7 on these problems
    assert np.linalg.norm(X - Xd) <= 1e-9 * np.linalg.norm(Xd)
    assert np.linalg.norm(H @ X - B) <= 1e-10 * np.linalg.norm(B)
    # a single right-hand side as a vector
    x1 = ulv.solve(h, fac, B[:, 1])
    assert x1.shape == (n,) and np.allclose(x1, X[:, 1], rtol=0, atol=1e-12 * np.abs(X).max())


def test_transform_maps_basis_to_skeleton_identity():
    h = _problem("laplace", 512, 32)
    T = h.tree
    checked = 0
    for t, nd in enumerate(h.nodes):
        if T.parent[t] < 0:
            continue
        for ids in (nd.idr, nd.idc):
            m = ids.rank + len(ids.rest)
            U = ids.basis(m)
            order = np.concatenate([ids.rest, ids.J])
            TU = ulv.transform(ids, m) @ U[order]
            k = len(ids.rest)
            assert np.array_equal(TU[:k], np.zeros((k, ids.rank)))
            assert np.array_equal(TU[k:], np.eye(ids.rank))
            checked += 1
    assert checked > 10


def test_nodes_without_redundant_rows():
    # a tolerance at rounding level keeps full rank on the small nodes (k = 0)
    h = _problem("toeplitz", 96, 8, rtol=1e-15)
    fac = ulv.factor(h)
    assert any(f["k"] == 0 for f in fac if not f["root"])
    b = inputs.gaussian_matrix(96, 1, 5)[:, 0]
    x = ulv.solve(h, fac, b)
    H = dense_from_generators(h)
    assert np.linalg.norm(H @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_nonsymmetric_dense_and_unequal_ranks():
    n = 600
    A = inputs.gaussian_matrix(n, n, 7) * 0.01 + 5.0 * np.eye(n)
    T = build_tree(n, 64)
    h = compress(PermutedOperator(Dense(A), T.perm), T, inputs.gaussian_matrix(n, n, 3), rtol=1e-6,
                 atol=1e-12, strategy="dbl_fnorm", d0=64, eta=1.0)
    fac = ulv.factor(h)
    b = inputs.gaussian_matrix(n, 2, 8)
    x = ulv.solve(h, fac, b)
    H = dense_from_generators(h)
    assert np.linalg.norm(H @ x - b) <= 1e-12 * np.linalg.norm(b)
    t = next(t for t in range(T.num_nodes) if T.parent[t] >= 0)
    h.nodes[t].idc = dataclasses.replace(h.nodes[t].idc, rank=h.nodes[t].idc.rank + 1)
    with pytest.raises(ValueError, match="equal ranks"):
        ulv.factor(h)
