"""Helpers shared by the GPU tests: move seeded inputs to the device and
build matching oracle problems."""
import numpy as np

from oracle.operators import Dense, Gauss, Laplace, PermutedOperator, Toeplitz
from oracle.tree import build_tree
from paper_1810_04125_amd import hss, inputs


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def dev_colmajor(x):
    return hss.colmajor(dev(np.asarray(x)))


def problem(family, n, leaf, seed=0, h=0.1, method=None, dense=None, symmetric=True):
    """(gpu generator, gpu tree, oracle tree, oracle operator)."""
    if family == "toeplitz":
        T = hss.Tree(n, leaf)
        ot = build_tree(n, leaf)
        return hss.toeplitz(n, h), T, ot, PermutedOperator(Toeplitz(n, h), ot.perm)
    if family in ("laplace", "gauss"):
        pts = inputs.sphere_points(n, seed) if family == "laplace" else inputs.cube_points(n, seed)
        method = method or ("rcb" if family == "laplace" else "kd")
        T = hss.Tree(n, leaf, pts, method)
        ot = build_tree(n, leaf, pts, method)
        if family == "laplace":
            return hss.laplace(dev(pts)), T, ot, PermutedOperator(Laplace(pts), ot.perm)
        return hss.gauss(dev(pts), 0.5, 1e-2), T, ot, PermutedOperator(Gauss(pts, 0.5, 1e-2), ot.perm)
    if family == "dense":
        T = hss.Tree(n, leaf)
        ot = build_tree(n, leaf)
        return (hss.dense(dev(dense), symmetric=symmetric), T, ot,
                PermutedOperator(Dense(dense), ot.perm))
    raise ValueError(family)
