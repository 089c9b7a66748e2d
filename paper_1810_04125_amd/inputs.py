"""Seeded synthetic inputs for HSS compression workloads.

This module only draws the raw inputs of a workload: point clouds, the
Gaussian random matrix R that the randomized method consumes column by
column, planted low-rank factors and the parameters of a batch of
problems.  It holds none of the compression method's arithmetic and none
of the matrix entry formulas, so both the HIP path and the CPU oracle can
take their inputs from here without sharing any of the computation.

All arrays are float64 numpy arrays.  Matrices that the library consumes
column by column (R) are returned in column-major (Fortran) order so that
each column is contiguous, which is the layout the C ABI expects.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(int(seed)))


def sphere_points(n: int, seed: int) -> np.ndarray:
    """n points uniform on the unit sphere S^2 (normalised Gaussian triples)."""
    g = _rng(seed).standard_normal((n, 3))
    nrm = np.sqrt((g * g).sum(axis=1))
    return np.ascontiguousarray(g / nrm[:, None])


def cube_points(n: int, seed: int) -> np.ndarray:
    """n points uniform in the unit cube [0,1]^3."""
    return np.ascontiguousarray(_rng(seed).random((n, 3)))


def gaussian_matrix(n: int, d: int, seed: int) -> np.ndarray:
    """An n x d matrix of iid N(0,1) entries, column-major.

    Column j is drawn after columns 0..j-1, so a prefix of the columns does
    not depend on how many columns are requested.
    """
    z = _rng(seed).standard_normal((d, n))
    return np.asfortranarray(z.T)


def orthonormal_columns(n: int, r: int, seed: int) -> np.ndarray:
    """An n x r matrix with orthonormal columns (QR of a Gaussian matrix)."""
    q, _ = np.linalg.qr(_rng(seed).standard_normal((n, r)))
    return np.asfortranarray(q)


def batch_problems(count: int, seed: int, n_lo: int = 2048, n_hi: int = 16384):
    """Parameters of a batch of independent problems.

    Half are Toeplitz problems with grid step h ~ U[0.05, 0.5], half are
    sphere-point Laplace problems; sizes are log-uniform in [n_lo, n_hi].
    Returns a list of dicts with keys family ('toeplitz' | 'laplace'), n,
    h (Toeplitz only) and points_seed (Laplace only).
    """
    rng = _rng(seed)
    out = []
    for i in range(count):
        u = rng.random()
        n = int(math.floor(n_lo * (n_hi / n_lo) ** u))
        n = max(n_lo, min(n_hi, n))
        if i < count // 2:
            out.append({"family": "toeplitz", "n": n, "h": float(0.05 + 0.45 * rng.random())})
        else:
            out.append({"family": "laplace", "n": n, "points_seed": 1000 + i})
    return out


def mlp_params(sizes, seed: int) -> np.ndarray:
    """Initial parameters of a fully connected network with layer widths
    `sizes`, flat float32 in the library's order [W_1, b_1, W_2, b_2, ...]
    with W_l of shape (sizes[l+1], sizes[l]) row-major: weights uniform in
    +-sqrt(6 / fan_in) (He et al., 2015), biases zero."""
    rng = _rng(seed)
    parts = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def mlp_samples(n: int, n_in: int, n_out: int, seed: int, keep: float = 0.8):
    """Random (X, T, M) for a network: X, T standard normal, M a 0/1 mask
    keeping each target with probability `keep`; float32, row-major."""
    rng = _rng(seed)
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = rng.standard_normal((n, n_out)).astype(np.float32)
    M = (rng.random((n, n_out)) < keep).astype(np.float32)
    return X, T, M


def learned_problems(count: int, seed: int, n_lo: int = 1024, n_hi: int = 32768):
    """Parameters of randomly parameterised problems for the d0 predictor's
    training set: family uniform over Toeplitz (h ~ U[0.05, 0.5], index
    bisection, leaf 64 or 128), sphere Laplace (RCB, leaf 128) and cube
    Gaussian (sigma ~ U[0.2, 1], diag 1e-2, kd tree, leaf 256); n
    log-uniform in [n_lo, n_hi]; relative tolerance log-uniform in
    [1e-8, 1e-4].  Each dict has family, n, leaf, rtol and h / sigma /
    points_seed as the family needs."""
    rng = _rng(seed)
    out = []
    for i in range(count):
        fam = ("toeplitz", "laplace", "gauss")[int(rng.integers(0, 3))]
        n = int(math.floor(n_lo * (n_hi / n_lo) ** rng.random()))
        n = max(n_lo, min(n_hi, n))
        rtol = float(10.0 ** rng.uniform(-8.0, -4.0))
        p = {"family": fam, "n": n, "rtol": rtol}
        if fam == "toeplitz":
            p.update(h=float(rng.uniform(0.05, 0.5)), leaf=int(rng.choice([64, 128])))
        elif fam == "laplace":
            p.update(leaf=128, points_seed=seed * 100000 + i)
        else:
            p.update(sigma=float(rng.uniform(0.2, 1.0)), leaf=256, points_seed=seed * 100000 + i)
        out.append(p)
    return out
