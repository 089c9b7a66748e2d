"""Matrix entries of the synthetic operator families (oracle).

The compression is partially matrix-free (Sec. 4, partially matrix-free
interface): it needs the products S^r = A R, S^c = A^T R and the entries
A(I,J) of sub-blocks.  Each family below gives a(i,j) on ORIGINAL indices;
`PermutedOperator` presents A_hat(i,j) = a(perm[i], perm[j]) on the
permuted index set of a cluster tree, which is the matrix the method
compresses.

Families (real arithmetic; the paper's conjugate transpose becomes the
transpose):
  toeplitz  symmetric Toeplitz, t(0) = pi^2/(6 h^2), t(k) = (-1)^k/(k^2 h^2)
  laplace   1/(4 pi |x_i - x_j|) for i != j, diag on the diagonal
  gauss     exp(-|x_i - x_j|^2 / (2 sigma^2)) + diag * delta_ij
  dense     an explicit n x n matrix
"""
from __future__ import annotations

import math

import numpy as np


class Family:
    symmetric = True

    def entries(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        raise NotImplementedError


class Toeplitz(Family):
    def __init__(self, n: int, h: float):
        self.n, self.h = n, float(h)
        k = np.arange(n, dtype=np.float64)
        t = np.empty(n)
        t[0] = math.pi ** 2 / (6.0 * self.h * self.h)
        sign = np.where(np.arange(1, n) % 2 == 0, 1.0, -1.0)
        t[1:] = sign / (k[1:] * k[1:] * self.h * self.h)
        self.t = t

    def entries(self, rows, cols):
        return self.t[np.abs(rows[:, None] - cols[None, :])]


class Laplace(Family):
    def __init__(self, points: np.ndarray, diag: float = 1.0):
        self.x = np.asarray(points, dtype=np.float64)
        self.n, self.diag = len(self.x), float(diag)

    def entries(self, rows, cols):
        diff = self.x[rows][:, None, :] - self.x[cols][None, :, :]
        dist = np.sqrt((diff * diff).sum(axis=2))
        same = rows[:, None] == cols[None, :]
        with np.errstate(divide="ignore"):
            a = 1.0 / (4.0 * math.pi * dist)
        a[same] = self.diag
        return a


class Gauss(Family):
    def __init__(self, points: np.ndarray, sigma: float = 0.5, diag: float = 1e-2):
        self.x = np.asarray(points, dtype=np.float64)
        self.n, self.sigma, self.diag = len(self.x), float(sigma), float(diag)

    def entries(self, rows, cols):
        diff = self.x[rows][:, None, :] - self.x[cols][None, :, :]
        d2 = (diff * diff).sum(axis=2)
        a = np.exp(-d2 / (2.0 * self.sigma * self.sigma))
        a = a + self.diag * (rows[:, None] == cols[None, :])
        return a


class Dense(Family):
    def __init__(self, a: np.ndarray):
        self.a = np.asarray(a, dtype=np.float64)
        self.n = self.a.shape[0]
        self.symmetric = bool(np.array_equal(self.a, self.a.T))

    def entries(self, rows, cols):
        return self.a[np.ix_(rows, cols)]


class PermutedOperator:
    """A_hat = P A P^T for the cluster-tree permutation."""

    def __init__(self, family: Family, perm: np.ndarray, block: int = 1024):
        self.f, self.perm = family, np.asarray(perm, dtype=np.int64)
        self.n = len(self.perm)
        self.block = block

    def extract(self, I, J) -> np.ndarray:
        """A_hat(I, J) for permuted index lists I, J."""
        I = np.asarray(I, dtype=np.int64)
        J = np.asarray(J, dtype=np.int64)
        if len(I) == 0 or len(J) == 0:
            return np.zeros((len(I), len(J)))
        return self.f.entries(self.perm[I], self.perm[J])

    def sample(self, R: np.ndarray):
        """(A_hat R, A_hat^T R) by dense row blocks of A_hat."""
        n, b = R.shape
        Sr = np.zeros((n, b))
        Sc = np.zeros((n, b))
        cols = np.arange(n)
        for i0 in range(0, n, self.block):
            rows = np.arange(i0, min(n, i0 + self.block))
            blk = self.extract(rows, cols)
            Sr[rows] = blk @ R
            if self.f.symmetric:
                Sc[rows] = Sr[rows]
            else:
                Sc += blk.T @ R[rows]
        return Sr, Sc

    def dense(self) -> np.ndarray:
        idx = np.arange(self.n)
        return self.extract(idx, idx)
