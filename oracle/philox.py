"""Counter-based Gaussian random matrix R (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method draws R as an N x d Gaussian matrix and appends new columns in
every adaptive round (Alg. 3, the randn of the sampling step).  The paper
does not fix a generator, so the random numbers are defined here
independently of any library state, by a published counter-based
generator: entry R(i, j) for permuted row i and column j is a function of
(seed, i, j) only, so columns appended later never change earlier ones and
any subset of entries can be recomputed on its own.

Definition (the HIP library implements the same definition in its own
code):
  * Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
    numbers: as easy as 1, 2, 3", SC 2011): 4 x 64-bit counter, 2 x 64-bit
    key, ten rounds of two 64 x 64 -> 128-bit multiplies with the
    constants M0, M1, the key bumped by the Weyl increments W0, W1 between
    rounds;
  * counter (i >> 2, j, 0, 0), key (seed, 0): one call gives four words
    w0..w3 for the rows 4q .. 4q+3 of column j, q = i >> 2;
  * uniforms u_t = ((w_t >> 11) + 1) 2^-53 in (0, 1];
  * Box and Muller (1958) in FP64 on the pairs (u0, u1) and (u2, u3):
    rho = sqrt(-2 log u_a), z_a = rho cos(2 pi u_b), z_b = rho sin(2 pi u_b),
    with 2 pi the double nearest to it, multiplied into u_b before the
    cosine and sine.
"""
from __future__ import annotations

import math

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
ROUNDS = 10
TWO_PI = 6.283185307179586
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: int):
    """(high, low) 64-bit halves of the 128-bit products a * b (uint64)."""
    b = np.uint64(b)
    lo = a * b                                    # wraps modulo 2^64
    a0, a1 = a & _MASK32, a >> _S32
    b0, b1 = b & _MASK32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _MASK32) + (p10 & _MASK32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64(ctr, key):
    """Philox4x64-10 of counters ctr (4 arrays or ints, uint64) under key
    (2 ints); returns the four output words as uint64 arrays."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
        x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
        k0, k1 = int(key[0]) & 0xFFFFFFFFFFFFFFFF, int(key[1]) & 0xFFFFFFFFFFFFFFFF
        for r in range(ROUNDS):
            if r:
                k0 = (k0 + W0) & 0xFFFFFFFFFFFFFFFF
                k1 = (k1 + W1) & 0xFFFFFFFFFFFFFFFF
            hi0, lo0 = _mulhilo(x0, M0)
            hi1, lo1 = _mulhilo(x2, M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0
        return x0, x1, x2, x3


def uniform53(w: np.ndarray) -> np.ndarray:
    """((w >> 11) + 1) 2^-53: a 64-bit word to a double in (0, 1]."""
    return ((w >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def box_muller(ua: np.ndarray, ub: np.ndarray):
    rho = np.sqrt(-2.0 * np.log(ua))
    ang = TWO_PI * ub
    return rho * np.cos(ang), rho * np.sin(ang)


def gaussian_columns(n: int, c0: int, c1: int, seed: int) -> np.ndarray:
    """Columns c0 .. c1-1 of R (n rows, permuted order), column-major."""
    ncol = max(0, c1 - c0)
    out = np.empty((n, ncol), order="F")
    nq = (n + 3) // 4
    q = np.arange(nq, dtype=np.uint64)
    for j in range(c0, c1):
        w = philox4x64((q, np.uint64(j), np.uint64(0), np.uint64(0)), (seed, 0))
        z0, z1 = box_muller(uniform53(w[0]), uniform53(w[1]))
        z2, z3 = box_muller(uniform53(w[2]), uniform53(w[3]))
        col = np.empty(4 * nq)
        col[0::4], col[1::4], col[2::4], col[3::4] = z0, z1, z2, z3
        out[:, j - c0] = col[:n]
    return out


def gaussian_matrix(n: int, d: int, seed: int) -> np.ndarray:
    """The first d columns of R, n x d column-major."""
    return gaussian_columns(n, 0, d, seed)


def entry(i: int, j: int, seed: int) -> float:
    """R(i, j) computed alone, with Python integers and the math module
    (the slow scalar route, for checks on a few entries)."""
    mask = (1 << 64) - 1
    x = [i >> 2, j, 0, 0]
    k0, k1 = seed & mask, 0
    for r in range(ROUNDS):
        if r:
            k0, k1 = (k0 + W0) & mask, (k1 + W1) & mask
        p0, p1 = M0 * x[0], M1 * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k0, p1 & mask, (p0 >> 64) ^ x[3] ^ k1, p0 & mask]
    u = [((w >> 11) + 1) * 2.0 ** -53 for w in x]
    t = i & 3
    a, b = (u[0], u[1]) if t < 2 else (u[2], u[3])
    rho = math.sqrt(-2.0 * math.log(a))
    ang = TWO_PI * b
    return rho * math.cos(ang) if t % 2 == 0 else rho * math.sin(ang)
