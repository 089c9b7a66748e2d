"""Error terms of the reduced-precision sampling, emulated on the CPU.

The FP32 and BF16x3 sampling kernels (k_sample_lp.hip) differ from the FP64
product by: entries generated in FP32 (exp / rsqrt of FP32 arguments); the
operands rounded to FP32; products accumulated in FP32 over chunks of
LP_CHUNK terms, then summed in FP64; for BF16x3, the split a = a_hi + a_lo
and r = r_hi + r_lo into BF16 parts with the a_lo r_lo product left out.
Each term is emulated here with numpy on rows of the n = 65536
Gaussian-kernel workload (sigma 0.5, points in the unit cube), as the
relative Frobenius error of those rows of S = A R, and held to the sizes the
GPU measurements agree with (full-product error of the FP32 kernel 1.4e-7,
of the BF16x3 kernel 4.0e-6).  The sequential FP32 sum stands for the
matrix cores' accumulation order, which it does not reproduce exactly."""
import os
import re

import numpy as np
import pytest

from paper_1810_04125_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lp_chunk():
    src = open(os.path.join(ROOT, "paper_1810_04125_amd", "csrc", "k_sample_lp.hip")).read()
    return int(re.search(r"constexpr int LP_CHUNK = (\d+);", src).group(1))


def _bf16(x):
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP32."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def _chunked_fp32(a32, r32, chunk):
    """Products in FP32, summed in FP32 within chunks and in FP64 across them."""
    p = (a32.astype(np.float64)[:, None] * r32.astype(np.float64)).astype(np.float32)
    out = np.zeros(r32.shape[1])
    for c0 in range(0, len(a32), chunk):
        out += np.cumsum(p[c0:c0 + chunk], axis=0, dtype=np.float32)[-1].astype(np.float64)
    return out


@pytest.fixture(scope="module")
def terms():
    n, sigma, diag = 65536, 0.5, 1e-2
    pts = inputs.cube_points(n, 2)
    R = inputs.gaussian_matrix(n, 32, 5)
    rows = np.random.default_rng(11).choice(n, 12, replace=False)
    inv2s2 = 1.0 / (2.0 * sigma * sigma)
    r32 = R.astype(np.float32)
    chunk = _lp_chunk()
    out = {k: [] for k in ("gen", "round_a", "round_r", "acc", "split")}
    S = []
    for i in rows:
        d2 = ((pts - pts[i]) ** 2).sum(axis=1)
        a = np.exp(-d2 * inv2s2)
        a[i] += diag
        s = a @ R
        S.append(s)
        ag = np.exp(-(d2 * inv2s2).astype(np.float32)).astype(np.float32)
        ag[i] += np.float32(diag)
        out["gen"].append(ag.astype(np.float64) @ R - s)
        a32 = a.astype(np.float32)
        out["round_a"].append(a32.astype(np.float64) @ R - s)
        out["round_r"].append(a @ r32.astype(np.float64) - s)
        ref32 = a32.astype(np.float64) @ r32.astype(np.float64)
        out["acc"].append(_chunked_fp32(a32, r32, chunk) - ref32)
        ah = _bf16(a32)
        al = _bf16(a32 - ah)
        rh = _bf16(r32)
        rl = _bf16(r32 - rh)
        f = lambda x: x.astype(np.float64)
        out["split"].append(f(ah) @ f(rh) + f(ah) @ f(rl) + f(al) @ f(rh) - ref32)
    nS = np.linalg.norm(np.array(S))
    res = {k: float(np.linalg.norm(np.array(v)) / nS) for k, v in out.items()}
    print("precision terms (relative to the sampled rows of S):", res, "chunk", chunk)
    return res


def test_fp32_generation_and_rounding_are_below_1e_7(terms):
    assert terms["gen"] <= 1e-7
    assert terms["round_a"] <= 5e-8 and terms["round_r"] <= 5e-8


def test_fp32_accumulation_dominates_and_sets_the_fp32_floor(terms):
    # accumulation over the kernel's chunk is the largest FP32 term and sits
    # below the FP32 floor (5e-7 per level)
    assert terms["acc"] >= max(terms["gen"], terms["round_a"], terms["round_r"])
    assert terms["acc"] <= 3e-7


def test_bf16_split_sets_the_bf16x3_floor(terms):
    # 16 significant bits per operand (2^-17 relative per part) and the
    # missing lo x lo product: about 4e-6, below the BF16x3 floor (1e-5)
    assert 1e-6 <= terms["split"] <= 1e-5
