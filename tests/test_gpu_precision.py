"""Reduced-precision sampling (FP32, BF16x3) and its effect on compression.

The oracle is FP64 only; these tests compare the reduced-precision HIP
path with the FP64 oracle product and with the FP64 HIP compression (which
the parity tests pin to the oracle).  Bounds are the measured accuracy of
the arithmetic with margin: FP32 products carry ~1e-6 relative error per
column, BF16x3 (hi/lo bf16 split, three products) ~2e-5.
"""
import numpy as np
import pytest

from paper_1810_04125_amd import hss, inputs
from tests.gpu_util import dev, dev_colmajor, problem

pytestmark = pytest.mark.gpu

BOUND = {"fp32": 5e-6, "bf16x3": 1e-4}


@pytest.mark.parametrize("family", ["toeplitz", "laplace", "gauss"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_sampling(family, prec):
    print("lp sample", family, prec, flush=True)
    n = 3000
    gen, T, ot, op = problem(family, n, 128, seed=2)
    R = inputs.gaussian_matrix(n, 80, 5)
    ref = op.dense() @ R
    S = hss.sample(gen, dev(T.perm), dev_colmajor(R), precision=prec).cpu().numpy()
    err = np.linalg.norm(S - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= BOUND[prec]
    S64 = hss.sample(gen, dev(T.perm), dev_colmajor(R), precision="fp64").cpu().numpy()
    assert np.linalg.norm(S64 - ref) <= 1e-12 * np.linalg.norm(ref)


# Compression floors of the reduced-precision samples (relative thresholds
# are not lowered below the sampling noise: kFloorFp32 = 5e-7 and
# kFloorBf16x3 = 1e-5 per level).  Below the floor the library answers
# HSS_TOL_BELOW_SAMPLING_PRECISION and the error settles at the floor's
# level, measured on the n = 65536 Gaussian-kernel workload at about 2e-6
# (FP32) and 3e-5 (BF16x3); the bounds here are that level with margin.
FLOOR_ERR = {"fp32": 5e-6, "bf16x3": 1e-4}


@pytest.mark.parametrize("prec,rtol", [("fp32", 1e-4), ("bf16x3", 1e-4), ("fp32", 1e-6), ("bf16x3", 1e-6)])
def test_reduced_precision_compression(prec, rtol):
    """Gaussian kernel n = 4096, leaf 256 (4 levels), eta 0.1: at rtol 1e-4
    FP32 is above its floor (0.1 * 1e-4 / 4 = 2.5e-6 >= 5e-7) and must
    return status OK with error <= rtol; BF16x3 is below its floor there,
    and both are at rtol 1e-6: status TOL_FLOOR, error at the floor's level."""
    print("lp compress", prec, rtol, flush=True)
    n = 4096
    gen, T, ot, op = problem("gauss", n, 256, seed=2)
    R = dev_colmajor(inputs.gaussian_matrix(n, 1024, 0))
    H64, st64 = hss.compress(gen, T, R, rtol=rtol, atol=1e-12, eta=0.1, strategy="inc_fnorm", d0=128, delta_d=64)
    H, st = hss.compress(gen, T, R, rtol=rtol, atol=1e-12, eta=0.1, strategy="inc_fnorm", d0=128, delta_d=64,
                         precision=prec)
    e64, e = H64.rel_error(), H.rel_error()
    print("status %d error %.3e (fp64 %.3e)" % (st, e, e64), flush=True)
    assert st64 == hss.OK and e64 <= rtol
    above_floor = 0.1 * rtol / 4 >= (5e-7 if prec == "fp32" else 1e-5)
    if above_floor:
        assert st == hss.OK and e <= rtol
    else:
        assert st == hss.TOL_FLOOR
        assert e <= max(rtol, FLOOR_ERR[prec])
