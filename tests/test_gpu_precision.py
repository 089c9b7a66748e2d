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


@pytest.mark.parametrize("prec,rtol,errmax", [("fp32", 1e-4, 1e-4), ("bf16x3", 1e-4, 3e-4),
                                              ("fp32", 1e-6, 2e-5)])
def test_reduced_precision_compression(prec, rtol, errmax):
    print("lp compress", prec, rtol, flush=True)
    n = 4096
    gen, T, ot, op = problem("gauss", n, 256, seed=2)
    R = dev_colmajor(inputs.gaussian_matrix(n, 1024, 0))
    H64, st64 = hss.compress(gen, T, R, rtol=rtol, atol=1e-12, eta=0.1, strategy="inc_fnorm", d0=128, delta_d=64)
    H, st = hss.compress(gen, T, R, rtol=rtol, atol=1e-12, eta=0.1, strategy="inc_fnorm", d0=128, delta_d=64,
                         precision=prec)
    e64, e = H64.rel_error(), H.rel_error()
    assert e64 <= rtol
    assert e <= errmax
    assert st in (hss.OK, hss.TOL_FLOOR)
    # the precision floor is flagged when the per-node tolerance is below it
    if rtol <= 1e-6:
        assert st == hss.TOL_FLOOR
