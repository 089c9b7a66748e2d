"""Learned d0 on the GPU: the predictor's forward pass against the FP64
oracle on the committed weights, and the gain it brings to the adaptive
compression, with the stopping tests still deciding every node.

The network's quality has no value in the paper to compare with; these
tests check that a predicted start keeps the accuracy of the adaptive run
(every node still passes its stopping test) and saves rounds on held-out
problems (seeds outside the training set's)."""
import os

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1810_04125_amd import hss, inputs, learned
from tests.gpu_util import dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not os.path.exists(learned.WEIGHTS), reason="no trained weights")]


def _unflatten(flat, sizes):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append((flat[o:o + a * b].reshape(b, a).astype(np.float64), flat[o + a * b:o + a * b + b].astype(np.float64)))
        o += a * b + b
    return out


def test_predictor_forward_matches_oracle():
    with np.load(learned.WEIGHTS, allow_pickle=False) as z:
        P = z["params"]
    T = hss.Tree(65536, 128)
    X = np.stack([learned.features(f, p, n, l, s, r)
                  for f, p, n, r in (("toeplitz", 0.1, 131072, 1e-6), ("laplace", 1.0, 65536, 1e-6),
                                     ("gauss", 0.5, 65536, 1e-4))
                  for l, s in enumerate(learned.level_sizes(T))])
    Y = hss.mlp_forward(learned.SIZES, dev(P), dev(X)).cpu().numpy()
    ref = omlp.forward(_unflatten(P, learned.SIZES), X)[-1]
    assert np.abs(Y - ref).max() <= 2e-5 * max(1.0, np.abs(ref).max())


def _laplace(n, seed):
    import torch
    pts = inputs.sphere_points(n, seed)
    return hss.laplace(torch.from_numpy(pts).cuda()), hss.Tree(n, 128, pts, "rcb")


@pytest.mark.parametrize("family,n", [("laplace", 8192), ("toeplitz", 32768)])
def test_learned_d0_saves_rounds_at_the_same_accuracy(family, n):
    print("learned gain", family, n, flush=True)
    if family == "laplace":
        gen, T = _laplace(n, 4)
        param = 1.0
    else:
        gen, T = hss.toeplitz(n, 0.1), hss.Tree(n, 128)
        param = 0.1
    d_max = 2048
    R = hss.colmajor(dev(np.ascontiguousarray(inputs.gaussian_matrix(n, d_max, 4).T)).t())
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm", delta_d=64, d_max=d_max)
    pred = learned.D0Predictor()
    d0 = pred.d0(family, param, n, T, 1e-6, 64, d_max)
    assert d0 % 64 == 0 and 64 <= d0 <= d_max
    Hb, stb = hss.compress(gen, T, R, d0=128, **kw)
    # the predictor runs inside hss_compress: its features and d0 equal the Python route's
    Hl, stl = hss.compress(gen, T, R, predictor=pred.handle(), **kw)
    ib, il = Hb.info(), Hl.info()
    assert il["d0"] == d0
    assert il["d_predicted"] == pytest.approx(pred.predict(family, param, n, T, 1e-6)["d_final"], rel=1e-5)
    print("baseline", ib, "learned d0", d0, il, flush=True)
    assert stb == stl == hss.OK
    assert il["rounds"] <= ib["rounds"]
    if family == "laplace":
        assert il["rounds"] < ib["rounds"] // 2
    eb = Hb.rel_error() if n <= 8192 else None
    el = Hl.rel_error() if n <= 8192 else None
    if el is not None:
        assert el <= 1e-6 and el <= 2.0 * eb
    # starting with enough columns gives generators no larger than the adaptive run's
    assert il["hss_rank"] <= ib["hss_rank"] + max(3, 0.05 * ib["hss_rank"])


def test_low_prediction_falls_back_to_the_adaptive_rounds():
    """A start far below the needed d: the stopping tests keep adding
    columns and reach the baseline's accuracy."""
    gen, T = _laplace(4096, 5)
    R = hss.colmajor(dev(np.ascontiguousarray(inputs.gaussian_matrix(4096, 2048, 5).T)).t())
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm", delta_d=64, d_max=2048)
    H, st = hss.compress(gen, T, R, d0=64, **kw)
    assert st == hss.OK and H.rel_error() <= 1e-6 and H.info()["rounds"] > 3


def test_low_prediction_outgrows_its_capacity_and_restarts():
    """A network that always predicts 64 final samples: the compression
    starts at d0 = 64 with a capacity of d0 + 4 delta_d = 320 columns, which
    a sphere-Laplace problem of n = 4096 outgrows; it is then restarted from
    320 with the caller's d_max and must reach the accuracy of the adaptive
    run (the stopping tests decide every node)."""
    import torch
    n = 4096
    gen, T = _laplace(n, 5)
    P = np.zeros(hss.mlp_num_params(learned.SIZES), np.float32)
    P[-1] = 6.0                                   # output 1 of the last layer: log2 d_final = 6
    pred = hss.Predictor(learned.SIZES, torch.from_numpy(P).cuda())
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.1, strategy="inc_fnorm", delta_d=64, d_max=2048)
    H, st = hss.compress(gen, T, None, predictor=pred, **kw)
    info = H.info()
    print("restarted", info, flush=True)
    assert st == hss.OK
    assert info["d_predicted"] == pytest.approx(64.0)
    assert info["d0"] == 320 and info["d_final"] > 320
    Hb, stb = hss.compress(gen, T, None, d0=128, **kw)
    assert stb == hss.OK
    e, eb = H.rel_error(), Hb.rel_error()
    assert e <= 1e-6 and e <= 2.0 * eb
