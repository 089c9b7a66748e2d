"""Host logic of the learned d0 predictor and its committed files (CPU only)."""
import json
import os

import numpy as np
import pytest

from paper_1810_04125_amd import hss, learned


def test_features_layout():
    f = learned.features("gauss", 0.5, 16384, 3, 2048, 1e-6)
    assert f.dtype == np.float32 and f.shape == (8,)
    assert list(f[:3]) == [0, 0, 1]
    assert f[3] == pytest.approx(0.5 * np.log2(0.5))
    assert f[4] == 0.0 and f[5] == pytest.approx(3 / 8) and f[6] == pytest.approx(0.25) and f[7] == 0.0
    assert learned.features("laplace", 123.0, 4096, 0, 4096, 1e-4)[3] == 0.0


def test_level_sizes_of_a_tree():
    T = hss.Tree(1000, 64)
    sizes = learned.level_sizes(T)
    assert sizes[0] == 1000 and len(sizes) == int(T.level.max()) + 1
    assert all(a > b for a, b in zip(sizes, sizes[1:]))


def test_rows_of_masks_root_and_levels():
    T = hss.Tree(4096, 128)
    spec = {"family": "toeplitz", "n": 4096, "h": 0.1, "rtol": 1e-6}
    ranks = np.arange(int(T.level.max()) + 1, dtype=float) * 10
    X, Tt, M = learned.rows_of(spec, T, ranks, 320)
    assert len(X) == len(ranks)
    assert M[0] == [0.0, 1.0] and Tt[0][1] == pytest.approx(np.log2(320))
    for lvl in range(1, len(ranks)):
        assert M[lvl] == [1.0, 0.0] and Tt[lvl][0] == pytest.approx(np.log2(1 + ranks[lvl]))


@pytest.mark.skipif(not os.path.exists(learned.WEIGHTS), reason="no trained weights")
def test_committed_weights_load_safely():
    with np.load(learned.WEIGHTS, allow_pickle=False) as z:
        assert list(z["sizes"]) == learned.SIZES
        P = z["params"]
        meta = json.loads(str(z["meta"]))
    assert P.dtype == np.float32 and P.size == hss.mlp_num_params(learned.SIZES) == 34434
    assert np.all(np.isfinite(P))
    assert meta["loss_last"] < meta["loss_first"]


@pytest.mark.skipif(not os.path.exists(learned.TRAIN_DATA), reason="no training set")
def test_committed_training_set_is_consistent():
    with np.load(learned.TRAIN_DATA, allow_pickle=False) as z:
        X, T, M = z["X"], z["T"], z["M"]
        nprob = len(z["p_n"])
        d_final = z["p_d_final"]
    assert X.shape[1] == 8 and T.shape == M.shape == (len(X), 2)
    root = X[:, 5] == 0.0
    assert root.sum() == nprob
    assert np.all(M[root] == [0, 1]) and np.all(M[~root] == [1, 0])
    assert np.allclose(2.0 ** T[root, 1], d_final)
    assert np.all(d_final % 64 == 0)


def _fake_set(nprob, d0, seed):
    """A training set of `nprob` problems with two rows each (root first)."""
    rng = np.random.default_rng(seed)
    X = rng.random((2 * nprob, 8)).astype(np.float32)
    X[0::2, 5] = 0.0   # root rows: level 0
    X[1::2, 5] = 0.125
    T = rng.random((2 * nprob, 2)).astype(np.float32)
    M = np.tile(np.array([[0, 1], [1, 0]], np.float32), (nprob, 1))
    return {"X": X, "T": T, "M": M, "p_n": np.arange(nprob) + 1000 * seed, "p_eta": np.array([0.05]),
            "p_d0": np.array([d0])}


def test_merge_interleaves_whole_problems_and_keeps_the_start():
    a, b = _fake_set(6, 128, 1), _fake_set(2, 128, 2)
    m = learned.merge(a, b, every=3)
    assert list(m["p_n"]) == [1000, 1001, 1002, 2000, 1003, 1004, 1005, 2001]
    assert len(m["X"]) == 16 and np.all(m["X"][0::2, 5] == 0.0)
    assert np.array_equal(m["X"][6:8], b["X"][0:2])   # b's first problem after a's third
    assert int(m["p_d0"][0]) == 128


def test_merge_refuses_sets_labelled_from_different_starts():
    with pytest.raises(ValueError):
        learned.merge(_fake_set(4, 128, 1), _fake_set(2, 64, 2), every=2)
