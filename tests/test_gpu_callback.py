"""Caller-supplied operators (HSS_FAM_CALLBACK, Sec. 4.1 partially matrix-free
interface): the library samples through the caller's product routine and
takes the sub-blocks D, B12, B21 from the caller's extraction routine, one
call per tree level (Sec. 4.2).  Compared with the FP64 oracle on the same
operator and R."""
import numpy as np
import pytest

from oracle.hss import compress as ocompress
from oracle.operators import Dense, Laplace, PermutedOperator, Toeplitz
from oracle.tree import build_tree
from paper_1810_04125_amd import hss, inputs
from tests.gpu_util import dev, dev_colmajor
from tests.test_gpu_parity import _compare

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


class FftToeplitz:
    """Symmetric Toeplitz operator applied by circulant embedding and FFT
    (O(n log n) per column, no n x n matrix anywhere), entries from its first
    column.  With index bisection the tree permutation is the identity."""

    def __init__(self, t):
        import torch
        self.n = len(t)
        self.t = dev(t)
        c = torch.zeros(2 * self.n, dtype=torch.float64, device="cuda")
        c[:self.n] = self.t
        c[self.n + 1:] = self.t[1:].flip(0)
        self.fc = torch.fft.rfft(c)
        self.calls = []

    def apply(self, X):
        import torch
        F = torch.fft.rfft(X, n=2 * self.n, dim=0)
        return torch.fft.irfft(F * self.fc[:, None], n=2 * self.n, dim=0)[:self.n]

    def sample(self, R, Sr, Sc):
        assert Sc is None   # symmetric: the library asks for S^r only
        Sr.copy_(self.apply(R))

    def extract(self, blocks):
        self.calls.append(len(blocks))
        for I, J, out in blocks:
            out.copy_(self.t[(I[:, None] - J[None, :]).abs()])


@pytest.mark.parametrize("strategy", ["dbl_fnorm", "inc_fnorm"])
def test_callback_fft_toeplitz_matches_oracle(strategy):
    _log("callback fft toeplitz 1024 " + strategy)
    n, leaf, h = 1024, 64, 0.1
    ref = Toeplitz(n, h)
    op_cb = FftToeplitz(ref.t)
    gen = hss.callback(n, op_cb.sample, op_cb.extract, symmetric=True)
    T = hss.Tree(n, leaf)
    ot = build_tree(n, leaf)
    assert np.array_equal(ot.perm, np.arange(n))
    op = PermutedOperator(ref, ot.perm)
    R = inputs.gaussian_matrix(n, 512, 0)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-6, atol=1e-12, strategy=strategy, d0=64, delta_d=64)
    oh = ocompress(op, ot, R, 1e-6, 1e-12, strategy, d0=64, delta_d=64)
    _compare(H, oh, ot, gen, op, T, 1e-6)
    assert H.info()["rounds"] == oh.rounds
    # the leaves' diagonal blocks come from the caller's table: bit-exact
    for t in range(ot.num_nodes):
        if ot.left[t] < 0:
            assert np.array_equal(H.node(t, "D"), oh.nodes[t].D)
    # extraction synchronized per level: the first call carries all 16 leaves
    assert op_cb.calls[0] == n // leaf


def test_callback_nonsymmetric_both_sides():
    """A nonsymmetric operator: the product routine is asked for S^r and S^c."""
    _log("callback nonsymmetric dense 400")
    n = 400
    pts = inputs.cube_points(n, 8)
    A = Laplace(pts).entries(np.arange(n), np.arange(n)) * (1.0 + 0.3 * pts[:, 0])[:, None]
    T = hss.Tree(n, 50)
    ot = build_tree(n, 50)
    op = PermutedOperator(Dense(A), ot.perm)
    Ah = dev(op.dense())
    asked = []

    def sample(R, Sr, Sc):
        asked.append((Sr is not None, Sc is not None))
        if Sr is not None:
            Sr.copy_(Ah @ R)
        if Sc is not None:
            Sc.copy_(Ah.t().contiguous() @ R)

    def extract(blocks):
        for I, J, out in blocks:
            out.copy_(Ah[I][:, J])

    gen = hss.callback(n, sample, extract, symmetric=False)
    R = inputs.gaussian_matrix(n, 400, 2)
    H, st = hss.compress(gen, T, dev_colmajor(R), rtol=1e-7, atol=1e-14, strategy="inc_fnorm", d0=32,
                         delta_d=16)
    ncomp = len(asked)
    assert ncomp >= 1 and all(a == (True, True) for a in asked)
    oh = ocompress(op, ot, R, 1e-7, 1e-14, "inc_fnorm", d0=32, delta_d=16)
    _compare(H, oh, ot, gen, op, T, 1e-6)
    # the exact error asks the product routine for columns of A_hat only
    assert len(asked) > ncomp and all(a == (True, False) for a in asked[ncomp:])


def test_callback_single_steps_forward_to_the_routines():
    n = 300
    A = inputs.gaussian_matrix(n, n, 11)
    Ah = dev(A)

    def sample(R, Sr, Sc):
        if Sr is not None:
            Sr.copy_(Ah @ R)
        if Sc is not None:
            Sc.copy_(Ah.t().contiguous() @ R)

    def extract(blocks):
        for I, J, out in blocks:
            out.copy_(Ah[I][:, J])

    gen = hss.callback(n, sample, extract, symmetric=False)
    perm = dev(np.arange(n))
    R = inputs.gaussian_matrix(n, 17, 12)
    for tr, ref in ((False, A @ R), (True, A.T @ R)):
        S = hss.sample(gen, perm, dev_colmajor(R), transpose=tr).cpu().numpy()
        assert np.linalg.norm(S - ref) <= 1e-13 * np.linalg.norm(ref)
    rng = np.random.default_rng(4)
    I, J = rng.integers(0, n, 23), rng.integers(0, n, 31)
    assert np.array_equal(hss.extract(gen, perm, dev(I), dev(J)).cpu().numpy(), A[np.ix_(I, J)])
    with pytest.raises(hss.HSSError):
        hss.sample(gen, perm, dev_colmajor(R), precision="fp32")


def test_callback_errors_abort_and_the_library_recovers():
    n, leaf, h = 512, 64, 0.1
    ref = Toeplitz(n, h)
    good = FftToeplitz(ref.t)
    T = hss.Tree(n, leaf)
    R = dev_colmajor(inputs.gaussian_matrix(n, 256, 1))

    class Boom(Exception):
        pass

    def bad_extract(blocks):
        raise Boom("no entries today")

    with pytest.raises(hss.HSSError) as ei:
        hss.compress(hss.callback(n, good.sample, bad_extract, symmetric=True), T, R, d0=64)
    assert ei.value.code == hss.ERR_CALLBACK and isinstance(ei.value.__cause__, Boom)

    def nan_sample(R_, Sr, Sc):
        Sr.copy_(good.apply(R_))
        Sr[3, 0] = float("nan")

    with pytest.raises(hss.HSSError) as ei:
        hss.compress(hss.callback(n, nan_sample, good.extract, symmetric=True), T, R, d0=64)
    assert ei.value.code == -5   # HSS_ERR_NONFINITE
    # a correct operator still compresses afterwards
    H, st = hss.compress(hss.callback(n, good.sample, good.extract, symmetric=True), T, R, rtol=1e-6, d0=64)
    assert st == hss.OK and H.rel_error() <= 1e-6


def test_callback_in_a_batch_with_builtin_families():
    """A batch mixing a caller operator and a generated family: each result
    equals that problem's own compression."""
    _log("callback batched")
    n, leaf, h = 1024, 64, 0.1
    cb = FftToeplitz(Toeplitz(n, h).t)
    gens = [hss.callback(n, cb.sample, cb.extract, symmetric=True), hss.toeplitz(n, 0.2)]
    trees = [hss.Tree(n, leaf), hss.Tree(n, leaf)]
    Rs = [dev_colmajor(inputs.gaussian_matrix(n, 512, 5)), dev_colmajor(inputs.gaussian_matrix(n, 512, 6))]
    Hb, st = hss.compress_batched(gens, trees, Rs, rtol=1e-6, strategy="dbl_fnorm", d0=64)
    for k in range(2):
        Hs, _ = hss.compress(gens[k], trees[k], Rs[k], rtol=1e-6, strategy="dbl_fnorm", d0=64)
        assert Hb[k].info()["rounds"] == Hs.info()["rounds"]
        for t in range(1, trees[k].num_nodes):
            assert Hb[k].node_info(t)["rank_r"] == Hs.node_info(t)["rank_r"]
            assert np.array_equal(Hb[k].node(t, "JR"), Hs.node(t, "JR"))
        assert Hb[k].rel_error() <= 1e-6
