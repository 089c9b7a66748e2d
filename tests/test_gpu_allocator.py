"""Device memory from the caller (hss_options.allocator): a compression and
its handle on torch's caching allocator give the same results as on the
library's own memory, every block taken is given back, and an allocator
that runs dry ends the call with HSS_ERR_OUT_OF_MEMORY after freeing what it
had taken (the condition is forced from the host: the allocator returns 0)."""
import numpy as np
import pytest

from paper_1810_04125_amd import hss
from tests.gpu_util import problem

pytestmark = pytest.mark.gpu

ERR_OUT_OF_MEMORY = -2


class Counting:
    """torch's caching allocator, counting blocks; returns 0 after `limit` blocks."""

    def __init__(self, limit=None):
        import torch
        self.live, self.taken, self.limit = {}, 0, limit
        dev = torch.cuda.current_device()

        def alloc(n, s):
            if self.limit is not None and self.taken >= self.limit:
                return 0
            p = torch.cuda.caching_allocator_alloc(n, dev, s)
            self.live[p] = n
            self.taken += 1
            return p

        def free(p, s):
            del self.live[p]
            torch.cuda.caching_allocator_delete(p)

        self.a = hss.Allocator(alloc, free)


KW = dict(rtol=1e-6, atol=1e-12, eta=0.05, strategy="inc_fnorm", d0=64, delta_d=32, d_max=1024, seed=9)


@pytest.mark.parametrize("family,n", [("laplace", 2048), ("toeplitz", 4096)])
def test_torch_allocator_gives_the_same_compression(family, n):
    import torch
    print("allocator", family, n, flush=True)
    gen, T, ot, op = problem(family, n, 64, seed=3)
    H0, st0 = hss.compress(gen, T, None, **KW)
    c = Counting()
    H1, st1 = hss.compress(gen, T, None, allocator=c.a, **KW)
    assert st0 == st1 == hss.OK and c.taken > 0
    i0, i1 = H0.info(), H1.info()
    assert (i0["rounds"], i0["d_final"], i0["hss_rank"]) == (i1["rounds"], i1["d_final"], i1["hss_rank"])
    for t in range(1, T.num_nodes):
        assert H0.node_info(t) == H1.node_info(t)
        assert np.array_equal(H0.node(t, "ER"), H1.node(t, "ER"))
    X = torch.randn(n, 3, dtype=torch.float64, device="cuda")
    Y0, Y1 = H0.matvec(X), H1.matvec(X)
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1)
    # only the handle's generators stay taken; destroying it gives them back
    assert 0 < len(c.live) < c.taken
    del H1
    torch.cuda.synchronize()
    assert not c.live


@pytest.mark.parametrize("limit", [0, 5])
def test_an_allocator_that_runs_dry_fails_cleanly(limit):
    import torch
    print("allocator limit", limit, flush=True)
    gen, T, ot, op = problem("laplace", 2048, 64, seed=3)
    c = Counting(limit)
    with pytest.raises(hss.HSSError) as e:
        hss.compress(gen, T, None, allocator=c.a, **KW)
    assert e.value.code == ERR_OUT_OF_MEMORY and "allocator" in str(e.value)
    torch.cuda.synchronize()
    assert c.taken == limit and not c.live
    # the library is usable afterwards
    H, st = hss.compress(gen, T, None, **KW)
    assert st == hss.OK and H.rel_error() <= 1e-6
