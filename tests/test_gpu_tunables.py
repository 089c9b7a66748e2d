"""Launch-shape tunables on the GPU: a compression under a table entry that
changes every tunable keeps the parity bar against the built-in shapes
(same rounds and d, ranks within 2, error at or below rtol; only the order
of sums changes), and the autotuner runs end to end and writes a table the
library reads back."""
import numpy as np
import pytest

from paper_1810_04125_amd import autotune, hss

pytestmark = pytest.mark.gpu


def test_table_entry_changes_shapes_within_parity(tmp_path):
    print("tunables parity", flush=True)
    n = 4096
    gen, T = autotune.problem("laplace", n, 128, 3)
    kw = dict(rtol=1e-6, atol=1e-12, eta=0.05, strategy="inc_fnorm", d0=64, delta_d=64, d_max=2048, seed=2)
    H0, st0 = hss.compress(gen, T, None, **kw)
    arch = autotune.device_arch()
    t = {"gemm_wg": 512, "gemm_max_split": 4, "sample_wg": 8192, "qrcp_wg": 256}
    path = tmp_path / "t.tune"
    path.write_text(autotune.table_line(arch, "laplace", "fp64", n, t) + "\n")
    hss.load_tunables(str(path))
    try:
        assert hss.lookup_tunables(arch, "laplace", "fp64", n) == t
        H1, st1 = hss.compress(gen, T, None, **kw)
    finally:
        hss.load_tunables(None)
    i0, i1 = H0.info(), H1.info()
    assert st0 == st1 == hss.OK
    assert (i0["rounds"], i0["d_final"]) == (i1["rounds"], i1["d_final"])
    for v in range(1, T.num_nodes):
        a, b = H0.node_info(v), H1.node_info(v)
        assert abs(a["rank_r"] - b["rank_r"]) <= 2 and abs(a["rank_c"] - b["rank_c"]) <= 2
    assert H1.rel_error() <= 1e-6


def test_autotuner_end_to_end(tmp_path):
    print("autotune small", flush=True)
    arch, best, t = autotune.tune("toeplitz", 8192, leaf=128, rtol=1e-6, d0=64, delta_d=64, d_max=1024, steps=1)
    assert set(best) == {"gemm_wg", "gemm_max_split", "sample_wg", "qrcp_wg"} and t > 0
    out = tmp_path / "table.tune"
    autotune.merge_table(str(out), autotune.table_line(arch, "toeplitz", "fp64", 8192, best))
    autotune.merge_table(str(out), autotune.table_line(arch, "toeplitz", "fp64", 8192, best))   # same key: replaced
    assert len(out.read_text().splitlines()) == 1
    hss.load_tunables(str(out))
    try:
        assert hss.lookup_tunables(arch, "toeplitz", "fp64", 8192) == best
    finally:
        hss.load_tunables(None)
