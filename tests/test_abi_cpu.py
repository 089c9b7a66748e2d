"""C-ABI library: loads, exports every declared symbol, host-side logic (CPU only)."""
import os
import re

import numpy as np
import pytest

from oracle.tree import build_tree
from paper_1810_04125_amd import hss, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hss_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hss.lib()
    names = _declared()
    assert "hss_compress" in names and "hss_matvec" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(hss.EXPORTS) == names


@pytest.mark.parametrize("method,n,leaf,seed", [("bisect", 1000, 64, 0), ("rcb", 4099, 128, 1),
                                                ("kd", 3000, 100, 2), ("rcb", 257, 128, 3),
                                                ("bisect", 1, 8, 0), ("kd", 65536, 256, 2)])
def test_tree_bit_exact_with_oracle(method, n, leaf, seed):
    pts = inputs.sphere_points(n, seed) if method == "rcb" else inputs.cube_points(n, seed)
    a = hss.Tree(n, leaf, None if method == "bisect" else pts, method)
    b = build_tree(n, leaf, None if method == "bisect" else pts, method)
    for f in ("perm", "lo", "hi", "left", "right", "parent", "level"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_tree_rejects_bad_input():
    with pytest.raises(hss.HSSError):
        hss.Tree(10, 0)
    bad = inputs.cube_points(10, 0)
    bad[3, 1] = np.nan
    with pytest.raises(hss.HSSError):
        hss.Tree(10, 4, bad, "rcb")


def test_bench_traffic_record_tracks_the_kernel_source(tmp_path, monkeypatch):
    import bench
    rec = dict(bench.TRAFFIC[("laplace-sphere-32768", "SAMPLE")])
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1")
    import hashlib
    rec.update(source=str(src), sha256=hashlib.sha256(b"kernel v1").hexdigest())
    monkeypatch.setattr(bench, "TRAFFIC", {("w", "C"): rec})
    monkeypatch.setattr(bench, "ROOT", "/")
    want = 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])
    assert bench.traffic_bytes("w", "C") == pytest.approx(want)
    src.write_bytes(b"kernel v2")
    assert bench.traffic_bytes("w", "C") is None
    assert bench.traffic_bytes("other", "C") is None


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes mirror in the binding has the size and field offsets of its C struct."""
    import ctypes as C
    import shutil
    import subprocess

    from paper_1810_04125_amd import hss as H
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    pairs = {"hss_generator": H._Gen, "hss_block": H._Block, "hss_tree": H._Tree, "hss_options": H._Opt,
             "hss_info": H._Info, "hss_kernel_stats": H._KStats, "hss_node_info": H._NodeInfo,
             "hss_mlp": H._Mlp, "hss_predictor": H._Predictor, "hss_allocator": H._Alloc}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hss.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    (tmp_path / "layout.c").write_text("\n".join(lines) + "\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, "-o", str(tmp_path / "layout"), str(tmp_path / "layout.c")],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(tmp_path / "layout")], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for cname, cls in pairs.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[cname + "." + f]) == getattr(cls, f).offset, cname + "." + f


def _host_compress(tree, **over):
    """hss_compress on a Toeplitz generator with host-only arguments (no
    stream, no device pointers): argument errors must come back before any
    HIP call, so this runs without a GPU."""
    import ctypes as C

    from paper_1810_04125_amd import hss as H
    g = H._Gen()
    g.family, g.symmetric, g.n, g.h = 0, 1, tree.n, 0.1
    o = H._Opt()
    o.rtol, o.atol, o.eta = 1e-6, 1e-12, 0.05
    o.strategy, o.d0, o.delta_d, o.oversample_p, o.d_max = 1, 16, 16, 10, 64
    o.R, o.seed = None, 0
    for k, v in over.items():
        setattr(o, k, v)
    h = C.c_void_p()
    st = H.lib().hss_compress(C.byref(g), tree._t, C.byref(o), C.byref(h))
    return st, H.lib().hss_last_error().decode()


def test_compress_rejects_a_perm_that_is_not_a_permutation():
    T = hss.Tree(64, 16)
    p = T._t.contents.perm
    saved = p[5]
    p[5] = p[6]               # index 6 twice, index 5 missing
    st, msg = _host_compress(T)
    assert st == -1 and "permutation" in msg
    p[5] = 64                 # outside [0, n)
    st, msg = _host_compress(T)
    assert st == -1 and "permutation" in msg
    p[5] = saved


def test_compress_rejects_a_root_off_level_zero():
    T = hss.Tree(64, 16)
    lv = T._t.contents.level
    for v in range(T.num_nodes):   # every level shifted: children still one below their parent
        lv[v] = lv[v] - 1
    st, msg = _host_compress(T)
    assert st == -1 and "level 0" in msg
    for v in range(T.num_nodes):
        lv[v] = lv[v] + 1


def test_compress_rejects_a_sample_cap_beyond_the_lds_vector():
    T = hss.Tree(40000, 2048)
    st, msg = _host_compress(T, d_max=hss.MAX_D + 1)
    assert st == -1 and "HSS_MAX_D" in msg
    # the cap that counts is min(d_max, n)
    T2 = hss.Tree(64, 16)
    st, msg = _host_compress(T2, d_max=hss.MAX_D + 1, rtol=-1.0)
    assert st == -1 and "rtol" in msg


def test_max_d_matches_the_header():
    src = open(os.path.join(ROOT, "include", "hss.h")).read()
    assert int(re.search(r"#define HSS_MAX_D (\d+)", src).group(1)) == hss.MAX_D


def test_compress_rejects_a_predictor_outside_its_scope():
    """The learned start applies to generated families with an incrementing
    strategy and rtol > 0; other uses are argument errors (host checks)."""
    import ctypes as C

    from paper_1810_04125_amd import hss as H
    pr = H._Predictor(H._mlp([8, 4, 2]), 8)   # never dereferenced on the device here
    ptr = C.cast(C.pointer(pr), C.c_void_p).value
    T = hss.Tree(64, 16)
    st, msg = _host_compress(T, predictor=ptr, strategy=0)
    assert st == -1 and "incrementing" in msg
    st, msg = _host_compress(T, predictor=ptr, rtol=0.0)
    assert st == -1 and "rtol" in msg


def test_compress_rejects_an_allocator_without_free():
    """alloc without free (or the reverse) is an argument error, caught on
    the host before any device call."""
    from paper_1810_04125_amd import hss as H
    a = H.Allocator(lambda n, s: 0, lambda p, s: None)
    half = H._Alloc()
    half.alloc = a._fa
    T = hss.Tree(64, 16)
    st, msg = _host_compress(T, allocator=half)
    assert st == -1 and "allocator" in msg


def test_tunables_table_lookup_and_errors(tmp_path):
    """The launch-shape table: a matching line by (arch, family, precision,
    n range), the defaults otherwise, bad files rejected with the table
    left as it was (host only)."""
    d = hss.default_tunables()
    assert d == {"gemm_wg": 2048, "gemm_max_split": 32, "sample_wg": 2048, "qrcp_wg": 1280}
    good = tmp_path / "t.tune"
    good.write_text("# arch family precision n_lo n_hi gemm_wg gemm_max_split sample_wg qrcp_wg\n"
                    "gfx950 1 0 16384 32768 4096 16 1024 2560\n"
                    "gfx950 1 0 32768 65536 1024 64 4096 640  # next bucket\n")
    try:
        hss.load_tunables(str(good))
        assert hss.lookup_tunables("gfx950", "laplace", "fp64", 20000) == \
            {"gemm_wg": 4096, "gemm_max_split": 16, "sample_wg": 1024, "qrcp_wg": 2560}
        assert hss.lookup_tunables("gfx950", "laplace", "fp64", 32768)["qrcp_wg"] == 640
        assert hss.lookup_tunables("gfx950", "laplace", "fp64", 65536) == d      # past the ranges
        assert hss.lookup_tunables("gfx950", "toeplitz", "fp64", 20000) == d     # other family
        assert hss.lookup_tunables("gfx950", "laplace", "fp32", 20000) == d      # other precision
        assert hss.lookup_tunables("gfx942", "laplace", "fp64", 20000) == d      # other device
        for text in ("gfx950 1 0 16384 32768 4096 16 1024\n",                   # 8 fields
                     "gfx950 1 0 16384 32768 4096 16 1024 9999\n",              # qrcp_wg > HSS_QRCP_WG_MAX
                     "gfx950 1 0 32768 16384 4096 16 1024 1280\n"):             # empty n range
            bad = tmp_path / "bad.tune"
            bad.write_text(text)
            with pytest.raises(hss.HSSError):
                hss.load_tunables(str(bad))
            assert hss.lookup_tunables("gfx950", "laplace", "fp64", 20000)["gemm_wg"] == 4096   # unchanged
        with pytest.raises(hss.HSSError):
            hss.load_tunables(str(tmp_path / "missing.tune"))
    finally:
        hss.load_tunables(None)
    assert hss.lookup_tunables("gfx950", "laplace", "fp64", 20000) == d


def test_qrcp_wg_max_matches_the_header():
    src = open(os.path.join(ROOT, "include", "hss.h")).read()
    assert int(re.search(r"#define HSS_QRCP_WG_MAX (\d+)", src).group(1)) == hss.QRCP_WG_MAX
