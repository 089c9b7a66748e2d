"""Python binding of libhss (argument marshalling only).

Every computation happens in libhss.so (HIP kernels for gfx950).  PyTorch
provides device memory and the stream; this module converts tensors to
pointers and strides, calls the C ABI of include/hss.h and turns status
codes into exceptions.  There is no fallback: if the library or a GPU is
missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhss.so")

FAMILY = {"toeplitz": 0, "laplace": 1, "gauss": 2, "dense": 3, "callback": 4}
STRATEGY = {"dbl_fnorm": 0, "inc_fnorm": 1, "dbl_hmt": 2, "inc_hmt": 3}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2}
TREE_METHOD = {"bisect": 0, "rcb": 1, "kd": 2}
NODE = {"D": 0, "B12": 1, "B21": 2, "JR": 3, "JC": 4, "ER": 5, "EC": 6, "IR": 7, "IC": 8}

OK, NOT_CONVERGED, TOL_FLOOR = 0, 1, 2


class HSSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libhss status %d: %s" % (code, msg))
        self.code = code


class _Gen(C.Structure):
    _fields_ = [("family", C.c_int32), ("symmetric", C.c_int32), ("n", C.c_int64),
                ("h", C.c_double), ("sigma", C.c_double), ("diag", C.c_double),
                ("points", C.c_void_p), ("dense", C.c_void_p), ("ld", C.c_int64),
                ("sample", C.c_void_p), ("extract", C.c_void_p), ("ctx", C.c_void_p)]


class _Block(C.Structure):
    _fields_ = [("nI", C.c_int32), ("nJ", C.c_int32), ("I", C.c_void_p), ("J", C.c_void_p),
                ("out", C.c_void_p), ("ldo", C.c_int64)]


_SAMPLE_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                         C.c_void_p, C.c_int64, C.c_void_p)
_EXTRACT_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_int32, C.POINTER(_Block), C.c_void_p)


class _Tree(C.Structure):
    _fields_ = [("n", C.c_int64), ("num_nodes", C.c_int32), ("perm", C.POINTER(C.c_int64)),
                ("lo", C.POINTER(C.c_int32)), ("hi", C.POINTER(C.c_int32)),
                ("left", C.POINTER(C.c_int32)), ("right", C.POINTER(C.c_int32)),
                ("parent", C.POINTER(C.c_int32)), ("level", C.POINTER(C.c_int32))]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Alloc(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class _Opt(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("eta", C.c_double),
                ("strategy", C.c_int32), ("d0", C.c_int32), ("delta_d", C.c_int32),
                ("oversample_p", C.c_int32), ("d_max", C.c_int32), ("sample_precision", C.c_int32),
                ("R", C.c_void_p), ("ldr", C.c_int64), ("ncols_R", C.c_int32),
                ("profile", C.c_int32), ("stream", C.c_void_p), ("hmt_alpha", C.c_double),
                ("seed", C.c_uint64), ("predictor", C.c_void_p), ("allocator", _Alloc)]


class Allocator:
    """Device memory for the library from Python callables (hss_allocator):
    alloc(nbytes, stream) returns an int device pointer (0 or an exception:
    none available), free(ptr, stream) gives a block back.  Keep the object
    alive while handles made with it exist (the handles hold a reference)."""

    def __init__(self, alloc, free):
        def _a(ctx, nbytes, stream):
            try:
                return alloc(int(nbytes), stream or 0) or None
            except Exception:
                return None

        def _f(ctx, ptr, stream):
            try:
                free(ptr, stream or 0)
            except Exception:
                pass

        self._fa, self._ff = _ALLOC_FN(_a), _FREE_FN(_f)
        self._c = _Alloc(self._fa, self._ff, None)


def torch_allocator(device=None):
    """An Allocator backed by torch's CUDA caching allocator."""
    import torch
    dev = torch.cuda.current_device() if device is None else device
    return Allocator(lambda n, s: torch.cuda.caching_allocator_alloc(n, dev, s),
                     lambda p, s: torch.cuda.caching_allocator_delete(p))


class _Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("num_nodes", C.c_int32), ("rounds", C.c_int32),
                ("d_final", C.c_int32), ("hss_rank", C.c_int32), ("status", C.c_int32),
                ("symmetric", C.c_int32), ("sample_ms", C.c_double), ("total_ms", C.c_double),
                ("sample_flops", C.c_double), ("d0", C.c_int32), ("pad", C.c_int32), ("d_predicted", C.c_double)]


class _KStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double), ("flops", C.c_double)]


KCLASS = ["SAMPLE", "SAMPLE_REDUCE", "EXTRACT", "GATHER", "GEMM", "TEST_NORMS", "QRCP_STEP", "QRCP_OTHER",
          "TRSM", "MISC", "QRCP_WG", "QFORM", "RNG", "TEST_QR", "ID"]

MAX_D = 16384   # HSS_MAX_D


class _NodeInfo(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("state", "is_leaf", "lo", "hi", "m_r", "m_c", "rank_r",
                                          "rank_c", "b_rows", "b_cols")]


_lib = None

EXPORTS = ["hss_tree_build", "hss_tree_free", "hss_compress", "hss_compress_batched", "hss_destroy",
           "hss_matvec", "hss_rel_error", "hss_get_info", "hss_get_node_info", "hss_copy_node",
           "hss_sample", "hss_extract", "hss_interpolative_batched", "hss_last_error", "hss_version",
           "hss_get_kernel_stats", "hss_release_cache", "hss_mlp_num_params", "hss_mlp_forward", "hss_mlp_gradient",
           "hss_mlp_adam", "hss_mlp_train", "hss_random_normal", "hss_random_words", "hss_matvec_noalloc",
           "hss_default_tunables", "hss_load_tunables", "hss_lookup_tunables", "hss_factor", "hss_solve"]

MLP_MAX_LAYERS = 6


class _Mlp(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("sizes", C.c_int32 * (MLP_MAX_LAYERS + 1))]


class _Predictor(C.Structure):
    _fields_ = [("net", _Mlp), ("params", C.c_void_p)]


class Predictor:
    """hss_predictor: a network (layer sizes 8 -> ... -> 2) and its device
    FP32 parameters, run by hss_compress to pick d0."""

    def __init__(self, sizes, params):
        self.params = params            # keeps the device tensor alive
        self._c = _Predictor(_mlp(sizes), params.data_ptr())


def lib():
    """Load libhss.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime torch was built with)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhss.so is not built; run `python -m paper_1810_04125_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.hss_last_error.restype = C.c_char_p
    L.hss_version.restype = C.c_char_p
    L.hss_tree_build.argtypes = [i64, vp, i32, i32, C.POINTER(C.POINTER(_Tree))]
    L.hss_tree_free.argtypes = [C.POINTER(_Tree)]
    L.hss_tree_free.restype = None
    L.hss_compress.argtypes = [C.POINTER(_Gen), C.POINTER(_Tree), C.POINTER(_Opt), C.POINTER(vp)]
    L.hss_compress_batched.argtypes = [i32, C.POINTER(_Gen), C.POINTER(C.POINTER(_Tree)),
                                       C.POINTER(_Opt), C.POINTER(vp)]
    L.hss_destroy.argtypes = [vp]
    L.hss_destroy.restype = None
    L.hss_matvec.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    L.hss_matvec_noalloc.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    L.hss_factor.argtypes = [vp]
    L.hss_solve.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    L.hss_rel_error.argtypes = [vp, C.POINTER(_Gen), C.POINTER(dbl)]
    L.hss_get_info.argtypes = [vp, C.POINTER(_Info)]
    L.hss_get_node_info.argtypes = [vp, i32, C.POINTER(_NodeInfo)]
    L.hss_get_kernel_stats.argtypes = [vp, i32, C.POINTER(_KStats)]
    L.hss_copy_node.argtypes = [vp, i32, i32, vp, C.c_size_t]
    L.hss_sample.argtypes = [C.POINTER(_Gen), vp, i32, vp, i64, vp, i64, i32, i32, vp]
    L.hss_extract.argtypes = [C.POINTER(_Gen), vp, i32, vp, i32, vp, vp, i64, vp]
    L.hss_interpolative_batched.argtypes = [i32, vp, vp, vp, vp, vp, dbl, dbl, vp, vp, vp, vp, vp]
    L.hss_release_cache.argtypes = []
    L.hss_random_normal.argtypes = [i64, i32, i32, C.c_uint64, vp, i64, vp]
    L.hss_random_words.argtypes = [i64, i32, i32, C.c_uint64, vp, i64, vp]
    flt, mp = C.c_float, C.POINTER(_Mlp)
    L.hss_mlp_num_params.argtypes = [mp, C.POINTER(i64)]
    L.hss_mlp_forward.argtypes = [mp, vp, vp, i64, vp, vp]
    L.hss_mlp_gradient.argtypes = [mp, vp, vp, vp, vp, i64, vp, vp, vp]
    L.hss_mlp_adam.argtypes = [i64, vp, vp, vp, vp, flt, flt, flt, flt, i64, vp]
    L.hss_mlp_train.argtypes = [mp, vp, vp, vp, C.POINTER(i64), vp, vp, vp, i64, i32, i32, flt, C.c_uint64,
                                vp, vp]
    for name in EXPORTS:
        if name not in ("hss_tree_free", "hss_destroy", "hss_last_error", "hss_version"):
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


ERR_CALLBACK = -4
_callback_exc = []   # exception raised inside a caller routine, re-raised by _check


def _check(code):
    if code < 0:
        err = HSSError(code, lib().hss_last_error().decode())
        cause = _callback_exc.pop() if (code == ERR_CALLBACK and _callback_exc) else None
        _callback_exc.clear()
        if cause is not None:
            raise err from cause
        raise err
    return code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _colmajor(t, name):
    """(rows, cols) float64 CUDA tensor with unit row stride -> leading dimension."""
    import torch
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    rows, cols = t.shape
    if cols <= 1:   # a single column: only the row stride matters
        if rows > 1 and t.stride(0) != 1:
            raise ValueError("%s must be column-major (use X.t().contiguous().t())" % name)
        return max(1, rows)
    if (rows > 1 and t.stride(0) != 1) or t.stride(1) < max(1, rows):
        raise ValueError("%s must be column-major (use X.t().contiguous().t())" % name)
    return t.stride(1)


def colmajor(x):
    """Copy a 2-D tensor into column-major layout."""
    return x.t().contiguous().t()


# --------------------------------------------------------------------------- tree
class Tree:
    """Cluster tree built by libhss on the host (hss_tree_build)."""

    def __init__(self, n, leaf_size, points=None, method="bisect"):
        L = lib()
        pts = None
        if points is not None:
            pts = np.ascontiguousarray(points, dtype=np.float64)
            if pts.shape != (n, 3):
                raise ValueError("points must be (n, 3)")
        out = C.POINTER(_Tree)()
        _check(L.hss_tree_build(n, pts.ctypes.data if pts is not None else None, leaf_size,
                                TREE_METHOD[method], C.byref(out)))
        self._t = out
        t = out.contents
        nn = t.num_nodes
        self.n, self.num_nodes = t.n, nn
        self.perm = np.ctypeslib.as_array(t.perm, shape=(n,)).copy()
        self.lo = np.ctypeslib.as_array(t.lo, shape=(nn,)).copy()
        self.hi = np.ctypeslib.as_array(t.hi, shape=(nn,)).copy()
        self.left = np.ctypeslib.as_array(t.left, shape=(nn,)).copy()
        self.right = np.ctypeslib.as_array(t.right, shape=(nn,)).copy()
        self.parent = np.ctypeslib.as_array(t.parent, shape=(nn,)).copy()
        self.level = np.ctypeslib.as_array(t.level, shape=(nn,)).copy()

    def __del__(self):
        if getattr(self, "_t", None) is not None and _lib is not None:
            _lib.hss_tree_free(self._t)
            self._t = None


# --------------------------------------------------------------------------- generator
@dataclass
class Generator:
    family: str
    n: int
    h: float = 0.0
    sigma: float = 0.0
    diag: float = 0.0
    points: object = None    # (n, 3) float64 CUDA tensor, original order
    dense: object = None     # (n, n) float64 CUDA tensor, column-major
    symmetric: bool = True
    routines: object = None  # callback family: (sample C function, extract C function)

    def _c(self):
        g = _Gen()
        g.family = FAMILY[self.family]
        g.symmetric = int(self.symmetric)
        g.n = self.n
        g.h, g.sigma, g.diag = self.h, self.sigma, self.diag
        g.points = self.points.data_ptr() if self.points is not None else None
        if self.dense is not None:
            g.ld = _colmajor(self.dense, "dense")
            g.dense = self.dense.data_ptr()
        if self.routines is not None:
            g.sample = C.cast(self.routines[0], C.c_void_p).value
            g.extract = C.cast(self.routines[1], C.c_void_p).value
        return g


def toeplitz(n, h):
    return Generator("toeplitz", n, h=h)


def laplace(points, diag=1.0):
    return Generator("laplace", points.shape[0], diag=diag, points=points.contiguous())


def gauss(points, sigma=0.5, diag=1e-2):
    return Generator("gauss", points.shape[0], sigma=sigma, diag=diag, points=points.contiguous())


def dense(A, symmetric=False):
    return Generator("dense", A.shape[0], dense=colmajor(A), symmetric=symmetric)


class _DevArray:
    """A block of library device memory, seen by torch.as_tensor without a copy."""

    def __init__(self, ptr, shape, strides, typestr):
        self.__cuda_array_interface__ = {"shape": shape, "strides": strides, "typestr": typestr,
                                         "data": (ptr, False), "version": 2}


def _device_view(ptr, rows, cols, ld, dtype="f8"):
    """(rows, cols) column-major view (leading dimension ld) of device memory at ptr;
    cols=None gives a 1-D view of rows entries."""
    import torch
    tdt = torch.float64 if dtype == "f8" else torch.int64
    if not ptr or rows == 0 or cols == 0:
        return torch.empty((rows,) if cols is None else (rows, cols), dtype=tdt, device="cuda")
    if cols is None:
        return torch.as_tensor(_DevArray(ptr, (rows,), (8,), "<" + dtype), device="cuda")
    return torch.as_tensor(_DevArray(ptr, (rows, cols), (8, 8 * ld), "<" + dtype), device="cuda")


def _on_stream(stream, fn):
    import torch
    if stream and stream != torch.cuda.current_stream().cuda_stream:
        with torch.cuda.stream(torch.cuda.ExternalStream(stream)):
            return fn()
    return fn()


def callback(n, sample, extract, symmetric=False):
    """Partially matrix-free operator (hss_generator with HSS_FAM_CALLBACK; Sec. 4.1).

    sample(R, Sr, Sc): R is an (n, k) float64 CUDA tensor; write A_hat @ R into
        Sr and A_hat.T @ R into Sc (each may be None: not wanted).
    extract(blocks): blocks is a list of (I, J, out), I and J int64 CUDA tensors
        of permuted positions and out a (len(I), len(J)) float64 tensor; write
        A_hat[I][:, J] into out.  One call serves all blocks of a tree level.
    A_hat is the operator in the tree's permuted order.  The tensors are views of
    library memory, valid during the call only; the routines run with the
    library's stream as torch's current stream.  An exception inside a routine
    aborts the library call, which raises HSSError from it."""

    def c_sample(ctx, nn, k, R, ldr, Sr, Sc, lds, stream):
        try:
            Rt = _device_view(R, nn, k, ldr)
            St = _device_view(Sr, nn, k, lds) if Sr else None
            Ct = _device_view(Sc, nn, k, lds) if Sc else None
            _on_stream(stream, lambda: sample(Rt, St, Ct))
            return 0
        except BaseException as e:   # noqa: BLE001  (handed back through the C call)
            _callback_exc.append(e)
            return 1

    def c_extract(ctx, nb, blocks, stream):
        try:
            bl = []
            for i in range(nb):
                b = blocks[i]
                bl.append((_device_view(b.I, b.nI, None, 0, "i8"), _device_view(b.J, b.nJ, None, 0, "i8"),
                           _device_view(b.out, b.nI, b.nJ, b.ldo)))
            _on_stream(stream, lambda: extract(bl))
            return 0
        except BaseException as e:   # noqa: BLE001
            _callback_exc.append(e)
            return 1

    return Generator("callback", n, symmetric=symmetric,
                     routines=(_SAMPLE_FN(c_sample), _EXTRACT_FN(c_extract)))


# --------------------------------------------------------------------------- compression
class HSSMatrix:
    def __init__(self, handle, keep):
        self._h = C.c_void_p(handle)
        self._keep = keep

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hss_destroy(self._h)
            self._h = None

    def info(self) -> dict:
        inf = _Info()
        _check(lib().hss_get_info(self._h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def kernel_stats(self) -> dict:
        """{class: {launches, ms, bytes, flops}} of the compression (ms only in profile mode)."""
        out = {}
        for i, name in enumerate(KCLASS):
            k = _KStats()
            _check(lib().hss_get_kernel_stats(self._h, i, C.byref(k)))
            out[name] = {f: getattr(k, f) for f, _ in _KStats._fields_}
        return out

    def node_info(self, node) -> dict:
        ni = _NodeInfo()
        _check(lib().hss_get_node_info(self._h, node, C.byref(ni)))
        return {k: getattr(ni, k) for k, _ in _NodeInfo._fields_}

    def node(self, node, what):
        """Host copy of a node generator (see hss_copy_node for the layouts)."""
        ni = self.node_info(node)
        if what == "D":
            m = ni["hi"] - ni["lo"]
            out = np.empty((m, m), order="F")
        elif what == "B12":
            out = np.empty((ni["b_rows"], ni["b_cols"]), order="F")
        elif what == "B21":
            # B21 is rank_r(right) x rank_c(left): ask the children
            raise ValueError("use node_b21()")
        elif what in ("JR", "JC"):
            out = np.empty(ni["m_r"] if what == "JR" else ni["m_c"], dtype=np.int32)
        elif what in ("ER", "EC"):
            r = ni["rank_r"] if what == "ER" else ni["rank_c"]
            m = ni["m_r"] if what == "ER" else ni["m_c"]
            out = np.empty((r, m - r), order="F")
        elif what in ("IR", "IC"):
            out = np.empty(ni["rank_r"] if what == "IR" else ni["rank_c"], dtype=np.int64)
        else:
            raise ValueError(what)
        if out.size:
            _check(lib().hss_copy_node(self._h, node, NODE[what], out.ctypes.data, out.nbytes))
        return out

    def node_b21(self, node, left, right):
        rr = self.node_info(right)["rank_r"]
        cl = self.node_info(left)["rank_c"]
        out = np.empty((rr, cl), order="F")
        if out.size:
            _check(lib().hss_copy_node(self._h, node, NODE["B21"], out.ctypes.data, out.nbytes))
        return out

    def matvec(self, X):
        """Y = H X (original ordering); X: (n,) or (n, k) float64 CUDA tensor."""
        import torch
        vec = X.dim() == 1
        Xc = colmajor(X[:, None] if vec else X)
        Y = torch.empty_like(Xc)
        Y = colmajor(Y)
        _check(lib().hss_matvec(self._h, Xc.shape[1], _ptr(Xc), _colmajor(Xc, "X"), _ptr(Y),
                                _colmajor(Y, "Y"), _stream()))
        return Y[:, 0] if vec else Y

    def factor(self):
        """hss_factor: the direct factorization for solve() (kept with the matrix)."""
        _check(lib().hss_factor(self._h))
        return self

    def solve(self, B):
        """X = H^{-1} B (original ordering, hss_solve); B: (n,) or (n, k) float64 CUDA tensor."""
        import torch
        vec = B.dim() == 1
        Bc = colmajor(B[:, None] if vec else B)
        X = colmajor(torch.empty_like(Bc))
        _check(lib().hss_solve(self._h, Bc.shape[1], _ptr(Bc), _colmajor(Bc, "B"), _ptr(X),
                               _colmajor(X, "X"), _stream()))
        return X[:, 0] if vec else X

    def matvec_noalloc(self, X, Y):
        """Y = H X through hss_matvec_noalloc (no device allocation in the call):
        X, Y (n, k) column-major float64 CUDA tensors, Y written in place."""
        _check(lib().hss_matvec_noalloc(self._h, X.shape[1], _ptr(X), _colmajor(X, "X"), _ptr(Y),
                                        _colmajor(Y, "Y"), _stream()))
        return Y

    def rel_error(self) -> float:
        e = C.c_double()
        gen = self._keep[0]
        g = C.byref(gen._c()) if gen.family == "callback" else None
        _check(lib().hss_rel_error(self._h, g, C.byref(e)))
        return e.value


def _opts(R, rtol, atol, eta, strategy, d0, delta_d, p, d_max, precision, profile=False, hmt_alpha=10.0,
          seed=0, n=None, predictor=None, allocator=None):
    o = _Opt()
    if allocator is not None:
        o.allocator = allocator._c
    o.rtol, o.atol, o.eta = rtol, atol, eta
    o.strategy = STRATEGY[strategy]
    o.d0, o.delta_d, o.oversample_p = d0, delta_d, p
    o.sample_precision = PRECISION[precision]
    if R is None:   # the library draws R from `seed`
        o.d_max = d_max if d_max is not None else min(n, MAX_D)
        o.R, o.ldr, o.ncols_R = None, 0, 0
    else:
        o.d_max = d_max if d_max is not None else R.shape[1]
        o.R = R.data_ptr()
        o.ldr = _colmajor(R, "R")
        o.ncols_R = R.shape[1]
    o.profile = int(bool(profile))
    o.stream = _stream()
    o.hmt_alpha = hmt_alpha
    o.seed = int(seed)
    o.predictor = C.cast(C.pointer(predictor._c), C.c_void_p).value if predictor is not None else None
    return o


def compress(gen: Generator, tree: Tree, R=None, rtol=1e-6, atol=1e-12, eta=1.0, strategy="dbl_fnorm",
             d0=64, delta_d=64, p=10, d_max=None, precision="fp64", profile=False, hmt_alpha=10.0, seed=0,
             predictor=None, allocator=None):
    """Adaptive HSS compression (hss_compress).  R: (n, d_cap) float64 CUDA tensor,
    column-major, rows in permuted order; or None, and the library draws R
    on the device from `seed` (hss_random_normal).  predictor: a Predictor
    (hss_predictor), whose d0 then replaces `d0`.  allocator: an Allocator
    (e.g. torch_allocator()) for all device memory of the compression and
    of the handle, or None for the library's own.  Returns (HSSMatrix, status)."""
    g = gen._c()
    o = _opts(R, rtol, atol, eta, strategy, d0, delta_d, p, d_max, precision, profile, hmt_alpha, seed, gen.n,
              predictor, allocator)
    h = C.c_void_p()
    st = _check(lib().hss_compress(C.byref(g), tree._t, C.byref(o), C.byref(h)))
    return HSSMatrix(h.value, (gen, tree, R, allocator)), st


def compress_batched(gens, trees, Rs, **kw):
    """Independent compressions in one job (hss_compress_batched).  Keyword
    options are those of compress(); a list or tuple gives one value per problem."""
    k = len(gens)

    def opt(name, i, default):
        v = kw.get(name, default)
        return v[i] if isinstance(v, (list, tuple)) else v

    G = (_Gen * k)(*[g._c() for g in gens])
    T = (C.POINTER(_Tree) * k)(*[t._t for t in trees])
    Rs = list(Rs) if Rs is not None else [None] * k
    O = (_Opt * k)(*[_opts(R, opt("rtol", i, 1e-6), opt("atol", i, 1e-12), opt("eta", i, 1.0),
                           opt("strategy", i, "dbl_fnorm"), opt("d0", i, 64), opt("delta_d", i, 64),
                           opt("p", i, 10), opt("d_max", i, None), opt("precision", i, "fp64"),
                           opt("profile", i, False), opt("hmt_alpha", i, 10.0), opt("seed", i, 0), gens[i].n,
                           opt("predictor", i, None), kw.get("allocator"))
                     for i, R in enumerate(Rs)])
    H = (C.c_void_p * k)()
    st = _check(lib().hss_compress_batched(k, G, T, O, H))
    return [HSSMatrix(H[i], (gens[i], trees[i], Rs[i], kw.get("allocator"))) for i in range(k)], st


def release_cache():
    """Free the device memory kept between compressions (hss_release_cache)."""
    _check(lib().hss_release_cache())


class _Tunables(C.Structure):
    _fields_ = [("gemm_wg", C.c_int32), ("gemm_max_split", C.c_int32), ("sample_wg", C.c_int32),
                ("qrcp_wg", C.c_int32)]


QRCP_WG_MAX = 4096   # HSS_QRCP_WG_MAX


def default_tunables() -> dict:
    """The built-in launch-shape tunables (hss_default_tunables)."""
    t = _Tunables()
    _check(lib().hss_default_tunables(C.byref(t)))
    return {k: getattr(t, k) for k, _ in _Tunables._fields_}


def load_tunables(path):
    """Load (path) or clear (None) the tunables table (hss_load_tunables)."""
    _check(lib().hss_load_tunables(path.encode() if path else None))


def lookup_tunables(arch, family, precision, n) -> dict:
    """The tunables a compression with this key takes (hss_lookup_tunables)."""
    t = _Tunables()
    _check(lib().hss_lookup_tunables(arch.encode(), FAMILY[family] if isinstance(family, str) else family,
                                     PRECISION[precision] if isinstance(precision, str) else precision,
                                     int(n), C.byref(t)))
    return {k: getattr(t, k) for k, _ in _Tunables._fields_}


# --------------------------------------------------------------------------- single steps
def sample(gen: Generator, perm, R, transpose=False, precision="fp64"):
    """S = op(A_hat) R (hss_sample); perm: int64 CUDA tensor; R (n, k) column-major."""
    import torch
    ldr = _colmajor(R, "R")
    S = colmajor(torch.empty((R.shape[0], R.shape[1]), dtype=torch.float64, device=R.device))
    g = gen._c()
    _check(lib().hss_sample(C.byref(g), _ptr(perm), R.shape[1], _ptr(R), ldr, _ptr(S),
                            _colmajor(S, "S"), int(transpose), PRECISION[precision], _stream()))
    return S


def random_normal(n, c0, ncols, seed, device="cuda"):
    """Columns c0 .. c0+ncols-1 of the library's Gaussian R (hss_random_normal),
    an (n, ncols) column-major float64 CUDA tensor."""
    import torch
    R = colmajor(torch.empty((n, ncols), dtype=torch.float64, device=device))
    _check(lib().hss_random_normal(n, c0, ncols, int(seed), _ptr(R), max(1, n), _stream()))
    return R


def random_words(n, c0, ncols, seed, device="cuda"):
    """The raw Philox words behind random_normal (hss_random_words), as an
    (n, ncols) column-major int64 CUDA tensor holding the uint64 bits."""
    import torch
    W = colmajor(torch.empty((n, ncols), dtype=torch.int64, device=device))
    _check(lib().hss_random_words(n, c0, ncols, int(seed), _ptr(W), max(1, n), _stream()))
    return W


def extract(gen: Generator, perm, I, J):
    """A_hat(I, J) (hss_extract); I, J int64 CUDA tensors of permuted indices."""
    import torch
    out = colmajor(torch.empty((len(I), len(J)), dtype=torch.float64, device=perm.device))
    g = gen._c()
    ldo = max(1, len(I))
    _check(lib().hss_extract(C.byref(g), _ptr(perm), len(I), _ptr(I), len(J), _ptr(J), _ptr(out),
                             ldo, _stream()))
    return out


def interpolative_batched(mats, eps_r, eps_a=0.0):
    """Batched ID (hss_interpolative_batched) of host matrices S_k (m_k x d_k).

    Returns a list of (rank, piv, E) with piv the pivot order followed by the
    other rows ascending and E = R1^{-1} R2 (rank x (m_k - rank))."""
    import torch
    dev = torch.device("cuda")
    k = len(mats)
    m = np.array([s.shape[0] for s in mats], dtype=np.int32)
    d = np.array([s.shape[1] for s in mats], dtype=np.int32)
    ld = np.maximum(d, 1).astype(np.int64)
    s_off = np.zeros(k, np.int64)
    p_off = np.zeros(k, np.int64)
    e_off = np.zeros(k, np.int64)
    so = po = eo = 0
    for i in range(k):
        s_off[i], p_off[i], e_off[i] = so, po, eo
        so += m[i] * ld[i]
        po += m[i]
        eo += m[i] * m[i]
    flat = np.zeros(max(so, 1))
    for i, s in enumerate(mats):
        flat[s_off[i]:s_off[i] + m[i] * ld[i]] = np.ascontiguousarray(s, dtype=np.float64).ravel()
    S = torch.from_numpy(flat).to(dev)
    piv = torch.zeros(max(po, 1), dtype=torch.int32, device=dev)
    E = torch.zeros(max(eo, 1), dtype=torch.float64, device=dev)
    rank = np.zeros(k, np.int32)
    _check(lib().hss_interpolative_batched(k, m.ctypes.data, d.ctypes.data, ld.ctypes.data, _ptr(S),
                                           s_off.ctypes.data, eps_r, eps_a, _ptr(piv), p_off.ctypes.data,
                                           _ptr(E), e_off.ctypes.data, rank.ctypes.data))
    pv, Ev = piv.cpu().numpy(), E.cpu().numpy()
    out = []
    for i in range(k):
        r = int(rank[i])
        Ei = Ev[e_off[i]:e_off[i] + m[i] * m[i]].reshape((m[i], m[i]), order="F")[:r, :m[i] - r]
        out.append((r, pv[p_off[i]:p_off[i] + m[i]].copy(), Ei.copy()))
    return out


# --------------------------------------------------------------------------- predictor network
def _mlp(sizes):
    if not 2 <= len(sizes) <= MLP_MAX_LAYERS + 1:
        raise ValueError("between 1 and %d layers" % MLP_MAX_LAYERS)
    net = _Mlp()
    net.n_layers = len(sizes) - 1
    for i, w in enumerate(sizes):
        net.sizes[i] = int(w)
    return net


def _f32(t, name, shape=None):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float32 CUDA tensor" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, not %s" % (name, tuple(shape), tuple(t.shape)))
    return _ptr(t)


def mlp_num_params(sizes) -> int:
    """Parameter count of the ReLU network `sizes` (hss_mlp_num_params)."""
    out = C.c_int64()
    _check(lib().hss_mlp_num_params(C.byref(_mlp(sizes)), C.byref(out)))
    return out.value


def mlp_forward(sizes, params, X):
    """Y = net(X) (hss_mlp_forward); X (n, sizes[0]) float32 CUDA, row-major."""
    import torch
    n = X.shape[0]
    Y = torch.empty((n, sizes[-1]), dtype=torch.float32, device=X.device)
    _check(lib().hss_mlp_forward(C.byref(_mlp(sizes)), _f32(params, "params", (mlp_num_params(sizes),)),
                                 _f32(X, "X", (n, sizes[0])), n, _ptr(Y), _stream()))
    return Y


def mlp_gradient(sizes, params, X, T, M):
    """(gradient, loss) of the masked squared error (hss_mlp_gradient)."""
    import torch
    n = X.shape[0]
    npar = mlp_num_params(sizes)
    g = torch.empty(npar, dtype=torch.float32, device=params.device)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    _check(lib().hss_mlp_gradient(C.byref(_mlp(sizes)), _f32(params, "params", (npar,)),
                                  _f32(X, "X", (n, sizes[0])), _f32(T, "T", (n, sizes[-1])),
                                  _f32(M, "M", (n, sizes[-1])), n, _ptr(g), _ptr(loss), _stream()))
    return g, loss


def mlp_adam(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place (hss_mlp_adam)."""
    np_ = params.numel()
    _check(lib().hss_mlp_adam(np_, _f32(params, "params"), _f32(grad, "grad", (np_,)), _f32(m, "m", (np_,)),
                              _f32(v, "v", (np_,)), lr, beta1, beta2, eps, step, _stream()))


def mlp_train(sizes, params, m, v, step, X, T, M, batch, epochs, lr, seed=0):
    """Mini-batch Adam on the device (hss_mlp_train).  Returns (loss per epoch, new step)."""
    n = X.shape[0]
    npar = mlp_num_params(sizes)
    st = C.c_int64(step)
    losses = np.zeros(max(1, epochs), dtype=np.float32)
    _check(lib().hss_mlp_train(C.byref(_mlp(sizes)), _f32(params, "params", (npar,)), _f32(m, "m", (npar,)),
                               _f32(v, "v", (npar,)), C.byref(st), _f32(X, "X", (n, sizes[0])),
                               _f32(T, "T", (n, sizes[-1])), _f32(M, "M", (n, sizes[-1])), n, batch, epochs,
                               lr, seed, losses.ctypes.data, _stream()))
    return losses[:epochs], st.value
