"""Python binding of libaqr (argument marshalling only).

Every function here forwards to the C-ABI entry point of the same name in
libaqr.so (declared in include/aqr.h); all computation happens in the
library's host code and gfx950 kernels.  PyTorch provides device memory
and streams.  If libaqr.so is missing the import of this module's
functions fails with an error: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaqr.so")

OK, INVALID_ARG, OOM, DEVICE, BUSY, CORRUPT, STATE = range(7)
NONE = 0xFFFFFFFF


class AqrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libaqr status {status}: {msg}")
        self.status = status


class QParams(C.Structure):
    _fields_ = [("k_rho", C.c_int32), ("threads", C.c_int32), ("n_sample", C.c_int64),
                ("sample_threshold", C.c_int64), ("eps", C.c_double), ("p_max", C.c_double),
                ("M0", C.c_int32), ("efc0", C.c_int32), ("weights", C.c_int32)]


class QInfo(C.Structure):
    _fields_ = [("d", C.c_int32), ("d_pad", C.c_int32), ("M", C.c_int32), ("efc", C.c_int32),
                ("delta", C.c_double), ("p_lo", C.c_double), ("p_hi", C.c_double),
                ("s_dist", C.c_double), ("eta", C.c_double), ("w_mean", C.c_double)]


class BParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("efc", C.c_int32), ("threads", C.c_int32),
                ("progress", C.c_int32), ("seed", C.c_uint64)]


class GInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("M", C.c_int32), ("efc", C.c_int32), ("L", C.c_int32),
                ("ep", C.c_uint32), ("upper_rows", C.c_int64)]


class SParams(C.Structure):
    _fields_ = [("ef_max", C.c_int32), ("out_stride", C.c_int32), ("m_ef", C.c_int32),
                ("waves_per_block", C.c_int32), ("blocks", C.c_int32),
                ("visited_log2", C.c_int32), ("order", C.c_void_p), ("ef_small", C.c_int32),
                ("small_waves", C.c_int32)]


class Taps(C.Structure):
    _fields_ = [("cap", C.c_int32), ("expanded", C.c_void_p), ("evaluated", C.c_void_p),
                ("counts", C.c_void_p)]


class RParams(C.Structure):
    _fields_ = [("n_rerank", C.c_int32), ("out_stride", C.c_int32), ("tau_gap", C.c_float),
                ("tau_ratio", C.c_float), ("eps", C.c_float), ("force_et", C.c_int32),
                ("waves_per_block", C.c_int32), ("assembly", C.c_int32)]


class RTaps(C.Structure):
    _fields_ = [("a_id", C.c_void_p), ("a_dist", C.c_void_p), ("et", C.c_void_p),
                ("nrr", C.c_void_p)]


class BatchBuffers(C.Structure):
    _fields_ = [("Q", C.c_void_p), ("nq_max", C.c_int64), ("k", C.c_void_p), ("ef", C.c_void_p),
                ("cand_id", C.c_void_p), ("cand_D", C.c_void_p), ("cand_cnt", C.c_void_p),
                ("out_id", C.c_void_p), ("out_dist", C.c_void_p), ("out_kind", C.c_void_p),
                ("order", C.c_void_p), ("ws", C.c_void_p), ("ws_bytes", C.c_size_t),
                ("counts", C.c_void_p)]


_lib = None

_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_u32 = C.c_uint32
_sz = C.c_size_t

# (name, restype, argtypes)
class ServerParams(C.Structure):
    _fields_ = [("ring", _i32), ("k_max", _i32), ("ef_max", _i32), ("m_ef", _i32),
                ("n_rerank", _i32), ("tau_gap", C.c_float), ("tau_ratio", C.c_float),
                ("eps", C.c_float), ("waves_per_block", _i32), ("visited_log2", _i32),
                ("idle_ms", _i32), ("reserved", _i32), ("state_budget", _i64),
                ("lds_budget_pages", _i64)]


class ServerUsage(C.Structure):
    _fields_ = [("ring", _i32), ("slots_used", _i32), ("lds_budget_pages", _i64),
                ("lds_used_pages", _i64), ("state_budget", _i64), ("state_used", _i64),
                ("blocks", _i32), ("run_pages", _i32)]


class IndexFileInfo(C.Structure):
    _fields_ = [("n", _i64), ("d", _i32), ("d_pad", _i32), ("M", _i32), ("reserved", _i32),
                ("upper_rows", _i64), ("file_bytes", C.c_uint64)]


_SIGS = [
    ("aqr_last_error", C.c_char_p, []),
    ("aqr_version", _i32, []),
    ("aqr_quantize", _i32, [_vp, _i64, _i32, C.POINTER(QParams), C.POINTER(_vp), _vp]),
    ("aqr_quantize_device", _i32, [_vp, _i64, _i32, C.POINTER(QParams), C.POINTER(_vp), _vp]),
    ("aqr_density", _i32, [_vp, _i64, _i32, C.POINTER(QParams), _i32, _vp]),
    ("aqr_quantizer_info", _i32, [_vp, C.POINTER(QInfo), _vp, _vp, _vp]),
    ("aqr_quantizer_create", _i32, [C.POINTER(QInfo), _vp, _vp, _vp, C.POINTER(_vp)]),
    ("aqr_quantizer_free", None, [_vp]),
    ("aqr_build", _i32, [_vp, _i64, _i32, _vp, C.POINTER(BParams), _vp, C.POINTER(_vp)]),
    ("aqr_build_batched", _i32, [_vp, _vp, _i64, _i32, _vp, C.POINTER(BParams), _vp, _i64, _i32,
                                 _i32, C.POINTER(_vp)]),
    ("aqr_graph_info", _i32, [_vp, C.POINTER(GInfo)]),
    ("aqr_graph_export", _i32, [_vp, _vp, _vp, _vp, _vp]),
    ("aqr_graph_import", _i32, [_i64, _i32, _vp, _vp, _vp, _vp, _u32, C.POINTER(_vp)]),
    ("aqr_graph_free", None, [_vp]),
    ("aqr_index_save", _i32, [C.c_char_p, _vp, _vp, _vp, _vp]),
    ("aqr_index_file_info", _i32, [C.c_char_p, C.POINTER(IndexFileInfo)]),
    ("aqr_index_load", _i32, [C.c_char_p, C.POINTER(_vp), C.POINTER(_vp), _vp, _vp]),
    ("aqr_index_bytes", _i32, [_vp, _vp, C.POINTER(_sz)]),
    ("aqr_index_bind", _i32, [_vp, _vp, _vp, _vp, _vp, _sz, _vp, C.POINTER(_vp)]),
    ("aqr_index_free", None, [_vp]),
    ("aqr_search_workspace_size", _sz, []),
    ("aqr_search", _i32, [_vp, _vp, _i64, _vp, _vp, _vp, C.POINTER(SParams), _vp, _vp, _vp,
                          _vp, _sz, C.POINTER(Taps), _vp]),
    ("aqr_encode_queries", _i32, [_vp, _vp, _i64, _vp, _vp]),
    ("aqr_rerank", _i32, [_vp, _vp, _i64, _vp, _vp, _i32, _vp, C.POINTER(RParams), _vp, _vp,
                          _vp, C.POINTER(RTaps), _vp]),
    ("aqr_search_fp32", _i32, [_vp, _vp, _i64, _vp, _vp, C.POINTER(SParams), _vp, _vp, _vp,
                               _sz, C.POINTER(Taps), _vp]),
    ("aqr_knn_workspace_size", _sz, [_i64, _i64, _i32]),
    ("aqr_knn_bruteforce", _i32, [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _sz,
                                  _vp]),
    ("aqr_knn_noalloc_max_bytes", _sz, []),
    ("aqr_knn_bruteforce_noalloc", _i32, [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _vp, _vp, _vp]),
    ("aqr_plan_create", _i32, [_vp, C.POINTER(SParams), C.POINTER(RParams),
                               C.POINTER(BatchBuffers), _i32, C.POINTER(_vp)]),
    ("aqr_plan_launch", _i32, [_vp, _i64, _vp]),
    ("aqr_plan_free", None, [_vp]),
    ("aqr_server_workspace_size", _sz, []),
    ("aqr_server_create", _i32, [_vp, C.POINTER(ServerParams), _vp, _sz, C.POINTER(_vp)]),
    ("aqr_server_submit", _i32, [_vp, _vp, _i32, _i32, C.POINTER(C.c_uint64)]),
    ("aqr_server_poll", _i32, [_vp, C.c_uint64, _vp, _vp, C.POINTER(_i32)]),
    ("aqr_server_request_cost", _i32, [_vp, _i32, _i32, C.POINTER(_i32), C.POINTER(_i64)]),
    ("aqr_server_usage", _i32, [_vp, C.POINTER(ServerUsage)]),
    ("aqr_server_stop", _i32, [_vp]),
    ("aqr_server_destroy", None, [_vp]),
    ("aqr_server_replay", _i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                 C.POINTER(C.c_double)]),
]

SYMBOLS = [s[0] for s in _SIGS]


def lib():
    """Load libaqr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libaqr.so not found at {LIB_PATH}; build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    # PyTorch loads its HIP runtime by path; importing it first makes libaqr's
    # dependency on libamdhip64.so.7 resolve to that same copy, so the process
    # holds a single HIP runtime shared by torch's allocations and libaqr.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    for name, res, args in _SIGS:
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st):
    if st != OK:
        raise AqrError(st, lib().aqr_last_error().decode(errors="replace"))


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t):
    """Device pointer of a torch CUDA tensor (None passes as NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _need(name, t, dtypes, ndim, rows=None, cols=None, optional=False):
    """Host-side argument checks of a device tensor before a launch: dtype,
    rank, at least `rows` rows and, for 2-D tensors, at least `cols` columns
    (exactly `cols` when cols is a tuple (n,)).  A kernel reads and writes
    through raw pointers, so a narrower dtype or a short buffer would be read
    or written past its end on the device."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name}: missing")
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor")
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype}, expected one of {dtypes}")
    if t.dim() != ndim:
        raise ValueError(f"{name}: {t.dim()}-D, expected {ndim}-D")
    if rows is not None and t.shape[0] < rows:
        raise ValueError(f"{name}: {t.shape[0]} rows, at least {rows} needed")
    if cols is not None and ndim == 2:
        if isinstance(cols, tuple):
            if t.shape[1] != cols[0]:
                raise ValueError(f"{name}: {t.shape[1]} columns, expected {cols[0]}")
        elif t.shape[1] < cols:
            raise ValueError(f"{name}: {t.shape[1]} columns, at least {cols} needed")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")


def _i32_types():
    import torch
    return (torch.int32,)


def _f32_types():
    import torch
    return (torch.float32,)


def _u8_types():
    import torch
    return (torch.uint8,)


def _check_queries(ix, Q):
    _need("Q", Q, _f32_types(), 2, cols=(ix.d,))
    return Q.shape[0]


def _check_search_args(ix, Q, k, ef, ws, order, nc=None):
    nq = _check_queries(ix, Q)
    _need("k", k, _i32_types(), 1, rows=nq)
    _need("ef", ef, _i32_types(), 1, rows=nq)
    _need("nc", nc, _i32_types(), 1, rows=nq, optional=True)
    _need("order", order, _i32_types(), 1, rows=nq, optional=True)
    _need("ws", ws, _u8_types(), 1)
    return nq


def _check_taps(taps, nq):
    if not taps:
        return
    cap = int(taps.get("cap", 0))
    _need("taps.counts", taps.get("counts"), _i32_types(), 2, rows=nq, cols=(8,), optional=True)
    for name in ("expanded", "evaluated"):
        _need(f"taps.{name}", taps.get(name), _i32_types(), 2, rows=nq, cols=cap, optional=True)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------------
# handles
# --------------------------------------------------------------------------

class _Handle:
    _free = None

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        p, self.ptr = getattr(self, "ptr", None), None
        if p and _lib is not None:
            getattr(_lib, self._free)(p)

    @property
    def as_parameter(self):
        return self.ptr


class Quantizer(_Handle):
    _free = "aqr_quantizer_free"


class Graph(_Handle):
    _free = "aqr_graph_free"


class Plan(_Handle):
    _free = "aqr_plan_free"

    def __init__(self, ptr, keep):
        super().__init__(ptr)
        self.keep = keep  # device buffers and parameter structs the plan points to


class Index(_Handle):
    _free = "aqr_index_free"

    def __init__(self, ptr, arena, d, d_pad):
        super().__init__(ptr)
        self.arena = arena  # keep the device memory alive
        self.d = d
        self.d_pad = d_pad


# --------------------------------------------------------------------------
# C-ABI wrappers
# --------------------------------------------------------------------------

def aqr_version():
    return int(lib().aqr_version())


def default_qparams(M0=16, efc0=200, p_max=0.01, threads=0, weights=0):
    return dict(k_rho=10, threads=threads, n_sample=5000, sample_threshold=10000, eps=1e-6,
                p_max=p_max, M0=M0, efc0=efc0, weights=weights)


def aqr_quantize(X, params=None, qz=None, codes=True, device=False):
    """Train (qz None) or reuse a quantiser; returns (Quantizer, codes or None).
    device=True: aqr_quantize_device (the density search on the current
    device, same result)."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    p = QParams(**(params or default_qparams()))
    h = C.c_void_p(qz.ptr if qz is not None else None)
    d_pad = (d + 15) // 16 * 16
    out = np.zeros((n, d_pad), np.uint8) if codes else None
    fn = lib().aqr_quantize_device if device else lib().aqr_quantize
    _check(fn(_np_ptr(X), n, d, C.byref(p), C.byref(h), _np_ptr(out)))
    return (qz if qz is not None else Quantizer(h.value)), out


def aqr_density(X, params=None, device=False):
    """Densities rho (n doubles) of the quantiser's Stage 1 (aqr_density)."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    p = QParams(**(params or default_qparams()))
    rho = np.zeros(n, np.float64)
    _check(lib().aqr_density(_np_ptr(X), n, d, C.byref(p), 1 if device else 0, _np_ptr(rho)))
    return rho


def aqr_quantizer_info(qz):
    info = QInfo()
    _check(lib().aqr_quantizer_info(qz.ptr, C.byref(info), None, None, None))
    d = info.d
    mn = np.zeros(d, np.float32)
    mx = np.zeros(d, np.float32)
    sc = np.zeros(d, np.float32)
    _check(lib().aqr_quantizer_info(qz.ptr, None, _np_ptr(mn), _np_ptr(mx), _np_ptr(sc)))
    res = {f: getattr(info, f) for f, _ in QInfo._fields_}
    res.update(min=mn, max=mx, scale=sc)
    return res


def aqr_quantizer_create(info, mn, mx, scale):
    qi = QInfo(**{f: info[f] for f, _ in QInfo._fields_})
    mn = np.ascontiguousarray(mn, np.float32)
    mx = np.ascontiguousarray(mx, np.float32)
    sc = np.ascontiguousarray(scale, np.float32)
    h = C.c_void_p()
    _check(lib().aqr_quantizer_create(C.byref(qi), _np_ptr(mn), _np_ptr(mx), _np_ptr(sc),
                                      C.byref(h)))
    return Quantizer(h.value)


def aqr_build(codes, d, qz, M=0, efc=0, threads=0, seed=0, level_u=None, progress=0):
    codes = np.ascontiguousarray(codes, np.uint8)
    n = codes.shape[0]
    bp = BParams(M=M, efc=efc, threads=threads, progress=progress, seed=seed)
    lu = None if level_u is None else np.ascontiguousarray(level_u, np.float64)
    h = C.c_void_p()
    _check(lib().aqr_build(_np_ptr(codes), n, d, qz.ptr, C.byref(bp), _np_ptr(lu), C.byref(h)))
    return Graph(h.value)


def aqr_build_batched(codes, X, d, qz, M=0, efc=0, threads=0, seed=0, level_u=None, progress=0,
                      seed_n=None, batch=16384, seed_batch=64):
    """Batched build with the chunk searches on the device (aqr_build_batched).
    seed_n defaults to max(20000, n / 64)."""
    codes = np.ascontiguousarray(codes, np.uint8)
    X = np.ascontiguousarray(X, np.float32)
    n = codes.shape[0]
    if X.shape != (n, d):
        raise ValueError("X must be n x d")
    seed_n = max(20000, n // 64) if seed_n is None else int(seed_n)
    bp = BParams(M=M, efc=efc, threads=threads, progress=progress, seed=seed)
    lu = None if level_u is None else np.ascontiguousarray(level_u, np.float64)
    h = C.c_void_p()
    _check(lib().aqr_build_batched(_np_ptr(codes), _np_ptr(X), n, d, qz.ptr, C.byref(bp),
                                   _np_ptr(lu), seed_n, int(seed_batch), int(batch), C.byref(h)))
    return Graph(h.value)


def aqr_graph_info(g):
    gi = GInfo()
    _check(lib().aqr_graph_info(g.ptr, C.byref(gi)))
    return {f: getattr(gi, f) for f, _ in GInfo._fields_}


def aqr_graph_export(g):
    gi = aqr_graph_info(g)
    n, M, rows = gi["n"], gi["M"], gi["upper_rows"]
    level = np.zeros(n, np.int32)
    adj0 = np.zeros((n, 2 * M), np.uint32)
    off = np.zeros(n + 1, np.int64)
    upper = np.zeros((max(rows, 1), M), np.uint32)
    _check(lib().aqr_graph_export(g.ptr, _np_ptr(level), _np_ptr(adj0), _np_ptr(off),
                                  _np_ptr(upper)))
    return dict(n=n, M=M, level=level, adj0=adj0, upper_off=off, upper_adj=upper, ep=gi["ep"],
                L=gi["L"], efc=gi["efc"])


def aqr_graph_import(gd):
    level = np.ascontiguousarray(gd["level"], np.int32)
    adj0 = np.ascontiguousarray(gd["adj0"], np.uint32)
    off = np.ascontiguousarray(gd["upper_off"], np.int64)
    upper = np.ascontiguousarray(gd["upper_adj"], np.uint32)
    h = C.c_void_p()
    _check(lib().aqr_graph_import(int(gd["n"]), int(gd["M"]), _np_ptr(level), _np_ptr(adj0),
                                  _np_ptr(off), _np_ptr(upper), int(gd["ep"]), C.byref(h)))
    return Graph(h.value)


def aqr_index_save(path, qz, g, codes, X):
    """Write quantiser, codes, FP32 rows and graph to one checksummed file."""
    codes = np.ascontiguousarray(codes, np.uint8)
    X = np.ascontiguousarray(X, np.float32)
    info = aqr_quantizer_info(qz)
    gi = aqr_graph_info(g)
    if codes.shape != (gi["n"], info["d_pad"]) or X.shape != (gi["n"], info["d"]):
        raise ValueError("codes / X do not match the quantiser and the graph")
    _check(lib().aqr_index_save(os.fsencode(path), qz.ptr, g.ptr, _np_ptr(codes), _np_ptr(X)))


def aqr_index_file_info(path):
    fi = IndexFileInfo()
    _check(lib().aqr_index_file_info(os.fsencode(path), C.byref(fi)))
    return {f: getattr(fi, f) for f, _ in IndexFileInfo._fields_ if f != "reserved"}


def aqr_index_load(path):
    """Returns (quantizer, graph, codes, X) from an index file."""
    fi = aqr_index_file_info(path)
    codes = np.empty((fi["n"], fi["d_pad"]), np.uint8)
    X = np.empty((fi["n"], fi["d"]), np.float32)
    q, g = _vp(), _vp()
    _check(lib().aqr_index_load(os.fsencode(path), C.byref(q), C.byref(g), _np_ptr(codes),
                                _np_ptr(X)))
    return Quantizer(q.value), Graph(g.value), codes, X


def aqr_index_bytes(qz, g):
    b = C.c_size_t()
    _check(lib().aqr_index_bytes(qz.ptr, g.ptr, C.byref(b)))
    return int(b.value)


def aqr_index_bind(qz, g, codes, X, device=None, stream=None):
    """Allocate the device arena with torch and bind the index into it."""
    import torch
    codes = np.ascontiguousarray(codes, np.uint8)
    X = np.ascontiguousarray(X, np.float32)
    nbytes = aqr_index_bytes(qz, g)
    arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    base = arena.data_ptr()
    pad = (-base) % 256
    h = C.c_void_p()
    _check(lib().aqr_index_bind(qz.ptr, g.ptr, _np_ptr(codes), _np_ptr(X),
                                C.c_void_p(base + pad), nbytes, _stream_ptr(stream), C.byref(h)))
    info = aqr_quantizer_info(qz)
    return Index(h.value, arena, info["d"], info["d_pad"])


def aqr_search_workspace_size():
    return int(lib().aqr_search_workspace_size())


def _taps(taps):
    if taps is None:
        return None
    t = Taps(cap=int(taps.get("cap", 0)), expanded=_dev_ptr(taps.get("expanded")),
             evaluated=_dev_ptr(taps.get("evaluated")), counts=_dev_ptr(taps.get("counts")))
    return C.byref(t), t


def aqr_search(ix, Q, k, ef, cand_id, cand_D, cand_cnt, ws, ef_max, out_stride, nc=None, m_ef=3,
               waves_per_block=0, blocks=0, visited_log2=0, order=None, taps=None, stream=None,
               ef_small=0, small_waves=0):
    nq = _check_search_args(ix, Q, k, ef, ws, order, nc)
    _need("cand_id", cand_id, _i32_types(), 2, rows=nq, cols=out_stride)
    _need("cand_D", cand_D, _i32_types(), 2, rows=nq, cols=out_stride)
    _need("cand_cnt", cand_cnt, _i32_types(), 1, rows=nq)
    if cand_id.shape[1] != out_stride or cand_D.shape[1] != out_stride:
        raise ValueError("cand_id/cand_D: the row stride must equal out_stride")
    _check_taps(taps, nq)
    sp = SParams(ef_max=ef_max, out_stride=out_stride, m_ef=m_ef,
                 waves_per_block=waves_per_block, blocks=blocks, visited_log2=visited_log2,
                 order=_dev_ptr(order), ef_small=ef_small, small_waves=small_waves)
    tp = _taps(taps)
    _check(lib().aqr_search(ix.ptr, _dev_ptr(Q), Q.shape[0], _dev_ptr(k), _dev_ptr(ef),
                            _dev_ptr(nc), C.byref(sp), _dev_ptr(cand_id), _dev_ptr(cand_D),
                            _dev_ptr(cand_cnt), _dev_ptr(ws), ws.numel() * ws.element_size(),
                            tp[0] if tp else None, _stream_ptr(stream)))


def aqr_search_fp32(ix, Q, k, ef, out_id, out_dist, ws, ef_max, out_stride, waves_per_block=0,
                    blocks=0, visited_log2=0, order=None, taps=None, stream=None, ef_small=0,
                    small_waves=0):
    nq = _check_search_args(ix, Q, k, ef, ws, order)
    _need("out_id", out_id, _i32_types(), 2, rows=nq, cols=(out_stride,))
    _need("out_dist", out_dist, _f32_types(), 2, rows=nq, cols=(out_stride,))
    _check_taps(taps, nq)
    sp = SParams(ef_max=ef_max, out_stride=out_stride, m_ef=1,
                 waves_per_block=waves_per_block, blocks=blocks, visited_log2=visited_log2,
                 order=_dev_ptr(order), ef_small=ef_small, small_waves=small_waves)
    tp = _taps(taps)
    _check(lib().aqr_search_fp32(ix.ptr, _dev_ptr(Q), Q.shape[0], _dev_ptr(k), _dev_ptr(ef),
                                 C.byref(sp), _dev_ptr(out_id), _dev_ptr(out_dist), _dev_ptr(ws),
                                 ws.numel() * ws.element_size(), tp[0] if tp else None,
                                 _stream_ptr(stream)))


def aqr_encode_queries(ix, Q, qcodes, stream=None):
    nq = _check_queries(ix, Q)
    _need("qcodes", qcodes, _u8_types(), 2, rows=nq, cols=(ix.d_pad,))
    _check(lib().aqr_encode_queries(ix.ptr, _dev_ptr(Q), Q.shape[0], _dev_ptr(qcodes),
                                    _stream_ptr(stream)))


def aqr_rerank(ix, Q, cand_id, cand_cnt, k, out_id, out_dist, out_kind=None, n_rerank=28,
               tau_gap=0.010, tau_ratio=1.008, eps=1e-6, force_et=-1, out_stride=None,
               waves_per_block=0, taps=None, stream=None, assembly=0):
    nq = _check_queries(ix, Q)
    _need("cand_id", cand_id, _i32_types(), 2, rows=nq)
    _need("cand_cnt", cand_cnt, _i32_types(), 1, rows=nq)
    _need("k", k, _i32_types(), 1, rows=nq)
    _need("out_id", out_id, _i32_types(), 2, rows=nq)
    out_stride = out_id.shape[1] if out_stride is None else out_stride
    if out_id.shape[1] != out_stride:
        raise ValueError("out_id: the row stride must equal out_stride")
    _need("out_dist", out_dist, _f32_types(), 2, rows=nq, cols=(out_stride,))
    _need("out_kind", out_kind, _u8_types(), 2, rows=nq, cols=(out_stride,), optional=True)
    if taps is not None:
        nc = cand_id.shape[1]
        _need("taps.a_id", taps.get("a_id"), _i32_types(), 2, rows=nq, cols=(nc,), optional=True)
        _need("taps.a_dist", taps.get("a_dist"), _f32_types(), 2, rows=nq, cols=(nc,),
              optional=True)
        _need("taps.et", taps.get("et"), _u8_types(), 1, rows=nq, optional=True)
        _need("taps.nrr", taps.get("nrr"), _i32_types(), 1, rows=nq, optional=True)
    rp = RParams(n_rerank=n_rerank, out_stride=out_stride, tau_gap=tau_gap, tau_ratio=tau_ratio,
                 eps=eps, force_et=force_et, waves_per_block=waves_per_block, assembly=assembly)
    rt = None
    if taps is not None:
        rt = RTaps(a_id=_dev_ptr(taps.get("a_id")), a_dist=_dev_ptr(taps.get("a_dist")),
                   et=_dev_ptr(taps.get("et")), nrr=_dev_ptr(taps.get("nrr")))
    _check(lib().aqr_rerank(ix.ptr, _dev_ptr(Q), Q.shape[0], _dev_ptr(cand_id),
                            _dev_ptr(cand_cnt), cand_id.shape[1], _dev_ptr(k), C.byref(rp),
                            _dev_ptr(out_id), _dev_ptr(out_dist), _dev_ptr(out_kind),
                            C.byref(rt) if rt is not None else None, _stream_ptr(stream)))


def aqr_knn_workspace_size(n, nq, k):
    return int(lib().aqr_knn_workspace_size(int(n), int(nq), int(k)))


def aqr_knn_bruteforce(X, Q, k, out_id=None, out_dist=None, certified=None, ws=None,
                       stream=None):
    """Exact k nearest neighbours of the rows of Q among the rows of X (device
    FP32 tensors) by brute force; returns (ids int32 [nq][k], dists FP64
    [nq][k], certified uint8 [nq]) as device tensors."""
    import torch
    _need("X", X, _f32_types(), 2)
    n, d = X.shape
    _need("Q", Q, _f32_types(), 2, cols=(d,))
    nq = Q.shape[0]
    dev = X.device
    if out_id is None:
        out_id = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if out_dist is None:
        out_dist = torch.empty((nq, k), dtype=torch.float64, device=dev)
    if certified is None:
        certified = torch.empty(nq, dtype=torch.uint8, device=dev)
    _need("out_id", out_id, _i32_types(), 2, rows=nq, cols=(k,))
    _need("out_dist", out_dist, (torch.float64,), 2, rows=nq, cols=(k,))
    _need("certified", certified, _u8_types(), 1, rows=nq)
    need = aqr_knn_workspace_size(n, nq, k)
    if ws is None:
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device=dev)
    _need("ws", ws, _u8_types(), 1, rows=need)
    _check(lib().aqr_knn_bruteforce(_dev_ptr(X), n, d, _dev_ptr(Q), nq, int(k), _dev_ptr(out_id),
                                    _dev_ptr(out_dist), _dev_ptr(certified), _dev_ptr(ws),
                                    ws.numel(), _stream_ptr(stream)))
    return out_id, out_dist, certified


def aqr_knn_bruteforce_noalloc(X, Q, k, out_id, out_dist, certified=None, stream=None):
    """aqr_knn_bruteforce into caller-given outputs, with the library's fixed
    device scratch instead of a workspace (nothing is allocated)."""
    import torch
    _need("X", X, _f32_types(), 2)
    n, d = X.shape
    _need("Q", Q, _f32_types(), 2, cols=(d,))
    nq = Q.shape[0]
    _need("out_id", out_id, _i32_types(), 2, rows=nq, cols=(k,))
    _need("out_dist", out_dist, (torch.float64,), 2, rows=nq, cols=(k,))
    _need("certified", certified, _u8_types(), 1, rows=nq, optional=True)
    _check(lib().aqr_knn_bruteforce_noalloc(_dev_ptr(X), n, d, _dev_ptr(Q), nq, int(k),
                                            _dev_ptr(out_id), _dev_ptr(out_dist),
                                            _dev_ptr(certified), _stream_ptr(stream)))
    return out_id, out_dist, certified


# --------------------------------------------------------------------------
# convenience: a bound index with preallocated query buffers
# --------------------------------------------------------------------------

class QueryPlan:
    """Device buffers for batches of up to nq queries (allocated with torch).

    run() issues Stage 1 and Stages 2-3 on the current stream: the whole
    query path of Alg. 2 for one batch.
    """

    def __init__(self, ix, nq, k_max, ef_max, m_ef=3, n_rerank=28, tau_gap=0.010,
                 tau_ratio=1.008, eps=1e-6, nc_max=None, visited_log2=0, waves_per_block=0,
                 blocks=0, assembly=0):
        import torch
        self.ix = ix
        self.nq = nq
        self.k_max = k_max
        self.ef_max = max(ef_max, k_max)
        self.m_ef = m_ef
        self.nc_max = nc_max or min(self.ef_max, max(k_max, self.ef_max // m_ef))
        self.rr = dict(n_rerank=n_rerank, tau_gap=tau_gap, tau_ratio=tau_ratio, eps=eps,
                       assembly=assembly)
        self.sp = dict(visited_log2=visited_log2, waves_per_block=waves_per_block, blocks=blocks)
        dev = ix.arena.device
        self.cand_id = torch.empty((nq, self.nc_max), dtype=torch.int32, device=dev)
        self.cand_D = torch.empty((nq, self.nc_max), dtype=torch.int32, device=dev)
        self.cand_cnt = torch.empty(nq, dtype=torch.int32, device=dev)
        self.out_id = torch.empty((nq, k_max), dtype=torch.int32, device=dev)
        self.out_dist = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
        self.out_kind = torch.empty((nq, k_max), dtype=torch.uint8, device=dev)
        self.ws = torch.zeros(aqr_search_workspace_size(), dtype=torch.uint8, device=dev)

    def run(self, Q, k, ef, nc=None, order=None):
        n = _check_queries(self.ix, Q)
        if n > self.nq:
            raise ValueError(f"Q: {n} queries, the plan holds {self.nq}")
        cid, cD, cc = self.cand_id[:n], self.cand_D[:n], self.cand_cnt[:n]
        aqr_search(self.ix, Q, k, ef, cid, cD, cc, self.ws, self.ef_max, self.nc_max, nc=nc,
                   m_ef=self.m_ef, order=order, **self.sp)
        aqr_rerank(self.ix, Q, cid, cc, k, self.out_id[:n], self.out_dist[:n],
                   self.out_kind[:n], **self.rr)
        return self.out_id[:n], self.out_dist[:n]


def aqr_plan_create(ix, sparams, rparams, buffers, use_graph=True):
    """sparams/rparams: dicts of SParams/RParams fields; buffers: dict of torch
    tensors (Q, k, ef, cand_id, cand_D, cand_cnt, out_id, out_dist, out_kind,
    order, ws, counts; optional entries may be None)."""
    sp = SParams(**sparams)
    rp = RParams(**rparams)
    t = buffers
    bb = BatchBuffers(Q=_dev_ptr(t["Q"]), nq_max=t["Q"].shape[0], k=_dev_ptr(t["k"]),
                      ef=_dev_ptr(t["ef"]), cand_id=_dev_ptr(t["cand_id"]),
                      cand_D=_dev_ptr(t["cand_D"]), cand_cnt=_dev_ptr(t["cand_cnt"]),
                      out_id=_dev_ptr(t["out_id"]), out_dist=_dev_ptr(t["out_dist"]),
                      out_kind=_dev_ptr(t.get("out_kind")), order=_dev_ptr(t.get("order")),
                      ws=_dev_ptr(t["ws"]), ws_bytes=t["ws"].numel(),
                      counts=_dev_ptr(t.get("counts")))
    h = C.c_void_p()
    _check(lib().aqr_plan_create(ix.ptr, C.byref(sp), C.byref(rp), C.byref(bb),
                                 1 if use_graph else 0, C.byref(h)))
    return Plan(h.value, (t, sp, rp, bb, ix))


def aqr_plan_launch(plan, nq, stream=None):
    _check(lib().aqr_plan_launch(plan.ptr, int(nq), _stream_ptr(stream)))


class BatchPlan:
    """Device buffers for uneven batches (per-query k and ef) and a plan over
    them: longest-first order, Stage 1 and Stages 2-3, optionally replayed
    as one captured graph.  Copy queries and parameters in with load(), then
    launch()."""

    def __init__(self, ix, nq_max, k_max, ef_max, m_ef=3, n_rerank=28, tau_gap=0.010,
                 tau_ratio=1.008, eps=1e-6, longest_first=True, use_graph=True, counts=False,
                 tuning=None, assembly=0):
        import torch
        tuning = dict(tuning or {})
        dev = ix.arena.device
        self.ix = ix
        self.nq_max = nq_max
        self.k_max = k_max
        self.ef_max = max(ef_max, k_max)
        self.nc_max = min(self.ef_max, max(k_max, self.ef_max // m_ef))
        i32 = torch.int32
        self.bufs = dict(
            Q=torch.zeros((nq_max, ix.d), dtype=torch.float32, device=dev),
            k=torch.ones(nq_max, dtype=i32, device=dev),
            ef=torch.ones(nq_max, dtype=i32, device=dev),
            cand_id=torch.zeros((nq_max, self.nc_max), dtype=i32, device=dev),
            cand_D=torch.zeros((nq_max, self.nc_max), dtype=i32, device=dev),
            cand_cnt=torch.zeros(nq_max, dtype=i32, device=dev),
            out_id=torch.zeros((nq_max, k_max), dtype=i32, device=dev),
            out_dist=torch.zeros((nq_max, k_max), dtype=torch.float32, device=dev),
            out_kind=torch.zeros((nq_max, k_max), dtype=torch.uint8, device=dev),
            order=torch.zeros(nq_max, dtype=i32, device=dev) if longest_first else None,
            ws=torch.zeros(aqr_search_workspace_size(), dtype=torch.uint8, device=dev),
            counts=torch.zeros((nq_max, 8), dtype=i32, device=dev) if counts else None)
        sp = dict(ef_max=self.ef_max, out_stride=self.nc_max, m_ef=m_ef,
                  waves_per_block=tuning.get("waves_per_block", 0),
                  blocks=tuning.get("blocks", 0), visited_log2=tuning.get("visited_log2", 0),
                  order=None, ef_small=tuning.get("ef_small", 0),
                  small_waves=tuning.get("small_waves", 0))
        rp = dict(n_rerank=n_rerank, out_stride=k_max, tau_gap=tau_gap, tau_ratio=tau_ratio,
                  eps=eps, force_et=-1, waves_per_block=tuning.get("rerank_waves_per_block", 0),
                  assembly=assembly)
        self.plan = aqr_plan_create(ix, sp, rp, self.bufs, use_graph)

    def load(self, Q, k, ef):
        n = _check_queries(self.ix, Q)
        if n > self.nq_max:
            raise ValueError(f"Q: {n} queries, the plan holds {self.nq_max}")
        _need("k", k, _i32_types(), 1, rows=n)
        _need("ef", ef, _i32_types(), 1, rows=n)
        self.bufs["Q"][:n].copy_(Q)
        self.bufs["k"][:n].copy_(k)
        self.bufs["ef"][:n].copy_(ef)
        return n

    def launch(self, nq, stream=None):
        aqr_plan_launch(self.plan, nq, stream)
        return self.bufs["out_id"][:nq], self.bufs["out_dist"][:nq]


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------

AQR_ERR_BUSY = 4


class Server(_Handle):
    """A resident persistent kernel fed from a ring of requests in pinned host
    memory (continuous admission).  submit() admits one query (host array of
    d floats) and returns a ticket; poll() returns None until the request is
    complete, then (ids, dists) rows of length k_max padded with (-1, inf)."""

    _free = "aqr_server_destroy"

    def __init__(self, ix, k_max, ef_max, ring=1024, m_ef=3, n_rerank=28, tau_gap=0.010,
                 tau_ratio=1.008, eps=1e-6, waves_per_block=0, visited_log2=0, idle_ms=50,
                 state_budget=0, lds_budget_pages=0):
        import torch
        self.ix = ix
        self.k_max = k_max
        self.ws = torch.zeros(int(lib().aqr_server_workspace_size()), dtype=torch.uint8,
                              device=ix.arena.device)
        p = ServerParams(ring=ring, k_max=k_max, ef_max=ef_max, m_ef=m_ef, n_rerank=n_rerank,
                         tau_gap=tau_gap, tau_ratio=tau_ratio, eps=eps,
                         waves_per_block=waves_per_block, visited_log2=visited_log2,
                         idle_ms=idle_ms, reserved=0,
                         state_budget=state_budget, lds_budget_pages=lds_budget_pages)
        h = _vp()
        _check(lib().aqr_server_create(ix.ptr, C.byref(p), _dev_ptr(self.ws), self.ws.numel(),
                                       C.byref(h)))
        super().__init__(h.value)

    def submit(self, q, k, ef):
        q = np.ascontiguousarray(q, np.float32).reshape(-1)
        if q.shape[0] != self.ix.d:
            raise ValueError(f"q: {q.shape[0]} values, the index has d = {self.ix.d}")
        t = C.c_uint64()
        st = lib().aqr_server_submit(self.ptr, _np_ptr(q), int(k), int(ef), C.byref(t))
        if st == AQR_ERR_BUSY:
            return None
        _check(st)
        return t.value

    def poll(self, ticket):
        ids = np.empty(self.k_max, np.int32)
        dist = np.empty(self.k_max, np.float32)
        done = _i32()
        _check(lib().aqr_server_poll(self.ptr, C.c_uint64(ticket), _np_ptr(ids), _np_ptr(dist),
                                     C.byref(done)))
        return (ids, dist) if done.value else None

    def stop(self):
        _check(lib().aqr_server_stop(self.ptr))

    def request_cost(self, k, ef):
        """(LDS pages, state bytes) a request of this k and ef is charged."""
        p, b = _i32(), _i64()
        _check(lib().aqr_server_request_cost(self.ptr, int(k), int(ef), C.byref(p), C.byref(b)))
        return p.value, b.value

    def usage(self):
        u = ServerUsage()
        _check(lib().aqr_server_usage(self.ptr, C.byref(u)))
        return {f: getattr(u, f) for f, _ in ServerUsage._fields_}

    def replay(self, arrival_s, Q, k, ef, service=False):
        """Replay an arrival trace natively; returns (ids, dists, latency_s, wall_s),
        plus the per-request device service times when service=True."""
        n = len(arrival_s)
        arr = np.ascontiguousarray(arrival_s, np.float64)
        Q = np.ascontiguousarray(Q, np.float32)
        k = np.ascontiguousarray(k, np.int32)
        ef = np.ascontiguousarray(ef, np.int32)
        if Q.ndim != 2 or Q.shape[0] != n or Q.shape[1] != self.ix.d:
            raise ValueError(f"Q: shape {Q.shape}, expected ({n}, {self.ix.d})")
        if k.shape != (n,) or ef.shape != (n,):
            raise ValueError("k, ef: one entry per request expected")
        ids = np.empty((n, self.k_max), np.int32)
        dist = np.empty((n, self.k_max), np.float32)
        lat = np.empty(n, np.float64)
        svc = np.empty(n, np.float64) if service else None
        wall = C.c_double()
        _check(lib().aqr_server_replay(self.ptr, n, _np_ptr(arr), _np_ptr(Q), _np_ptr(k),
                                       _np_ptr(ef), _np_ptr(ids), _np_ptr(dist), _np_ptr(lat),
                                       _np_ptr(svc), C.byref(wall)))
        if service:
            return ids, dist, lat, wall.value, svc
        return ids, dist, lat, wall.value
