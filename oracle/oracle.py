"""ctypes wrapper of the C oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.

Each function is a thin marshalling layer over one C function of
aqr_oracle.c; the arithmetic lives there, with the citations.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NONE = 0xFFFFFFFF

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_u32 = C.c_uint32
_f64 = C.c_double


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    lib = C.CDLL(_LIB_PATH)
    lib.orc_set_threads.argtypes = [_i32]
    lib.orc_get_threads.restype = _i32
    lib.orc_density.argtypes = [_f32p, _i64, _i32, _i32, _f64, _i64, _i64, _f64p]
    lib.orc_density.restype = _i32
    lib.orc_delta.argtypes = [_f64p, _i64, _f64]
    lib.orc_delta.restype = _f64
    lib.orc_percentile_sorted.argtypes = [_f64p, _i64, _f64]
    lib.orc_percentile_sorted.restype = _f64
    lib.orc_train_ranges.argtypes = [_f32p, _i64, _i32, _f64p, _f64, _f64, _f32p, _f32p, _f32p,
                                     _f64p, C.c_void_p]
    lib.orc_train_ranges.restype = _i32
    lib.orc_dim_weights.argtypes = [_f32p, _i64, _i32, _i32, _f64, _i64, _i64, _f64p]
    lib.orc_dim_weights.restype = _i32
    lib.orc_build_params.argtypes = [_i32, _i32, _f64, _f64, _i32p]
    lib.orc_encode.argtypes = [_f32p, _i64, _i32, _f32p, _f32p, _u8p, _i32]
    lib.orc_encode.restype = _i32
    lib.orc_decode.argtypes = [_u8p, _i64, _i32, _i32, _f32p, _f32p, _f32p]
    lib.orc_levels.argtypes = [_f64p, _i64, _i32, _i32p]
    lib.orc_levels.restype = _i32
    lib.orc_select_heuristic_f32.argtypes = [_f32p, _i32, _u32, _u32p, _i32, _i32, _u32p]
    lib.orc_select_heuristic_f32.restype = _i32
    lib.orc_build.argtypes = [_u8p, _i64, _i32, _i32, _i32, _i32, _i32p, _u32p, _i64p, _u32p,
                              _i32p]
    lib.orc_build.restype = _i32
    lib.orc_build_batched.argtypes = [_u8p, _i64, _i32, _i32, _i32, _i32, _i32p, _i64, _i32,
                                      _i32, _u32p, _i64p, _u32p, _i32p]
    lib.orc_build_batched.restype = _i32
    lib.orc_param_map.argtypes = [_i32, _i32, _i32, _i32p]
    lib.orc_search_codes.argtypes = [_u8p, _i64, _i32, _i32, _i32, _i32p, _u32p, _i64p, _u32p,
                                     _u32, _i32, _u8p, _i64, _i32p, _i32p, _i32, _u32p, _u32p,
                                     _i32p, _i32, _vp, _vp, _vp, _vp]
    lib.orc_search_codes.restype = _i32
    lib.orc_search_f32.argtypes = [_f32p, _i64, _i32, _i32, _i32p, _u32p, _i64p, _u32p, _u32,
                                   _i32, _f32p, _i64, _i32p, _i32p, _i32, _i32p, _f64p, _vp,
                                   _vp, _i32, _vp]
    lib.orc_search_f32.restype = _i32
    lib.orc_rerank.argtypes = [_f32p, _u8p, _i64, _i32, _i32, _f32p, _f32p, _f32p, _i64, _u32p,
                               _i32p, _i32, _i32p, _i32, _i32, _f64, _f64, _f64, _vp, _i32, _vp,
                               _i32p, _f64p, _vp, _vp, _vp, _vp, _vp]
    lib.orc_rerank.restype = _i32
    lib.orc_knn_f32.argtypes = [_f32p, _i64, _i32, _f32p, _i64, _i32, _i32p, _f64p]
    lib.orc_knn_f32.restype = _i32
    lib.orc_knn_codes.argtypes = [_u8p, _i64, _i32, _i32, _u8p, _i64, _i32, _u32p, _u32p]
    lib.orc_knn_codes.restype = _i32
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle: {what} failed (rc={rc})")


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def get_threads() -> int:
    return int(_load().orc_get_threads())


# --------------------------------------------------------------------------
# Section 3.1: density, heterogeneity, quantiser training, encoding
# --------------------------------------------------------------------------

def density(X, k_rho=10, eps=1e-6, n_s=5000, threshold=10000):
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    rho = np.zeros(n, np.float64)
    _check(_load().orc_density(X, n, d, k_rho, eps, n_s, threshold, rho), "density")
    return rho


def delta(rho, eps=1e-6):
    rho = np.ascontiguousarray(rho, np.float64)
    return float(_load().orc_delta(rho, rho.size, eps))


def percentile_sorted(v, p):
    v = np.ascontiguousarray(v, np.float64)
    return float(_load().orc_percentile_sorted(v, v.size, p))


def build_params(M0, efc0, delta_, eta):
    out = np.zeros(2, np.int32)
    _load().orc_build_params(int(M0), int(efc0), float(delta_), float(eta), out)
    return int(out[0]), int(out[1])


def dim_weights(X, k_rho=10, eps=1e-6, n_s=5000, threshold=10000):
    """Per-dimension density weights w_j (the per-dimension reading of
    Algorithm 1's w_j): mean one-dimensional k_rho-NN density along j."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    w = np.zeros(d, np.float64)
    _check(_load().orc_dim_weights(X, n, d, k_rho, eps, n_s, threshold, w), "dim_weights")
    return w


def train(X, p_max=0.01, M0=16, efc0=200, k_rho=10, eps=1e-6, n_s=5000, threshold=10000,
          rho=None, weights=0):
    """Alg. 1 stages 1-2 plus the build parameters.  Returns a dict.
    weights 0: every w_j is the mean density (the literal reading);
    1: per-dimension weights (dim_weights)."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    if rho is None:
        rho = density(X, k_rho, eps, n_s, threshold)
    w = dim_weights(X, k_rho, eps, n_s, threshold) if weights == 1 else None
    mn = np.zeros(d, np.float32)
    mx = np.zeros(d, np.float32)
    sc = np.zeros(d, np.float32)
    s = np.zeros(6, np.float64)
    _check(_load().orc_train_ranges(X, n, d, rho, eps, p_max, mn, mx, sc, s,
                                    None if w is None else w.ctypes.data), "train_ranges")
    M_i, efc = build_params(M0, efc0, s[0], s[4])
    return dict(rho=rho, delta=float(s[0]), p_lo=float(s[1]), p_hi=float(s[2]),
                s_dist=float(s[3]), eta=float(s[4]), w_mean=float(s[5]), min=mn, max=mx,
                scale=sc, M=M_i, efc=efc, d=d, p_max=p_max, w=w)


def encode(X, mn, scale, stride=None):
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    stride = d if stride is None else int(stride)
    codes = np.zeros((n, stride), np.uint8)
    rc = _load().orc_encode(X, n, d, np.ascontiguousarray(mn, np.float32),
                            np.ascontiguousarray(scale, np.float32), codes, stride)
    if rc != 0:
        raise ValueError("oracle: encode rejected the input (non-finite value)")
    return codes


def decode(codes, d, mn, scale):
    codes = np.ascontiguousarray(codes, np.uint8)
    n, stride = codes.shape
    out = np.zeros((n, d), np.float32)
    _load().orc_decode(codes, n, d, stride, np.ascontiguousarray(mn, np.float32),
                       np.ascontiguousarray(scale, np.float32), out)
    return out


# --------------------------------------------------------------------------
# Section 3.1 stage 3: HNSW graph over the codes
# --------------------------------------------------------------------------

def levels(u, M):
    u = np.ascontiguousarray(u, np.float64)
    lv = np.zeros(u.size, np.int32)
    _check(_load().orc_levels(u, u.size, int(M), lv), "levels")
    return lv


def upper_offsets(level):
    """Row offsets of the upper-layer rows: node i owns level[i] rows."""
    off = np.zeros(level.size + 1, np.int64)
    np.cumsum(level.astype(np.int64), out=off[1:])
    return off


def select_heuristic_f32(X, base, ids, M):
    X = np.ascontiguousarray(X, np.float32)
    ids = np.ascontiguousarray(ids, np.uint32)
    out = np.zeros(max(M, 1), np.uint32)
    r = _load().orc_select_heuristic_f32(X, X.shape[1], int(base), ids, ids.size, int(M), out)
    _check(0 if r >= 0 else -1, "select_heuristic")
    return out[:r].copy()


def build(codes, d, M, efc, level):
    """Sequential HNSW build; returns the graph as plain arrays."""
    codes = np.ascontiguousarray(codes, np.uint8)
    n, stride = codes.shape
    level = np.ascontiguousarray(level, np.int32)
    off = upper_offsets(level)
    adj0 = np.zeros((n, 2 * M), np.uint32)
    upper = np.zeros((max(int(off[-1]), 1), M), np.uint32)
    out2 = np.zeros(2, np.int32)
    _check(_load().orc_build(codes, n, d, stride, int(M), int(efc), level, adj0, off, upper,
                             out2), "build")
    return dict(n=n, M=int(M), level=level, adj0=adj0, upper_off=off, upper_adj=upper,
                ep=int(out2[0]), L=int(out2[1]))


def build_batched(codes, d, M, efc, level, seed_n, batch, seed_batch=64):
    """Batched HNSW build: chunks of at most seed_batch seed points that plan
    on every level against the graph as it stood before the chunk, then
    chunks of at most batch level-0 points that search it the same way."""
    codes = np.ascontiguousarray(codes, np.uint8)
    n, stride = codes.shape
    level = np.ascontiguousarray(level, np.int32)
    off = upper_offsets(level)
    adj0 = np.zeros((n, 2 * M), np.uint32)
    upper = np.zeros((max(int(off[-1]), 1), M), np.uint32)
    out2 = np.zeros(2, np.int32)
    _check(_load().orc_build_batched(codes, n, d, stride, int(M), int(efc), level, int(seed_n),
                                     int(seed_batch), int(batch), adj0, off, upper, out2),
           "build_batched")
    return dict(n=n, M=int(M), level=level, adj0=adj0, upper_off=off, upper_adj=upper,
                ep=int(out2[0]), L=int(out2[1]))


def _g(graph):
    return (graph["M"], np.ascontiguousarray(graph["level"], np.int32),
            np.ascontiguousarray(graph["adj0"], np.uint32),
            np.ascontiguousarray(graph["upper_off"], np.int64),
            np.ascontiguousarray(graph["upper_adj"], np.uint32), graph["ep"], graph["L"])


# --------------------------------------------------------------------------
# Section 3.2: search and re-rank
# --------------------------------------------------------------------------

def param_map(k, ef, m_ef=3):
    out = np.zeros(2, np.int32)
    _load().orc_param_map(int(k), int(ef), int(m_ef), out)
    return int(out[0]), int(out[1])


def search_codes(graph, codes, d, qcodes, ef_eff, nc, nc_stride=None, tap_cap=0):
    """Stage 1 for a batch of encoded queries.  Returns a dict."""
    codes = np.ascontiguousarray(codes, np.uint8)
    n, stride = codes.shape
    qcodes = np.ascontiguousarray(qcodes, np.uint8)
    nq = qcodes.shape[0]
    assert qcodes.shape[1] == stride
    ef_eff = np.ascontiguousarray(np.broadcast_to(ef_eff, (nq,)), np.int32)
    nc = np.ascontiguousarray(np.broadcast_to(nc, (nq,)), np.int32)
    nc_stride = int(nc.max()) if nc_stride is None else int(nc_stride)
    cid = np.full((nq, nc_stride), NONE, np.uint32)
    cD = np.full((nq, nc_stride), NONE, np.uint32)
    cnt = np.zeros(nq, np.int32)
    exp = vis = nexp = nvis = None
    if tap_cap > 0:
        exp = np.zeros((nq, tap_cap), np.uint32)
        vis = np.zeros((nq, tap_cap), np.uint32)
        nexp = np.zeros(nq, np.int64)
        nvis = np.zeros(nq, np.int64)
    M, lv, a0, off, up, ep, L = _g(graph)
    _check(_load().orc_search_codes(codes, n, d, stride, M, lv, a0, off, up, ep, L, qcodes, nq,
                                    ef_eff, nc, nc_stride, cid, cD, cnt, int(tap_cap), _ptr(exp),
                                    _ptr(nexp), _ptr(vis), _ptr(nvis)), "search_codes")
    res = dict(cand_id=cid, cand_D=cD, cand_cnt=cnt)
    if tap_cap > 0:
        res.update(expanded=exp, n_expanded=nexp, visited=vis, n_visited=nvis)
    return res


def search_f32(graph, X, Q, ef_eff, k, k_stride=None, with_visits=False, tap_cap=0):
    """Baseline FP32 HNSW (distances in FP64).  Returns (ids, dists), plus the
    visit counts with with_visits, plus (expanded, n_expanded) with tap_cap."""
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    Q = np.ascontiguousarray(Q, np.float32)
    nq = Q.shape[0]
    ef_eff = np.ascontiguousarray(np.broadcast_to(ef_eff, (nq,)), np.int32)
    k = np.ascontiguousarray(np.broadcast_to(k, (nq,)), np.int32)
    k_stride = int(k.max()) if k_stride is None else int(k_stride)
    oid = np.zeros((nq, k_stride), np.int32)
    od = np.zeros((nq, k_stride), np.float64)
    nvis = np.zeros(nq, np.int64) if with_visits else None
    exp = np.zeros((nq, tap_cap), np.uint32) if tap_cap else None
    nexp = np.zeros(nq, np.int32) if tap_cap else None
    M, lv, a0, off, up, ep, L = _g(graph)
    _check(_load().orc_search_f32(X, n, d, M, lv, a0, off, up, ep, L, Q, nq, ef_eff, k, k_stride,
                                  oid, od, _ptr(nvis), _ptr(exp), int(tap_cap), _ptr(nexp)),
           "search_f32")
    out = (oid, od)
    if with_visits:
        out = out + (nvis,)
    if tap_cap:
        out = out + (exp, nexp)
    return out


def rerank(X, codes, mn, scale, Q, cand_id, cand_cnt, k, n_rerank=28, tau_gap=0.010,
           tau_ratio=1.008, eps=1e-6, force_et=None, a_order=None, k_stride=None, taps=False,
           assembly=0):
    """Stages 2-3, early termination and assembly.  Returns a dict.

    assembly 0 fills R from A only while it holds fewer than k entries (the
    reading "as needed to ensure at least k"); 1 joins every remaining
    candidate of A to the exact results (the union reading)."""
    if assembly not in (0, 1):
        raise ValueError("assembly must be 0 (fill) or 1 (union)")
    X = np.ascontiguousarray(X, np.float32)
    n, d = X.shape
    codes = np.ascontiguousarray(codes, np.uint8)
    stride = codes.shape[1]
    Q = np.ascontiguousarray(Q, np.float32)
    nq = Q.shape[0]
    cand_id = np.ascontiguousarray(cand_id, np.uint32)
    nc_stride = cand_id.shape[1]
    cand_cnt = np.ascontiguousarray(cand_cnt, np.int32)
    k = np.ascontiguousarray(np.broadcast_to(k, (nq,)), np.int32)
    k_stride = int(k.max()) if k_stride is None else int(k_stride)
    fe = None if force_et is None else np.ascontiguousarray(
        np.broadcast_to(force_et, (nq,)), np.int32)
    ao = None if a_order is None else np.ascontiguousarray(a_order, np.uint32)
    oid = np.zeros((nq, k_stride), np.int32)
    od = np.zeros((nq, k_stride), np.float64)
    ok = np.zeros((nq, k_stride), np.uint8)
    aid = ad = et = nrr = None
    if taps:
        aid = np.zeros((nq, nc_stride), np.uint32)
        ad = np.zeros((nq, nc_stride), np.float64)
        et = np.zeros(nq, np.uint8)
        nrr = np.zeros(nq, np.int32)
    _check(_load().orc_rerank(X, codes, n, d, stride, np.ascontiguousarray(mn, np.float32),
                              np.ascontiguousarray(scale, np.float32), Q, nq, cand_id, cand_cnt,
                              nc_stride, k, k_stride, int(n_rerank), float(tau_gap),
                              float(tau_ratio), float(eps), _ptr(fe), int(assembly), _ptr(ao),
                              oid, od, _ptr(ok),
                              _ptr(aid), _ptr(ad), _ptr(et), _ptr(nrr)), "rerank")
    res = dict(id=oid, dist=od, kind=ok)
    if taps:
        res.update(a_id=aid, a_dist=ad, et=et, nrr=nrr)
    return res


def knn_f32(X, Q, k):
    X = np.ascontiguousarray(X, np.float32)
    Q = np.ascontiguousarray(Q, np.float32)
    n, d = X.shape
    nq = Q.shape[0]
    oid = np.zeros((nq, k), np.int32)
    od = np.zeros((nq, k), np.float64)
    _check(_load().orc_knn_f32(X, n, d, Q, nq, int(k), oid, od), "knn_f32")
    return oid, od


def knn_codes(codes, d, qcodes, k):
    codes = np.ascontiguousarray(codes, np.uint8)
    qcodes = np.ascontiguousarray(qcodes, np.uint8)
    n, stride = codes.shape
    nq = qcodes.shape[0]
    oid = np.zeros((nq, k), np.uint32)
    oD = np.zeros((nq, k), np.uint32)
    _check(_load().orc_knn_codes(codes, n, d, stride, qcodes, nq, int(k), oid, oD), "knn_codes")
    return oid, oD


# --------------------------------------------------------------------------
# whole query path (Alg. 2): encode, Stage 1, Stages 2-3
# --------------------------------------------------------------------------

def query(index, Q, k, ef, m_ef=3, n_rerank=28, tau_gap=0.010, tau_ratio=1.008, eps=1e-6,
          taps=False, assembly=0):
    """index: dict with X, codes, d, min, scale, graph.  Returns a dict."""
    Q = np.ascontiguousarray(Q, np.float32)
    nq = Q.shape[0]
    k = np.broadcast_to(np.asarray(k, np.int32), (nq,))
    ef = np.broadcast_to(np.asarray(ef, np.int32), (nq,))
    efe = np.zeros(nq, np.int32)
    nc = np.zeros(nq, np.int32)
    for i in range(nq):
        efe[i], nc[i] = param_map(int(k[i]), int(ef[i]), m_ef)
    qc = encode(Q, index["min"], index["scale"], stride=index["codes"].shape[1])
    s1 = search_codes(index["graph"], index["codes"], index["d"], qc, efe, nc,
                      tap_cap=(65536 if taps else 0))
    rr = rerank(index["X"], index["codes"], index["min"], index["scale"], Q, s1["cand_id"],
                s1["cand_cnt"], k, n_rerank, tau_gap, tau_ratio, eps, taps=taps,
                assembly=assembly)
    rr["stage1"] = s1
    rr["qcodes"] = qc
    return rr
