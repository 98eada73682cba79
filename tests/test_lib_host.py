"""Host-side checks of libaqr (no GPU): exported symbols, quantiser and graph
builder parity with the oracle, and argument validation."""
import os
import re

import numpy as np
import pytest

from paper_2602_21600_amd import aqr
from paper_2602_21600_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return aqr.lib()


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "aqr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aqr_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    declared = _declared_symbols()
    assert len(declared) >= 19
    for name in declared:
        assert hasattr(L, name), name
    assert set(aqr.SYMBOLS) == set(declared)
    assert aqr.aqr_version() == 1


def _train_both(orc, X, M0=16, efc0=100, p_max=0.01, threads=0, **kw):
    params = aqr.default_qparams(M0=M0, efc0=efc0, p_max=p_max, threads=threads)
    params.update(kw)
    qz, codes = aqr.aqr_quantize(X, params)
    ref = orc.train(X, p_max=p_max, M0=M0, efc0=efc0,
                    n_s=params["n_sample"], threshold=params["sample_threshold"])
    return qz, codes, ref


@pytest.mark.parametrize("n,d,threshold", [(2000, 24, 10000), (3000, 20, 1000), (1500, 100, 10000)])
def test_quantize_matches_oracle(orc, n, d, threshold):
    X, _ = W.tiny(n, d, seed=n + d, clusters=7)
    qz, codes, ref = _train_both(orc, X, sample_threshold=threshold, n_sample=500)
    info = aqr.aqr_quantizer_info(qz)
    # same definitions, same FP64 summation order: identical values
    assert info["delta"] == ref["delta"]
    assert info["p_lo"] == ref["p_lo"] and info["p_hi"] == ref["p_hi"]
    assert info["eta"] == ref["eta"] == 0.0
    assert info["s_dist"] == ref["s_dist"]
    assert (info["M"], info["efc"]) == (ref["M"], ref["efc"])
    np.testing.assert_array_equal(info["min"], ref["min"])
    np.testing.assert_array_equal(info["max"], ref["max"])
    np.testing.assert_array_equal(info["scale"], ref["scale"])
    d_pad = (d + 15) // 16 * 16
    assert codes.shape == (n, d_pad) and info["d_pad"] == d_pad
    oc = orc.encode(X, ref["min"], ref["scale"], stride=d_pad)
    np.testing.assert_array_equal(codes, oc)


def test_quantize_small_workload_matches_oracle(orc):
    X = W.base("small")
    qz, codes, ref = _train_both(orc, X)
    info = aqr.aqr_quantizer_info(qz)
    assert info["delta"] == ref["delta"]
    np.testing.assert_array_equal(info["min"], ref["min"])
    np.testing.assert_array_equal(info["max"], ref["max"])
    np.testing.assert_array_equal(codes, orc.encode(X, ref["min"], ref["scale"], stride=128))


def test_quantize_image_like_rows_match_oracle(orc):
    # 784 dimensions with about half the values zero (the Fashion-MNIST
    # shape): many dimensions have a zero lower bound, some are almost
    # constant
    X = W.base("fmnist", 3000)
    assert 0.3 < float((X == 0).mean()) < 0.7
    qz, codes, ref = _train_both(orc, X)
    info = aqr.aqr_quantizer_info(qz)
    assert info["delta"] == ref["delta"]
    np.testing.assert_array_equal(info["min"], ref["min"])
    np.testing.assert_array_equal(info["max"], ref["max"])
    np.testing.assert_array_equal(codes, orc.encode(X, ref["min"], ref["scale"], stride=784))


@pytest.mark.parametrize("n,d,k_rho,threshold", [(2500, 20, 10, 1000), (900, 13, 64, 10000),
                                                 (3, 5, 10, 10000)])
def test_host_density_matches_oracle(orc, n, d, k_rho, threshold):
    X, _ = W.tiny(n, d, seed=n + k_rho, clusters=4) if n > 50 else (
        np.random.default_rng(0).standard_normal((n, d)).astype(np.float32), None)
    p = aqr.default_qparams()
    p.update(k_rho=k_rho, n_sample=400, sample_threshold=threshold)
    ref = orc.density(X, k_rho=k_rho, n_s=400, threshold=threshold)
    np.testing.assert_array_equal(aqr.aqr_density(X, p), ref)


def test_density_rejects_bad_parameters():
    X = np.ones((10, 4), np.float32)
    for bad in (dict(k_rho=0), dict(k_rho=65), dict(n_sample=0), dict(eps=0.0)):
        p = aqr.default_qparams()
        p.update(bad)
        with pytest.raises(aqr.AqrError):
            aqr.aqr_density(X, p)


@pytest.mark.parametrize("n,d,threshold", [(2000, 12, 10000), (3000, 20, 1000), (900, 37, 10000)])
def test_quantize_per_dimension_weights_match_oracle(orc, n, d, threshold):
    # the per-dimension reading of w_j: eta > 0, and with it M_i, ef^c and
    # s_dist, identical to the oracle's; the codes do not depend on w_j
    X, _ = W.tiny(n, d, seed=n, clusters=5)
    X[100:140] = X[5]
    p = aqr.default_qparams(weights=1)
    p.update(sample_threshold=threshold, n_sample=500)
    qz, codes = aqr.aqr_quantize(X, p)
    a = aqr.aqr_quantizer_info(qz)
    r = orc.train(X, weights=1, n_s=500, threshold=threshold)
    assert a["eta"] == r["eta"] and a["eta"] > 0.0
    assert (a["s_dist"], a["w_mean"], a["M"], a["efc"]) == (r["s_dist"], r["w_mean"], r["M"],
                                                            r["efc"])
    assert a["M"] > orc.train(X, n_s=500, threshold=threshold)["M"]
    np.testing.assert_array_equal(codes, orc.encode(X, r["min"], r["scale"], stride=a["d_pad"]))


def test_quantize_rejects_unknown_weights():
    X = np.random.default_rng(0).standard_normal((50, 4)).astype(np.float32)
    with pytest.raises(aqr.AqrError):
        aqr.aqr_quantize(X, aqr.default_qparams(weights=2))


def test_quantize_encode_only(orc):
    X, Y = W.tiny(800, 16, seed=2, nq=50)
    qz, codes = aqr.aqr_quantize(X, aqr.default_qparams())
    _, ycodes = aqr.aqr_quantize(Y, qz=qz)
    info = aqr.aqr_quantizer_info(qz)
    np.testing.assert_array_equal(ycodes, orc.encode(Y, info["min"], info["scale"], stride=16))


def test_quantize_rejects_bad_input(L):
    X = np.ones((10, 4), np.float32)
    X[3, 2] = np.nan
    with pytest.raises(aqr.AqrError) as e:
        aqr.aqr_quantize(X, aqr.default_qparams())
    assert e.value.status == aqr.INVALID_ARG
    X[3, 2] = np.inf
    with pytest.raises(aqr.AqrError):
        aqr.aqr_quantize(X, aqr.default_qparams())
    bad = aqr.default_qparams()
    bad["k_rho"] = 0
    with pytest.raises(aqr.AqrError) as e:
        aqr.aqr_quantize(np.ones((10, 4), np.float32), bad)
    assert "out of range" in str(e.value)
    qz, _ = aqr.aqr_quantize(np.random.default_rng(0).random((20, 4)).astype(np.float32),
                             aqr.default_qparams())
    with pytest.raises(aqr.AqrError):
        aqr.aqr_quantize(np.ones((10, 5), np.float32), qz=qz)


def _both_graphs(orc, X, M0, efc0, seed):
    qz, codes, ref = _train_both(orc, X, M0=M0, efc0=efc0)
    info = aqr.aqr_quantizer_info(qz)
    u = 1.0 - np.random.default_rng(seed).random(X.shape[0])
    g = aqr.aqr_build(codes, X.shape[1], qz, threads=1, level_u=u)
    lv = orc.levels(u, info["M"])
    og = orc.build(codes, X.shape[1], info["M"], info["efc"], lv)
    return aqr.aqr_graph_export(g), og, info


@pytest.mark.parametrize("n,d,M0,efc0", [(1500, 16, 6, 40), (2500, 32, 16, 100)])
def test_sequential_build_matches_oracle(orc, n, d, M0, efc0):
    X, _ = W.tiny(n, d, seed=n, clusters=5)
    eg, og, info = _both_graphs(orc, X, M0, efc0, seed=n)
    np.testing.assert_array_equal(eg["level"], og["level"])
    assert (eg["ep"], eg["L"]) == (og["ep"], og["L"])
    np.testing.assert_array_equal(eg["upper_off"], og["upper_off"])
    np.testing.assert_array_equal(eg["adj0"], og["adj0"])
    np.testing.assert_array_equal(eg["upper_adj"][: og["upper_off"][-1]],
                                  og["upper_adj"][: og["upper_off"][-1]])


def test_sequential_build_small_workload_matches_oracle(orc):
    X = W.base("small", 4000)
    eg, og, _ = _both_graphs(orc, X, 16, 100, seed=7)
    np.testing.assert_array_equal(eg["adj0"], og["adj0"])
    assert (eg["ep"], eg["L"]) == (og["ep"], og["L"])


def test_parallel_build_invariants(orc):
    from test_oracle_graph import check_invariants
    X, _ = W.tiny(3000, 24, seed=5, clusters=6)
    qz, codes = aqr.aqr_quantize(X, aqr.default_qparams(M0=8, efc0=40))
    g = aqr.aqr_build(codes, 24, qz, threads=4, seed=99)
    eg = aqr.aqr_graph_export(g)
    check_invariants(eg, eg["M"])
    # most points are found by an exhaustive search from the entry point
    from test_oracle_search import _reachable
    assert _reachable(eg["adj0"], eg["ep"]).size > 0.99 * 3000


def test_graph_import_round_trip_and_corruption(orc):
    X, _ = W.tiny(600, 8, seed=1)
    qz, codes = aqr.aqr_quantize(X, aqr.default_qparams(M0=4, efc0=20))
    eg = aqr.aqr_graph_export(aqr.aqr_build(codes, 8, qz, threads=1, seed=3))
    g2 = aqr.aqr_graph_import(eg)
    e2 = aqr.aqr_graph_export(g2)
    for key in ("level", "adj0", "upper_off"):
        np.testing.assert_array_equal(eg[key], e2[key])
    bad = dict(eg)
    bad["adj0"] = eg["adj0"].copy()
    bad["adj0"][5, 0] = 10 ** 6
    with pytest.raises(aqr.AqrError) as e:
        aqr.aqr_graph_import(bad)
    assert e.value.status == aqr.CORRUPT
    bad = dict(eg)
    bad["level"] = eg["level"].copy()
    bad["level"][0] += 1
    with pytest.raises(aqr.AqrError) as e:
        aqr.aqr_graph_import(bad)
    assert e.value.status == aqr.CORRUPT


def test_null_handles_are_rejected(L):
    import ctypes as C
    assert L.aqr_search(None, None, 1, None, None, None, None, None, None, None, None, 0, None,
                        None) == aqr.INVALID_ARG
    assert b"null" in L.aqr_last_error()
    assert L.aqr_rerank(None, None, 1, None, None, 1, None, None, None, None, None, None,
                        None) == aqr.INVALID_ARG
    assert L.aqr_search_fp32(None, None, 1, None, None, None, None, None, None, 0, None,
                             None) == aqr.INVALID_ARG
    assert L.aqr_index_bind(None, None, None, None, None, 0, None, C.byref(C.c_void_p())) == \
        aqr.INVALID_ARG
    assert L.aqr_build(None, 1, 1, None, None, None, C.byref(C.c_void_p())) == aqr.INVALID_ARG


def test_server_entry_points_reject_bad_arguments(L):
    import ctypes as C
    h = C.c_void_p()
    p = aqr.ServerParams(ring=8, k_max=10, ef_max=64, m_ef=3, n_rerank=28, tau_gap=0.01,
                         tau_ratio=1.008, eps=1e-6)
    assert L.aqr_server_workspace_size() >= 24
    assert L.aqr_server_create(None, C.byref(p), None, 0, C.byref(h)) == aqr.INVALID_ARG
    assert b"null" in L.aqr_last_error()
    t = C.c_uint64()
    assert L.aqr_server_submit(None, None, 1, 1, C.byref(t)) == aqr.INVALID_ARG
    done = C.c_int32()
    assert L.aqr_server_poll(None, 0, None, None, C.byref(done)) == aqr.INVALID_ARG
    assert L.aqr_server_stop(None) == aqr.INVALID_ARG
    assert L.aqr_server_replay(None, 0, None, None, None, None, None, None, None, None,
                               None) == aqr.INVALID_ARG
    L.aqr_server_destroy(None)


def test_binding_rejects_malformed_buffers():
    # The binding checks dtype, rank and size of every buffer before any
    # launch: a narrower dtype or a short buffer would be read or written
    # past its end by the kernels.  Checked on the host with CPU tensors
    # (the device check comes last, so a well-formed CPU tensor fails only
    # for being on the host).
    import types
    import torch
    from paper_2602_21600_amd import aqr
    ix = types.SimpleNamespace(d=8, d_pad=16, ptr=None)
    nq, ns = 5, 12
    Q = torch.zeros((nq, 8), dtype=torch.float32)
    k = torch.ones(nq, dtype=torch.int32)
    ef = torch.ones(nq, dtype=torch.int32)
    cid = torch.zeros((nq, ns), dtype=torch.int32)
    cD = torch.zeros((nq, ns), dtype=torch.int32)
    cnt = torch.zeros(nq, dtype=torch.int32)
    ws = torch.zeros(256, dtype=torch.uint8)

    def search(**kw):
        a = dict(Q=Q, k=k, ef=ef, cand_id=cid, cand_D=cD, cand_cnt=cnt, ws=ws)
        a.update(kw)
        aqr.aqr_search(ix, a["Q"], a["k"], a["ef"], a["cand_id"], a["cand_D"], a["cand_cnt"],
                       a["ws"], 64, ns)

    bad = [
        (dict(Q=Q.double()), "Q: dtype"),
        (dict(Q=torch.zeros((nq, 9), dtype=torch.float32)), "Q: 9 columns"),
        (dict(Q=torch.zeros(8, dtype=torch.float32)), "Q: 1-D"),
        (dict(k=k.long()), "k: dtype"),
        (dict(k=k[:3]), "k: 3 rows"),
        (dict(ef=ef[:4]), "ef: 4 rows"),
        (dict(cand_id=cid[:, :6].contiguous()), "cand_id: 6 columns"),
        (dict(cand_D=torch.zeros((2, ns), dtype=torch.int32)), "cand_D: 2 rows"),
        (dict(cand_cnt=cnt.float()), "cand_cnt: dtype"),
        (dict(ws=ws.int()), "ws: dtype"),
    ]
    for kw, msg in bad:
        with pytest.raises(ValueError, match=msg):
            search(**kw)
    # well-formed host tensors pass the shape checks and stop at the device check
    with pytest.raises(ValueError, match="device tensor"):
        search()

    out_id = torch.zeros((nq, 10), dtype=torch.int32)
    out_d = torch.zeros((nq, 10), dtype=torch.float32)
    with pytest.raises(ValueError, match="out_dist: dtype"):
        aqr.aqr_rerank(ix, Q, cid, cnt, k, out_id, out_d.double())
    with pytest.raises(ValueError, match="out_dist: 7 columns"):
        aqr.aqr_rerank(ix, Q, cid, cnt, k, out_id, torch.zeros((nq, 7)))
    with pytest.raises(ValueError, match="k: 2 rows"):
        aqr.aqr_rerank(ix, Q, cid, cnt, k[:2], out_id, out_d)
    with pytest.raises(ValueError, match="out_id: 4 rows"):
        aqr.aqr_search_fp32(ix, Q, k, ef, out_id[:4], out_d, ws, 64, 10)
    with pytest.raises(ValueError, match="out_id: 10 columns, expected 12"):
        aqr.aqr_search_fp32(ix, Q, k, ef, out_id, out_d, ws, 64, 12)
    with pytest.raises(ValueError, match="qcodes: 8 columns, expected 16"):
        aqr.aqr_encode_queries(ix, Q, torch.zeros((nq, 8), dtype=torch.uint8))
    with pytest.raises(ValueError, match="taps.counts"):
        aqr.aqr_search(ix, Q, k, ef, cid, cD, cnt, ws, 64, ns,
                       taps=dict(cap=0, counts=torch.zeros((nq, 4), dtype=torch.int32)))


def test_chunked_seed_is_thread_independent_and_matches_oracle(orc):
    # seed_n = n: every point is seeded, so aqr_build_batched inserts them all
    # in chunks on the host and never needs a device; the graph must be the
    # same on one and on eight threads and equal the oracle's chunked build,
    # and chunks of one point must give the sequential build
    X, _ = W.tiny(2500, 20, seed=17, clusters=5)
    qz, codes, ref = _train_both(orc, X, M0=8, efc0=40)
    info = aqr.aqr_quantizer_info(qz)
    n = X.shape[0]
    u = 1.0 - np.random.default_rng(23).random(n)
    g1 = aqr.aqr_graph_export(aqr.aqr_build_batched(codes, X, 20, qz, threads=1, level_u=u,
                                                    seed_n=n, batch=64))
    g8 = aqr.aqr_graph_export(aqr.aqr_build_batched(codes, X, 20, qz, threads=8, level_u=u,
                                                    seed_n=n, batch=64))
    og = orc.build_batched(codes, 20, info["M"], info["efc"], orc.levels(u, info["M"]), n, 64)
    rows = og["upper_off"][-1]
    for eg in (g1, g8):
        np.testing.assert_array_equal(eg["adj0"], og["adj0"])
        np.testing.assert_array_equal(eg["upper_adj"][:rows], og["upper_adj"][:rows])
        assert (eg["ep"], eg["L"]) == (og["ep"], og["L"])
    seq = aqr.aqr_graph_export(aqr.aqr_build(codes, 20, qz, threads=1, level_u=u))
    unit = aqr.aqr_graph_export(aqr.aqr_build_batched(codes, X, 20, qz, threads=4, level_u=u,
                                                      seed_n=n, batch=1))
    np.testing.assert_array_equal(unit["adj0"], seq["adj0"])
    np.testing.assert_array_equal(unit["upper_adj"][:rows], seq["upper_adj"][:rows])
    assert (unit["ep"], unit["L"]) == (seq["ep"], seq["L"])
    assert not np.array_equal(g1["adj0"], seq["adj0"])  # chunks of up to 64 points differ
