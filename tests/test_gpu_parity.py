"""GPU parity of the query path against the oracle, through the C-ABI.

Integer work (query codes, Stage-1 distances, expansion order, distinct
visited set, candidate order) must be bit-exact.  FP32 distances must be
within 1e-5 relative of the oracle's FP64 values; early-termination
decisions may differ only when the oracle's gap or ratio is within 1e-5
relative of its threshold, and then the oracle is rerun with the GPU's
decision and A order before the top-k ids are compared.
"""
import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-5
NONE = 0xFFFFFFFF


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def make_index(orc, X, M0, efc0, p_max=0.01, seed=1, stride=None):
    """Oracle-trained quantiser and oracle-built graph, imported into libaqr."""
    from paper_2602_21600_amd import aqr
    n, d = X.shape
    tr = orc.train(X, p_max=p_max, M0=M0, efc0=efc0)
    d_pad = (d + 15) // 16 * 16
    codes = orc.encode(X, tr["min"], tr["scale"], stride=d_pad)
    u = 1.0 - np.random.default_rng(seed).random(n)
    lv = orc.levels(u, tr["M"])
    g = orc.build(codes, d, tr["M"], tr["efc"], lv)
    info = dict(d=d, d_pad=d_pad, M=tr["M"], efc=tr["efc"], delta=tr["delta"], p_lo=tr["p_lo"],
                p_hi=tr["p_hi"], s_dist=tr["s_dist"], eta=tr["eta"], w_mean=tr["w_mean"])
    qz = aqr.aqr_quantizer_create(info, tr["min"], tr["max"], tr["scale"])
    gh = aqr.aqr_graph_import(g)
    ix = aqr.aqr_index_bind(qz, gh, codes, X)
    return dict(X=X, codes=codes, d=d, min=tr["min"], max=tr["max"], scale=tr["scale"], graph=g,
                ix=ix, qz=qz, gh=gh, tr=tr)


@pytest.fixture(scope="module")
def small(orc):
    X = W.base("small")
    Q = W.queries("small")
    ix = make_index(orc, X, 16, 100)
    ix["Q"] = Q
    return ix


def run_stage1(index, Q, k, ef, nc=None, ef_max=None, out_stride=None, tap_cap=0, vb=0,
               order=None, waves_per_block=0, blocks=0, m_ef=3):
    torch = _torch()
    from paper_2602_21600_amd import aqr
    nq = Q.shape[0]
    k = np.broadcast_to(np.asarray(k, np.int32), (nq,)).copy()
    ef = np.broadcast_to(np.asarray(ef, np.int32), (nq,)).copy()
    efe = np.maximum(ef, k)
    if ef_max is None:
        ef_max = int(efe.max())
    if out_stride is None:
        out_stride = int(nc.max()) if nc is not None else int(
            np.minimum(np.maximum(efe // m_ef, k), efe).max())
    dev = "cuda"
    Qd = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).to(dev)
    kd = torch.from_numpy(k).to(dev)
    efd = torch.from_numpy(ef).to(dev)
    ncd = None if nc is None else torch.from_numpy(np.ascontiguousarray(nc, np.int32)).to(dev)
    cid = torch.full((nq, out_stride), -1, dtype=torch.int32, device=dev)
    cD = torch.full((nq, out_stride), -1, dtype=torch.int32, device=dev)
    cnt = torch.zeros(nq, dtype=torch.int32, device=dev)
    ws = torch.zeros(aqr.aqr_search_workspace_size(), dtype=torch.uint8, device=dev)
    taps = None
    if tap_cap:
        taps = dict(cap=tap_cap,
                    expanded=torch.zeros((nq, tap_cap), dtype=torch.int32, device=dev),
                    evaluated=torch.zeros((nq, tap_cap), dtype=torch.int32, device=dev),
                    counts=torch.zeros((nq, 8), dtype=torch.int32, device=dev))
    od = None if order is None else torch.from_numpy(np.ascontiguousarray(order, np.int32)).to(dev)
    aqr.aqr_search(index["ix"], Qd, kd, efd, cid, cD, cnt, ws, ef_max, out_stride, nc=ncd,
                   m_ef=m_ef, visited_log2=vb, taps=taps, order=od,
                   waves_per_block=waves_per_block, blocks=blocks)
    torch.cuda.synchronize()
    res = dict(cand_id=cid.cpu().numpy().view(np.uint32), cand_D=cD.cpu().numpy().view(np.uint32),
               cand_cnt=cnt.cpu().numpy(), Qd=Qd, kd=kd, cid_d=cid, cnt_d=cnt)
    if taps:
        res.update({kk: v.cpu().numpy().view(np.uint32) for kk, v in taps.items() if kk != "cap"})
    return res


def oracle_stage1(orc, index, Q, k, ef, nc=None, tap_cap=0, m_ef=3):
    nq = Q.shape[0]
    k = np.broadcast_to(np.asarray(k, np.int32), (nq,))
    ef = np.broadcast_to(np.asarray(ef, np.int32), (nq,))
    efe = np.zeros(nq, np.int32)
    ncc = np.zeros(nq, np.int32)
    for i in range(nq):
        efe[i], ncc[i] = orc.param_map(int(k[i]), int(ef[i]), m_ef)
    if nc is not None:
        ncc = np.asarray(nc, np.int32)
    qc = orc.encode(Q, index["min"], index["scale"], stride=index["codes"].shape[1])
    return orc.search_codes(index["graph"], index["codes"], index["d"], qc, efe, ncc,
                            tap_cap=tap_cap), qc


def compare_stage1(g, o, nq):
    np.testing.assert_array_equal(g["cand_cnt"], o["cand_cnt"])
    for q in range(nq):
        c = o["cand_cnt"][q]
        np.testing.assert_array_equal(g["cand_id"][q, :c], o["cand_id"][q, :c], err_msg=f"q={q}")
        np.testing.assert_array_equal(g["cand_D"][q, :c], o["cand_D"][q, :c], err_msg=f"q={q}")


def test_query_encoding_bit_exact(orc, small):
    torch = _torch()
    from paper_2602_21600_amd import aqr
    rng = np.random.default_rng(5)
    Q = np.vstack([small["Q"], small["X"][:50],
                   small["min"][None, :] + (np.arange(128)[None, :] % 7 - 3) * 0.5 /
                   small["scale"][None, :]]).astype(np.float32)
    Q = np.vstack([Q, Q[:20] + rng.normal(0, 5, Q[:20].shape).astype(np.float32)])
    Qd = torch.from_numpy(Q).cuda()
    out = torch.zeros((Q.shape[0], 128), dtype=torch.uint8, device="cuda")
    aqr.aqr_encode_queries(small["ix"], Qd, out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(),
                                  orc.encode(Q, small["min"], small["scale"], stride=128))


@pytest.mark.parametrize("ef", [10, 64, 210, 512, 1000])
def test_stage1_bit_exact_small(orc, small, ef):
    Q = small["Q"]
    cap = 1 << 15
    g = run_stage1(small, Q, 10, ef, tap_cap=cap)
    o, _ = oracle_stage1(orc, small, Q, 10, ef, tap_cap=cap)
    compare_stage1(g, o, Q.shape[0])
    for q in range(Q.shape[0]):
        ne = int(o["n_expanded"][q])
        assert g["counts"][q, 0] == ne
        np.testing.assert_array_equal(g["expanded"][q, :ne], o["expanded"][q, :ne])
        # distinct layer-0 visited set: the GPU's evaluations plus the layer-0
        # entry point (scored during the descent) equal the oracle's set
        nv = int(o["n_visited"][q])
        ge = int(g["counts"][q, 1])
        assert ge < cap
        gset = set(g["evaluated"][q, :ge].tolist()) | {int(o["expanded"][q, 0])}
        assert gset == set(o["visited"][q, :nv].tolist())


@pytest.mark.parametrize("m_ef", [1, 2, 5])
def test_stage1_candidate_count_mapping(orc, small, m_ef):
    # N_c = clamp(floor(ef_eff / m_ef), k, ef_eff) derived on the device for
    # other ratios than 3, with mixed k and ef; then Stages 2-3 on the longer
    # (or shorter) candidate lists
    Q = small["Q"][:300]
    nq = Q.shape[0]
    rng = np.random.default_rng(m_ef)
    k = rng.choice([1, 10, 50], nq).astype(np.int32)
    ef = rng.choice([16, 100, 288], nq).astype(np.int32)
    g = run_stage1(small, Q, k, ef, ef_max=288, m_ef=m_ef)
    o, _ = oracle_stage1(orc, small, Q, k, ef, m_ef=m_ef)
    compare_stage1(g, o, nq)
    k10 = np.full(nq, 10, np.int32)
    g = run_stage1(small, Q, k10, 288, m_ef=m_ef)
    gr = _rerank_gpu(small, g, 10, force_et=0, n_rerank=50)
    check_rerank(orc, small, Q, g, 10, gr, force_et=0, n_rerank=50)


def test_stage1_forgetful_cache_is_exact(orc, small):
    # 16 buckets (64 ids): the visited cache forgets constantly, results and
    # the expansion order stay identical; only re-evaluations grow
    Q = small["Q"][:40]
    cap = 1 << 16
    g = run_stage1(small, Q, 10, 128, vb=4, tap_cap=cap)
    o, _ = oracle_stage1(orc, small, Q, 10, 128, tap_cap=cap)
    compare_stage1(g, o, Q.shape[0])
    re_eval = 0
    for q in range(Q.shape[0]):
        ne = int(o["n_expanded"][q])
        np.testing.assert_array_equal(g["expanded"][q, :ne], o["expanded"][q, :ne])
        ge = int(g["counts"][q, 1])
        gset = set(g["evaluated"][q, :ge].tolist()) | {int(o["expanded"][q, 0])}
        nv = int(o["n_visited"][q])
        assert gset == set(o["visited"][q, :nv].tolist())
        re_eval += ge + 1 - nv
    assert re_eval > 0


def test_stage1_mixed_k_ef_ragged_batch(orc, small):
    rng = np.random.default_rng(3)
    Q = np.vstack([small["Q"], W.queries("small", 237)[100:]])
    nq = Q.shape[0]
    k = rng.choice(np.array([1, 10, 100], np.int32), nq)
    ef = rng.choice(np.array([16, 32, 64, 128, 256, 512], np.int32), nq)
    g = run_stage1(small, Q, k, ef, ef_max=512, out_stride=200)
    o, _ = oracle_stage1(orc, small, Q, k, ef)
    compare_stage1(g, o, nq)


def test_stage1_alone_equals_in_batch_and_order(orc, small):
    Q = small["Q"]
    full = run_stage1(small, Q, 10, 96)
    perm = np.random.default_rng(0).permutation(Q.shape[0]).astype(np.int32)
    alt = run_stage1(small, Q, 10, 96, order=perm, waves_per_block=1, blocks=7, vb=6)
    for q in (0, 17, 99):
        one = run_stage1(small, Q[q:q + 1], 10, 96)
        c = one["cand_cnt"][0]
        np.testing.assert_array_equal(one["cand_id"][0, :c], full["cand_id"][q, :c])
    np.testing.assert_array_equal(alt["cand_id"], full["cand_id"])
    np.testing.assert_array_equal(alt["cand_D"], full["cand_D"])


def test_invalid_queries_flagged(orc, small):
    Q = small["Q"][:6].copy()
    Q[2, 5] = np.nan
    Q[3, 0] = np.inf
    k = np.array([10, 0, 10, 10, 10, 10], np.int32)
    ef = np.array([64, 64, 64, 64, 2000, 64], np.int32)
    g = run_stage1(small, Q, k, ef, ef_max=64, out_stride=21)
    assert g["cand_cnt"].tolist()[:5] == [21, -1, -1, -1, -1]
    assert g["cand_cnt"][5] == 21


def test_exhaustive_search_and_exact_pipeline(orc):
    torch = _torch()
    from paper_2602_21600_amd import aqr
    X, Q = W.tiny(500, 24, seed=8, clusters=5, nq=20)
    index = make_index(orc, X, 6, 40)
    n = X.shape[0]
    g = run_stage1(index, Q, 10, n, nc=np.full(20, n, np.int32), ef_max=n, out_stride=n)
    o, _ = oracle_stage1(orc, index, Q, 10, n, nc=np.full(20, n, np.int32))
    compare_stage1(g, o, 20)
    # N_c = N_rerank = N, early termination off: exact kNN
    out_id = torch.zeros((20, 10), dtype=torch.int32, device="cuda")
    out_d = torch.zeros((20, 10), dtype=torch.float32, device="cuda")
    aqr.aqr_rerank(index["ix"], g["Qd"], g["cid_d"], g["cnt_d"], g["kd"], out_id, out_d,
                   n_rerank=n, force_et=0)
    torch.cuda.synchronize()
    gt_id, gt_d = orc.knn_f32(X, Q, 10)
    got = out_id.cpu().numpy()
    gd = out_d.cpu().numpy()
    np.testing.assert_allclose(gd, gt_d, rtol=RTOL)
    for q in range(20):
        for t in np.nonzero(got[q] != gt_id[q])[0]:
            # only entries whose exact distances tie within tolerance may swap
            close = np.abs(gt_d[q] - gt_d[q, t]) <= RTOL * gt_d[q, t]
            assert close.sum() >= 2, (q, t)


def _rerank_gpu(index, s1, k, n_rerank=28, force_et=-1, tau_gap=0.010, tau_ratio=1.008,
                assembly=0):
    torch = _torch()
    from paper_2602_21600_amd import aqr
    nq = s1["cand_id"].shape[0]
    ncs = s1["cand_id"].shape[1]
    km = int(np.max(k))
    out_id = torch.zeros((nq, km), dtype=torch.int32, device="cuda")
    out_d = torch.zeros((nq, km), dtype=torch.float32, device="cuda")
    out_k = torch.zeros((nq, km), dtype=torch.uint8, device="cuda")
    taps = dict(a_id=torch.zeros((nq, ncs), dtype=torch.int32, device="cuda"),
                a_dist=torch.zeros((nq, ncs), dtype=torch.float32, device="cuda"),
                et=torch.zeros(nq, dtype=torch.uint8, device="cuda"),
                nrr=torch.zeros(nq, dtype=torch.int32, device="cuda"))
    kd = torch.from_numpy(np.broadcast_to(np.asarray(k, np.int32), (nq,)).copy()).cuda()
    aqr.aqr_rerank(index["ix"], s1["Qd"], s1["cid_d"], s1["cnt_d"], kd, out_id, out_d, out_k,
                   n_rerank=n_rerank, force_et=force_et, tau_gap=tau_gap, tau_ratio=tau_ratio,
                   taps=taps, assembly=assembly)
    torch.cuda.synchronize()
    r = dict(id=out_id.cpu().numpy(), dist=out_d.cpu().numpy(), kind=out_k.cpu().numpy())
    r.update({kk: v.cpu().numpy() for kk, v in taps.items()})
    r["a_id"] = r["a_id"].view(np.uint32)
    return r


def check_rerank(orc, index, Q, s1, k, gr, n_rerank=28, tau_gap=0.010, tau_ratio=1.008,
                 force_et=-1, assembly=0):
    """Parity protocol for Stages 2-3 (see module docstring)."""
    nq = Q.shape[0]
    kk = np.broadcast_to(np.asarray(k, np.int32), (nq,))
    ref = orc.rerank(index["X"], index["codes"], index["min"], index["scale"], Q, s1["cand_id"],
                     s1["cand_cnt"], kk, n_rerank, tau_gap, tau_ratio, taps=True,
                     force_et=force_et, k_stride=gr["id"].shape[1], assembly=assembly)
    flips = 0
    for q in range(nq):
        c = s1["cand_cnt"][q]
        # d^a: same set, within tolerance, GPU order non-decreasing in oracle d^a
        da_ref = dict(zip(ref["a_id"][q, :c].tolist(), ref["a_dist"][q, :c].tolist()))
        ga = gr["a_id"][q, :c].tolist()
        assert sorted(ga) == sorted(da_ref)
        gd = gr["a_dist"][q, :c].astype(np.float64)
        rd = np.array([da_ref[i] for i in ga])
        np.testing.assert_allclose(gd, rd, rtol=RTOL, atol=1e-30)
        assert np.all(np.diff(rd) >= -RTOL * np.abs(rd[1:]))
        et_g, et_o = int(gr["et"][q]), int(ref["et"][q])
        if et_g != et_o:
            kq = int(kk[q])
            dk, dk1 = ref["a_dist"][q, kq - 1], ref["a_dist"][q, kq]
            gap = (dk1 - dk) / (dk + 1e-6)
            ratio = dk1 / (dk + 1e-6)
            near = abs(gap - tau_gap) <= RTOL * tau_gap or abs(ratio - tau_ratio) <= RTOL * tau_ratio
            assert near, f"q={q}: early-termination decision differs away from the threshold"
            flips += 1
    # rerun the oracle from the GPU's A order and decision
    ref2 = orc.rerank(index["X"], index["codes"], index["min"], index["scale"], Q, s1["cand_id"],
                      s1["cand_cnt"], kk, n_rerank, tau_gap, tau_ratio,
                      force_et=gr["et"].astype(np.int32),
                      a_order=np.ascontiguousarray(gr["a_id"][:, :s1["cand_id"].shape[1]]),
                      taps=True, k_stride=gr["id"].shape[1], assembly=assembly)
    np.testing.assert_array_equal(gr["nrr"], ref2["nrr"])
    for q in range(nq):
        gi, oi = gr["id"][q], ref2["id"][q]
        np.testing.assert_allclose(gr["dist"][q], ref2["dist"][q], rtol=RTOL)
        if not np.array_equal(gi, oi):
            # ids may differ only between entries whose distances tie within tolerance
            for t in np.nonzero(gi != oi)[0]:
                d = ref2["dist"][q, t]
                close = np.abs(ref2["dist"][q] - d) <= RTOL * max(d, 1e-30)
                assert close.sum() >= 2, f"q={q} slot {t}"
        # kinds where the ids agree (a tie may swap an exact and an approximate entry)
        same = gi == oi
        np.testing.assert_array_equal(gr["kind"][q][same], ref2["kind"][q][same])
    return flips


@pytest.mark.parametrize("ef,k", [(64, 10), (210, 10), (300, 100), (16, 1)])
def test_rerank_matches_oracle(orc, small, ef, k):
    Q = small["Q"]
    s1 = run_stage1(small, Q, k, ef)
    gr = _rerank_gpu(small, s1, k)
    check_rerank(orc, small, Q, s1, k, gr)


def test_rerank_forced_modes(orc, small):
    Q = small["Q"][:30]
    s1 = run_stage1(small, Q, 10, 128)
    for f in (0, 1):
        gr = _rerank_gpu(small, s1, 10, force_et=f)
        assert np.all(gr["et"] == f)
        check_rerank(orc, small, Q, s1, 10, gr, force_et=f)


@pytest.mark.parametrize("ef,k,f", [(128, 10, 1), (128, 10, -1), (512, 100, 1)])
def test_rerank_union_matches_oracle(orc, small, ef, k, f):
    # the union reading of the assembly: every candidate not re-ranked joins
    # the exact results with its d^a
    Q = small["Q"]
    s1 = run_stage1(small, Q, k, ef)
    gr = _rerank_gpu(small, s1, k, force_et=f, assembly=1)
    check_rerank(orc, small, Q, s1, k, gr, force_et=f, assembly=1)
    if f == 1:
        # ET forced on re-ranks k candidates: the rest of A joins the results
        assert np.all(s1["cand_cnt"] > k) and np.any(gr["kind"] == 2)
        from paper_2602_21600_amd import aqr
        with pytest.raises(aqr.AqrError):
            _rerank_gpu(small, s1, k, force_et=f, assembly=2)


def test_fp32_baseline_matches_oracle(orc, small):
    # every query's list equals the FP64 oracle's, or differs only through an
    # FP32 rounding tie shown at the output or on the search path
    Q = small["Q"]
    for ef, k in [(64, 10), (256, 10), (128, 100)]:
        same, out_ties, path_ties = check_fp32_baseline(orc, small, small["X"], Q, k, ef)
        assert same + out_ties + path_ties == Q.shape[0]


def fp32_search(index, Q, k, ef, tap_cap=0, vb=0):
    """The FP32 baseline on the GPU: ids, FP32 distances, and the layer-0
    expansion order when tap_cap > 0."""
    torch = _torch()
    from paper_2602_21600_amd import aqr
    nq = Q.shape[0]
    Qd = torch.from_numpy(Q).cuda()
    kd = torch.full((nq,), k, dtype=torch.int32, device="cuda")
    efd = torch.full((nq,), ef, dtype=torch.int32, device="cuda")
    oid = torch.zeros((nq, k), dtype=torch.int32, device="cuda")
    odist = torch.zeros((nq, k), dtype=torch.float32, device="cuda")
    ws = torch.zeros(aqr.aqr_search_workspace_size(), dtype=torch.uint8, device="cuda")
    taps = None
    if tap_cap:
        taps = dict(cap=tap_cap, expanded=torch.zeros((nq, tap_cap), dtype=torch.int32,
                                                      device="cuda"),
                    counts=torch.zeros((nq, 8), dtype=torch.int32, device="cuda"))
    aqr.aqr_search_fp32(index["ix"], Qd, kd, efd, oid, odist, ws, max(ef, k), k,
                        visited_log2=vb, taps=taps)
    torch.cuda.synchronize()
    r = dict(id=oid.cpu().numpy(), dist=odist.cpu().numpy())
    if tap_cap:
        r["expanded"] = taps["expanded"].cpu().numpy().view(np.uint32)
        r["n_expanded"] = taps["counts"].cpu().numpy()[:, 0]
    return r


def check_fp32_baseline(orc, index, X, Q, k, ef, tap_cap=1 << 14, vb=0):
    """The FP32 baseline against the oracle's FP64 search, query by query.
    Identical lists must agree in distance within RTOL.  A query whose list
    differs must be explained by an FP32 rounding tie, one of:
      - a tie at the output: position by position the distances agree within
        RTOL, and every differing id's exact distance equals the oracle's at
        that position within RTOL;
      - a tie on the path: at the first expansion where the two searches
        part, the two nodes they expand have exact distances within RTOL of
        each other (FP32 ordered them one way, FP64 the other).
    Returns the numbers of (identical, output ties, path ties)."""
    nq = Q.shape[0]
    g = fp32_search(index, Q, k, ef, tap_cap=tap_cap, vb=vb)
    rid, rd, oexp, onexp = orc.search_f32(index["graph"], X, Q, max(ef, k), k, tap_cap=tap_cap)
    X64 = X.astype(np.float64)

    def dist(q, i):
        e = X64[int(i)] - Q[q].astype(np.float64)
        return float(e @ e)

    same = out_ties = path_ties = 0
    for q in range(nq):
        gi, gd = g["id"][q], g["dist"][q].astype(np.float64)
        if np.array_equal(gi, rid[q]):
            np.testing.assert_allclose(gd, rd[q], rtol=RTOL)
            same += 1
            continue
        if np.allclose(gd, rd[q], rtol=RTOL) and all(
                gi[t] >= 0 and abs(dist(q, gi[t]) - rd[q, t]) <= RTOL * rd[q, t]
                for t in np.nonzero(gi != rid[q])[0]):
            out_ties += 1
            continue
        ge = g["expanded"][q, :min(int(g["n_expanded"][q]), tap_cap)]
        oe = oexp[q, :min(int(onexp[q]), tap_cap)]
        m = min(len(ge), len(oe))
        diff = np.nonzero(ge[:m] != oe[:m])[0]
        assert diff.size, f"q={q}: lists differ but the expansion orders agree"
        i = int(diff[0])
        da, db = dist(q, ge[i]), dist(q, oe[i])
        assert abs(da - db) <= RTOL * max(da, db), \
            f"q={q}: paths part at expansion {i} on nodes {ge[i]} ({da}) and {oe[i]} ({db}), " \
            f"not a rounding tie"
        path_ties += 1
    return same, out_ties, path_ties


@pytest.mark.parametrize("d", [100, 20])
def test_ragged_dimension_pipeline(orc, d):
    # d not a multiple of 16: code rows carry zero padding up to d_pad, which
    # must add nothing to Stage-1, Stage-2 or Stage-3 distances
    X, Q = W.tiny(4000, d, seed=30 + d, clusters=6, nq=60)
    index = make_index(orc, X, 12, 80)
    s1 = run_stage1(index, Q, 10, 96)
    o, _ = oracle_stage1(orc, index, Q, 10, 96)
    compare_stage1(s1, o, Q.shape[0])
    gr = _rerank_gpu(index, s1, 10)
    check_rerank(orc, index, Q, s1, 10, gr)
    gr = _rerank_gpu(index, s1, 10, force_et=0, n_rerank=20)
    check_rerank(orc, index, Q, s1, 10, gr, force_et=0, n_rerank=20)


@pytest.mark.parametrize("nq", [40, 1100])
def test_wide_rows_pipeline(orc, nq):
    # 960-dimensional rows (the GIST-1M shape, M_0 = 32): code rows take 8
    # chunks per lane on 8-lane groups and FP32 rows 8 chunks per lane on
    # 32-lane groups.  A batch of at most one wave per SIMD (40 queries)
    # keeps four row sets in flight, a larger one (1,100 queries) two.
    torch = _torch()
    from paper_2602_21600_amd import aqr
    X, Q = W.tiny(2500, 960, seed=77, clusters=6, nq=nq)
    index = make_index(orc, X, 32, 60)
    s1 = run_stage1(index, Q, 10, 128, tap_cap=1 << 14)
    o, _ = oracle_stage1(orc, index, Q, 10, 128, tap_cap=1 << 14)
    compare_stage1(s1, o, Q.shape[0])
    for q in range(Q.shape[0]):
        ne = int(o["n_expanded"][q])
        np.testing.assert_array_equal(s1["expanded"][q, :ne], o["expanded"][q, :ne])
    gr = _rerank_gpu(index, s1, 10, force_et=0, n_rerank=40)
    check_rerank(orc, index, Q, s1, 10, gr, force_et=0, n_rerank=40)
    # the FP32 baseline: identical lists, or differences explained by FP32
    # rounding ties
    same, out_ties, path_ties = check_fp32_baseline(orc, index, X, Q, 10, 96)
    assert same + out_ties + path_ties == nq


def test_empty_batches(orc, small):
    # nq = 0 is accepted by every batch entry point and launches nothing
    torch = _torch()
    from paper_2602_21600_amd import aqr
    z = torch.zeros((0, small["d"]), dtype=torch.float32, device="cuda")
    zi = torch.zeros(0, dtype=torch.int32, device="cuda")
    cid = torch.zeros((0, 21), dtype=torch.int32, device="cuda")
    ws = torch.zeros(aqr.aqr_search_workspace_size(), dtype=torch.uint8, device="cuda")
    aqr.aqr_search(small["ix"], z, zi, zi, cid, cid.clone(), zi.clone(), ws, 64, 21)
    out_id = torch.zeros((0, 10), dtype=torch.int32, device="cuda")
    out_d = torch.zeros((0, 10), dtype=torch.float32, device="cuda")
    aqr.aqr_rerank(small["ix"], z, cid, zi, zi, out_id, out_d)
    aqr.aqr_search_fp32(small["ix"], z, zi, zi, out_id, out_d, ws, 64, 10)
    plan = aqr.BatchPlan(small["ix"], 8, 10, 64, use_graph=False)
    plan.launch(0)
    torch.cuda.synchronize()


def test_bench_ground_truth_matches_oracle(orc, small):
    # the bench's exact kNN (aqr_knn_bruteforce, in query chunks) equals the
    # oracle's FP64 brute force: ids and distances identical
    import bench
    X, Q = small["X"], small["Q"]
    gi, gd, cert = bench.ground_truth(X, Q, 10, "cuda:0", qchunk=37)
    ri, rd = orc.knn_f32(X, Q, 10)
    np.testing.assert_array_equal(gi, ri)
    np.testing.assert_array_equal(gd.view(np.uint64), rd.view(np.uint64))
    assert cert.shape == (Q.shape[0],)


def test_full_rows_at_m32_match_oracle(orc):
    # M = 32: layer-0 rows hold 2M = 64 neighbours and upper rows 32, so a
    # row can be full with no unused entry; Stage 1 on codes stays bit-exact
    # and the FP32 baseline follows the FP64 oracle but for rounding ties,
    # whatever the visited-cache size
    torch = _torch()
    from paper_2602_21600_amd import aqr
    X = W.base("sift1m", 12000)
    Q = W.queries("sift1m", 200)
    n, d = X.shape
    tr = orc.train(X, M0=16, efc0=100)
    codes = orc.encode(X, tr["min"], tr["scale"], stride=128)
    u = 1.0 - np.random.default_rng(3).random(n)
    g = orc.build(codes, d, 32, 100, orc.levels(u, 32))
    assert (g["adj0"] != 0xFFFFFFFF).all(axis=1).sum() > 0  # some full layer-0 rows
    info = dict(d=d, d_pad=128, M=32, efc=100, delta=tr["delta"], p_lo=tr["p_lo"],
                p_hi=tr["p_hi"], s_dist=tr["s_dist"], eta=tr["eta"], w_mean=tr["w_mean"])
    qz = aqr.aqr_quantizer_create(info, tr["min"], tr["max"], tr["scale"])
    gh = aqr.aqr_graph_import(g)
    index = dict(X=X, codes=codes, d=d, min=tr["min"], scale=tr["scale"], graph=g,
                 ix=aqr.aqr_index_bind(qz, gh, codes, X))
    s1 = run_stage1(index, Q, 10, 200)
    o, _ = oracle_stage1(orc, index, Q, 10, 200)
    compare_stage1(s1, o, Q.shape[0])
    nq = Q.shape[0]
    prev = None
    for vb in (6, 10):
        gid = fp32_search(index, Q, 10, 200, vb=vb)["id"]
        if prev is not None:
            np.testing.assert_array_equal(gid, prev)
        prev = gid
        same, out_ties, path_ties = check_fp32_baseline(orc, index, X, Q, 10, 200, vb=vb)
        assert same + out_ties + path_ties == nq


def _library_index(name, n, M0, efc0, nq, batched=True):
    """A library-built index (quantiser and graph from libaqr) of n rows of a
    workload, with its graph exported for the oracle."""
    from paper_2602_21600_amd import aqr
    X = W.base(name, n)
    Q = W.queries(name, nq)
    d = X.shape[1]
    qz, codes = aqr.aqr_quantize(X, aqr.default_qparams(M0=M0, efc0=efc0))
    if batched:
        g = aqr.aqr_build_batched(codes, X, d, qz, level_u=W.level_draws(name, n))
    else:
        g = aqr.aqr_build(codes, d, qz, threads=0, level_u=W.level_draws(name, n))
    info = aqr.aqr_quantizer_info(qz)
    return dict(X=X, Q=Q, codes=codes, d=d, min=info["min"], scale=info["scale"],
                graph=aqr.aqr_graph_export(g), ix=aqr.aqr_index_bind(qz, g, codes, X))


def test_stage1_at_19_bit_ids(orc):
    # 262,145 rows need 19-bit ids.  With 16 visited buckets the cache stores
    # the full 15-bit remainder of each hashed id (the widest entry it has)
    # and forgets most of what it sees; with 512 buckets it stores 10 bits.
    # Stage 1 (candidates, D values, expansion order, distinct visited set)
    # stays bit-exact against the oracle on the library-built graph, and
    # Stages 2-3 follow the parity protocol.
    print("index: serving rows, n = 262,145", flush=True)
    index = _library_index("serving", 262_145, 16, 100, 200)
    Q = index["Q"]
    cap = 1 << 15
    o, _ = oracle_stage1(orc, index, Q, 10, 160, tap_cap=cap)
    for vb in (4, 9):
        g = run_stage1(index, Q, 10, 160, vb=vb, tap_cap=cap)
        compare_stage1(g, o, Q.shape[0])
        for q in range(Q.shape[0]):
            ne = int(o["n_expanded"][q])
            np.testing.assert_array_equal(g["expanded"][q, :ne], o["expanded"][q, :ne])
            ge = int(g["counts"][q, 1])
            assert ge < cap
            gset = set(g["evaluated"][q, :ge].tolist()) | {int(o["expanded"][q, 0])}
            assert gset == set(o["visited"][q, :int(o["n_visited"][q])].tolist())
    gr = _rerank_gpu(index, g, 10, force_et=0, n_rerank=50)
    check_rerank(orc, index, Q, g, 10, gr, force_et=0, n_rerank=50)


def test_stage1_at_20_bit_ids_with_16_bit_entries(orc):
    # 524,289 rows need 20-bit ids.  With 2^4 visited buckets plus the ones
    # the launch adds from spare LDS, each entry holds 16 bits: the scaled
    # place of the hashed id in its bucket.  With 2^9 buckets it holds 11.
    # Stage 1 stays bit-exact against the oracle (same expansions, same
    # distinct visited set), so no entry ever names an id the cache has not
    # seen.
    print("index: serving rows, n = 524,289", flush=True)
    index = _library_index("serving", 524_289, 16, 100, 120)
    Q = index["Q"]
    cap = 1 << 15
    o, _ = oracle_stage1(orc, index, Q, 10, 160, tap_cap=cap)
    for vb in (4, 9):
        g = run_stage1(index, Q, 10, 160, vb=vb, tap_cap=cap)
        compare_stage1(g, o, Q.shape[0])
        for q in range(Q.shape[0]):
            ne = int(o["n_expanded"][q])
            np.testing.assert_array_equal(g["expanded"][q, :ne], o["expanded"][q, :ne])
            ge = int(g["counts"][q, 1])
            assert ge < cap
            gset = set(g["evaluated"][q, :ge].tolist()) | {int(o["expanded"][q, 0])}
            assert gset == set(o["visited"][q, :int(o["n_visited"][q])].tolist())


def test_image_shaped_rows_pipeline(orc):
    # 784-dimensional rows (the Fashion-MNIST shape): 49 chunks of 16 codes
    # per row, four chunks per lane; code rows at a 896-byte stride and FP32
    # rows at 800 floats in the device arena.  Stage 1 bit-exact, Stages 2-3
    # by the parity protocol, the FP32 baseline up to rounding ties.
    print("index: fmnist rows, n = 12,000", flush=True)
    index = _library_index("fmnist", 12_000, 16, 100, 120, batched=False)
    Q = index["Q"]
    cap = 1 << 14
    g = run_stage1(index, Q, 10, 96, tap_cap=cap)
    o, _ = oracle_stage1(orc, index, Q, 10, 96, tap_cap=cap)
    compare_stage1(g, o, Q.shape[0])
    for q in range(Q.shape[0]):
        ne = int(o["n_expanded"][q])
        np.testing.assert_array_equal(g["expanded"][q, :ne], o["expanded"][q, :ne])
    gr = _rerank_gpu(index, g, 10)
    check_rerank(orc, index, Q, g, 10, gr)
    same, out_ties, path_ties = check_fp32_baseline(orc, index, index["X"], Q, 10, 96)
    assert same + out_ties + path_ties == Q.shape[0]
