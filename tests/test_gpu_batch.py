"""Uneven batches in one launch: per-query k and ef, longest-first order,
graph capture and replay, and tuning choices.

Each query's result must be the same alone, in the mixed batch, under graph
replay and under every tuning choice (integers bit-exact; the FP32 stages run
the same arithmetic per query, so their outputs are bit-identical too), and
the batch must match the oracle (Stage 1 bit-exact, Stages 2-3 by the parity
protocol of test_gpu_parity).
"""
import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small(orc):
    from test_gpu_parity import make_index
    X = W.base("small")
    ix = make_index(orc, X, 16, 100)
    rng = np.random.default_rng(11)
    Q = np.vstack([W.queries("small"), W.queries("small", 357)[100:]])
    nq = Q.shape[0]
    ix["Q"] = Q
    ix["k"] = rng.choice(np.array([1, 10, 100], np.int32), nq)
    ix["ef"] = rng.choice(np.array([16, 32, 64, 128, 256, 512], np.int32), nq)
    return ix


def run_plan(index, Q, k, ef, use_graph=False, longest_first=True, tuning=None, launches=1,
             between=None, **plan_kw):
    import torch
    from paper_2602_21600_amd import aqr
    plan = aqr.BatchPlan(index["ix"], Q.shape[0], 100, 512, use_graph=use_graph,
                         longest_first=longest_first, tuning=tuning, **plan_kw)
    n = plan.load(torch.from_numpy(Q).cuda(), torch.from_numpy(k).cuda(),
                  torch.from_numpy(ef).cuda())
    outs = []
    for i in range(launches):
        if between is not None:
            between(i)
        plan.launch(n)
        torch.cuda.synchronize()
        b = plan.bufs
        outs.append(dict(cand_id=b["cand_id"][:n].cpu().numpy().view(np.uint32).copy(),
                         cand_cnt=b["cand_cnt"][:n].cpu().numpy().copy(),
                         id=b["out_id"][:n].cpu().numpy().copy(),
                         dist=b["out_dist"][:n].cpu().numpy().copy(),
                         kind=b["out_kind"][:n].cpu().numpy().copy()))
    return outs


def same(a, b, nq):
    np.testing.assert_array_equal(a["cand_cnt"], b["cand_cnt"])
    for q in range(nq):
        c = a["cand_cnt"][q]
        np.testing.assert_array_equal(a["cand_id"][q, :c], b["cand_id"][q, :c], err_msg=f"q={q}")
    np.testing.assert_array_equal(a["id"], b["id"])
    np.testing.assert_array_equal(a["dist"].view(np.uint32), b["dist"].view(np.uint32))
    np.testing.assert_array_equal(a["kind"], b["kind"])


@pytest.mark.parametrize("et", ["table3", "off"])
def test_batch_matches_oracle(orc, small, et):
    # Stage 1 of the whole uneven batch bit-exact against the oracle; Stages
    # 2-3 by the parity protocol (distances within 1e-5, ids equal up to ties
    # inside that tolerance, early-termination decisions equal except within
    # 1e-5 of a threshold), with Table 3's thresholds and with early
    # termination off
    import torch
    from paper_2602_21600_amd import aqr
    from test_gpu_parity import check_rerank, oracle_stage1
    Q, k, ef = small["Q"], small["k"], small["ef"]
    inf = float("inf")
    tau = dict(tau_gap=0.010, tau_ratio=1.008) if et == "table3" else dict(tau_gap=inf,
                                                                           tau_ratio=inf)
    out = run_plan(small, Q, k, ef, **tau)[0]
    o, _ = oracle_stage1(orc, small, Q, k, ef)
    np.testing.assert_array_equal(out["cand_cnt"], o["cand_cnt"])
    for q in range(Q.shape[0]):
        c = o["cand_cnt"][q]
        np.testing.assert_array_equal(out["cand_id"][q, :c], o["cand_id"][q, :c])
    # the plan's Stages 2-3 once more on its own candidates, with the taps the
    # protocol needs: the same kernel on the same inputs gives the same rows
    nq, ncs = out["cand_id"].shape
    dev = "cuda"
    Qd = torch.from_numpy(Q).to(dev)
    cid = torch.from_numpy(np.ascontiguousarray(out["cand_id"]).view(np.int32)).to(dev)
    cnt = torch.from_numpy(out["cand_cnt"]).to(dev)
    kd = torch.from_numpy(k).to(dev)
    oid = torch.zeros((nq, 100), dtype=torch.int32, device=dev)
    od = torch.zeros((nq, 100), dtype=torch.float32, device=dev)
    ok = torch.zeros((nq, 100), dtype=torch.uint8, device=dev)
    taps = dict(a_id=torch.zeros((nq, ncs), dtype=torch.int32, device=dev),
                a_dist=torch.zeros((nq, ncs), dtype=torch.float32, device=dev),
                et=torch.zeros(nq, dtype=torch.uint8, device=dev),
                nrr=torch.zeros(nq, dtype=torch.int32, device=dev))
    aqr.aqr_rerank(small["ix"], Qd, cid, cnt, kd, oid, od, ok, n_rerank=28, taps=taps, **tau)
    torch.cuda.synchronize()
    gr = dict(id=oid.cpu().numpy(), dist=od.cpu().numpy(), kind=ok.cpu().numpy())
    gr.update({kk: v.cpu().numpy() for kk, v in taps.items()})
    gr["a_id"] = gr["a_id"].view(np.uint32)
    np.testing.assert_array_equal(gr["id"], out["id"])
    np.testing.assert_array_equal(gr["dist"].view(np.uint32), out["dist"].view(np.uint32))
    s1 = dict(cand_id=np.ascontiguousarray(out["cand_id"]), cand_cnt=out["cand_cnt"])
    check_rerank(orc, small, Q, s1, k, gr, n_rerank=28, **tau)
    if et == "table3":
        assert gr["et"].sum() > 0  # the termination test acted on part of the batch
    for q in range(nq):
        assert np.all(out["id"][q, k[q]:] == -1)


def test_alone_equals_batch_and_orders(orc, small):
    Q, k, ef = small["Q"], small["k"], small["ef"]
    nq = Q.shape[0]
    batch = run_plan(small, Q, k, ef, longest_first=True)[0]
    natural = run_plan(small, Q, k, ef, longest_first=False)[0]
    same(batch, natural, nq)
    for q in (0, 5, 77, 200, nq - 1):
        one = run_plan(small, Q[q:q + 1], k[q:q + 1], ef[q:q + 1])[0]
        c = one["cand_cnt"][0]
        assert c == batch["cand_cnt"][q]
        np.testing.assert_array_equal(one["cand_id"][0, :c], batch["cand_id"][q, :c])
        np.testing.assert_array_equal(one["id"][0], batch["id"][q])
        np.testing.assert_array_equal(one["dist"][0].view(np.uint32),
                                      batch["dist"][q].view(np.uint32))


def test_graph_replays_equal_eager(orc, small):
    import torch
    Q, k, ef = small["Q"], small["k"], small["ef"]
    nq = Q.shape[0]
    eager = run_plan(small, Q, k, ef)[0]
    scratch = torch.zeros(1 << 20, device="cuda")

    def between(i):
        # the program's own eager work and a synchronisation between replays
        scratch.add_(float(i + 1))
        torch.cuda.synchronize()

    outs = run_plan(small, Q, k, ef, use_graph=True, launches=4, between=between)
    for o in outs:
        same(o, eager, nq)


@pytest.mark.parametrize("tuning", [
    dict(waves_per_block=1, visited_log2=8, rerank_waves_per_block=2),
    dict(waves_per_block=2, visited_log2=10, rerank_waves_per_block=4),
    dict(waves_per_block=4, visited_log2=6, rerank_waves_per_block=1, blocks=5),
    # two list sizes in one launch
    dict(waves_per_block=4, visited_log2=8, ef_small=128, small_waves=2),
    dict(waves_per_block=4, visited_log2=9, ef_small=256, small_waves=3),
    dict(waves_per_block=2, visited_log2=7, ef_small=64, small_waves=1, blocks=3),
])
def test_tuning_does_not_change_results(orc, small, tuning):
    Q, k, ef = small["Q"], small["k"], small["ef"]
    base = run_plan(small, Q, k, ef)[0]
    other = run_plan(small, Q, k, ef, tuning=tuning)[0]
    same(base, other, Q.shape[0])


def _split_words(Q, k, ef, small, tuning, longest_first):
    # the plan's search workspace after a launch: claims of positions [0, c),
    # the split point c (-1: the order is not split), claims of [c, nq)
    import torch
    from paper_2602_21600_amd import aqr
    plan = aqr.BatchPlan(small["ix"], Q.shape[0], 100, 512, use_graph=False,
                         longest_first=longest_first, tuning=tuning)
    n = plan.load(torch.from_numpy(Q).cuda(), torch.from_numpy(k).cuda(),
                  torch.from_numpy(ef).cuda())
    plan.launch(n)
    torch.cuda.synchronize()
    return plan.bufs["ws"][:12].cpu().numpy().view(np.int32)


def test_two_list_sizes_split_and_fall_back(orc, small):
    # longest first: the split point is the number of queries whose list is
    # above ef_small, and both claim counters pass their ranges; in the
    # given order (not split) the small-list waves leave and the others
    # take every query; a batch already in longest-first order splits
    # without the order array; results are the same in every case
    Q, k, ef = small["Q"], small["k"], small["ef"]
    nq = Q.shape[0]
    tuning = dict(waves_per_block=4, visited_log2=8, ef_small=128, small_waves=2)
    big = int((np.maximum(ef, k) > 128).sum())
    assert 0 < big < nq
    w = _split_words(Q, k, ef, small, tuning, True)
    assert w[1] == big and w[0] >= big and w[2] >= nq - big
    base = run_plan(small, Q, k, ef)[0]
    w = _split_words(Q, k, ef, small, tuning, False)
    assert w[1] == -1 and w[0] >= nq
    same(base, run_plan(small, Q, k, ef, longest_first=False, tuning=tuning)[0], nq)
    srt = np.argsort(-np.maximum(ef, k), kind="stable")
    w = _split_words(Q[srt], k[srt], ef[srt], small, tuning, False)
    assert w[1] == big
    out = run_plan(small, Q[srt], k[srt], ef[srt], longest_first=False, tuning=tuning)[0]
    for key in ("cand_cnt", "id", "kind"):
        np.testing.assert_array_equal(out[key], base[key][srt])
    np.testing.assert_array_equal(out["dist"].view(np.uint32), base["dist"][srt].view(np.uint32))


@pytest.mark.parametrize("bad", [dict(small_waves=4), dict(small_waves=-1),
                                 dict(small_waves=1, ef_small=512),
                                 dict(small_waves=1, ef_small=0)])
def test_two_list_sizes_reject_bad_arguments(orc, small, bad):
    import torch
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"][:8], small["k"][:8], small["ef"][:8]
    nc = 170
    cid = torch.empty((8, nc), dtype=torch.int32, device="cuda")
    cD = torch.empty_like(cid)
    cnt = torch.empty(8, dtype=torch.int32, device="cuda")
    ws = torch.zeros(aqr.aqr_search_workspace_size(), dtype=torch.uint8, device="cuda")
    with pytest.raises(aqr.AqrError):
        aqr.aqr_search(small["ix"], torch.from_numpy(Q).cuda(), torch.from_numpy(k).cuda(),
                       torch.from_numpy(ef).cuda(), cid, cD, cnt, ws, 512, nc,
                       waves_per_block=4, **bad)


def test_autotune_picks_a_valid_config(orc, small, tmp_path):
    import torch
    from paper_2602_21600_amd import tune
    Q, k, ef = small["Q"], small["k"], small["ef"]
    best, table = tune.autotune(small["ix"], torch.from_numpy(Q).cuda(),
                                torch.from_numpy(k).cuda(), torch.from_numpy(ef).cuda(), 100, 512,
                                cache_path=str(tmp_path / "tune.json"), reps=1)
    assert len(table) >= 6
    assert best in [t for t, _ in table]
    again, _ = tune.autotune(small["ix"], None, None, None, 100, 512,
                             cache_path=str(tmp_path / "tune.json"))
    assert again == best


def test_two_list_sizes_fp32_baseline(orc, small):
    # the FP32 search keeps its query in LDS ahead of the other arrays; with
    # two list sizes (longest-first order, a split order and the natural
    # order that is not split) its rows equal the single-size launch's
    import torch
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"], small["k"], small["ef"]
    nq = Q.shape[0]
    Qd, kd, efd = (torch.from_numpy(a).cuda() for a in (Q, k, ef))
    ws = torch.zeros(aqr.aqr_search_workspace_size(), dtype=torch.uint8, device="cuda")
    order = torch.from_numpy(np.argsort(-np.maximum(ef, k), kind="stable").astype(np.int32)).cuda()

    def run(**kw):
        oid = torch.full((nq, 100), -7, dtype=torch.int32, device="cuda")
        od = torch.zeros((nq, 100), dtype=torch.float32, device="cuda")
        aqr.aqr_search_fp32(small["ix"], Qd, kd, efd, oid, od, ws, 512, 100, **kw)
        torch.cuda.synchronize()
        return oid.cpu().numpy(), od.cpu().numpy()

    base_id, base_d = run(waves_per_block=4, visited_log2=8)
    for kw in (dict(order=order, ef_small=128, small_waves=2),
               dict(order=order, ef_small=256, small_waves=3),
               dict(ef_small=128, small_waves=1)):
        oid, od = run(waves_per_block=4, visited_log2=8, **kw)
        np.testing.assert_array_equal(oid, base_id, err_msg=str(kw))
        np.testing.assert_array_equal(od.view(np.uint32), base_d.view(np.uint32), err_msg=str(kw))
