"""Pins of the oracle's query path (Section 3.2, Alg. 2).

  * ef >= N makes the layer-0 search exhaustive over the nodes reachable
    from its entry point, so Stage 1 must equal brute force (numpy) there,
    bit-exact including order, and the baseline FP32 search must equal the
    exact k nearest neighbours.
  * N_c = N_rerank = N with early termination off reduces Alg. 2 to exact
    k-NN.
  * Hand cases for early termination, the re-rank depth and assembly.
"""
import json
import os
from collections import deque

import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NONE = 0xFFFFFFFF


def _index(orc, n=400, d=20, M0=6, efc0=40, seed=21, nq=12):
    X, Q = W.tiny(n, d, seed=seed, clusters=5, nq=nq)
    tr = orc.train(X, p_max=0.01, M0=M0, efc0=efc0)
    stride = (d + 15) // 16 * 16
    codes = orc.encode(X, tr["min"], tr["scale"], stride=stride)
    lv = orc.levels(W.level_draws("small", n), tr["M"])
    g = orc.build(codes, d, tr["M"], tr["efc"], lv)
    return dict(X=X, Q=Q, codes=codes, d=d, min=tr["min"], max=tr["max"], scale=tr["scale"],
                graph=g, tr=tr)


def _reachable(adj0, start):
    seen = {int(start)}
    dq = deque([int(start)])
    while dq:
        x = dq.popleft()
        for y in adj0[x]:
            if y == NONE:
                break
            y = int(y)
            if y not in seen:
                seen.add(y)
                dq.append(y)
    return np.array(sorted(seen), np.int64)


def test_param_map_reproduces_table3(orc):
    spec = json.load(open(os.path.join(GOLDEN, "table3_presets.json")))
    for _, nc, rr, gap, ratio, mult in spec["rows"]:
        efe, got = orc.param_map(10, nc * mult, mult)
        assert (efe, got) == (nc * mult, nc)
    # k > ef: ef_eff = k and N_c = k; N_c never exceeds ef_eff
    assert orc.param_map(100, 16, 3) == (100, 100)
    assert orc.param_map(10, 20, 3) == (20, 10)
    assert orc.param_map(1, 16, 3) == (16, 5)


def test_stage1_exhaustive_equals_bruteforce(orc):
    ix = _index(orc)
    n = ix["X"].shape[0]
    qc = orc.encode(ix["Q"], ix["min"], ix["scale"], stride=ix["codes"].shape[1])
    s1 = orc.search_codes(ix["graph"], ix["codes"], ix["d"], qc, n, n, tap_cap=n + 8)
    codes64 = ix["codes"][:, : ix["d"]].astype(np.int64)
    for q in range(qc.shape[0]):
        ep0 = s1["expanded"][q, 0]
        reach = _reachable(ix["graph"]["adj0"], ep0)
        vis = np.sort(s1["visited"][q, : s1["n_visited"][q]].astype(np.int64))
        np.testing.assert_array_equal(vis, reach)
        D = ((codes64[reach] - qc[q, : ix["d"]].astype(np.int64)) ** 2).sum(axis=1)
        order = np.lexsort((reach, D))
        cnt = s1["cand_cnt"][q]
        assert cnt == reach.size
        np.testing.assert_array_equal(s1["cand_id"][q, :cnt], reach[order])
        np.testing.assert_array_equal(s1["cand_D"][q, :cnt], D[order])


def test_f32_baseline_exhaustive_equals_exact_knn(orc):
    ix = _index(orc)
    n = ix["X"].shape[0]
    k = 10
    oid, od = orc.search_f32(ix["graph"], ix["X"], ix["Q"], n, k)
    X64 = ix["X"].astype(np.float64)
    for q in range(ix["Q"].shape[0]):
        # the layer-0 entry point of the FP32 search may differ from the code
        # search; every node reachable from any entry is compared
        reach = _reachable(ix["graph"]["adj0"], oid[q, 0])
        Dq = ((X64[reach] - ix["Q"][q].astype(np.float64)) ** 2).sum(axis=1)
        order = np.lexsort((reach, Dq))[:k]
        np.testing.assert_array_equal(oid[q], reach[order])
        np.testing.assert_allclose(od[q], Dq[order], rtol=1e-12)


def test_f32_expansion_tap(orc):
    # the expansion tap of the FP32 baseline: with ef >= N every node
    # reachable in layer 0 from the entry is expanded exactly once, nearest
    # first (the first expansion is the layer-0 entry point, the rest follow
    # the search order; tap-free and tapped runs return the same lists)
    ix = _index(orc)
    n = ix["X"].shape[0]
    oid, od = orc.search_f32(ix["graph"], ix["X"], ix["Q"], n, 10)
    oid2, od2, exp, nexp = orc.search_f32(ix["graph"], ix["X"], ix["Q"], n, 10, tap_cap=n)
    np.testing.assert_array_equal(oid, oid2)
    np.testing.assert_array_equal(od, od2)
    X64 = ix["X"].astype(np.float64)
    for q in range(ix["Q"].shape[0]):
        e = exp[q, :nexp[q]].astype(np.int64)
        assert len(set(e.tolist())) == len(e)
        reach = _reachable(ix["graph"]["adj0"], e[0])
        assert sorted(e.tolist()) == sorted(reach.tolist())
        # after the first expansion W holds every node seen, so each next
        # expansion is the nearest not yet expanded among those evaluated:
        # the distances of expansions 2.. never undercut an earlier one by
        # more than the order of discovery allows; the last expanded node is
        # no closer than the k-th result
        dq = ((X64[e] - ix["Q"][q].astype(np.float64)) ** 2).sum(axis=1)
        assert dq[-1] >= od[q, 9]


def test_exact_pipeline_equals_knn(orc):
    # N_c = N_rerank = N and early termination off: Alg. 2 returns exact kNN
    ix = _index(orc)
    n = ix["X"].shape[0]
    k = 10
    qc = orc.encode(ix["Q"], ix["min"], ix["scale"], stride=ix["codes"].shape[1])
    s1 = orc.search_codes(ix["graph"], ix["codes"], ix["d"], qc, n, n, tap_cap=n + 8)
    rr = orc.rerank(ix["X"], ix["codes"], ix["min"], ix["scale"], ix["Q"], s1["cand_id"],
                    s1["cand_cnt"], k, n_rerank=n, tau_gap=np.inf, tau_ratio=np.inf)
    X64 = ix["X"].astype(np.float64)
    for q in range(ix["Q"].shape[0]):
        reach = _reachable(ix["graph"]["adj0"], s1["expanded"][q, 0])
        Dq = ((X64[reach] - ix["Q"][q].astype(np.float64)) ** 2).sum(axis=1)
        order = np.lexsort((reach, Dq))[:k]
        np.testing.assert_array_equal(rr["id"][q], reach[order])
        np.testing.assert_allclose(rr["dist"][q], Dq[order], rtol=1e-12)
        assert np.all(rr["kind"][q] == 1)


def test_asymmetric_distance_uses_decoded_vectors(orc):
    ix = _index(orc, n=300, d=12)
    qc = orc.encode(ix["Q"], ix["min"], ix["scale"], stride=ix["codes"].shape[1])
    s1 = orc.search_codes(ix["graph"], ix["codes"], ix["d"], qc, 60, 20)
    rr = orc.rerank(ix["X"], ix["codes"], ix["min"], ix["scale"], ix["Q"], s1["cand_id"],
                    s1["cand_cnt"], 5, taps=True)
    # decode with numpy in FP32: x~ = code / scale + min (two FP32 operations)
    dec = (ix["codes"][:, :12].astype(np.float32) / ix["scale"]).astype(np.float32) + ix["min"]
    for q in range(ix["Q"].shape[0]):
        cnt = s1["cand_cnt"][q]
        ids = rr["a_id"][q, :cnt].astype(np.int64)
        da = ((dec[ids].astype(np.float64) - ix["Q"][q].astype(np.float64)) ** 2).sum(axis=1)
        np.testing.assert_allclose(rr["a_dist"][q, :cnt], da, rtol=1e-12)
        # A is sorted by (d^a, id)
        assert np.all(np.diff(rr["a_dist"][q, :cnt]) >= 0)
        assert sorted(ids.tolist()) == sorted(s1["cand_id"][q, :cnt].tolist())


def _et_setup(codes):
    codes = np.array(codes, np.uint8).reshape(-1, 1)
    mn = np.array([90.0], np.float32)
    sc = np.array([10.0], np.float32)
    X = (codes.astype(np.float32) / sc + mn).astype(np.float32)
    Q = np.zeros((1, 1), np.float32)
    cid = np.arange(codes.shape[0], dtype=np.uint32).reshape(1, -1)
    cnt = np.array([codes.shape[0]], np.int32)
    return codes, mn, sc, X, Q, cid, cnt


def test_early_termination_hand_cases(orc):
    spec = json.load(open(os.path.join(GOLDEN, "early_termination.json")))
    for case in spec["cases"]:
        codes, mn, sc, X, Q, cid, cnt = _et_setup(case["codes"])
        rr = orc.rerank(X, codes, mn, sc, Q, cid, cnt, 2, n_rerank=28, tau_gap=0.010,
                        tau_ratio=1.008, taps=True)
        np.testing.assert_allclose(rr["a_dist"][0, : cnt[0]], case["d_a"], rtol=1e-6)
        assert bool(rr["et"][0]) == case["et"], case["why"]
        # re-rank depth: min(|A|, k) under ET, else min(|A|, max(N_rerank, k))
        want = min(cnt[0], 2) if case["et"] else min(cnt[0], 28)
        assert rr["nrr"][0] == want


def test_ratio_gap_identity():
    # ratio = gap + d_k/(d_k + eps): with tau_ratio - 1 < tau_gap (every row of
    # Table 3) the ratio test is the one that decides.
    rng = np.random.default_rng(1)
    eps = 1e-6
    dk = rng.uniform(0.1, 100, 1000)
    dk1 = dk * rng.uniform(1.0, 1.05, 1000)
    gap = (dk1 - dk) / (dk + eps)
    ratio = dk1 / (dk + eps)
    np.testing.assert_allclose(ratio, gap + dk / (dk + eps), rtol=1e-12)
    spec = json.load(open(os.path.join(GOLDEN, "table3_presets.json")))
    for row in spec["rows"]:
        assert row[4] - 1.0 < row[3]


def test_force_et_switch(orc):
    codes, mn, sc, X, Q, cid, cnt = _et_setup([0, 100, 120, 130, 140])
    for f, et, nrr in [(-1, 1, 2), (0, 0, 5), (1, 1, 2)]:
        rr = orc.rerank(X, codes, mn, sc, Q, cid, cnt, 2, n_rerank=28, force_et=f, taps=True)
        assert (rr["et"][0], rr["nrr"][0]) == (et, nrr)


def test_assembly_padding_ties_and_kinds(orc):
    # three candidates, k = 5: every candidate is re-ranked exactly, results
    # padded with (-1, +inf); equal exact distances are ordered by id
    codes = np.array([[10, 0], [20, 0], [30, 0]], np.uint8)
    mn = np.zeros(2, np.float32)
    sc = np.ones(2, np.float32)
    X = np.array([[2.0, 0.0], [-2.0, 0.0], [1.0, 0.0]], np.float32)
    Q = np.zeros((1, 2), np.float32)
    cid = np.array([[2, 1, 0]], np.uint32)
    cnt = np.array([3], np.int32)
    rr = orc.rerank(X, codes, mn, sc, Q, cid, cnt, 5, n_rerank=28, taps=True)
    assert rr["id"][0].tolist() == [2, 0, 1, -1, -1]
    np.testing.assert_array_equal(rr["dist"][0], [1.0, 4.0, 4.0, np.inf, np.inf])
    assert rr["kind"][0].tolist() == [1, 1, 1, 0, 0]
    assert rr["nrr"][0] == 3 and rr["et"][0] == 0


def test_assembly_union_hand_case(orc):
    # d = 1, decoded x~ = code: d^a = 1, 4, 9, 16 for ids 0..3.  The exact
    # vectors differ (5, 6, 0.5, 0.25): d^e = 25, 36, 0.25, 0.0625.  ET forced
    # on with k = 2 re-ranks ids 0 and 1 only.  Fill mode stops at k exact
    # results; the union reading lets the approximate 9 and 16 of ids 2 and 3
    # win over the exact 25 and 36.
    codes = np.array([[1], [2], [3], [4]], np.uint8)
    mn = np.zeros(1, np.float32)
    sc = np.ones(1, np.float32)
    X = np.array([[5.0], [6.0], [0.5], [0.25]], np.float32)
    Q = np.zeros((1, 1), np.float32)
    cid = np.array([[0, 1, 2, 3]], np.uint32)
    cnt = np.array([4], np.int32)
    fill = orc.rerank(X, codes, mn, sc, Q, cid, cnt, 2, force_et=1, taps=True)
    assert fill["id"][0].tolist() == [0, 1] and fill["dist"][0].tolist() == [25.0, 36.0]
    assert fill["kind"][0].tolist() == [1, 1] and fill["nrr"][0] == 2
    union = orc.rerank(X, codes, mn, sc, Q, cid, cnt, 2, force_et=1, taps=True, assembly=1)
    assert union["id"][0].tolist() == [2, 3] and union["dist"][0].tolist() == [9.0, 16.0]
    assert union["kind"][0].tolist() == [2, 2]
    with pytest.raises(ValueError):
        orc.rerank(X, codes, mn, sc, Q, cid, cnt, 2, assembly=2)


def test_assembly_union_properties(orc):
    # on a random index: the union's k-th distance never exceeds fill's (it
    # chooses from a superset); every approximate entry carries its Stage-2
    # distance; with every candidate re-ranked the two readings agree
    ix = _index(orc, n=300, d=12)
    qc = orc.encode(ix["Q"], ix["min"], ix["scale"], stride=ix["codes"].shape[1])
    s1 = orc.search_codes(ix["graph"], ix["codes"], ix["d"], qc, 60, 20)
    args = (ix["X"], ix["codes"], ix["min"], ix["scale"], ix["Q"], s1["cand_id"], s1["cand_cnt"], 5)
    fill = orc.rerank(*args, n_rerank=5, force_et=1, taps=True)
    union = orc.rerank(*args, n_rerank=5, force_et=1, taps=True, assembly=1)
    assert np.all(union["dist"][:, -1] <= fill["dist"][:, -1])
    assert np.any(union["kind"] == 2)
    for q in range(ix["Q"].shape[0]):
        da = dict(zip(union["a_id"][q].tolist(), union["a_dist"][q].tolist()))
        for t in np.nonzero(union["kind"][q] == 2)[0]:
            assert union["dist"][q, t] == da[int(union["id"][q, t])]
    full_f = orc.rerank(*args, n_rerank=60, force_et=0)
    full_u = orc.rerank(*args, n_rerank=60, force_et=0, assembly=1)
    np.testing.assert_array_equal(full_f["id"], full_u["id"])
    np.testing.assert_array_equal(full_f["dist"], full_u["dist"])


def test_rerank_from_supplied_order(orc):
    # a supplied A order replaces the Stage-2 sort: with ET forced on and k=1
    # only the first supplied candidate is re-ranked
    codes = np.array([[10], [20], [30]], np.uint8)
    mn = np.zeros(1, np.float32)
    sc = np.ones(1, np.float32)
    X = np.array([[10.0], [20.0], [30.0]], np.float32)
    Q = np.zeros((1, 1), np.float32)
    cid = np.array([[0, 1, 2]], np.uint32)
    cnt = np.array([3], np.int32)
    rr = orc.rerank(X, codes, mn, sc, Q, cid, cnt, 1, force_et=1,
                    a_order=np.array([[2, 0, 1]], np.uint32))
    assert rr["id"][0].tolist() == [2]
    assert rr["dist"][0].tolist() == [900.0]


def test_library_presets_match_table3(orc):
    from paper_2602_21600_amd import presets
    spec = json.load(open(os.path.join(GOLDEN, "table3_presets.json")))
    assert len(presets.TABLE3) == len(spec["rows"])
    for row, (lo, nc, rr, gap, ratio, mult) in zip(spec["rows"], presets.TABLE3):
        assert float(row[0].split("-")[0].rstrip("+")) == lo
        assert (row[1], row[2], row[3], row[4], row[5]) == (nc, rr, gap, ratio, mult)
    for t, first in ((0.80, 0.85), (0.87, 0.85), (0.90, 0.90), (0.93, 0.90), (0.96, 0.95),
                     (0.98, 0.97), (0.999, 0.97)):
        p = presets.table3(t)
        row = next(r for r in presets.TABLE3 if r[0] == first)
        assert (p["nc"], p["n_rerank"], p["m_ef"]) == (row[1], row[2], row[5])
        # the search width of the row maps back to its N_c (Section 3.2)
        assert orc.param_map(10, p["ef"], p["m_ef"]) == (p["ef"], p["nc"])
