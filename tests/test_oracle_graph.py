"""Pins of the oracle's HNSW construction (Alg. 1 stage 3, HNSW of Section 2).

The paper delegates insertion to HNSW and prints no graph, so the pins are
hand-derived special cases and structural invariants.
"""
import json
import os

import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NONE = 0xFFFFFFFF


def check_invariants(g, M):
    """Degree caps, no self loops or duplicates, layer membership, entry point."""
    n = g["n"]
    lv = g["level"]
    adj0 = g["adj0"]
    assert adj0.shape == (n, 2 * M)
    for i in range(n):
        row = adj0[i]
        nb = row[row != NONE]
        # valid entries form a prefix
        assert np.all(row[: nb.size] != NONE)
        assert i not in nb
        assert np.unique(nb).size == nb.size
        assert np.all(nb < n)
    off = g["upper_off"]
    assert off[0] == 0 and off[-1] == lv.sum()
    for i in np.nonzero(lv > 0)[0]:
        for layer in range(1, lv[i] + 1):
            row = g["upper_adj"][off[i] + layer - 1]
            nb = row[row != NONE]
            assert nb.size <= M
            assert i not in nb
            assert np.unique(nb).size == nb.size
            assert np.all(lv[nb.astype(np.int64)] >= layer)
    assert g["L"] == lv.max()
    assert lv[g["ep"]] == g["L"]


def test_levels_closed_form(orc):
    M = 16
    u = np.array([1.0, 0.5, 1.0 / 16 + 1e-12, 1.0 / 16 - 1e-12, 1.0 / 256 + 1e-15,
                  1.0 / 256 - 1e-15, 1e-9])
    # floor(-ln(u) / ln(M)): level l when M^-(l+1) < u <= M^-l
    np.testing.assert_array_equal(orc.levels(u, M), [0, 0, 0, 1, 1, 2, 7])


def test_levels_distribution(orc):
    u = W.level_draws("small", 200000)
    lv = orc.levels(u, 16)
    # P(level >= l) = M^-l
    for l, p in [(1, 1 / 16), (2, 1 / 256)]:
        frac = np.mean(lv >= l)
        assert abs(frac - p) < 4 * np.sqrt(p / 200000)


def test_heuristic_hand_example(orc):
    spec = json.load(open(os.path.join(GOLDEN, "heuristic_circle.json")))
    pts = [spec["base"]]
    for r, deg in spec["points_polar"]:
        a = np.deg2rad(deg)
        pts.append([r * np.cos(a), r * np.sin(a)])
    # ids 0..4 are the candidates, id 5 the base
    X = np.array(pts[1:] + pts[:1], np.float32)
    ids = np.array([4, 2, 0, 3, 1], np.uint32)  # order of the input must not matter
    for key, want in spec["expected"].items():
        M = int(key.split("=")[1])
        got = orc.select_heuristic_f32(X, 5, ids, M)
        assert got.tolist() == want


def test_line_inserted_in_order_gives_path(orc):
    # 1-D codes 0,1,2,...: when node i is inserted every earlier node lies to
    # its left, the nearest (i-1) is kept and all others are closer to i-1
    # than to i, so each node links to i-1 and receives i+1: a path graph.
    n = 200
    codes = np.arange(n, dtype=np.uint8).reshape(n, 1)
    level = np.zeros(n, np.int32)
    for efc in (4, 300):
        g = orc.build(codes, 1, 8, efc, level)
        check_invariants(g, 8)
        for i in range(n):
            nb = sorted(int(x) for x in g["adj0"][i] if x != NONE)
            want = [j for j in (i - 1, i + 1) if 0 <= j < n]
            assert nb == want


def test_first_insert_links_all_when_few(orc):
    # With n <= M + 1 nodes on a line inserted in order and efc >= n the graph
    # is the path as above; inserting in reverse order gives the same path.
    n = 20
    codes = np.arange(n, dtype=np.uint8)[::-1].reshape(n, 1).copy()
    g = orc.build(codes, 1, 4, 50, np.zeros(n, np.int32))
    for i in range(n):
        nb = sorted(int(x) for x in g["adj0"][i] if x != NONE)
        assert nb == [j for j in (i - 1, i + 1) if 0 <= j < n]


def test_overflow_shrinks_with_heuristic(orc):
    # A star: centre 0 and 12 points on distinct directions (no pruning
    # between them since they are far apart relative to the centre).  With
    # M = 2 (cap 4 on layer 0) the centre's list must be shrunk and stay <= 4.
    rng = np.random.default_rng(0)
    d = 16
    n = 13
    codes = np.full((n, d), 128, np.uint8)
    for i in range(1, n):
        codes[i, (i - 1) % d] = 128 + 100 if i % 2 else 128 - 100
    g = orc.build(codes, d, 2, 32, np.zeros(n, np.int32))
    check_invariants(g, 2)
    deg = (g["adj0"] != NONE).sum(axis=1)
    assert deg.max() <= 4
    assert deg[0] == 4


@pytest.mark.parametrize("M,efc", [(8, 40), (31, 100)])
def test_invariants_on_mixture(orc, M, efc):
    X, _ = W.tiny(3000, 24, seed=7, clusters=6)
    tr = orc.train(X, p_max=0.01)
    codes = orc.encode(X, tr["min"], tr["scale"], stride=32)
    lv = orc.levels(W.level_draws("small", 3000), M)
    g = orc.build(codes, 24, M, efc, lv)
    check_invariants(g, M)


def test_build_is_deterministic(orc):
    X, _ = W.tiny(1500, 16, seed=9)
    tr = orc.train(X)
    codes = orc.encode(X, tr["min"], tr["scale"])
    lv = orc.levels(W.level_draws("small", 1500), 12)
    g1 = orc.build(codes, 16, 12, 40, lv)
    g2 = orc.build(codes, 16, 12, 40, lv)
    for k in ("adj0", "upper_adj", "upper_off"):
        np.testing.assert_array_equal(g1[k], g2[k])
    assert (g1["ep"], g1["L"]) == (g2["ep"], g2["L"])


def _codes(orc, n, d, seed):
    X, Q = W.tiny(n, d, seed=seed, clusters=6, nq=40)
    tr = orc.train(X, p_max=0.01)
    stride = (d + 15) // 16 * 16
    return X, Q, tr, orc.encode(X, tr["min"], tr["scale"], stride=stride)


def _same_graph(a, b):
    for key in ("adj0", "upper_adj", "upper_off", "level"):
        np.testing.assert_array_equal(a[key], b[key])
    assert (a["ep"], a["L"]) == (b["ep"], b["L"])


def test_batched_build_with_everything_seeded_in_unit_chunks_is_sequential(orc):
    X, _, _, codes = _codes(orc, 1200, 16, 3)
    lv = orc.levels(W.level_draws("small", 1200), 10)
    _same_graph(orc.build_batched(codes, 16, 10, 40, lv, seed_n=1200, batch=1),
                orc.build(codes, 16, 10, 40, lv))


def test_chunked_seed_keeps_invariants_and_recall(orc):
    # every point seeded, in chunks of up to 64: points of a chunk plan on
    # every level against the graph before the chunk, so the graph differs
    # from the sequential one but keeps the invariants and its recall
    n, M, efc, d = 3000, 12, 60, 24
    X, Q, tr, codes = _codes(orc, n, d, 6)
    lv = orc.levels(W.level_draws("small", n), M)
    gb = orc.build_batched(codes, d, M, efc, lv, seed_n=n, batch=64)
    gs = orc.build(codes, d, M, efc, lv)
    check_invariants(gb, M)
    assert not np.array_equal(gb["adj0"], gs["adj0"])
    qc = orc.encode(Q, tr["min"], tr["scale"], stride=codes.shape[1])
    truth, _ = orc.knn_codes(codes, d, qc, 10)
    rec = []
    for g in (gb, gs):
        s1 = orc.search_codes(g, codes, d, qc, 40, 40)
        hits = [len(set(s1["cand_id"][q, :10].tolist()) & set(truth[q].tolist()))
                for q in range(Q.shape[0])]
        rec.append(np.mean(hits) / 10)
    assert rec[0] >= rec[1] - 0.02, rec


def test_batched_build_with_unit_chunks_is_sequential(orc):
    # every upper-level point lies below seed_n, so the seed is the prefix
    # [0, seed_n) and chunks of one point continue in id order: the batched
    # build must then be the sequential build
    n, M = 1500, 10
    X, _, _, codes = _codes(orc, n, 16, 4)
    lv = orc.levels(W.level_draws("small", n), M)
    seed_n = 300
    lv[seed_n:] = 0
    lv[0] = max(lv[0], 1)
    _same_graph(orc.build_batched(codes, 16, M, 40, lv, seed_n=seed_n, batch=1),
                orc.build(codes, 16, M, 40, lv))


def test_batched_build_chunks_differ_but_keep_invariants_and_recall(orc):
    # chunks of up to 1/8 of the graph: points of a chunk do not see each
    # other, so the graph differs from the sequential one, but it keeps the
    # invariants and finds the exact neighbours about as often
    n, M, efc, d = 3000, 12, 60, 24
    X, Q, tr, codes = _codes(orc, n, d, 5)
    lv = orc.levels(W.level_draws("small", n), M)
    gb = orc.build_batched(codes, d, M, efc, lv, seed_n=200, batch=256)
    gs = orc.build(codes, d, M, efc, lv)
    check_invariants(gb, M)
    assert not np.array_equal(gb["adj0"], gs["adj0"])
    qc = orc.encode(Q, tr["min"], tr["scale"], stride=codes.shape[1])
    truth, _ = orc.knn_codes(codes, d, qc, 10)
    rec = []
    for g in (gb, gs):
        s1 = orc.search_codes(g, codes, d, qc, 40, 40)
        hits = [len(set(s1["cand_id"][q, :10].tolist()) & set(truth[q].tolist()))
                for q in range(Q.shape[0])]
        rec.append(np.mean(hits) / 10)
    assert rec[0] >= rec[1] - 0.02, rec
