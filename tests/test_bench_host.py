"""Host-side checks of the benchmark's bookkeeping (no GPU): the one-GPU
contract of --gpus, tie-inclusive recall, the parity classification of top-k
rows, the algorithmic byte count of a Stage-1 launch, the sweep's settings
and the tie rule of the launch-shape loop."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_recall_counts_ties_at_the_kth_distance(bench):
    # points on a line at 0, 1, 1, 2, 3 (ids 0..4); the query sits at 0
    X = np.array([[0.0], [1.0], [1.0], [2.0], [3.0]], np.float32)
    Q = np.zeros((1, 1), np.float32)
    gt_ids = np.array([[0, 1]])
    gt_d = np.array([[0.0, 1.0]])
    # id 2 ties the 2nd true distance exactly: it counts
    assert bench.recall_at(np.array([[0, 2]]), X, Q, gt_ids, gt_d, 2) == 1.0
    # id 3 is farther: it does not
    assert bench.recall_at(np.array([[0, 3]]), X, Q, gt_ids, gt_d, 2) == 0.5
    # padding (-1) never counts, and recall is capped at 1
    assert bench.recall_at(np.array([[-1, 1]]), X, Q, gt_ids, gt_d, 2) == 0.5
    assert bench.recall_at(np.array([[2, 1]]), X, Q, gt_ids, gt_d, 2) == 1.0
    # per-query k
    r = bench.recall_per_query(np.array([[0, 3], [3, 0]]), X, np.zeros((2, 1), np.float32),
                               np.array([[0, 1], [0, 1]]), np.array([[0.0, 1.0], [0.0, 1.0]]),
                               [1, 2])
    np.testing.assert_array_equal(r, [1.0, 0.5])


def test_topk_agreement_separates_ties_from_errors(bench):
    X = np.array([[0.0], [1.0], [1.0], [2.0]], np.float32)
    Q = np.zeros((3, 1), np.float32)
    ref = dict(id=np.array([[0, 1]] * 3), dist=np.array([[0.0, 1.0]] * 3))
    gid = np.array([[0, 1], [0, 2], [0, 3]])
    gdist = np.array([[0.0, 1.0], [0.0, 1.0], [0.0, 4.0]], np.float32)
    same, tied = bench.topk_agreement(gid, gdist, ref, X, Q, [2, 2, 2])
    assert (same, tied) == (1, 1)


def test_search_bytes_by_hand(bench):
    # per query: [expansions, layer-0 evaluations, upper evaluations, -, upper expansions]
    cnt = np.array([[10, 300, 20, 0, 4, 0, 0, 0], [12, 340, 22, 0, 5, 0, 0, 0]], np.int64)
    code, adj, io = bench.search_bytes(cnt, nq=2, d=100, d_pad=112, s0=64, s1=32, nc_total=150)
    assert code == (640 + 42 + 2) * 112
    assert adj == 22 * 64 * 4 + 9 * 32 * 4
    assert io == 2 * (400 + 4 + 8) + 8 * 150


def test_sweep_settings_follow_table3_then_cost_order(bench):
    from paper_2602_21600_amd import presets
    names = [c[0] for c in bench.RERANK_CONFIGS]
    assert len(set(names)) == len(names)
    # the Table 3 rows first, each with its own depth, thresholds and m_ef
    for (lo, _, nrr, gap, ratio, mef), cfg in zip(presets.TABLE3, bench.RERANK_CONFIGS):
        assert cfg[1:] == (nrr, gap, ratio, mef)
    # early termination on before off; deeper re-rank after shallower
    et_on = [np.isfinite(c[2]) for c in bench.RERANK_CONFIGS]
    assert et_on == sorted(et_on, reverse=True)
    off = [c for c in bench.RERANK_CONFIGS if not np.isfinite(c[2])]
    assert [c[1] for c in off if c[4] == 3] == sorted(c[1] for c in off if c[4] == 3)
    assert bench.rerank_by_name("no-et-50-nc2")[4] == 2


def test_launch_shape_ties_go_to_the_larger_cache_then_block(bench):
    # shapes within 1% of the fastest are equal; among them the larger visited
    # cache, then the larger block, is taken; a clearly faster shape still wins
    t = [(47.35, 9, 1), (47.30, 9, 2), (47.22, 9, 4), (60.5, 10, 1)]
    assert bench.pick_shape(t, None) == {"visited_log2": 9, "waves_per_block": 4}
    t = [(1.011, 12, 1), (1.014, 11, 1), (1.015, 12, 4), (1.2, 9, 1)]
    assert bench.pick_shape(t, None) == {"visited_log2": 12, "waves_per_block": 4}
    t = [(2.0, 8, 4), (2.5, 12, 4)]
    assert bench.pick_shape(t, None) == {"visited_log2": 8, "waves_per_block": 4}
    assert bench.pick_shape([], {"visited_log2": 7}) == {"visited_log2": 7}


def test_autotune_keeps_one_list_size_unless_two_win_clearly():
    from paper_2602_21600_amd import tune
    one = dict(waves_per_block=4, visited_log2=8)
    two = dict(waves_per_block=4, visited_log2=8, ef_small=128, small_waves=1)
    assert tune.pick([(one, 12.80), (two, 12.78)]) == one      # within 1%
    assert tune.pick([(one, 12.80), (two, 12.50)]) == two      # more than 1% faster
    assert tune.pick([(one, 12.70), (two, 12.90)]) == one
    assert tune.pick([(two, 12.90)]) == two                    # nothing else ran
