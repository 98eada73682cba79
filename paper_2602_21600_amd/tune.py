"""Autotuner of the batch launch: waves per block, resident waves per CU,
visited-cache size and re-rank waves per block, chosen by timing a sample
batch through libaqr; then, on the best of those, a second list size for
part of each block's waves (waves whose LDS holds lists of ef_small only).

The search result does not depend on these choices (only the speed does);
the tests check that.  Results are cached in a JSON file keyed by the index
shape, ef_max, k_max and the device name.
"""
import itertools
import json
import os
import time

from . import aqr

SEARCH_WPB = (1, 2, 4)
VISITED_LOG2 = (6, 7, 8, 9, 10)
RERANK_WPB = (2, 4)
# resident search waves per CU: 0 = as many as occupancy allows, else the
# persistent grid is cut to this many waves per CU
WAVES_PER_CU = (0, 8)
# second list size: ef_small as a fraction of ef_max (rounded up to whole
# 64-entry slots), on 1 .. waves_per_block - 1 waves of each block
SMALL_FRACTIONS = (4, 2)


def small_choices(wpb, ef_max):
    """(ef_small, small_waves) pairs tried for a block of wpb waves."""
    out = []
    for f in SMALL_FRACTIONS:
        es = (ef_max // f + 63) // 64 * 64
        if 1 <= es < ef_max:
            for sw in range(1, wpb):
                if (es, sw) not in out:
                    out.append((es, sw))
    return out


def _key(ix, ef_max, k_max, device_name):
    return f"n{ix.arena.numel()}-d{ix.d}-ef{ef_max}-k{k_max}-{device_name}"


def time_config(ix, Q, k, ef, k_max, ef_max, tuning, reps=3):
    import torch
    plan = aqr.BatchPlan(ix, Q.shape[0], k_max, ef_max, use_graph=False, tuning=tuning)
    n = plan.load(Q, k, ef)
    plan.launch(n)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        plan.launch(n)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / reps


def spin_up(ix, Q, k, ef, k_max, ef_max, seconds=0.5):
    """Keep the device busy for about `seconds` with the default launch shape:
    an idle GPU runs at a low clock, and configurations timed before the clock
    has ramped up would look slower than they are."""
    import torch
    plan = aqr.BatchPlan(ix, Q.shape[0], k_max, ef_max, use_graph=False, tuning={})
    n = plan.load(Q, k, ef)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        plan.launch(n)
        torch.cuda.synchronize()


def pick(table, tie=0.01):
    """The fastest tuning; two list sizes only when they beat the fastest
    single size by more than `tie` (repeat timings differ by about 0.5%, and
    one size is the simpler launch)."""
    best = min(table, key=lambda t: t[1])
    if best[0].get("small_waves"):
        single = [t for t in table if not t[0].get("small_waves")]
        if single:
            s = min(single, key=lambda t: t[1])
            if s[1] <= best[1] * (1.0 + tie):
                return s[0]
    return best[0]


def autotune(ix, Q, k, ef, k_max, ef_max, cache_path=None, reps=3, log=None):
    """Returns (best tuning dict, table of (tuning, ms))."""
    import torch
    name = torch.cuda.get_device_name()
    key = _key(ix, ef_max, k_max, name)
    if cache_path and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
            if cached:
                return cached["best"], cached["table"]
        except ValueError:
            pass
    table = []
    spin_up(ix, Q, k, ef, k_max, ef_max)
    n_cu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    for wpb, vb, rwpb, wpc in itertools.product(SEARCH_WPB, VISITED_LOG2, RERANK_WPB,
                                                WAVES_PER_CU):
        tuning = dict(waves_per_block=wpb, visited_log2=vb, rerank_waves_per_block=rwpb,
                      blocks=(n_cu * wpc) // wpb if wpc else 0)
        try:
            ms = time_config(ix, Q, k, ef, k_max, ef_max, tuning, reps)
        except aqr.AqrError as e:
            if log:
                log(f"tune {tuning}: skipped ({e})")
            continue
        table.append((tuning, round(ms, 4)))
        if log:
            log(f"tune {tuning}: {ms:.3f} ms")
    if not table:
        raise RuntimeError("autotune: no configuration could run")
    best = min(table, key=lambda t: t[1])[0]
    # second list size, on the best single-size choice and each block size
    for wpb in SEARCH_WPB:
        for es, sw in small_choices(wpb, max(ef_max, k_max)):
            tuning = dict(best, waves_per_block=wpb, ef_small=es, small_waves=sw)
            if best.get("blocks"):
                tuning["blocks"] = best["blocks"] * best["waves_per_block"] // wpb
            try:
                ms = time_config(ix, Q, k, ef, k_max, ef_max, tuning, reps)
            except aqr.AqrError as e:
                if log:
                    log(f"tune {tuning}: skipped ({e})")
                continue
            table.append((tuning, round(ms, 4)))
            if log:
                log(f"tune {tuning}: {ms:.3f} ms")
    best = pick(table)
    if cache_path:
        data = {}
        if os.path.exists(cache_path):
            try:
                data = json.load(open(cache_path))
            except ValueError:
                data = {}
        data[key] = {"best": best, "table": table}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        json.dump(data, open(cache_path, "w"), indent=1)
    return best, table
