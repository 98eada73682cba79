"""Benchmark: QPS at recall@10 >= 0.98 of the AQR-HNSW query path on one MI355X.

Workload (default): 1,000,000 x 128 FP32 base vectors drawn from a seeded
256-cluster Gaussian mixture with Zipf(1.1) cluster sizes and values clipped
at 0 (a SIFT-1M-shaped synthetic set), 10,000 queries from the same mixture,
HNSW M_0 = 16, ef_0^construction = 200, k = 10.

One step = the whole query path for the batch of queries: encode + Stage 1
(aqr_search) + Stages 2-3 (aqr_rerank), inputs resident in device memory.
ef is swept and the cheapest ef whose mean recall@10 reaches 0.98 is timed;
the baseline FP32 HNSW search on the same graph is swept and timed the same
way.  The CPU oracle (test infrastructure) is timed on a sample of the same
queries on the host cores.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2602_21600_amd import presets as PRESETS  # noqa: E402  (Table 3 rows, no torch)

HBM_PEAK_GBS = 8000.0
TARGET_RECALL = 0.98
# further points of the recall-QPS curve, each timed like the headline point
CURVE_TARGETS = (0.90, 0.95, 0.99)
CURVE_EXTRA_EF = (576, 640, 768, 896, 1024)
# ef sweep per workload (the cheapest ef reaching the target is timed); the
# default list is the workload's own ef values plus finer steps above them
SWEEP_EF = {
    "serving": [128, 192, 256, 320, 384, 448, 512, 576, 640, 768, 896, 1024],
}
# the default run: the metric on the largest configuration (10M x 96), then
# the other full-size configurations as extra keys, each with its roofline
DEFAULT_LEGS = ("sift1m", "gist1m")
# oracle time budget of the CPU baseline (seconds of host work)
CPU_SECONDS = 15.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def ground_truth(X, Q, k, device, qchunk=131072):
    """Exact k nearest neighbours (ids, FP64 squared distances, certified
    flags) from the library's brute-force kernel: FP32 screening on the
    matrix cores, FP64 re-score of the best k + 32."""
    import torch
    from paper_2602_21600_amd import aqr
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(device)
    ids_all, d_all, c_all = [], [], []
    for q0 in range(0, Q.shape[0], qchunk):
        Qd = torch.from_numpy(np.ascontiguousarray(Q[q0:q0 + qchunk])).to(device)
        i, dd, c = aqr.aqr_knn_bruteforce(Xd, Qd, k)
        ids_all.append(i.cpu().numpy())
        d_all.append(dd.cpu().numpy())
        c_all.append(c.cpu().numpy())
    del Xd
    torch.cuda.empty_cache()
    return np.concatenate(ids_all), np.concatenate(d_all), np.concatenate(c_all)


PARITY_RTOL = 1e-5  # FP32 device distances against the oracle's FP64 ones


def topk_agreement(gid, gdist, ref, X, Q, kq):
    """Rows whose top-k ids equal the oracle's, and rows that differ only by
    ties: device distances within PARITY_RTOL of the oracle's position by
    position, and each differing id's exact FP64 distance within PARITY_RTOL
    of the oracle's distance at that position."""
    same = tied = 0
    for q in range(gid.shape[0]):
        kk = int(kq[q])
        gi, oi = gid[q, :kk], ref["id"][q, :kk]
        if np.array_equal(gi, oi):
            same += 1
            continue
        rd = ref["dist"][q, :kk]
        ok = np.allclose(gdist[q, :kk].astype(np.float64), rd, rtol=PARITY_RTOL)
        for t in np.nonzero(gi != oi)[0]:
            if not ok or gi[t] < 0:
                ok = False
                break
            e = X[gi[t]].astype(np.float64) - Q[q].astype(np.float64)
            ok = abs(float(e @ e) - rd[t]) <= PARITY_RTOL * abs(rd[t])
        tied += int(ok)
    return same, tied


def recall_per_query(ids, X, Q, gt_ids, gt_d, kk, chunk=16384):
    """Per-query recall@kk[q]; a returned id also counts when its exact
    distance ties the kk-th true distance within a factor 1 + 1e-6."""
    ids = np.asarray(ids)
    nq = ids.shape[0]
    kk = np.broadcast_to(np.asarray(kk), (nq,)).astype(np.int64)
    kmax = int(kk.max()) if nq else 0
    out = np.zeros(nq)
    if nq == 0:
        return out
    r = ids[:, :kmax].astype(np.int64)
    g = gt_ids[:, :kmax].astype(np.int64)
    col = np.arange(kmax)
    rv = (col[None, :] < kk[:, None]) & (r >= 0)        # returned entries that count
    gv = col[None, :] < kk[:, None]                     # true neighbours that count
    hit = np.zeros((nq, kmax), bool)
    for s in range(0, nq, chunk):
        e = min(nq, s + chunk)
        eq = (r[s:e, :, None] == g[s:e, None, :]) & gv[s:e, None, :]
        hit[s:e] = eq.any(2)
    hit &= rv
    h = hit.sum(1)
    # tie-inclusive: a returned id outside the true list still counts when its
    # exact distance is within (1 + 1e-6) of the kk-th true distance
    miss = rv & ~hit & (h < kk)[:, None]
    qi, ci = np.nonzero(miss)
    if qi.size:
        thr = gt_d[np.arange(nq), kk - 1] * (1 + 1e-6)
        extra = np.zeros(nq, np.int64)
        for s in range(0, qi.size, 1 << 18):
            a, b = qi[s:s + (1 << 18)], ci[s:s + (1 << 18)]
            dv = X[r[a, b]].astype(np.float64) - Q[a].astype(np.float64)
            dd = np.einsum("ij,ij->i", dv, dv)
            np.add.at(extra, a, (dd <= thr[a]).astype(np.int64))
        h = h + extra
    out[:] = np.minimum(h, kk) / kk
    return out


def recall_at(ids, X, Q, gt_ids, gt_d, k=10):
    """Mean recall@k over the queries."""
    return float(recall_per_query(ids, X, Q, gt_ids, gt_d, k).mean())


# Re-rank settings swept after ef, cheapest first: the rows of Table 3 below
# "0.97+", its "0.97+" row, the upper ends of the ranges of the sensitivity
# analysis (Section 4.4), early termination switched off with growing exact
# re-rank depth, and then a longer candidate list A (N_c = ef/2 instead of
# ef/3).  Fields: name, N_rerank, tau_gap, tau_ratio, m_ef
# (N_c = clamp(floor(ef_eff / m_ef), k, ef_eff)).
RERANK_CONFIGS = [
    *((f"table3-{lo:.2f}", nrr, gap, ratio, mef)
      for lo, _, nrr, gap, ratio, mef in PRESETS.TABLE3[:-1]),
    ("table3", 28, 0.010, 1.008, 3),
    ("sec4.4", 28, 0.03, 1.02, 3),
    ("no-et", 28, float("inf"), float("inf"), 3),
    ("no-et-50", 50, float("inf"), float("inf"), 3),
    ("no-et-100", 100, float("inf"), float("inf"), 3),
    ("no-et-50-nc2", 50, float("inf"), float("inf"), 2),
    ("no-et-100-nc2", 100, float("inf"), float("inf"), 2),
]


ASSEMBLY = 0  # re-rank assembly: 0 fill (default reading), 1 union (--assembly union)
WEIGHTS = {"equal": 0, "per-dim": 1}  # aqr_qparams.weights (--weights)


class AqrRunner:
    def __init__(self, aqr, ix, nq, k, ef, device, visited_log2=0, waves_per_block=0,
                 rerank=RERANK_CONFIGS[0]):
        import torch
        self.torch = torch
        self.aqr = aqr
        self.rerank = rerank
        _, nrr, tg, tr, m_ef = rerank
        self.plan = aqr.QueryPlan(ix, nq, k, max(ef, k), m_ef=m_ef, visited_log2=visited_log2,
                                  waves_per_block=waves_per_block, n_rerank=nrr, tau_gap=tg,
                                  tau_ratio=tr, assembly=ASSEMBLY)
        self.k = torch.full((nq,), k, dtype=torch.int32, device=device)
        self.ef = torch.full((nq,), ef, dtype=torch.int32, device=device)

    def step(self, Qd):
        return self.plan.run(Qd, self.k, self.ef)

    def search_only(self, Qd, taps=None):
        p = self.plan
        n = Qd.shape[0]
        self.aqr.aqr_search(p.ix, Qd, self.k, self.ef, p.cand_id[:n], p.cand_D[:n],
                            p.cand_cnt[:n], p.ws, p.ef_max, p.nc_max, m_ef=p.m_ef, taps=taps,
                            **p.sp)

    def rerank_only(self, Qd):
        p = self.plan
        n = Qd.shape[0]
        self.aqr.aqr_rerank(p.ix, Qd, p.cand_id[:n], p.cand_cnt[:n], self.k, p.out_id[:n],
                            p.out_dist[:n], p.out_kind[:n], **p.rr)


class Fp32Runner:
    def __init__(self, aqr, ix, nq, k, ef, device, visited_log2=0, waves_per_block=0):
        import torch
        self.aqr = aqr
        self.ix = ix
        self.sp = dict(visited_log2=visited_log2, waves_per_block=waves_per_block)
        self.k_ = k
        self.ef_ = max(ef, k)
        self.k = torch.full((nq,), k, dtype=torch.int32, device=device)
        self.ef = torch.full((nq,), ef, dtype=torch.int32, device=device)
        self.out_id = torch.empty((nq, k), dtype=torch.int32, device=device)
        self.out_d = torch.empty((nq, k), dtype=torch.float32, device=device)
        self.ws = torch.zeros(aqr.aqr_search_workspace_size(), dtype=torch.uint8, device=device)

    def step(self, Qd, taps=None):
        self.aqr.aqr_search_fp32(self.ix, Qd, self.k, self.ef, self.out_id, self.out_d, self.ws,
                                 self.ef_, self.k_, taps=taps, **self.sp)
        return self.out_id, self.out_d


def spin_up(torch, fn, seconds=0.5):
    """Run fn(None) back to back for about `seconds`, so that an idle GPU's
    clock has ramped up before launch shapes are compared by timing."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn(None)
        torch.cuda.synchronize()


def timed(torch, fn, steps, warmup, kernel_events=None):
    """Run warmup then `steps` timed calls; returns (ms_per_step, per-kernel ms)."""
    for _ in range(warmup):
        fn(None)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(kernel_events or 0)]
        fn(marks)
        evs.append(marks)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    per = None
    if kernel_events:
        per = [np.mean([m[i].elapsed_time(m[i + 1]) for m in evs])
               for i in range(kernel_events - 1)]
    return ms, per


def source_sha():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2602_21600_amd", "csrc", "device.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(name, sha):
    """HBM bytes per launch from a committed rocprofv3 counter summary of the
    same kernel source, or None."""
    p = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except ValueError:
        return None
    if rec.get("device_hip_sha") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def search_bytes(cnt_big, nq, d, d_pad, s0, s1, nc_total):
    """Algorithmic bytes of one Stage-1 launch from distinct-evaluation counts:
    one code row per distinct evaluation (layer 0 and upper layers) plus the
    entry point, one adjacency row per expansion, the FP32 queries in and
    the candidate lists out."""
    code = int((cnt_big[:, 1].sum() + cnt_big[:, 2].sum() + nq) * d_pad)
    adj = int(cnt_big[:, 0].sum() * s0 * 4 + cnt_big[:, 4].sum() * s1 * 4)
    io = int(nq * (4 * d + 4 + 8) + 8 * nc_total)
    return code, adj, io


def tune_vbs(n):
    """Visited-cache sizes the launch-shape loop tries: 2^6 .. 2^12 buckets,
    from the smallest the id width allows (the stored part of a hashed id is
    at most 16 bits, and 16 only when the launch adds buckets beyond 2^vb;
    where it cannot, the library takes the next size)."""
    idbits = max(1, int(np.ceil(np.log2(max(n, 2)))))
    return list(range(max(6, idbits - 16), 13))


def pick_shape(timings, fallback, tie=0.01):
    """Launch shape from the tuning loop's (ms, visited_log2, waves_per_block)
    timings: shapes within `tie` of the fastest count as equal (repeat runs
    differ by about 0.5%), and among those the larger visited cache (fewer
    re-scored rows), then the larger block, is taken, so that noise does not
    flip the choice between runs."""
    if not timings:
        return fallback
    best = min(t[0] for t in timings)
    _, vb, wpb = max((t for t in timings if t[0] <= best * (1 + tie)), key=lambda t: (t[1], t[2]))
    return {"visited_log2": vb, "waves_per_block": wpb}


def finite_or_none(x):
    """JSON has no infinities: thresholds that switch early termination off
    are reported as null."""
    return x if x is None or np.isfinite(x) else None


def rerank_by_name(name):
    return next(c for c in RERANK_CONFIGS if c[0] == name)


def common_out(args, metric_value, ms, dtype="u8"):
    return {
        "metric": "QPS at recall@10>=0.98 on 1 MI355X, AQR-int8 vs FP32 HNSW; p50/p99 latency",
        "value": round(metric_value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
    }


def fp32_batched(args, torch, aqr, ix, Qd, kd, efd, b, X, Q, gt_ids, gt_d, efq, k10, kk, k_max,
                 ef_max):
    """FP32 HNSW on the batched workload's batch and order, its launch shape
    tuned on the same batch."""
    nq = Q.shape[0]
    dev = Qd.device
    out_id = torch.empty((nq, k_max), dtype=torch.int32, device=dev)
    out_d = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
    ws = torch.zeros(aqr.aqr_search_workspace_size(), dtype=torch.uint8, device=dev)

    # the baseline's launch shape is tuned on the same batch, as the AQR plan's is
    fp_sp, best_fp = {}, None
    spin_up(torch, lambda m: aqr.aqr_search_fp32(ix, Qd, kd, efd, out_id, out_d, ws, ef_max,
                                                 k_max, order=b["order"]))
    for vb in (7, 8, 9, 10, 11):
        for wpb in (1, 2, 4):
            cand = dict(visited_log2=vb, waves_per_block=wpb)
            try:
                ms_t, _ = timed(torch, lambda m: aqr.aqr_search_fp32(
                    ix, Qd, kd, efd, out_id, out_d, ws, ef_max, k_max, order=b["order"], **cand),
                    2, 1)
            except aqr.AqrError as e:  # LDS limit of the device
                log(f"tune fp32 {cand}: skipped ({e})")
                continue
            if best_fp is None or ms_t < best_fp:
                best_fp, fp_sp = ms_t, cand
    log(f"fp32 tuning picked {fp_sp}")

    def fp_step(marks):
        if marks:
            marks[0].record()
        aqr.aqr_search_fp32(ix, Qd, kd, efd, out_id, out_d, ws, ef_max, k_max, order=b["order"],
                            **fp_sp)
        if marks:
            marks[1].record()

    log("timing FP32 HNSW on the same batch")
    ms_fp, per_fp = timed(torch, fp_step, args.steps, args.warmup, kernel_events=2)
    rq_fp = recall_per_query(out_id.cpu().numpy(), X, Q, gt_ids, gt_d, kk)
    fp = {"value": round(nq / (ms_fp / 1e3), 1), "unit": "queries/s", "tuning": fp_sp,
          "ms_per_step": round(ms_fp, 4), "recall@min(k,10)": round(float(rq_fp.mean()), 5),
          "recall@10_by_ef": {int(v): round(float(rq_fp[k10 & (efq == v)].mean()), 5)
                              for v in np.unique(efq)}}
    log(f"FP32 {fp['value']:,.0f} QPS; recall {rq_fp.mean():.4f}")
    return fp


def bench_batched(args, torch, aqr, W, wl, dev, threads):
    """Uneven batch in one captured launch: per-query k and ef, longest first,
    tuning chosen by the autotuner; FP32 HNSW on the same batch beside it."""
    from paper_2602_21600_amd import tune
    t_all = time.perf_counter()
    log(f"generating {args.workload}")
    X = W.base(args.workload, args.n)
    nq = args.nq or wl.nq
    Q = W.queries(args.workload, nq)
    kq, efq = W.query_params(args.workload, nq)
    n, d = X.shape
    qz, g, codes, info, ginfo, t_quant, t_build = build_index(args, wl, X, threads)
    ix = aqr.aqr_index_bind(qz, g, codes, X, device=dev)
    k_max, ef_max = int(kq.max()), int(efq.max())
    log("ground truth")
    gt_ids, gt_d, _ = ground_truth(X, Q, 10, dev)
    Qd = torch.from_numpy(Q).to(dev)
    kd = torch.from_numpy(kq).to(dev)
    efd = torch.from_numpy(efq).to(dev)
    cfg = rerank_by_name(args.rerank or "table3")
    _, nrr, tg, tr, _ = cfg

    if args.profile:
        # a fixed launch shape, so that a profiler sees only the timed one
        best = dict(waves_per_block=args.wpb or 4, visited_log2=args.vb or 8,
                    rerank_waves_per_block=2, blocks=0)
        table = []
        log(f"--profile: fixed tuning {best}")
    else:
        S = min(nq, args.tune_sample)
        log(f"autotune on {S} queries")
        best, table = tune.autotune(ix, Qd[:S], kd[:S], efd[:S], k_max, ef_max, reps=2, log=log)
        log(f"autotune picked {best}")
    plan = aqr.BatchPlan(ix, nq, k_max, ef_max, n_rerank=nrr, tau_gap=tg, tau_ratio=tr,
                         use_graph=True, tuning=best)
    plan.load(Qd, kd, efd)

    def step(marks):
        plan.launch(nq)

    log(f"timing the captured batch: warmup {args.warmup}, steps {args.steps}")
    ms, _ = timed(torch, step, args.steps, args.warmup)
    qps = nq / (ms / 1e3)
    b = plan.bufs
    ids = b["out_id"][:nq].cpu().numpy()
    kk = np.minimum(kq, 10)
    rq = recall_per_query(ids, X, Q, gt_ids, gt_d, kk)
    rec_by_k = {int(v): round(float(rq[kq == v].mean()), 5) for v in np.unique(kq)}
    k10 = kq >= 10
    rec_by_ef = {int(v): round(float(rq[k10 & (efq == v)].mean()), 5) for v in np.unique(efq)}
    log(f"batch {qps:,.0f} QPS ({ms:.3f} ms/launch); recall@min(k,10) {rq.mean():.4f}; "
        f"recall@10 by ef {rec_by_ef}")

    # Stage-1 kernel alone, same order and tuning, for the roofline
    sp = dict(waves_per_block=best.get("waves_per_block", 0), blocks=best.get("blocks", 0),
              visited_log2=best.get("visited_log2", 0))

    def search_step(marks):
        if marks:
            marks[0].record()
        aqr.aqr_search(ix, Qd, kd, efd, b["cand_id"], b["cand_D"], b["cand_cnt"], b["ws"],
                       plan.ef_max, plan.nc_max, order=b["order"], **sp)
        if marks:
            marks[1].record()

    _, per = timed(torch, search_step, args.steps, 1, kernel_events=2)
    search_ms = per[0]
    counts = torch.zeros((nq, 8), dtype=torch.int32, device=dev)
    aqr.aqr_search(ix, Qd, kd, efd, b["cand_id"], b["cand_D"], b["cand_cnt"], b["ws"],
                   plan.ef_max, plan.nc_max, order=b["order"], visited_log2=14, waves_per_block=1,
                   taps=dict(cap=0, counts=counts))
    torch.cuda.synchronize()
    cnt_big = counts.cpu().numpy().astype(np.int64)
    nc_total = int(b["cand_cnt"][:nq].sum().item())
    s0 = (2 * ginfo["M"] + 15) // 16 * 16
    s1 = (ginfo["M"] + 15) // 16 * 16
    code_b, adj_b, io_b = search_bytes(cnt_big, nq, d, info["d_pad"], s0, s1, nc_total)
    alg = code_b + adj_b + io_b
    achieved = alg / (search_ms / 1e3) / 1e9
    lat_us = cnt_big[:, 5] / 100.0
    prof_name = (f"search_u8_batched_vb{best.get('visited_log2', 0)}"
                 f"_wpb{best.get('waves_per_block', 0)}"
                 + (f"_es{best['ef_small']}_sw{best['small_waves']}"
                    if best.get("small_waves") else ""))
    traffic = traffic_from_profile(prof_name, source_sha())

    copy_info = None
    fp = None
    if args.profile:
        # a plain copy of known size: its FETCH_SIZE/WRITE_SIZE readings scale
        # the counters of the search kernel to bytes
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        copy_info = {"bytes": args.copy_mib << 20}
        log("--profile: no FP32 baseline")
    else:
        fp = fp32_batched(args, torch, aqr, ix, Qd, kd, efd, b, X, Q, gt_ids, gt_d, efq, k10, kk,
                          k_max, ef_max)

    cpu = parity = None
    if not args.no_cpu:
        import oracle as orc
        orc.set_threads(threads)
        S = min(args.cpu_sample, nq)
        gx = aqr.aqr_graph_export(g)
        index = dict(X=X, codes=codes, d=d, min=info["min"], scale=info["scale"], graph=gx)
        log(f"CPU oracle on {S} queries with {orc.get_threads()} threads")
        t = time.perf_counter()
        ref = orc.query(index, Q[:S], kq[:S], efq[:S], n_rerank=nrr, tau_gap=tg, tau_ratio=tr)
        dt = time.perf_counter() - t
        cpu = {"value": round(S / dt, 1), "unit": "queries/s", "cores": orc.get_threads(),
               "kind": "oracle",
               "sample": f"first {S} of the {nq} queries with their own k and ef, same index; "
                         f"encode + Stage 1 + Stages 2-3 in FP64"}
        plan.launch(nq)
        torch.cuda.synchronize()
        s1r = ref["stage1"]
        gid = b["cand_id"][:S].cpu().numpy().view(np.uint32)
        gcnt = b["cand_cnt"][:S].cpu().numpy()
        exact = sum(int(gcnt[q] == s1r["cand_cnt"][q] and
                        np.array_equal(gid[q, :gcnt[q]], s1r["cand_id"][q, :gcnt[q]]))
                    for q in range(S))
        same, tied = topk_agreement(b["out_id"][:S].cpu().numpy(),
                                    b["out_dist"][:S].cpu().numpy(), ref, X, Q, kq)
        parity = {"queries": S, "stage1_bit_exact": exact, "topk_identical": same,
                  "topk_differ_only_by_ties": tied}
        log(f"oracle {cpu['value']:,.1f} QPS; parity {parity}")

    out = common_out(args, qps, ms)
    out.update({
        "config": {
            "workload": f"batched: {n:,} x {d} FP32 unit vectors (cosine as L2), "
                        f"{wl.n_clusters}-cluster mixture with Pareto(1.5) sizes; {nq:,} queries "
                        f"with k in {{1,10,100}} and ef in {{16,...,512}} in one captured launch",
            "n": n, "d": d, "nq": nq, "M0": wl.M0, "efc0": wl.efc0, "M_i": ginfo["M"],
            "graph_build": ("batched, device searches; quantiser density on the device"
                            if args.gpu_build else "host"),
            "delta": round(info["delta"], 6), "rerank": cfg[0], "n_rerank": nrr,
            "tau_gap": finite_or_none(tg), "tau_ratio": finite_or_none(tr), "tuning": best,
            "recall@min(k,10)": round(float(rq.mean()), 5), "recall_by_k": rec_by_k,
            "recall@10_by_ef": rec_by_ef, "global_batch": nq,
            "parallelism": "single GPU, one wavefront per query, persistent",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_profile": prof_name,
            "kernel": "k_search (Stage 1, 8-bit codes)", "kernel_ms": round(search_ms, 4),
            "alg_bytes_per_launch": alg, "code_bytes": code_b, "adjacency_bytes": adj_b,
            "io_bytes": io_b, "expansions_per_query": round(float(cnt_big[:, 0].mean()), 2),
            "distinct_evaluations_per_query": round(float(cnt_big[:, 1].mean()), 1),
        },
        "latency_us": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                       "p99": round(float(np.percentile(lat_us, 99)), 2),
                       "what": "per-query Stage-1 device time inside the batch"},
        "fp32_hnsw": fp,
        "speedup_vs_fp32": round(qps / fp["value"], 3) if fp else None,
        "autotune": table,
        "copy_kernel": copy_info,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "build_s": {"quantize": t_quant and round(t_quant, 1),
                    "graph": t_build and round(t_build, 1)},
        "device_hip_sha": source_sha(),
        "wall_s": round(time.perf_counter() - t_all, 1),
    })
    print(json.dumps(out, allow_nan=False), flush=True)


def bench_serving(args, torch, aqr, W, wl, dev, threads):
    """Continuous admission from Poisson arrival traces into the resident
    server kernel; latency from each request's arrival to its completion."""
    t_all = time.perf_counter()
    log(f"generating {args.workload}")
    X = W.base(args.workload, args.n)
    nq = args.nq or 50_000
    Q = W.queries(args.workload, nq)
    kq, efq = W.query_params(args.workload, nq)
    n, d = X.shape
    qz, g, codes, info, ginfo, t_quant, t_build = build_index(args, wl, X, threads)
    ix = aqr.aqr_index_bind(qz, g, codes, X, device=dev)
    log("ground truth")
    gt_ids, gt_d, _ = ground_truth(X, Q, 10, dev)
    Qd = torch.from_numpy(Q).to(dev)
    k_max, ef_max = 100, 512

    # calibration: cheapest ef (k = 10) reaching recall@10 >= 0.98 in batch mode
    C = min(nq, 10_000)
    efs = [int(e) for e in args.efs.split(",")] if args.efs else [64, 96, 128, 192, 256, 384,
                                                                   512]
    pick, sweep = None, []
    for ef in efs:
        for cfg in RERANK_CONFIGS:
            r = AqrRunner(aqr, ix, C, 10, ef, dev, rerank=cfg)
            ids, _ = r.step(Qd[:C])
            torch.cuda.synchronize()
            rec = recall_at(ids.cpu().numpy(), X, Q[:C], gt_ids[:C], gt_d[:C], 10)
            sweep.append((ef, cfg[0], round(rec, 5)))
            log(f"calibrate ef={ef} rerank={cfg[0]} recall@10={rec:.4f}")
            if rec >= TARGET_RECALL:
                pick = (ef, cfg)
                break
        if pick:
            break
    if pick is None:
        best = max(sweep, key=lambda t: t[2])
        pick = (best[0], rerank_by_name(best[1]))
    ef98, cfg = pick
    rec98 = next(r for e, c, r in sweep if e == ef98 and c == cfg[0])
    _, nrr, tg, tr, mef = cfg
    # the mixed stream's ef is log-uniform in [16, 512], so most of its
    # requests sit below ef_0.98; the same draws mapped onto [ef_0.98, 512]
    # give the stream whose k >= 10 requests reach the recall target
    lo, hi = np.log(16.0), np.log(512.0)
    u = np.clip((np.log(efq.astype(np.float64)) - lo) / (hi - lo), 0.0, 1.0)
    ef_hi = np.clip(np.exp(np.log(ef98) + u * (hi - np.log(ef98))).astype(np.int32), ef98, 512)
    streams = {
        "fixed": (np.full(nq, 10, np.int32), np.full(nq, ef98, np.int32)),
        "mixed": (kq, efq),
        "mixed_from_ef98": (kq, ef_hi.astype(np.int32)),
    }
    # batch capacity of each stream (same queries, one launch)
    batch_qps = {}
    for name, (ks, es) in streams.items():
        plan = aqr.BatchPlan(ix, nq, k_max, ef_max, m_ef=mef, n_rerank=nrr, tau_gap=tg,
                             tau_ratio=tr, use_graph=True)
        plan.load(Qd, torch.from_numpy(ks).to(dev), torch.from_numpy(es).to(dev))
        ms, _ = timed(torch, lambda m: plan.launch(nq), 3, 1)
        batch_qps[name] = nq / (ms / 1e3)
        log(f"batch capacity {name}: {batch_qps[name]:,.0f} QPS")
        del plan

    # Stage-1 roofline of the fixed stream run as one batch: the 8-bit search
    # kernel alone, timed with HIP events, against its algorithmic bytes from
    # distinct-evaluation counts (a run with a large visited cache)
    s_run = AqrRunner(aqr, ix, nq, 10, ef98, dev, rerank=cfg)
    spin_up(torch, lambda m: s_run.search_only(Qd))

    def s_step(marks):
        if marks:
            marks[0].record()
        s_run.search_only(Qd)
        if marks:
            marks[1].record()

    _, per_s = timed(torch, s_step, 5, 2, kernel_events=2)
    s_ms = per_s[0]
    counts = torch.zeros((nq, 8), dtype=torch.int32, device=dev)
    AqrRunner(aqr, ix, nq, 10, ef98, dev, visited_log2=14, waves_per_block=1,
              rerank=cfg).search_only(Qd, taps=dict(cap=0, counts=counts))
    torch.cuda.synchronize()
    cnt_big = counts.cpu().numpy().astype(np.int64)
    s0 = (2 * ginfo["M"] + 15) // 16 * 16
    s1 = (ginfo["M"] + 15) // 16 * 16
    nc_total = int(s_run.plan.cand_cnt[:nq].sum().item())
    code_b, adj_b, io_b = search_bytes(cnt_big, nq, d, info["d_pad"], s0, s1, nc_total)
    s_alg = code_b + adj_b + io_b
    s_achieved = s_alg / (s_ms / 1e3) / 1e9
    log(f"Stage-1 batch of the fixed stream: {s_ms:.3f} ms, {s_achieved:,.0f} GB/s algorithmic")
    serve_roofline = {
        "bound": "hbm", "achieved": round(s_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(s_achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "kernel": f"k_search (Stage 1, 8-bit codes) on the fixed stream as one batch of {nq:,}",
        "kernel_ms": round(s_ms, 4), "alg_bytes_per_launch": s_alg, "code_bytes": code_b,
        "adjacency_bytes": adj_b, "io_bytes": io_b,
    }

    sv = aqr.Server(ix, k_max, ef_max, ring=args.ring, m_ef=mef, n_rerank=nrr, tau_gap=tg,
                    tau_ratio=tr, idle_ms=200, visited_log2=args.serve_vb)
    results = {}
    try:
        # warm up the server (kernel launch, caches)
        w = min(nq, 2000)
        sv.replay(np.zeros(w), Q[:w], streams["fixed"][0][:w], streams["fixed"][1][:w])
        for si, (name, (ks, es)) in enumerate(streams.items()):
            # saturation: every request arrives at time 0
            _, _, lat, wall, svc = sv.replay(np.zeros(nq), Q, ks, es, service=True)
            sat = nq / wall
            log(f"server saturation {name}: {sat:,.0f} QPS; device service time p50 "
                f"{np.percentile(svc, 50) * 1e3:.3f} ms p99 {np.percentile(svc, 99) * 1e3:.3f} ms")
            rows = []
            for li, load in enumerate(args.loads):
                rate = load * sat
                cnt = int(min(4 * nq, max(5000, rate * args.serve_seconds)))
                idx = np.arange(cnt) % nq
                arr = W.poisson_arrivals(rate, cnt, seed=5000 + 100 * si + li)
                ids, _, lat, wall, svc = sv.replay(arr, Q[idx], ks[idx], es[idx], service=True)
                rq = recall_per_query(ids[:nq], X, Q[idx[:nq]], gt_ids[idx[:nq]],
                                      gt_d[idx[:nq]], np.minimum(ks[idx[:nq]], 10))
                k10 = ks[idx[:nq]] >= 10
                row = {"load": load, "offered_qps": round(rate, 1),
                       "achieved_qps": round(cnt / wall, 1), "requests": cnt,
                       "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
                       "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
                       "service_p50_ms": round(float(np.percentile(svc, 50)) * 1e3, 4),
                       "service_p99_ms": round(float(np.percentile(svc, 99)) * 1e3, 4),
                       "recall@min(k,10)": round(float(rq.mean()), 5),
                       "recall@10_of_k_ge_10": round(float(rq[k10].mean()), 5)}
                rows.append(row)
                log(f"{name} load {load}: {row}")
            results[name] = {"saturation_qps": round(sat, 1),
                             "batch_capacity_qps": round(batch_qps[name], 1), "loads": rows}
    finally:
        sv.stop()

    # the summary row: the highest offered load at or below saturation
    under = [r for r in results["fixed"]["loads"] if r["load"] <= 1.0] or results["fixed"]["loads"]
    head = max(under, key=lambda r: r["load"])
    out = common_out(args, head["achieved_qps"], 1e3 / max(head["achieved_qps"], 1e-9))
    out["steps"] = head["requests"]
    out.update({
        "config": {
            "workload": f"serving: {n:,} x {d} FP32 L2, {wl.n_clusters}-cluster mixture with "
                        f"log-uniform weights; Poisson arrivals; value = achieved QPS of the "
                        f"k=10, ef={ef98} stream at load {head['load']} of the server's "
                        f"saturation rate; ef is the cheapest reaching recall@10 >= 0.98 in "
                        f"batch mode, else the best reachable (calibrated recall@10 {rec98})",
            "n": n, "d": d, "M0": wl.M0, "efc0": wl.efc0, "M_i": ginfo["M"],
            "graph_build": ("batched, device searches; quantiser density on the device"
                            if args.gpu_build else "host"),
            "delta": round(info["delta"], 6), "ef": ef98, "recall@10": rec98,
            "rerank": cfg[0], "n_rerank": nrr, "m_ef": mef,
            "tau_gap": finite_or_none(tg), "tau_ratio": finite_or_none(tr), "ring": args.ring, "k_max": k_max,
            "ef_max": ef_max, "parallelism": "single GPU, resident persistent server kernel",
        },
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"],
                       "what": "arrival to completion seen by the host, queueing included"},
        "serving": results,
        "calibration": sweep,
        "roofline": serve_roofline,
        "cpu_baseline": None,
        "build_s": {"quantize": t_quant and round(t_quant, 1),
                    "graph": t_build and round(t_build, 1)},
        "device_hip_sha": source_sha(),
        "wall_s": round(time.perf_counter() - t_all, 1),
    })
    print(json.dumps(out, allow_nan=False), flush=True)


def build_index(args, wl, X, threads, name=None, cache="args"):
    """Quantiser and graph of the workload (built, or loaded from an index file)."""
    from paper_2602_21600_amd import aqr
    from paper_2602_21600_amd import workloads as W
    n, d = X.shape
    t_quant = t_build = None
    name = name or args.workload
    cache = args.cache if cache == "args" else cache
    if cache and os.path.exists(cache):
        # one checksummed index file (aqr_index_save / aqr_index_load)
        log(f"loading index from {cache}")
        qz, g, codes, Xf = aqr.aqr_index_load(cache)
        if Xf.shape != X.shape or not np.array_equal(Xf[:1000], X[:1000]):
            raise SystemExit(f"{cache} holds an index of other data")
    else:
        # --sq8: the paper's plain scalar-quantisation baseline, min/max bounds
        # (P_max = 0) and a graph at the configured M_0 and ef_0^c, with no
        # density adaptation
        p_max = 0.0 if args.sq8 else 0.01
        log(f"quantize n={n} d={d} threads={threads} p_max={p_max} "
            f"density on the {'GPU' if args.gpu_build else 'host'}")
        t = time.perf_counter()
        qz, codes = aqr.aqr_quantize(X, aqr.default_qparams(M0=wl.M0, efc0=wl.efc0,
                                                            p_max=p_max, threads=threads,
                                                            weights=WEIGHTS[args.weights]),
                                     device=args.gpu_build)
        t_quant = time.perf_counter() - t
        t = time.perf_counter()
        if args.gpu_build:
            g = aqr.aqr_build_batched(codes, X, d, qz, threads=threads,
                                      M=wl.M0 if args.sq8 else 0,
                                      efc=wl.efc0 if args.sq8 else 0,
                                      level_u=W.level_draws(name, n), progress=20)
        else:
            g = aqr.aqr_build(codes, d, qz, threads=threads,
                              M=wl.M0 if args.sq8 else 0, efc=wl.efc0 if args.sq8 else 0,
                              level_u=W.level_draws(name, n), progress=20)
        t_build = time.perf_counter() - t
        if cache:
            t = time.perf_counter()
            aqr.aqr_index_save(cache, qz, g, codes, X)
            log(f"index saved to {cache} in {time.perf_counter() - t:.1f} s")
    info = aqr.aqr_quantizer_info(qz)
    ginfo = aqr.aqr_graph_info(g)
    log(f"index ready: quantize {t_quant}s, build {t_build}s, delta={info['delta']:.4f} "
        f"M_i={info['M']} L={ginfo['L']}")
    return qz, g, codes, info, ginfo, t_quant, t_build


def recall_qps_curve(args, torch, aqr, ix, Qd, nq, k, dev, efs, aqr_table, fp_table, tuning,
                     fp_tuning, recall_of):
    """For each of CURVE_TARGETS: the cheapest AQR setting (smallest ef, then
    the re-rank settings in cost order) and the smallest FP32 ef whose recall
    reaches it, each timed over args.steps steps; None where no swept ef
    reaches the target."""
    a_tab = list(aqr_table)
    f_tab = list(fp_table)
    more = sorted(set(efs) | set(CURVE_EXTRA_EF))
    top = max(CURVE_TARGETS)

    def a_first(t):
        return next(((e, c, r) for e, c, r in a_tab if r >= t), None)

    def f_first(t):
        return next(((e, r) for e, r in f_tab if r >= t), None)

    done_a = {(e, c) for e, c, _ in a_tab}
    for ef in more:
        if a_first(top) is not None:
            break
        for cfg in RERANK_CONFIGS:
            if (ef, cfg[0]) in done_a:
                continue
            r = AqrRunner(aqr, ix, nq, k, ef, dev, rerank=cfg)
            ids, _ = r.step(Qd)
            torch.cuda.synchronize()
            rec = recall_of(ids)
            a_tab.append((ef, cfg[0], round(rec, 5)))
            log(f"curve aqr ef={ef} rerank={cfg[0]} recall@10={rec:.4f}")
            if rec >= top:
                break
    done_f = {e for e, _ in f_tab}
    for ef in more:
        if f_first(top) is not None:
            break
        if ef in done_f:
            continue
        r = Fp32Runner(aqr, ix, nq, k, ef, dev)
        ids, _ = r.step(Qd)
        torch.cuda.synchronize()
        rec = recall_of(ids)
        f_tab.append((ef, round(rec, 5)))
        log(f"curve fp32 ef={ef} recall@10={rec:.4f}")
    a_tab.sort(key=lambda t: (t[0], [c[0] for c in RERANK_CONFIGS].index(t[1])))
    f_tab.sort()
    out = []
    for t in CURVE_TARGETS:
        pa, pf = a_first(t), f_first(t)
        pt = {"target": t, "aqr": None, "fp32": None, "speedup": None}
        if pa is not None:
            cfg = rerank_by_name(pa[1])
            r = AqrRunner(aqr, ix, nq, k, pa[0], dev, rerank=cfg, **tuning)
            ms, _ = timed(torch, lambda m: r.step(Qd), args.steps, 50)
            pt["aqr"] = {"ef": pa[0], "rerank": pa[1], "recall@10": pa[2],
                         "qps": round(nq / (ms / 1e3), 1)}
        if pf is not None and fp_tuning is not None:
            r = Fp32Runner(aqr, ix, nq, k, pf[0], dev, **fp_tuning)
            ms, _ = timed(torch, lambda m: r.step(Qd), args.steps, 50)
            pt["fp32"] = {"ef": pf[0], "recall@10": pf[1], "qps": round(nq / (ms / 1e3), 1)}
        if pt["aqr"] and pt["fp32"]:
            pt["speedup"] = round(pt["aqr"]["qps"] / pt["fp32"]["qps"], 3)
        log(f"curve target {t}: {pt}")
        out.append(pt)
    return out


def bench_build(args, wl, threads):
    """--build-only: quantiser and graph of the workload, timed on the host clock
    around each call (the device parts wait for their own work)."""
    from paper_2602_21600_amd import workloads as W
    t_all = time.perf_counter()
    log(f"generating {args.workload}")
    X = W.base(args.workload, args.n)
    n, d = X.shape
    args.cache = None
    _, _, _, info, ginfo, t_quant, t_build = build_index(args, wl, X, threads)
    print(json.dumps({
        "metric": "index build time (quantiser training + encoding + HNSW graph)",
        "value": round(t_quant + t_build, 3), "unit": "s", "n_gpus": 1,
        "higher_is_better": False, "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n:,} x {d} FP32 base set", "n": n, "d": d,
                   "M0": wl.M0, "efc0": wl.efc0,
                   "M_i": ginfo["M"], "efc": info["efc"], "host_threads": threads,
                   "quantiser": "density on the device" if args.gpu_build else "host",
                   "graph_build": "batched, device searches" if args.gpu_build else "host"},
        "build_s": {"quantize": round(t_quant, 3), "graph": round(t_build, 3)},
        "wall_s": round(time.perf_counter() - t_all, 1)}), flush=True)


def run_search(args, torch, aqr, W, name, dev, threads, nq=None, curve_leg=True, cpu_leg=True,
               cache=None):
    """QPS at recall@10 >= 0.98 of one workload: build (or load) the index,
    exact ground truth on the device, sweep ef and the re-rank settings, time
    the cheapest AQR point and the cheapest FP32 HNSW point on the same graph,
    the Stage-1 roofline, optionally the recall-QPS curve and the CPU oracle
    leg.  Returns (the result dict, the context for further legs)."""
    wl = W.WORKLOADS[name]
    k = 10 if 10 in wl.k else wl.k[0]
    t_all = time.perf_counter()

    log(f"generating {name}")
    X = W.base(name, args.n)
    Q = W.queries(name, nq)
    n, d = X.shape
    nq = Q.shape[0]

    qz, g, codes, info, ginfo, t_quant, t_build = build_index(args, wl, X, threads, name=name, cache=cache)
    ix = aqr.aqr_index_bind(qz, g, codes, X, device=dev)
    gt_ids = gt_d = None
    gt_info = None
    if not args.profile:
        log("ground truth")
        t = time.perf_counter()
        gt_ids, gt_d, gt_cert = ground_truth(X, Q, k, dev)
        gt_info = {"kernel": "aqr_knn_bruteforce", "s": round(time.perf_counter() - t, 2),
                   "certified": int(gt_cert.sum()), "queries": nq}
        log(f"ground truth: {gt_info}")
    Qd = torch.from_numpy(Q).to(dev)

    # the workload's ef list, then finer steps above it, so the cheapest ef that
    # reaches the recall target is found for both searches alike
    efs = ([int(e) for e in args.efs.split(",")] if args.efs else SWEEP_EF.get(
        name, sorted(set(wl.ef) | {288, 304, 320, 352, 384, 448, 512})))

    def recall_of(ids):
        return recall_at(ids.cpu().numpy(), X, Q, gt_ids, gt_d, k)

    aqr_table, fp_table = [], []
    aqr_pick = fp_pick = None
    if args.profile:
        cfg = rerank_by_name(args.rerank or "no-et")
        aqr_pick = (args.ef or 256, float("nan"), cfg)
    else:
        def trial(ef, cfg):
            r = AqrRunner(aqr, ix, nq, k, ef, dev, rerank=cfg)
            ids, _ = r.step(Qd)
            torch.cuda.synchronize()
            rec = recall_of(ids)
            aqr_table.append((ef, cfg[0], round(rec, 5)))
            log(f"aqr ef={ef} rerank={cfg[0]} recall@10={rec:.4f}")
            return rec

        if args.full_sweep:
            # the sensitivity grid: every re-rank setting at every ef (Section
            # 4.4, Figure 3, Table 3); the headline point is chosen from it
            for ef in efs:
                for cfg in RERANK_CONFIGS:
                    trial(ef, cfg)
        for ef in efs:
            if args.full_sweep:
                hit = [(c, r) for e, c, r in aqr_table if e == ef and r >= TARGET_RECALL]
                if hit:
                    first = min(hit, key=lambda t: [c[0] for c in RERANK_CONFIGS].index(t[0]))
                    aqr_pick = (ef, first[1], rerank_by_name(first[0]))
                    break
                continue
            # the most exhaustive re-rank setting first: when it misses the
            # target at this ef, the cheaper settings (fewer candidates, fewer
            # exact distances) are not tried
            top = RERANK_CONFIGS[-1]
            if trial(ef, top) < TARGET_RECALL:
                continue
            for cfg in RERANK_CONFIGS[:-1]:
                rec = trial(ef, cfg)
                if rec >= TARGET_RECALL:
                    aqr_pick = (ef, rec, cfg)
                    break
            if aqr_pick is None:
                aqr_pick = (ef, next(r for e, c, r in aqr_table if e == ef and c == top[0]), top)
            break
        if aqr_pick is None:
            best = max(aqr_table, key=lambda t: t[2])
            aqr_pick = (best[0], best[2], next(c for c in RERANK_CONFIGS if c[0] == best[1]))
        for ef in efs:
            r = Fp32Runner(aqr, ix, nq, k, ef, dev)
            ids, _ = r.step(Qd)
            torch.cuda.synchronize()
            rec = recall_of(ids)
            fp_table.append((ef, round(rec, 5)))
            log(f"fp32 ef={ef} recall@10={rec:.4f}")
            if rec >= TARGET_RECALL:
                fp_pick = (ef, rec)
                break
        if fp_pick is None:
            # the target is out of reach on this sweep: the best recall reached
            best_f = max(fp_table, key=lambda t: t[1])
            fp_pick = (best_f[0], best_f[1])

    # ---- tuning (results do not depend on it) and the timed AQR path ----
    ef_a = aqr_pick[0]
    # launch shape of the timed search with --no-tune (results do not depend
    # on it); the library raises the visited cache to the id width's minimum
    tuning = {"visited_log2": 8, "waves_per_block": 4}
    if args.vb or args.wpb:
        tuning = {"visited_log2": args.vb, "waves_per_block": args.wpb}
    elif args.tune and not args.profile:
        timings = []
        r0 = AqrRunner(aqr, ix, nq, k, ef_a, dev, rerank=aqr_pick[2], **tuning)
        spin_up(torch, lambda m: r0.search_only(Qd))
        for vb in tune_vbs(n):
            for wpb in (1, 2, 4):
                try:
                    r = AqrRunner(aqr, ix, nq, k, ef_a, dev, visited_log2=vb,
                                  waves_per_block=wpb, rerank=aqr_pick[2])
                    ms_t, _ = timed(torch, lambda m: r.search_only(Qd), 3, 1)
                except aqr.AqrError as e:  # LDS limit of the device
                    log(f"tune visited_log2={vb} waves_per_block={wpb}: skipped ({e})")
                    continue
                log(f"tune visited_log2={vb} waves_per_block={wpb}: {ms_t:.3f} ms")
                timings.append((ms_t, vb, wpb))
        tuning = pick_shape(timings, tuning)
        log(f"tuning picked {tuning}")
    runner = AqrRunner(aqr, ix, nq, k, ef_a, dev, rerank=aqr_pick[2], **tuning)

    def aqr_step(marks):
        if marks:
            marks[0].record()
            runner.search_only(Qd)
            marks[1].record()
            runner.rerank_only(Qd)
            marks[2].record()
        else:
            runner.step(Qd)

    log(f"timing AQR at ef={ef_a}: warmup {args.warmup}, steps {args.steps}")
    ms_aqr, per = timed(torch, aqr_step, args.steps, args.warmup, kernel_events=3)
    qps_aqr = nq / (ms_aqr / 1e3)
    search_ms, rerank_ms = per
    log(f"AQR {qps_aqr:,.0f} QPS ({ms_aqr:.3f} ms/step; search {search_ms:.3f} ms, "
        f"rerank {rerank_ms:.3f} ms)")

    # per-query counters (separate, untimed run with a large visited cache so
    # that evaluations count distinct nodes)
    counts = torch.zeros((nq, 8), dtype=torch.int32, device=dev)
    big = AqrRunner(aqr, ix, nq, k, ef_a, dev, visited_log2=14, waves_per_block=1,
                    rerank=aqr_pick[2])
    big.search_only(Qd, taps=dict(cap=0, counts=counts))
    torch.cuda.synchronize()
    cnt_big = counts.cpu().numpy().astype(np.int64)
    counts.zero_()
    runner.search_only(Qd, taps=dict(cap=0, counts=counts))
    torch.cuda.synchronize()
    cnt = counts.cpu().numpy().astype(np.int64)
    d_pad = info["d_pad"]
    s0 = (2 * ginfo["M"] + 15) // 16 * 16
    s1 = (ginfo["M"] + 15) // 16 * 16
    nc = min(max(max(ef_a, k) // aqr_pick[2][4], k), max(ef_a, k))
    # algorithmic bytes of one search launch (distinct evaluations)
    code_bytes = int((cnt_big[:, 1].sum() + cnt_big[:, 2].sum() + nq) * d_pad)
    adj_bytes = int(cnt_big[:, 0].sum() * s0 * 4 + cnt_big[:, 4].sum() * s1 * 4)
    io_bytes = int(nq * (4 * d + 8 * nc + 4))
    alg_bytes = code_bytes + adj_bytes + io_bytes
    achieved = alg_bytes / (search_ms / 1e3) / 1e9
    reeval = float(cnt[:, 1].sum() / max(1, cnt_big[:, 1].sum()) - 1.0)
    lat_us = cnt[:, 5] / 100.0  # 100 MHz real-time clock
    sha = source_sha()
    prof_name = (f"search_{'sq8' if args.sq8 else 'u8'}_{name}_ef{ef_a}"
                 f"_vb{tuning['visited_log2']}"
                 f"_wpb{tuning['waves_per_block']}")
    traffic = traffic_from_profile(prof_name, sha)

    copy_info = None
    if args.profile:
        # a plain copy of known size: its FETCH_SIZE/WRITE_SIZE readings scale
        # the counters of the search kernel to bytes
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        copy_info = {"bytes": args.copy_mib << 20}

    # ---- timed FP32 baseline ----
    fp = None
    if fp_pick is not None:
        ef_f = fp_pick[0]
        # the baseline gets the same launch-shape treatment as the AQR search;
        # with --no-tune, a fixed shape (FP32 rows are 4x the bytes, so a
        # larger visited cache pays)
        fp_tuning = ({"visited_log2": args.vb, "waves_per_block": args.wpb}
                     if (args.vb or args.wpb) else {"visited_log2": 10, "waves_per_block": 4})
        if args.tune and not args.profile and not (args.vb or args.wpb):
            timings = []
            r0 = Fp32Runner(aqr, ix, nq, k, ef_f, dev, **fp_tuning)
            spin_up(torch, lambda m: r0.step(Qd))
            for vb in tune_vbs(n):
                for wpb in (1, 2, 4):
                    try:
                        r = Fp32Runner(aqr, ix, nq, k, ef_f, dev, visited_log2=vb,
                                       waves_per_block=wpb)
                        ms_t, _ = timed(torch, lambda m: r.step(Qd), 3, 1)
                    except aqr.AqrError as e:
                        log(f"tune fp32 visited_log2={vb} waves_per_block={wpb}: skipped ({e})")
                        continue
                    log(f"tune fp32 visited_log2={vb} waves_per_block={wpb}: {ms_t:.3f} ms")
                    timings.append((ms_t, vb, wpb))
            fp_tuning = pick_shape(timings, fp_tuning)
            log(f"fp32 tuning picked {fp_tuning}")
        frun = Fp32Runner(aqr, ix, nq, k, ef_f, dev, **fp_tuning)

        def fp_step(marks):
            if marks:
                marks[0].record()
                frun.step(Qd)
                marks[1].record()
            else:
                frun.step(Qd)

        log(f"timing FP32 HNSW at ef={ef_f}")
        ms_fp, per_fp = timed(torch, fp_step, args.steps, args.warmup, kernel_events=2)
        counts.zero_()
        frun.step(Qd, taps=dict(cap=0, counts=counts))
        torch.cuda.synchronize()
        cf = counts.cpu().numpy().astype(np.int64)
        xs = (d + 3) // 4 * 4
        fp_bytes = int((cf[:, 1].sum() + cf[:, 2].sum() + nq) * xs * 4 +
                       cf[:, 0].sum() * s0 * 4 + cf[:, 4].sum() * s1 * 4 + nq * (4 * d + 8 * k))
        fp = {"value": round(nq / (ms_fp / 1e3), 1), "unit": "queries/s", "ef": ef_f,
              "tuning": fp_tuning,
              "recall@10": round(fp_pick[1], 5),
              "reached_target": bool(fp_pick[1] >= TARGET_RECALL),
              "ms_per_step": round(ms_fp, 4),
              "kernel_ms": round(per_fp[0], 4),
              "achieved_GBps": round(fp_bytes / (per_fp[0] / 1e3) / 1e9, 1),
              "p50_query_us": round(float(np.percentile(cf[:, 5] / 100.0, 50)), 2),
              "p99_query_us": round(float(np.percentile(cf[:, 5] / 100.0, 99)), 2),
              "sweep": fp_table}
        log(f"FP32 {fp['value']:,.0f} QPS at ef={ef_f}")

    # ---- recall-QPS curve: the cheapest setting of each search at further
    # recall targets, timed the same way (the sweeps above stop at 0.98, so
    # they are continued for higher targets) ----
    curve = None
    if curve_leg and not args.profile and not args.no_curve:
        curve = recall_qps_curve(args, torch, aqr, ix, Qd, nq, k, dev, efs, aqr_table, fp_table,
                                 tuning, fp_tuning if fp is not None else None, recall_of)
        curve.append({"target": TARGET_RECALL,
                      "aqr": {"ef": ef_a, "rerank": aqr_pick[2][0],
                              "recall@10": round(aqr_pick[1], 5), "qps": round(qps_aqr, 1)},
                      "fp32": ({"ef": fp["ef"], "recall@10": fp["recall@10"],
                                "qps": fp["value"]} if fp else None),
                      "speedup": round(qps_aqr / fp["value"], 3) if fp else None})
        curve.sort(key=lambda c: c["target"])

    # ---- CPU oracle baseline on a bounded sample of the same queries ----
    cpu = None
    parity = None
    if cpu_leg and not args.no_cpu and not args.profile:
        cpu, parity = cpu_oracle_leg(args, aqr, g, X, Q, codes, info, d, k, ef_a, aqr_pick[2],
                                     runner.plan, threads, nq)

    out = {
        "metric": "QPS at recall@10>=0.98 on 1 MI355X, AQR-int8 vs FP32 HNSW; p50/p99 latency",
        "value": round(qps_aqr, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_aqr, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": f"{name}: {n:,} x {d} FP32 L2, {wl.n_clusters}-cluster "
                        f"Gaussian mixture; {nq:,} queries; k={k}"
                        + ("; plain SQ8 baseline (P_max 0, graph at M_0)" if args.sq8 else "")
                        + ("" if args.gpu_build else "; graph from the host build")
                        + ("; per-dimension density weights" if args.weights == "per-dim"
                           else ""),
            "n": n, "d": d, "nq": nq, "k": k, "ef": ef_a, "M0": wl.M0, "efc0": wl.efc0,
            "M_i": ginfo["M"], "efc": ginfo["efc"], "weights": args.weights,
            "eta": round(info["eta"], 6),
            "graph_build": ("batched, device searches; quantiser density on the device"
                            if args.gpu_build else "host"),
            "delta": round(info["delta"], 6), "m_ef": aqr_pick[2][4],
            "rerank": aqr_pick[2][0], "n_rerank": aqr_pick[2][1],
            "assembly": "union" if ASSEMBLY else "fill",
            "tau_gap": finite_or_none(aqr_pick[2][2]),
            "tau_ratio": finite_or_none(aqr_pick[2][3]),
            "recall@10": finite_or_none(round(aqr_pick[1], 5)), "tuning": tuning,
            "global_batch": nq, "parallelism": "single GPU, one wavefront per query",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "traffic_profile": prof_name,
            "kernel": "k_search (Stage 1, 8-bit codes)",
            "kernel_ms": round(search_ms, 4),
            "alg_bytes_per_launch": alg_bytes,
            "code_bytes": code_bytes, "adjacency_bytes": adj_bytes, "io_bytes": io_bytes,
            "code_gather_GBps": round(code_bytes / (search_ms / 1e3) / 1e9, 1),
            "code_gather_frac": round(code_bytes / (search_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "reevaluation_overhead": round(reeval, 4),
            "expansions_per_query": round(float(cnt[:, 0].mean()), 2),
            "evaluations_per_query": round(float(cnt[:, 1].mean()), 1),
        },
        "rerank_ms": round(rerank_ms, 4),
        "stage1_device_us": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                             "p99": round(float(np.percentile(lat_us, 99)), 2),
                             "what": "per-query Stage-1 device time inside the batch"},
        "ground_truth": gt_info,
        "fp32_hnsw": fp,
        "speedup_vs_fp32": (round(qps_aqr / fp["value"], 3) if fp else None),
        "aqr_sweep": aqr_table,
        "recall_qps_curve": curve,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "build_s": {"quantize": t_quant and round(t_quant, 1),
                    "graph": t_build and round(t_build, 1)},
        "device_hip_sha": sha,
        "copy_kernel": copy_info,
        "wall_s": round(time.perf_counter() - t_all, 1),
    }
    ctx = dict(ix=ix, X=X, Q=Q, Qd=Qd, gt_ids=gt_ids, gt_d=gt_d, ef=ef_a, cfg=aqr_pick[2], k=k,
               info=info, ginfo=ginfo, g=g, codes=codes, tuning=tuning, n=n, d=d, nq=nq,
               t_all=t_all)
    return out, ctx


def host_info():
    """Host CPU description for the CPU baseline."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"nproc": os.cpu_count(), "affinity": affinity, "model": model}


def cpu_oracle_leg(args, aqr, g, X, Q, codes, info, d, k, ef, cfg, plan, threads, nq):
    """The oracle (plain C, FP64) on the host cores the job may use, on a
    sample of the same queries sized to about CPU_SECONDS of work, and the
    parity of the device results with it on that sample."""
    import oracle as orc
    gx = aqr.aqr_graph_export(g)
    index = dict(X=X, codes=codes, d=d, min=info["min"], scale=info["scale"], graph=gx)
    _, nrr, tg, tr, mef = cfg

    def run(S, th):
        orc.set_threads(th)
        t = time.perf_counter()
        r = orc.query(index, Q[:S], k, ef, m_ef=mef, n_rerank=nrr, tau_gap=tg, tau_ratio=tr,
                      assembly=ASSEMBLY)
        return r, time.perf_counter() - t

    # size the sample from a short pilot on all threads
    S0 = min(nq, 256)
    _, dt0 = run(S0, threads)
    S = int(min(args.cpu_sample or nq, nq, max(S0, S0 * CPU_SECONDS / max(dt0, 1e-3))))
    log(f"CPU oracle on {S} queries with {threads} threads (pilot {S0} in {dt0:.2f} s)")
    ref, dt = run(S, threads)
    S1 = max(16, min(S, int(S0 * 2.0 / max(dt0 * threads, 1e-3))))
    _, dt1 = run(S1, 1)
    orc.set_threads(threads)
    cpu = {"value": round(S / dt, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": f"first {S} of the {nq} queries, same index and settings (ef={ef}, k={k}, "
                     f"re-rank {cfg[0]}); encode + Stage 1 + Stages 2-3, FP64 re-rank; "
                     f"{dt:.1f} s of host time",
           "one_thread_value": round(S1 / dt1, 1), "one_thread_sample": S1,
           "host": host_info()}
    s1 = ref["stage1"]
    gid = plan.cand_id[:S].cpu().numpy().view(np.uint32)
    gcnt = plan.cand_cnt[:S].cpu().numpy()
    exact = sum(int(gcnt[q] == s1["cand_cnt"][q] and
                    np.array_equal(gid[q, :gcnt[q]], s1["cand_id"][q, :gcnt[q]]))
                for q in range(S))
    same, tied = topk_agreement(plan.out_id[:S].cpu().numpy(), plan.out_dist[:S].cpu().numpy(),
                                ref, X, Q, np.full(S, k))
    parity = {"queries": S, "stage1_bit_exact": exact, "topk_identical": same,
              "topk_differ_only_by_ties": tied}
    log(f"oracle {cpu['value']:,.1f} QPS; parity {parity}")
    return cpu, parity


def serving_leg(args, torch, aqr, W, name, ctx, dev, loads=(0.5, 0.9), seconds=1.0):
    """Request latency on the same index: the resident server at the headline
    setting (k = 10, the timed ef and re-rank), Poisson arrivals at fractions
    of its saturation rate, and the workload's mixed stream (k in {1,10,100},
    per-query ef) at the highest load.  Latency runs from each request's
    arrival to the poll that finds it complete."""
    ix, Q, X = ctx["ix"], ctx["Q"], ctx["X"]
    gt_ids, gt_d = ctx["gt_ids"], ctx["gt_d"]
    _, nrr, tg, tr, mef = ctx["cfg"]
    ef = ctx["ef"]
    nq = Q.shape[0]
    ks_mix, efs_mix = W.query_params(name, nq)
    efs_mix = np.minimum(efs_mix, 1024)
    k_max, ef_max = 100, max(ef, int(efs_mix.max()))
    sv = aqr.Server(ix, k_max, ef_max, ring=args.ring, m_ef=mef, n_rerank=nrr, tau_gap=tg,
                    tau_ratio=tr, idle_ms=200, visited_log2=args.serve_vb)
    streams = {"fixed": (np.full(nq, 10, np.int32), np.full(nq, ef, np.int32)),
               "mixed": (ks_mix.astype(np.int32), efs_mix.astype(np.int32))}
    res = {}
    try:
        w = min(nq, 2000)
        sv.replay(np.zeros(w), Q[:w], streams["fixed"][0][:w], streams["fixed"][1][:w])
        for si, (sname, (ks, es)) in enumerate(streams.items()):
            # saturation from the whole query set at t = 0 (with fewer
            # requests the ramp and the tail lower the rate: 20,000 of the
            # 10M x 96 set read 1.64M QPS, all 100,000 read 1.93M)
            _, _, _, wall, svc = sv.replay(np.zeros(nq), Q, ks, es, service=True)
            sat = nq / wall
            rows = []
            for li, load in enumerate(loads if sname == "fixed" else loads[-1:]):
                rate = load * sat
                cnt = int(min(nq, max(5000, rate * seconds)))
                arr = W.poisson_arrivals(rate, cnt, seed=7000 + 100 * si + li)
                ids, _, lat, wall, svc = sv.replay(arr, Q[:cnt], ks[:cnt], es[:cnt], service=True)
                rq = recall_per_query(ids, X, Q[:cnt], gt_ids[:cnt], gt_d[:cnt],
                                      np.minimum(ks[:cnt], 10))
                row = {"load": load, "offered_qps": round(rate, 1),
                       "achieved_qps": round(cnt / wall, 1), "requests": cnt,
                       "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
                       "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
                       "service_p50_ms": round(float(np.percentile(svc, 50)) * 1e3, 4),
                       "service_p99_ms": round(float(np.percentile(svc, 99)) * 1e3, 4),
                       "recall@min(k,10)": round(float(rq.mean()), 5)}
                rows.append(row)
                log(f"serving {sname} load {load}: {row}")
            res[sname] = {"saturation_qps": round(sat, 1), "loads": rows}
    finally:
        sv.stop()
    return res


def main():
    T0 = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps before each timed region: an idle GPU sits at a low "
                         "clock and needs a fraction of a second of steady load to leave it")
    ap.add_argument("--workload", default="serving",
                    help="workload of the headline line (default: the 10M x 96 configuration, "
                         "followed by the --legs workloads as extra keys)")
    ap.add_argument("--legs", default=",".join(DEFAULT_LEGS),
                    help="further workloads measured after the default headline")
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--no-serve-leg", action="store_true",
                    help="skip the request-latency leg through the server kernel")
    ap.add_argument("--n", type=int, default=None, help="base subset (testing only)")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--efs", default=None, help="comma-separated ef sweep")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="cap of the CPU oracle's sample (0: sized to about 15 s of host work)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="skip sweeps and the CPU leg; time the AQR path at --ef (batched: "
                         "the fixed launch shape --vb/--wpb, no autotune, no FP32 baseline)")
    ap.add_argument("--ef", type=int, default=None)
    ap.add_argument("--rerank", default=None,
                    help="re-rank setting (--profile: default no-et; batched: table3)")
    ap.add_argument("--tune-sample", type=int, default=100_000,
                    help="batched: queries timed per launch shape (shapes that win on a small "
                         "sample can lose on the whole batch, whose occupancy matters more)")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the launch-shape loop of the timed searches (AQR and FP32) and "
                         "use fixed shapes (results do not depend on the shape)")
    ap.add_argument("--vb", type=int, default=0, help="visited_log2 of the timed search (skips tuning)")
    ap.add_argument("--wpb", type=int, default=0, help="waves per block of the timed search (skips tuning)")
    ap.add_argument("--serve", action="store_true",
                    help="serving only: Poisson traces through the resident server kernel")
    ap.add_argument("--ring", type=int, default=4096, help="serving: request slots")
    ap.add_argument("--serve-vb", type=int, default=0,
                    help="serving: visited_log2 of the server kernel (0: the library default)")
    ap.add_argument("--loads", default="0.1,0.25,0.5,0.75,0.9,1.1",
                    help="serving: offered loads as fractions of the saturation rate")
    ap.add_argument("--serve-seconds", type=float, default=1.0)
    ap.add_argument("--cache", default=None,
                    help="index file: loaded when it exists, else written after the build")
    ap.add_argument("--assembly", choices=("fill", "union"), default="fill",
                    help="re-rank assembly: fill from A while fewer than k (default), or the "
                         "union of the exact results with the rest of A")
    ap.add_argument("--host-build", dest="gpu_build", action="store_false",
                    help="train the quantiser and build the graph on the host (aqr_quantize, "
                         "aqr_build) instead of with the density search and the batched "
                         "build's chunk searches on the GPU (aqr_quantize_device, "
                         "aqr_build_batched)")
    ap.add_argument("--weights", choices=tuple(WEIGHTS), default="equal",
                    help="density weights w_j of Eq. 1 and eta: 'equal' (the printed formula, "
                         "eta = 0) or 'per-dim' (one-dimensional densities per dimension, "
                         "eta > 0, which raises M_i and lowers ef^c)")
    ap.add_argument("--sq8", action="store_true",
                    help="plain 8-bit scalar quantisation (P_max = 0) and a plain HNSW graph at "
                         "M_0 and ef_0^c: the paper's scalar-quantisation baseline")
    ap.add_argument("--full-sweep", action="store_true",
                    help="evaluate every re-rank setting at every ef of the sweep (the "
                         "sensitivity grid of Section 4.4) before choosing the timed point")
    ap.add_argument("--no-curve", action="store_true",
                    help="skip the recall-QPS curve at recall targets "
                         + ", ".join(str(t) for t in CURVE_TARGETS))
    ap.add_argument("--build-only", action="store_true",
                    help="train the quantiser and build the graph of the workload, then print "
                         "one JSON line with the build times (no search)")
    ap.add_argument("--copy-mib", type=int, default=256,
                    help="size of the plain copy kernel timed in --profile mode")
    args = ap.parse_args()
    global ASSEMBLY
    ASSEMBLY = 1 if args.assembly == "union" else 0

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2602_21600_amd import aqr
    from paper_2602_21600_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(3)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    wl = W.WORKLOADS[args.workload]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = threads if threads > 0 else min(16, os.cpu_count() or 1)
    args.loads = [float(x) for x in args.loads.split(",")]
    if args.build_only:
        return bench_build(args, wl, threads)
    if args.workload == "batched":
        if args.cpu_sample == 0:
            args.cpu_sample = 300
        return bench_batched(args, torch, aqr, W, wl, dev, threads)
    if args.serve:
        return bench_serving(args, torch, aqr, W, wl, dev, threads)
    nq = args.nq
    single = args.profile or args.no_legs or args.workload != "serving"
    out, ctx = run_search(args, torch, aqr, W, args.workload, dev, threads, nq=nq,
                          curve_leg=args.workload != "serving", cpu_leg=True, cache=args.cache)
    if not args.profile and not args.no_serve_leg:
        log("serving leg on the same index")
        sres = serving_leg(args, torch, aqr, W, args.workload, ctx, dev)
        head = sres["fixed"]["loads"][-1]
        out["latency_ms"] = {
            "p50": head["p50_ms"], "p99": head["p99_ms"], "load": head["load"],
            "achieved_qps": head["achieved_qps"],
            "what": "request latency from arrival to completion through the resident server "
                    "(Poisson arrivals at this fraction of its saturation rate; k=10 at the "
                    "headline ef and re-rank setting), queueing included"}
        out["serving"] = sres
    if not single:
        import gc
        out["legs"] = {}
        for leg in [x for x in args.legs.split(",") if x]:
            del ctx
            gc.collect()
            torch.cuda.empty_cache()
            log(f"leg {leg}")
            lo, ctx = run_search(args, torch, aqr, W, leg, dev, threads, nq=None,
                                 curve_leg=False, cpu_leg=False, cache=None)
            out["legs"][leg] = {f: lo[f] for f in (
                "value", "unit", "ms_per_step", "config", "roofline", "rerank_ms",
                "stage1_device_us", "fp32_hnsw", "speedup_vs_fp32", "ground_truth", "build_s",
                "wall_s")}
    out["wall_s"] = round(time.perf_counter() - T0, 1)
    print(json.dumps(out, allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
