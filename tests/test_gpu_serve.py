"""Serving: continuous admission into a resident persistent kernel.

Each request's result must be the same when it is served alone, in a stream
of overlapping requests, replayed from an arrival trace, and after the
kernel has gone idle and been relaunched; and it must equal the batch
path's result for the same query, k and ef (ids bit-exact, distances
bit-identical: both run the same per-query code).
"""
import time

import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

pytestmark = pytest.mark.gpu

K_MAX, EF_MAX = 100, 512


@pytest.fixture(scope="module")
def small(orc):
    from test_gpu_parity import make_index
    X = W.base("small")
    ix = make_index(orc, X, 16, 100)
    rng = np.random.default_rng(21)
    Q = np.vstack([W.queries("small"), W.queries("small", 300)[100:]])
    nq = Q.shape[0]
    ix["Q"] = Q
    ix["k"] = rng.choice(np.array([1, 10, 100], np.int32), nq)
    ix["ef"] = rng.choice(np.array([16, 64, 128, 512], np.int32), nq)
    return ix


def batch_results(index, Q, k, ef):
    import torch
    from test_gpu_batch import run_plan
    return run_plan(index, Q, k, ef)[0]


def wait(server, ticket, timeout=30.0):
    t0 = time.monotonic()
    while True:
        r = server.poll(ticket)
        if r is not None:
            return r
        assert time.monotonic() - t0 < timeout, "request not completed"
        time.sleep(1e-4)


def check_row(ids, dist, ref, q):
    np.testing.assert_array_equal(ids, ref["id"][q], err_msg=f"q={q}")
    np.testing.assert_array_equal(dist.view(np.uint32), ref["dist"][q].view(np.uint32),
                                  err_msg=f"q={q}")


def test_serve_overlapping_requests_equal_batch(small):
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"], small["k"], small["ef"]
    ref = batch_results(small, Q, k, ef)
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=64)
    try:
        pending = {}
        nq = Q.shape[0]
        nxt = 0
        done = 0
        # keep up to 48 requests in flight; collect in a different order
        while done < nq:
            while nxt < nq and len(pending) < 48:
                t = sv.submit(Q[nxt], k[nxt], ef[nxt])
                assert t is not None
                pending[t] = nxt
                nxt += 1
            for t in sorted(pending, reverse=True):
                r = sv.poll(t)
                if r is not None:
                    check_row(r[0], r[1], ref, pending.pop(t))
                    done += 1
    finally:
        sv.stop()


def test_serve_alone_and_after_idle_relaunch(small):
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"], small["k"], small["ef"]
    ref = batch_results(small, Q, k, ef)
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=8, idle_ms=1)
    try:
        for q in (0, 3, 77):
            r = wait(sv, sv.submit(Q[q], k[q], ef[q]))
            check_row(r[0], r[1], ref, q)
            time.sleep(0.02)  # the kernel leaves after 1 ms idle; the next submit relaunches
        sv.stop()
        r = wait(sv, sv.submit(Q[5], k[5], ef[5]))
        check_row(r[0], r[1], ref, 5)
    finally:
        sv.stop()


def test_serve_ring_admission(small):
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"], small["k"], small["ef"]
    ref = batch_results(small, Q, k, ef)
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=4)
    try:
        tickets = [sv.submit(Q[q], k[q], ef[q]) for q in range(4)]
        assert None not in tickets
        # every slot holds an uncollected request: admission refuses
        assert sv.submit(Q[4], k[4], ef[4]) is None
        r = wait(sv, tickets[0])
        check_row(r[0], r[1], ref, 0)
        t4 = sv.submit(Q[4], k[4], ef[4])
        assert t4 is not None
        for q, t in zip((1, 2, 3, 4), tickets[1:] + [t4]):
            r = wait(sv, t)
            check_row(r[0], r[1], ref, q)
        with pytest.raises(aqr.AqrError):
            sv.poll(t4)  # already collected
        with pytest.raises(aqr.AqrError):
            sv.submit(Q[0], K_MAX + 1, 64)  # beyond the server's k_max
    finally:
        sv.stop()


def test_serve_replay_trace(small):
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"], small["k"], small["ef"]
    ref = batch_results(small, Q, k, ef)
    nq = Q.shape[0]
    arrivals = W.poisson_arrivals(20000.0, nq, seed=7)
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=256)
    try:
        ids, dist, lat, wall, svc = sv.replay(arrivals, Q, k, ef, service=True)
    finally:
        sv.stop()
    for q in range(nq):
        check_row(ids[q], dist[q], ref, q)
    assert np.all(lat > 0) and wall >= arrivals[-1]
    assert np.all(svc > 0) and np.all(svc <= lat + 1e-3)


def test_serve_longer_candidate_list_equals_batch(small):
    # m_ef = 2 (N_c = ef/2): the server sizes its candidate lists by m_ef and
    # must still return the batch path's rows for the same settings
    from paper_2602_21600_amd import aqr
    from test_gpu_batch import run_plan
    Q, k, ef = small["Q"][:200], small["k"][:200], small["ef"][:200]
    ref = run_plan(small, Q, k, ef, m_ef=2, n_rerank=50, tau_gap=float("inf"),
                   tau_ratio=float("inf"))[0]
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=256, m_ef=2, n_rerank=50,
                    tau_gap=float("inf"), tau_ratio=float("inf"))
    try:
        tickets = [sv.submit(Q[q], k[q], ef[q]) for q in range(Q.shape[0])]
        assert all(t is not None for t in tickets)
        for q, t in enumerate(tickets):
            r = wait(sv, t)
            check_row(r[0], r[1], ref, q)
    finally:
        sv.stop()


def _near_threshold(ref, q, k, tau_gap, tau_ratio, rtol=1e-5):
    """The oracle's early-termination statistics of query q lie within rtol of
    a threshold (the FP32 device may then decide the other way)."""
    a = ref["a_dist"][q]
    if not np.isfinite(tau_gap) or k >= int(ref["stage1"]["cand_cnt"][q]):
        return False
    dk, dk1 = a[k - 1], a[k]
    gap = (dk1 - dk) / (dk + 1e-6)
    ratio = dk1 / (dk + 1e-6)
    return abs(gap - tau_gap) <= rtol * tau_gap or abs(ratio - tau_ratio) <= rtol * tau_ratio


@pytest.mark.parametrize("et", ["off", "table3"])
def test_serve_matches_oracle(orc, small, et):
    # every served row of a mixed k/ef stream against the oracle's Alg. 2:
    # distances within 1e-5 of its FP64 values, ids equal up to ties inside
    # that tolerance (rows whose early-termination statistics sit within 1e-5
    # of a threshold may take the other branch and are counted, not compared)
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"], small["k"], small["ef"]
    inf = float("inf")
    tg, tr = (inf, inf) if et == "off" else (0.010, 1.008)
    index = dict(X=small["X"], codes=small["codes"], d=small["d"], min=small["min"],
                 scale=small["scale"], graph=small["graph"])
    ref = orc.query(index, Q, k, ef, n_rerank=28, tau_gap=tg, tau_ratio=tr, taps=True)
    nq = Q.shape[0]
    arrivals = W.poisson_arrivals(50000.0, nq, seed=9)
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=128, tau_gap=tg, tau_ratio=tr)
    try:
        ids, dist, lat, wall = sv.replay(arrivals, Q, k, ef)
    finally:
        sv.stop()
    skipped = 0
    for q in range(nq):
        kq = int(k[q])
        if _near_threshold(ref, q, kq, tg, tr):
            skipped += 1
            continue
        rd = ref["dist"][q, :kq]
        np.testing.assert_allclose(dist[q, :kq].astype(np.float64), rd, rtol=1e-5,
                                   err_msg=f"q={q}")
        gi, oi = ids[q, :kq], ref["id"][q, :kq]
        for t in np.nonzero(gi != oi)[0]:
            close = np.abs(rd - rd[t]) <= 1e-5 * max(rd[t], 1e-30)
            assert close.sum() >= 2, f"q={q} slot {t}: ids differ away from a tie"
        assert np.all(ids[q, kq:] == -1)
    assert skipped <= nq // 50


def test_serve_budget_admission(small):
    # admission charges each request its own LDS pages and state bytes:
    # requests beyond the budget are refused, and admitted again once earlier
    # results are collected; rows admitted under budget pressure equal the
    # batch rows
    from paper_2602_21600_amd import aqr
    Q, k, ef = small["Q"], small["k"], small["ef"]
    ref = batch_results(small, Q, k, ef)
    probe = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=16)
    big_p, big_b = probe.request_cost(100, 512)
    small_p, small_b = probe.request_cost(1, 16)
    del probe
    assert small_p < big_p and small_b < big_b
    # LDS budget: one large request and one small request at a time
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=16, lds_budget_pages=big_p + small_p)
    try:
        big = [q for q in range(len(k)) if k[q] == 100 and ef[q] == 512][:2]
        tiny = [q for q in range(len(k)) if k[q] == 1 and ef[q] == 16][:2]
        assert len(big) == 2 and len(tiny) == 2
        t0 = sv.submit(Q[big[0]], 100, 512)
        assert t0 is not None
        assert sv.submit(Q[big[1]], 100, 512) is None          # over the LDS budget
        u = sv.usage()
        assert u["lds_used_pages"] == big_p and u["slots_used"] == 1
        t1 = sv.submit(Q[tiny[0]], 1, 16)                      # fits beside it
        assert t1 is not None
        assert sv.submit(Q[tiny[1]], 1, 16) is None           # budget full
        r = wait(sv, t0)
        check_row(r[0], r[1], ref, big[0])
        t2 = sv.submit(Q[big[1]], 100, 512)                    # admitted again
        assert t2 is not None
        for q, t in ((tiny[0], t1), (big[1], t2)):
            r = wait(sv, t)
            check_row(r[0], r[1], ref, q)
        assert sv.usage()["lds_used_pages"] == 0 and sv.usage()["state_used"] == 0
    finally:
        sv.stop()
    # state budget: room for two k = 100 requests
    sv = aqr.Server(small["ix"], K_MAX, EF_MAX, ring=16, state_budget=2 * big_b)
    try:
        qs = [q for q in range(len(k)) if k[q] == 100][:3]
        ts = [sv.submit(Q[q], 100, int(ef[q])) for q in qs[:2]]
        assert None not in ts
        assert sv.submit(Q[qs[2]], 100, int(ef[qs[2]])) is None  # state budget exhausted
        assert sv.usage()["state_used"] == 2 * big_b
        r = wait(sv, ts[0])
        check_row(r[0], r[1], ref, qs[0])
        t3 = sv.submit(Q[qs[2]], 100, int(ef[qs[2]]))
        assert t3 is not None
        for q, t in ((qs[1], ts[1]), (qs[2], t3)):
            r = wait(sv, t)
            check_row(r[0], r[1], ref, q)
    finally:
        sv.stop()
    with pytest.raises(aqr.AqrError):
        aqr.Server(small["ix"], K_MAX, EF_MAX, ring=4, lds_budget_pages=1)  # below one request
