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
