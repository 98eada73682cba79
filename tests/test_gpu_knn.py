"""GPU parity of aqr_knn_bruteforce (MFMA screening + FP64 re-score) against
the oracle's brute force: ids and FP64 distances identical element by
element (the re-score sums (q_j - x_j)^2 in the same order), ties by id."""
import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(X, Q, k):
    import torch
    from paper_2602_21600_amd import aqr
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    ids, dist, cert = aqr.aqr_knn_bruteforce(Xd, Qd, k)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dist.cpu().numpy(), cert.cpu().numpy()


CASES = [
    # (n, d, nq, k, seed): several query blocks and tiles, ragged tails in
    # rows, dimensions and queries, one and several row partitions, k > n
    (5_000, 96, 300, 10, 1),
    (1_037, 37, 130, 17, 2),
    (40_000, 32, 64, 10, 3),      # eight row partitions
    (2_000, 960, 70, 10, 4),      # wide rows: 30 staged dimension chunks
    (3_001, 128, 65, 100, 5),
    (7, 20, 9, 10, 6),            # fewer rows than k: padding
    (1, 5, 3, 1, 7),
]


@pytest.mark.parametrize("n,d,nq,k,seed", CASES)
def test_knn_matches_oracle(orc, n, d, nq, k, seed):
    print(f"knn case n={n} d={d} nq={nq} k={k}", flush=True)
    X, Q = W.tiny(n, d, seed=seed, clusters=7, nq=nq)
    ids, dist, cert = _run(X, Q, k)
    rid, rd = orc.knn_f32(X, Q, k)
    np.testing.assert_array_equal(ids, rid)
    np.testing.assert_array_equal(dist.view(np.uint64), rd.view(np.uint64))
    # the certificate is a worst-case rounding bound (it grows with d): it
    # may decline a query whose result is exact, never the other way round
    assert cert.sum() >= 0.9 * nq


def test_knn_ties_and_duplicates(orc):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((3_000, 24)).astype(np.float32)
    X[100:140] = X[7]            # 41 identical rows
    X[2_000] = X[7]
    Q = rng.standard_normal((50, 24)).astype(np.float32)
    Q[:5] = X[7]                 # distance 0 to 42 rows: ids in order
    Q[5:10] = X[7] + 1e-3
    ids, dist, cert = _run(X, Q, 20)
    rid, rd = orc.knn_f32(X, Q, 20)
    np.testing.assert_array_equal(ids, rid)
    np.testing.assert_array_equal(dist.view(np.uint64), rd.view(np.uint64))
    assert list(ids[0, :3]) == [7, 100, 101]


def test_knn_rejects_bad_arguments():
    import torch
    from paper_2602_21600_amd import aqr
    X = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    Q = torch.zeros((2, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(aqr.AqrError):
        aqr.aqr_knn_bruteforce(X, Q, 129)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError, match="ws"):
        aqr.aqr_knn_bruteforce(X, Q, 5, ws=ws)
