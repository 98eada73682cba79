"""Pins of the oracle's brute-force k nearest neighbours (the exact truth that
recall and several parity tests are measured against).

  * orc_knn_f32: squared L2 in FP64 from FP32 inputs, ordered by
    (distance, id).  Pinned by scipy's cdist in FP64 and a lexicographic sort
    written here, on data with exact duplicate rows (ties broken by id) and
    with k > n (padding -1 / +inf).
  * orc_knn_codes: the integer code distance sum_j (a_j - b_j)^2 of Stage 1
    (Section 3.2), ordered by (D, id).  Pinned by numpy integer arithmetic in
    int64 on codes with repeated rows, k > n (padding 0xFFFFFFFF) and a
    stride wider than d (padding bytes must not count).
"""
import numpy as np
from scipy.spatial.distance import cdist

NONE = 0xFFFFFFFF


def _lexi_topk(dist, k):
    """Indices of the k smallest entries per row under (distance, index)."""
    n = dist.shape[1]
    out = np.full((dist.shape[0], k), -1, np.int64)
    for q in range(dist.shape[0]):
        order = np.lexsort((np.arange(n), dist[q]))  # last key sorts first
        m = min(k, n)
        out[q, :m] = order[:m]
    return out


def _with_duplicates(rng, n, d, nq):
    X = rng.standard_normal((n, d)).astype(np.float32)
    # exact duplicates, some of them placed before their original
    X[5] = X[40]
    X[41] = X[40]
    X[77] = X[3]
    Q = rng.standard_normal((nq, d)).astype(np.float32)
    Q[0] = X[40]          # distance 0 to three rows: order 5, 40, 41
    Q[1] = X[3] * 0.5     # equidistant from the duplicates 3 and 77
    return X, Q


def test_knn_f32_matches_cdist_with_ties(orc):
    rng = np.random.default_rng(101)
    X, Q = _with_duplicates(rng, 120, 7, 9)
    k = 12
    oid, od = orc.knn_f32(X, Q, k)
    D = cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    # cdist's squared Euclidean may round differently in the last place;
    # recompute exactly in FP64 by direct differences for the ordering
    diff = Q.astype(np.float64)[:, None, :] - X.astype(np.float64)[None, :, :]
    E = (diff * diff).sum(-1)
    np.testing.assert_allclose(D, E, rtol=1e-12, atol=1e-12)
    ref = _lexi_topk(E, k)
    np.testing.assert_array_equal(oid, ref)
    np.testing.assert_allclose(od, np.take_along_axis(E, ref, 1), rtol=1e-12, atol=0)
    # the tie protocol: duplicates come in id order
    assert list(oid[0, :3]) == [5, 40, 41] and np.all(od[0, :3] == 0.0)
    i3, i77 = list(oid[1]).index(3), list(oid[1]).index(77)
    assert i77 == i3 + 1 and od[1, i3] == od[1, i77]


def test_knn_f32_pads_when_k_exceeds_n(orc):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, 3)).astype(np.float32)
    Q = rng.standard_normal((2, 3)).astype(np.float32)
    oid, od = orc.knn_f32(X, Q, 6)
    diff = Q.astype(np.float64)[:, None, :] - X.astype(np.float64)[None, :, :]
    E = (diff * diff).sum(-1)
    ref = _lexi_topk(E, 6)
    np.testing.assert_array_equal(oid[:, :4], ref[:, :4])
    assert np.all(oid[:, 4:] == -1) and np.all(np.isinf(od[:, 4:]))


def test_knn_codes_matches_integer_brute_force(orc):
    rng = np.random.default_rng(77)
    n, d, stride, nq, k = 150, 21, 32, 8, 15
    codes = np.zeros((n, stride), np.uint8)
    codes[:, :d] = rng.integers(0, 256, (n, d))
    codes[:, d:] = rng.integers(0, 256, (n, stride - d))  # padding must be ignored
    codes[9, :d] = codes[100, :d]
    codes[120, :d] = codes[100, :d]
    qc = np.zeros((nq, stride), np.uint8)
    qc[:, :d] = rng.integers(0, 256, (nq, d))
    qc[0, :d] = codes[100, :d]
    qc[:, d:] = 255
    oid, oD = orc.knn_codes(codes, d, qc, k)
    diff = qc[:, None, :d].astype(np.int64) - codes[None, :, :d].astype(np.int64)
    E = (diff * diff).sum(-1)
    ref = _lexi_topk(E, k)
    np.testing.assert_array_equal(oid.astype(np.int64), ref)
    np.testing.assert_array_equal(oD.astype(np.int64), np.take_along_axis(E, ref, 1))
    assert list(oid[0, :3]) == [9, 100, 120] and np.all(oD[0, :3] == 0)


def test_knn_codes_pads_when_k_exceeds_n(orc):
    codes = np.array([[3, 0], [1, 0], [3, 0]], np.uint8)
    qc = np.array([[2, 0]], np.uint8)
    oid, oD = orc.knn_codes(codes, 1, qc, 5)
    # distances 1, 1, 1: all tied, id order; then two padded entries
    assert list(oid[0]) == [0, 1, 2, NONE, NONE]
    assert list(oD[0]) == [1, 1, 1, NONE, NONE]


def test_knn_codes_largest_distance_fits(orc):
    # d * 255^2 for a wide row stays exact in the oracle's integer path
    d = 960
    codes = np.zeros((2, d), np.uint8)
    codes[1] = 255
    qc = np.full((1, d), 255, np.uint8)
    oid, oD = orc.knn_codes(codes, d, qc, 2)
    assert list(oid[0]) == [1, 0]
    assert int(oD[0, 1]) == d * 255 * 255
