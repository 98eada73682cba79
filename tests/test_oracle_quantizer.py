"""Pins of the oracle's quantiser (Section 3.1, Alg. 1 stages 1-2).

Each test checks the oracle against something other than itself: a library
routine (numpy.percentile, scipy distances), a closed form, or a special case
whose answer is known by construction.
"""
import itertools

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from paper_2602_21600_amd import workloads as W


def _hypercube(dim, scale=1.0, offset=0.0):
    v = np.array(list(itertools.product([0.0, 1.0], repeat=dim)))
    return (v * scale + offset).astype(np.float32)


def test_density_matches_bruteforce(orc):
    X, _ = W.tiny(300, 12, seed=3)
    rho = orc.density(X, k_rho=10, eps=1e-6)
    D = cdist(X.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    np.fill_diagonal(D, np.inf)
    dk = np.sort(D, axis=1)[:, :10].mean(axis=1)
    np.testing.assert_allclose(rho, 1.0 / (dk + 1e-6), rtol=1e-12)


def test_density_hypercube_closed_form(orc):
    # Vertices of {0,1}^6: every vertex has 6 neighbours at squared distance 1
    # and 15 at 2, so the 10 nearest average (6*1 + 4*2)/10 = 1.4 exactly.
    X = _hypercube(6)
    rho = orc.density(X, k_rho=10, eps=1e-6)
    assert np.all(rho == 1.0 / (1.4 + 1e-6))
    assert orc.delta(rho) == 0.0


def test_density_two_scales_closed_form(orc):
    # Two far-apart hypercubes with edge 1 and edge 2: the 10 nearest stay in
    # the own cube, so mean squared distance is 1.4 and 1.4*4 = 5.6.
    A = _hypercube(6, 1.0, 0.0)
    B = _hypercube(6, 2.0, 100.0)
    X = np.vstack([A, B])
    rho = orc.density(X, k_rho=10, eps=1e-6)
    r1, r2 = 1.0 / (1.4 + 1e-6), 1.0 / (5.6 + 1e-6)
    np.testing.assert_allclose(rho[:64], r1, rtol=1e-15)
    np.testing.assert_allclose(rho[64:], r2, rtol=1e-15)
    np.testing.assert_allclose(orc.delta(rho), (r1 - r2) / (r1 + 1e-6), rtol=1e-14)


def test_density_sampling_stride_and_mean(orc):
    # n > threshold: only points floor(s*n/n_s) are measured, the others get
    # the sample mean (Section 3.1, "efficient computation").
    X, _ = W.tiny(200, 8, seed=5)
    rho = orc.density(X, k_rho=10, eps=1e-6, n_s=20, threshold=50)
    full = orc.density(X, k_rho=10, eps=1e-6)
    S = np.array([(s * 200) // 20 for s in range(20)])
    np.testing.assert_array_equal(rho[S], full[S])
    rest = np.setdiff1d(np.arange(200), S)
    assert np.all(rho[rest] == rho[rest][0])
    np.testing.assert_allclose(rho[rest][0], full[S].mean(), rtol=1e-14)


def test_density_small_n_uses_all_other_points(orc):
    X = np.array([[0.0], [1.0], [3.0]], np.float32)
    rho = orc.density(X, k_rho=10, eps=1e-6)
    # only n-1 = 2 neighbours exist
    np.testing.assert_allclose(rho, 1.0 / (np.array([5.0, 2.5, 6.5]) + 1e-6), rtol=1e-15)


@pytest.mark.parametrize("p", [0.0, 0.01, 0.0137, 0.25, 0.5, 0.77, 0.99, 1.0])
def test_percentile_matches_numpy(orc, p):
    rng = np.random.default_rng(11)
    v = np.sort(rng.standard_normal(1001))
    got = orc.percentile_sorted(v, p)
    np.testing.assert_allclose(got, np.percentile(v, 100.0 * p, method="linear"), rtol=1e-14,
                               atol=1e-15)


def test_ranges_match_numpy_percentiles(orc):
    X = W.base("small", 2000)
    tr = orc.train(X, p_max=0.01, M0=16, efc0=100)
    d = X.shape[1]
    for j in range(d):
        lo = np.percentile(X[:, j].astype(np.float64), 100.0 * tr["p_lo"], method="linear")
        hi = np.percentile(X[:, j].astype(np.float64), 100.0 * tr["p_hi"], method="linear")
        # equal after rounding to FP32, up to one FP32 ulp for a last-bit
        # difference in the interpolation formula
        assert abs(float(tr["min"][j]) - np.float32(lo)) <= abs(np.spacing(np.float32(lo)))
        assert abs(float(tr["max"][j]) - np.float32(hi)) <= abs(np.spacing(np.float32(hi)))
    assert tr["p_lo"] == tr["delta"] * 0.01
    assert tr["p_hi"] == 1.0 - tr["delta"] * 0.01


def test_scalars_closed_forms(orc):
    X = W.base("small", 3000)
    tr = orc.train(X, p_max=0.01, M0=16, efc0=100)
    assert 0.0 <= tr["delta"] < 1.0
    # the printed weights have no j, so they are all equal: eta = 0 and Eq. 1
    # reduces to the RMS range over 255
    assert tr["eta"] == 0.0
    rng_ = tr["max"].astype(np.float64) - tr["min"].astype(np.float64)
    np.testing.assert_allclose(tr["s_dist"], np.sqrt(np.mean(rng_ ** 2)) / 255.0, rtol=1e-13)
    assert tr["M"] == int(np.floor(16 * (1.0 + tr["delta"])))
    assert tr["efc"] == 100
    # scale = 255 / (range + 1e-6), each operation in FP32
    sc = np.float32(255.0) / ((tr["max"] - tr["min"]) + np.float32(1e-6))
    np.testing.assert_array_equal(tr["scale"], sc.astype(np.float32))


@pytest.mark.parametrize("M0,efc0,delta,eta,M,efc", [
    (16, 200, 0.0, 0.0, 16, 200),
    (16, 200, 0.5, 0.0, 24, 200),
    (16, 200, 0.5, 1.0, 32, 133),
    (32, 200, 0.9971, 0.0, 63, 200),
    (24, 100, 1.0 / 3.0, 0.5, 36, 85),
])
def test_build_params_hand_values(orc, M0, efc0, delta, eta, M, efc):
    # M_i = floor(M0 (1 + delta (1 + eta))), ef_c = floor(ef0 / (1 + delta eta))
    assert orc.build_params(M0, efc0, delta, eta) == (M, efc)


def test_equal_density_reduces_to_minmax(orc):
    # delta = 0 (every point has the same density): the percentile bounds
    # are 0 and 1, i.e. the plain min/max 8-bit quantiser.
    X = _hypercube(7, 1.0) * np.linspace(1.0, 2.0, 7, dtype=np.float32) - 0.5
    X = X.astype(np.float32)
    rho = orc.density(X)
    tr = orc.train(X, p_max=0.01, rho=rho)
    assert tr["delta"] == 0.0
    np.testing.assert_array_equal(tr["min"], X.min(axis=0))
    np.testing.assert_array_equal(tr["max"], X.max(axis=0))
    codes = orc.encode(X, tr["min"], tr["scale"])
    # column extremes map to 0 and 255
    assert np.all(codes.min(axis=0) == 0) and np.all(codes.max(axis=0) == 255)


def test_encode_round_trip_bound(orc):
    X = W.base("small", 4000)
    tr = orc.train(X, p_max=0.01)
    codes = orc.encode(X, tr["min"], tr["scale"], stride=128)
    assert codes.dtype == np.uint8
    xt = orc.decode(codes, 128, tr["min"], tr["scale"]).astype(np.float64)
    clip = np.clip(X.astype(np.float64), tr["min"].astype(np.float64),
                   tr["max"].astype(np.float64))
    # rounding to the nearest code loses at most half a step 1/scale; the
    # 1e-6 in the scale and FP32 rounding add a few ulps
    mag = np.maximum(np.abs(clip), np.abs(tr["max"]).astype(np.float64))
    bound = 0.5 / tr["scale"].astype(np.float64) + 1e-6 + 8 * np.abs(np.spacing(mag.astype(np.float32)))
    assert np.all(np.abs(xt - clip) <= bound)
    # values outside the range saturate
    below = X < tr["min"]
    above = X > tr["max"]
    assert np.all(codes[:, :128][below] == 0)
    assert np.all(codes[:, :128][above] == 255)


def test_encode_rounds_half_to_even(orc):
    # min 0, scale 1: the code is rint(x) with ties to even, then clipped
    X = np.array([[0.5, 1.5, 2.5, 254.5, -3.0, 300.0, 7.49999, 7.5]], np.float32)
    mn = np.zeros(8, np.float32)
    sc = np.ones(8, np.float32)
    codes = orc.encode(X, mn, sc)
    np.testing.assert_array_equal(codes[0], [0, 2, 2, 254, 0, 255, 7, 8])


def test_encode_rejects_non_finite(orc):
    X = np.array([[0.0, np.nan]], np.float32)
    with pytest.raises(ValueError):
        orc.encode(X, np.zeros(2, np.float32), np.ones(2, np.float32))


def test_encode_pads_stride_with_zeros(orc):
    X = np.ones((3, 5), np.float32)
    codes = orc.encode(X, np.zeros(5, np.float32), np.full(5, 10.0, np.float32), stride=16)
    assert codes.shape == (3, 16)
    assert np.all(codes[:, :5] == 10) and np.all(codes[:, 5:] == 0)


# ---- per-dimension density weights (the per-dimension reading of w_j) ----

def _spaced_columns(n, steps, seed):
    """Column j holds 0, a_j, 2 a_j, ... (exact in FP32), rows shuffled."""
    rng = np.random.default_rng(seed)
    X = np.stack([np.arange(n, dtype=np.float64) * a for a in steps], 1).astype(np.float32)
    return X[rng.permutation(n)]


@pytest.mark.parametrize("k", [2, 4])
def test_dim_weights_evenly_spaced_closed_form(orc, k):
    # on an evenly spaced column with step a, an inner point's k nearest
    # squared differences are a^2 {1,1,4,4,...}; the two points at each end
    # have one-sided neighbourhoods
    n, eps = 400, 1e-6
    steps = [0.5, 1.0, 2.0, 4.0]
    X = _spaced_columns(n, steps, seed=k)
    w = orc.dim_weights(X, k_rho=k, eps=eps)
    for j, a in enumerate(steps):
        a2 = a * a
        if k == 2:
            inner = 1.0 / (a2 + eps)
            ends = 2 * [1.0 / (2.5 * a2 + eps)]
            n_inner = n - 2
        else:
            inner = 1.0 / (2.5 * a2 + eps)
            ends = 2 * [1.0 / (3.75 * a2 + eps), 1.0 / (7.5 * a2 + eps)]
            n_inner = n - 4
        want = (n_inner * inner + sum(ends)) / n
        np.testing.assert_allclose(w[j], want, rtol=1e-12)
    # the weights differ across dimensions, so eta > 0 and follows from them
    tr = orc.train(X, M0=16, efc0=200, k_rho=k, weights=1)
    np.testing.assert_array_equal(tr["w"], w)
    np.testing.assert_allclose(tr["eta"], np.std(w) / np.mean(w), rtol=1e-12)
    rng_ = tr["max"].astype(np.float64) - tr["min"].astype(np.float64)
    np.testing.assert_allclose(tr["s_dist"], np.sqrt(np.sum(rng_ ** 2 * w) / np.sum(255.0 ** 2 * w)),
                               rtol=1e-12)
    assert tr["M"] == int(np.floor(16 * (1.0 + tr["delta"] * (1.0 + tr["eta"]))))
    assert tr["efc"] == int(np.floor(200 / (1.0 + tr["delta"] * tr["eta"])))


def test_dim_weights_match_bruteforce_with_sampling_and_ties(orc):
    rng = np.random.default_rng(5)
    n, d, k, eps = 90, 3, 5, 1e-6
    X = rng.standard_normal((n, d)).astype(np.float32)
    X[10:20, 1] = X[3, 1]  # ties at difference 0 in one column
    for n_s, threshold in ((90, 1000), (25, 40)):
        m = min(n_s, n)
        S = [(s * n) // m for s in range(m)] if n > threshold else list(range(n))
        want = []
        for j in range(d):
            col = X[:, j].astype(np.float64)
            dens = []
            for i in S:
                diff = np.delete((col[i] - col) ** 2, i)
                dens.append(1.0 / (np.sort(diff)[:k].mean() + eps))
            want.append(np.mean(dens))
        got = orc.dim_weights(X, k_rho=k, eps=eps, n_s=n_s, threshold=threshold)
        np.testing.assert_allclose(got, want, rtol=1e-12)


def test_dim_weights_equal_columns_give_zero_eta(orc):
    # identical columns have identical weights: eta = 0 exactly, and the
    # per-dimension reading then leaves M_i and ef^c as the literal one does
    rng = np.random.default_rng(2)
    c = rng.standard_normal(500).astype(np.float32)
    X = np.stack([c, c, c, c], 1)
    tr1 = orc.train(X, M0=16, efc0=200, weights=1)
    tr0 = orc.train(X, M0=16, efc0=200)
    assert tr1["eta"] == 0.0
    assert (tr1["M"], tr1["efc"]) == (tr0["M"], tr0["efc"])
