"""The quantiser's density search on the device (Section 3.1, Stage 1).

Every distance is summed in the same FP64 order as the oracle's and the k
smallest are summed in ascending order, so the device densities must equal
the oracle's bit for bit, and the quantiser trained with them must equal the
oracle's (and the host library's) exactly: scalars, ranges, scales and codes.
Cases cover sampled and unsampled densities, dimensions that are and are not
multiples of 4 (the two row-load paths), partitions with a ragged last batch
of rows, a partial last tile of samples, k from 1 to 64, exact duplicate
rows (ties at distance 0 that must still exclude only the point itself), and
the degenerate sizes n = 1, 2 and n - 1 < k_rho.
"""
import numpy as np
import pytest

from paper_2602_21600_amd import workloads as W

pytestmark = pytest.mark.gpu


def _aqr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    from paper_2602_21600_amd import aqr
    return aqr


def _params(aqr, k_rho=10, n_sample=5000, threshold=10000, **kw):
    p = aqr.default_qparams(**kw)
    p.update(k_rho=k_rho, n_sample=n_sample, sample_threshold=threshold)
    return p


@pytest.mark.parametrize("n,d,k_rho,n_sample,threshold", [
    (3000, 20, 10, 500, 1000),    # sampled, d % 4 == 0, 12 partitions of 250 rows
    (1500, 37, 10, 5000, 10000),  # every point measured, scalar row loads, 47 tiles
    (2000, 16, 1, 300, 1000),     # k = 1
    (2000, 24, 64, 100, 1000),    # k = 64: a list element in every lane
    (700, 9, 5, 5000, 10000),
])
def test_density_matches_oracle(orc, n, d, k_rho, n_sample, threshold):
    aqr = _aqr()
    X, _ = W.tiny(n, d, seed=n + d + k_rho, clusters=5)
    ref = orc.density(X, k_rho=k_rho, n_s=n_sample, threshold=threshold)
    got = aqr.aqr_density(X, _params(aqr, k_rho, n_sample, threshold), device=True)
    np.testing.assert_array_equal(got, ref)


def test_density_with_duplicate_rows(orc):
    aqr = _aqr()
    X, _ = W.tiny(600, 12, seed=3, clusters=4)
    X[300:330] = X[0]          # 31 copies of row 0: its 10 nearest are at distance 0
    X[400:402] = X[401]
    ref = orc.density(X, k_rho=10)
    got = aqr.aqr_density(X, _params(aqr), device=True)
    np.testing.assert_array_equal(got, ref)
    assert got[0] == 1.0 / 1e-6


@pytest.mark.parametrize("n,d,k_rho", [(1, 8, 10), (2, 3, 10), (5, 4, 10), (64, 7, 63),
                                       (65, 8, 64)])
def test_density_degenerate_sizes(orc, n, d, k_rho):
    aqr = _aqr()
    X = np.random.default_rng(n).standard_normal((n, d)).astype(np.float32)
    ref = orc.density(X, k_rho=k_rho)
    got = aqr.aqr_density(X, _params(aqr, k_rho), device=True)
    np.testing.assert_array_equal(got, ref)


def test_density_rejects_k_above_64():
    aqr = _aqr()
    X = np.zeros((100, 4), np.float32)
    with pytest.raises(aqr.AqrError):
        aqr.aqr_density(X, _params(aqr, 65), device=True)


@pytest.mark.parametrize("name,n", [("sift1m", 20000), ("fmnist", 3000), ("gist1m", 12000)])
def test_quantize_device_matches_oracle(orc, name, n):
    aqr = _aqr()
    X = W.base(name, n)
    params = aqr.default_qparams(M0=16, efc0=200)
    qz, codes = aqr.aqr_quantize(X, params, device=True)
    info = aqr.aqr_quantizer_info(qz)
    ref = orc.train(X, M0=16, efc0=200, n_s=params["n_sample"],
                    threshold=params["sample_threshold"])
    for f in ("delta", "p_lo", "p_hi", "s_dist", "eta", "w_mean", "M", "efc"):
        assert info[f] == ref[f], f
    np.testing.assert_array_equal(info["min"], ref["min"])
    np.testing.assert_array_equal(info["max"], ref["max"])
    np.testing.assert_array_equal(info["scale"], ref["scale"])
    d_pad = info["d_pad"]
    np.testing.assert_array_equal(codes, orc.encode(X, ref["min"], ref["scale"], stride=d_pad))


def test_quantize_device_equals_host_library_at_200k():
    # 200,000 x 128 with 5,000 samples: 157 tiles of samples, each over many row
    # partitions of several thousand rows
    aqr = _aqr()
    X = W.base("sift1m", 200_000)
    p = aqr.default_qparams(M0=16, efc0=200)
    qd, cd = aqr.aqr_quantize(X, p, device=True)
    qh, ch = aqr.aqr_quantize(X, p)
    a, b = aqr.aqr_quantizer_info(qd), aqr.aqr_quantizer_info(qh)
    for f in ("delta", "p_lo", "p_hi", "s_dist", "eta", "w_mean", "M", "efc"):
        assert a[f] == b[f], f
    for f in ("min", "max", "scale"):
        np.testing.assert_array_equal(a[f], b[f])
    np.testing.assert_array_equal(cd, ch)
