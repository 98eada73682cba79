"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

The paper evaluates on public datasets (Table 1) that are not available
here.  These generators stand in for their shapes with Gaussian mixtures:

  small    10,000 x 128, L2, 32 isotropic clusters, equal weights, per-cluster
           std log-uniform [0.05, 1.0]; 100 queries; M=16, efC=100; k=10, ef=64
  sift1m   1,000,000 x 128 (SIFT-1M shape), 256 isotropic clusters, sizes
           Zipf(1.1), std log-uniform [0.02, 1.0], values clipped to >= 0;
           10,000 queries; M=16, efC=200; k=10, ef 32..256
  gist1m   1,000,000 x 960 (GIST-1M shape), 128 anisotropic clusters,
           per-dimension std log-uniform [0.01, 1.0]; 1,000 queries; M=32,
           efC=200; k=10, ef 64..512
  batched  1,200,000 x 100, cosine (unit vectors), 512 clusters with Pareto
           (alpha=1.5) sizes, std log-uniform [0.05, 1.0]; 100,000 queries with
           per-query ef in {16,...,512} and k in {1,10,100}; M=24, efC=200
  serving  10,000,000 x 96, L2, 1,024 clusters with log-uniform weights in
           [1, 100], std log-uniform [0.05, 1.0]; M=16, efC=200; Poisson
           arrivals with k in {1,10,100} and ef log-uniform in [16, 512]
  fmnist   60,000 x 784 (Fashion-MNIST shape), L2, 10 clusters (one per
           class) with equal weights; each cluster varies along 16 random
           directions of its own (scale log-uniform [0.3, 1.0]) plus noise of
           std 0.02, so pixels are correlated as in images; values clipped to
           >= 0 (zero background); 10,000 queries; M=16, efC=200; k=10, ef 16..256

Cluster centres are N(0, I_d).  Samples are drawn in FP64 from NumPy's PCG64
generator and stored as FP32.  Seeds: base 1000*c+1, queries 1000*c+2,
level draws 1000*c+3, per-query parameters 1000*c+4 (c = workload number).
Every generator accepts a smaller n / nq for parity-test subsets; the first
rows do not depend on n (rows are drawn in fixed-size blocks).
"""
from dataclasses import dataclass, field

import numpy as np

_BLOCK = 65536


@dataclass(frozen=True)
class Workload:
    name: str
    number: int
    n: int
    d: int
    nq: int
    n_clusters: int
    sizes: str            # "equal" | "zipf" | "pareto" | "loguniform"
    size_param: float
    std_lo: float
    std_hi: float
    anisotropic: bool
    clip_nonneg: bool
    cosine: bool
    M0: int
    efc0: int
    k: tuple = (10,)
    ef: tuple = (64,)
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "small": Workload("small", 1, 10_000, 128, 100, 32, "equal", 0.0, 0.05, 1.0, False, False,
                      False, 16, 100, (10,), (64,)),
    "sift1m": Workload("sift1m", 2, 1_000_000, 128, 10_000, 256, "zipf", 1.1, 0.02, 1.0, False,
                       True, False, 16, 200, (10,), (32, 48, 64, 96, 128, 192, 256)),
    "gist1m": Workload("gist1m", 3, 1_000_000, 960, 1_000, 128, "equal", 0.0, 0.01, 1.0, True,
                       False, False, 32, 200, (10,), (64, 96, 128, 192, 256, 384, 512)),
    "batched": Workload("batched", 4, 1_200_000, 100, 100_000, 512, "pareto", 1.5, 0.05, 1.0,
                        False, False, True, 24, 200, (1, 10, 100), (16, 32, 64, 128, 256, 512)),
    "serving": Workload("serving", 5, 10_000_000, 96, 100_000, 1024, "loguniform", 100.0, 0.05,
                        1.0, False, False, False, 16, 200, (1, 10, 100), (16, 512)),
    "fmnist": Workload("fmnist", 6, 60_000, 784, 10_000, 10, "equal", 0.0, 0.3, 1.0, False, True,
                       False, 16, 200, (10,), (16, 24, 32, 48, 64, 96, 128, 192, 256),
                       extra={"latent": 16, "noise": 0.02}),
}


def _mixture(w: Workload, rng: np.random.Generator):
    """Cluster centres, per-cluster std (scalar or per dimension) and weights."""
    c = w.n_clusters
    centres = rng.standard_normal((c, w.d))
    lo, hi = np.log(w.std_lo), np.log(w.std_hi)
    if w.anisotropic:
        std = np.exp(rng.uniform(lo, hi, size=(c, w.d)))
    else:
        std = np.exp(rng.uniform(lo, hi, size=(c, 1)))
    if w.sizes == "equal":
        weights = np.full(c, 1.0 / c)
    elif w.sizes == "zipf":
        rank = rng.permutation(c) + 1
        weights = rank.astype(np.float64) ** (-w.size_param)
    elif w.sizes == "pareto":
        u = 1.0 - rng.random(c)
        weights = u ** (-1.0 / w.size_param)
    elif w.sizes == "loguniform":
        weights = np.exp(rng.uniform(0.0, np.log(w.size_param), size=c))
    else:
        raise ValueError(w.sizes)
    weights = weights / weights.sum()
    basis = None
    r = w.extra.get("latent", 0)
    if r:
        # low-rank clusters: each has its own random basis of r directions
        basis = rng.standard_normal((c, w.d, r)) / np.sqrt(r)
    return centres, std, weights, basis


def _draw(w: Workload, seed: int, count: int) -> np.ndarray:
    mix_rng = np.random.default_rng(1000 * w.number)
    centres, std, weights, basis = _mixture(w, mix_rng)
    rng = np.random.default_rng(seed)
    out = np.empty((count, w.d), np.float32)
    for s in range(0, count, _BLOCK):
        e = min(count, s + _BLOCK)
        labels = rng.choice(w.n_clusters, size=_BLOCK, p=weights)[: e - s]
        if basis is None:
            z = rng.standard_normal((_BLOCK, w.d))[: e - s]
            x = centres[labels] + std[labels] * z
        else:
            # centre + std * (basis @ latent) + small independent noise
            u = rng.standard_normal((_BLOCK, basis.shape[2]))[: e - s]
            z = rng.standard_normal((_BLOCK, w.d))[: e - s]
            x = centres[labels] + w.extra["noise"] * z
            for c in np.unique(labels):
                m = labels == c
                x[m] += std[c] * (u[m] @ basis[c].T)
        if w.clip_nonneg:
            np.maximum(x, 0.0, out=x)
        if w.cosine:
            nrm = np.sqrt((x * x).sum(axis=1, keepdims=True))
            x = x / np.maximum(nrm, 1e-300)
        out[s:e] = x
    return out


def base(name: str, n: int = None) -> np.ndarray:
    w = WORKLOADS[name]
    return _draw(w, 1000 * w.number + 1, w.n if n is None else int(n))


def queries(name: str, nq: int = None) -> np.ndarray:
    w = WORKLOADS[name]
    return _draw(w, 1000 * w.number + 2, w.nq if nq is None else int(nq))


def level_draws(name: str, n: int = None) -> np.ndarray:
    """Uniform draws u in (0, 1], one per base point, for the HNSW levels."""
    w = WORKLOADS[name]
    rng = np.random.default_rng(1000 * w.number + 3)
    return 1.0 - rng.random(w.n if n is None else int(n))


def query_params(name: str, nq: int = None):
    """Per-query (k, ef).  Fixed-k workloads use their first k and ef."""
    w = WORKLOADS[name]
    nq = w.nq if nq is None else int(nq)
    rng = np.random.default_rng(1000 * w.number + 4)
    if name == "batched":
        k = rng.choice(np.array(w.k, np.int32), size=nq)
        ef = rng.choice(np.array(w.ef, np.int32), size=nq)
    elif name == "serving":
        k = rng.choice(np.array(w.k, np.int32), size=nq)
        ef = np.exp(rng.uniform(np.log(w.ef[0]), np.log(w.ef[1]), size=nq)).astype(np.int32)
    else:
        k = np.full(nq, w.k[0], np.int32)
        ef = np.full(nq, w.ef[0], np.int32)
    return k.astype(np.int32), ef.astype(np.int32)


def poisson_arrivals(rate_qps: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_qps, size=count))


def tiny(n: int, d: int, seed: int, clusters: int = 4, nq: int = 8):
    """Small mixtures for unit tests: (base, queries)."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((clusters, d))
    std = np.exp(rng.uniform(np.log(0.05), 0.0, size=(clusters, 1)))
    lab = rng.integers(0, clusters, size=n + nq)
    x = centres[lab] + std[lab] * rng.standard_normal((n + nq, d))
    x = x.astype(np.float32)
    return x[:n].copy(), x[n:].copy()
