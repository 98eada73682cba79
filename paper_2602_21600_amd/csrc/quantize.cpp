// quantize.cpp -- host quantiser of libaqr (Section 3.1, Alg. 1 stages 1-2).
//
// Density: rho_i = 1 / (mean of the k_rho smallest squared L2 distances from
// x_i to the other points + eps), FP64; with n above the sampling threshold
// only the points floor(s*n/n_s), s < n_s, are measured and the others get
// the sample mean.  Each distance is summed dimension by dimension in order,
// in FP64; a tile of sample points is scored against one base row at a time
// so that the base set streams through the cache once per tile.
//
// Ranges: P_l = delta*P_max and P_h = 1 - delta*P_max; min_j / max_j are the
// linear-interpolation percentiles of column j (order statistics at
// h = p*(n-1), interpolated in FP64, rounded to FP32); scale_j =
// 255 / ((max_j - min_j) + eps) in FP32.  The density weights w_j are the
// mean density for every j (the printed formula), or with weights = 1 the
// mean one-dimensional density along j; Eq. 1 gives s_dist,
// eta = sigma_w / mean_w.
// Build parameters M_i = floor(M_0 (1 + delta (1 + eta))) and
// ef^c = floor(ef_0 / (1 + delta eta)).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>

#include "internal.hpp"

namespace aqr {

namespace {

constexpr int kTile = 8;  // sample points scored together against one base row

// Keep the k smallest values of a stream, ascending.
struct TopK {
    int k = 0, cnt = 0;
    double v[64];
    void push(double x) {
        if (cnt < k) {
            int p = cnt++;
            while (p > 0 && v[p - 1] > x) {
                v[p] = v[p - 1];
                --p;
            }
            v[p] = x;
        } else if (x < v[k - 1]) {
            int p = k - 1;
            while (p > 0 && v[p - 1] > x) {
                v[p] = v[p - 1];
                --p;
            }
            v[p] = x;
        }
    }
};

aqr_status densities(const float* X, int64_t n, int32_t d, const aqr_qparams& p, int T,
                     bool device, std::vector<double>& rho) {
    const int64_t ns = std::min<int64_t>(p.n_sample, n);
    const bool sampled = n > p.sample_threshold;
    const int64_t m = sampled ? ns : n;
    const int k = (int)std::min<int64_t>(p.k_rho, n - 1);
    if (p.k_rho > 64) return fail(AQR_ERR_INVALID_ARG, "aqr_quantize: k_rho must be <= 64");
    std::vector<int64_t> S(m);
    for (int64_t s = 0; s < m; ++s) S[s] = sampled ? (s * n) / ns : s;
    rho.assign(n, 0.0);
    if (device && k > 0) {
        std::vector<double> sums(m);
        aqr_status st = device_density_sums(X, n, d, S.data(), m, k, T, sums.data());
        if (st != AQR_OK) return st;
        for (int64_t s = 0; s < m; ++s) rho[S[s]] = 1.0 / (sums[s] / (double)k + p.eps);
    }
    const int64_t ntiles = device && k > 0 ? 0 : (m + kTile - 1) / kTile;
    std::atomic<int64_t> next{0};
    parallel_for_threads(T, [&](int) {
        std::vector<double> tileT((size_t)d * kTile);  // [dim][t]
        TopK top[kTile];
        for (;;) {
            int64_t tile = next.fetch_add(1);
            if (tile >= ntiles) break;
            int64_t s0 = tile * kTile;
            int tn = (int)std::min<int64_t>(kTile, m - s0);
            for (int t = 0; t < kTile; ++t) {
                top[t].k = k;
                top[t].cnt = 0;
                int64_t i = S[s0 + std::min(t, tn - 1)];
                for (int32_t j = 0; j < d; ++j) tileT[(size_t)j * kTile + t] = X[i * d + j];
            }
            for (int64_t r = 0; r < n; ++r) {
                const float* xr = X + r * d;
                double acc[kTile];
                for (int t = 0; t < kTile; ++t) acc[t] = 0.0;
                for (int32_t j = 0; j < d; ++j) {
                    const double xv = (double)xr[j];
                    const double* a = &tileT[(size_t)j * kTile];
                    for (int t = 0; t < kTile; ++t) {
                        double df = a[t] - xv;
                        acc[t] += df * df;
                    }
                }
                for (int t = 0; t < tn; ++t)
                    if (S[s0 + t] != r) top[t].push(acc[t]);
            }
            for (int t = 0; t < tn; ++t) {
                double mean = 0.0;
                if (k > 0) {
                    double sum = 0.0;
                    for (int u = 0; u < k; ++u) sum += top[t].v[u];
                    mean = sum / (double)k;
                }
                rho[S[s0 + t]] = 1.0 / (mean + p.eps);
            }
        }
    });
    if (sampled) {
        double sum = 0.0;
        for (int64_t s = 0; s < m; ++s) sum += rho[S[s]];
        const double mean = sum / (double)m;
        std::vector<char> in(n, 0);
        for (int64_t s = 0; s < m; ++s) in[S[s]] = 1;
        for (int64_t i = 0; i < n; ++i)
            if (!in[i]) rho[i] = mean;
    }
    return AQR_OK;
}

// Per-dimension weights (aqr_qparams.weights = 1): w_j = mean over the
// measured points of 1 / (mean of the k smallest squared differences to the
// other values of column j + eps).  Each column is sorted once; a point's k
// nearest values are then the nearer of the two sides, taken outward from
// one copy of its own value, so they arrive in ascending order and are
// summed in that order.
aqr_status dim_weights(const float* X, int64_t n, int32_t d, const aqr_qparams& p, int T,
                       std::vector<double>& w) {
    const int64_t ns = std::min<int64_t>(p.n_sample, n);
    const bool sampled = n > p.sample_threshold;
    const int64_t m = sampled ? ns : n;
    const int k = (int)std::min<int64_t>(p.k_rho, n - 1);
    if (p.k_rho > 64) return fail(AQR_ERR_INVALID_ARG, "aqr_quantize: k_rho must be <= 64");
    w.assign(d, 0.0);
    const double inf = std::numeric_limits<double>::infinity();
    std::atomic<int32_t> next{0};
    parallel_for_threads(std::max(1, std::min<int>(T, d)), [&](int) {
        std::vector<double> col(n);
        for (;;) {
            const int32_t j = next.fetch_add(1);
            if (j >= d) break;
            for (int64_t i = 0; i < n; ++i) col[i] = (double)X[i * d + j];
            std::sort(col.begin(), col.end());
            double sum = 0.0;
            for (int64_t s = 0; s < m; ++s) {
                const int64_t i = sampled ? (s * n) / ns : s;
                const double v = (double)X[i * d + j];
                const int64_t at = std::lower_bound(col.begin(), col.end(), v) - col.begin();
                int64_t lo = at - 1, hi = at + 1;
                double acc = 0.0;
                for (int u = 0; u < k; ++u) {
                    const double tl = lo >= 0 ? v - col[lo] : 0.0;
                    const double th = hi < n ? col[hi] - v : 0.0;
                    const double dl = lo >= 0 ? tl * tl : inf;
                    const double dh = hi < n ? th * th : inf;
                    if (dl <= dh) {
                        acc += dl;
                        --lo;
                    } else {
                        acc += dh;
                        ++hi;
                    }
                }
                const double mean = k > 0 ? acc / (double)k : 0.0;
                sum += 1.0 / (mean + p.eps);
            }
            w[j] = sum / (double)m;
        }
    });
    return AQR_OK;
}

// Linear-interpolation percentile from the two order statistics around h,
// interpolated in FP64.  The column may hold the FP32 values themselves:
// widening to FP64 is exact and keeps the order, so the order statistics
// are the same.
template <class T>
double percentile_of(std::vector<T>& col, double p) {
    const int64_t n = (int64_t)col.size();
    if (n == 1) return (double)col[0];
    const double h = p * (double)(n - 1);
    if (h <= 0.0) return (double)*std::min_element(col.begin(), col.end());
    if (h >= (double)(n - 1)) return (double)*std::max_element(col.begin(), col.end());
    const int64_t lo = (int64_t)std::floor(h);
    std::nth_element(col.begin(), col.begin() + lo, col.end());
    const double a = (double)col[lo];
    const double b = (double)*std::min_element(col.begin() + lo + 1, col.end());
    return a + (h - (double)lo) * (b - a);
}

void encode_rows(const float* X, int64_t n, int32_t d, int32_t d_pad, const Quantizer& q,
                 uint8_t* codes, int T) {
    std::atomic<int64_t> next{0};
    const int64_t chunk = 4096;
    parallel_for_threads(T, [&](int) {
        for (;;) {
            int64_t s = next.fetch_add(chunk);
            if (s >= n) break;
            int64_t e = std::min(n, s + chunk);
            for (int64_t i = s; i < e; ++i) {
                uint8_t* c = codes + i * d_pad;
                for (int32_t j = 0; j < d; ++j) {
                    float t = X[i * d + j] - q.mn[j];
                    float u = t * q.scale[j];
                    float r = std::nearbyint(u);
                    r = r < 0.0f ? 0.0f : (r > 255.0f ? 255.0f : r);
                    c[j] = (uint8_t)r;
                }
                for (int32_t j = d; j < d_pad; ++j) c[j] = 0;
            }
        }
    });
}

bool all_finite(const float* X, int64_t count) {
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(X[i])) return false;
    return true;
}

aqr_status train(const float* X, int64_t n, int32_t d, const aqr_qparams& p, int T,
                 bool device, Quantizer& q) {
    std::vector<double> rho;
    aqr_status st = densities(X, n, d, p, T, device, rho);
    if (st != AQR_OK) return st;
    double rmax = rho[0], rmin = rho[0];
    for (int64_t i = 1; i < n; ++i) {
        rmax = std::max(rmax, rho[i]);
        rmin = std::min(rmin, rho[i]);
    }
    const double delta = (rmax - rmin) / (rmax + p.eps);
    const double p_lo = delta * p.p_max;
    const double p_hi = 1.0 - delta * p.p_max;
    q.mn.assign(d, 0.f);
    q.mx.assign(d, 0.f);
    q.scale.assign(d, 0.f);
    // columns are gathered a group at a time, so that one pass over the rows
    // reads each cache line of X once for the whole group
    constexpr int32_t G = 8;
    const int32_t ngroups = (d + G - 1) / G;
    std::atomic<int32_t> next{0};
    parallel_for_threads(std::max(1, std::min<int>(T, ngroups)), [&](int) {
        std::vector<float> cols((size_t)G * n), work(n);
        for (;;) {
            const int32_t gi = next.fetch_add(1);
            if (gi >= ngroups) break;
            const int32_t j0 = gi * G, gw = std::min(G, d - j0);
            for (int64_t i = 0; i < n; ++i) {
                const float* r = X + i * d + j0;
                for (int32_t c = 0; c < gw; ++c) cols[(size_t)c * n + i] = r[c];
            }
            for (int32_t c = 0; c < gw; ++c) {
                const float* col = &cols[(size_t)c * n];
                const int32_t j = j0 + c;
                work.assign(col, col + n);
                q.mn[j] = (float)percentile_of(work, p_lo);
                work.assign(col, col + n);
                q.mx[j] = (float)percentile_of(work, p_hi);
                float range = q.mx[j] - q.mn[j];
                float denom = range + (float)p.eps;
                q.scale[j] = 255.0f / denom;
            }
        }
    });
    // density weights: the mean density for every dimension, or per dimension
    std::vector<double> w;
    if (p.weights == 1) {
        st = dim_weights(X, n, d, p, T, w);
        if (st != AQR_OK) return st;
    } else {
        double rsum = 0.0;
        for (int64_t i = 0; i < n; ++i) rsum += rho[i];
        w.assign(d, rsum / (double)n);
    }
    double shift = 0.0;
    for (int32_t j = 0; j < d; ++j) shift += w[j] - w[0];
    const double wbar = w[0] + shift / (double)d;
    double var = 0.0;
    for (int32_t j = 0; j < d; ++j) var += (w[j] - wbar) * (w[j] - wbar);
    const double eta = std::sqrt(var / (double)d) / wbar;
    double num = 0.0, den = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        const double r = (double)q.mx[j] - (double)q.mn[j];
        num += r * r * w[j];
        den += 255.0 * 255.0 * w[j];
    }
    aqr_qinfo& I = q.info;
    I.d = d;
    I.d_pad = round_up(d, 16);
    I.delta = delta;
    I.p_lo = p_lo;
    I.p_hi = p_hi;
    I.s_dist = std::sqrt(num / den);
    I.eta = eta;
    I.w_mean = wbar;
    I.M = (int32_t)std::floor((double)p.M0 * (1.0 + delta * (1.0 + eta)));
    I.efc = (int32_t)std::floor((double)p.efc0 * (1.0 / (1.0 + delta * eta)));
    return AQR_OK;
}

}  // namespace

}  // namespace aqr

using namespace aqr;

namespace {

aqr_status quantize(const float* X, int64_t n, int32_t d, const aqr_qparams* p,
                    aqr_quantizer** qz, uint8_t* codes_out, bool device, const char* who) {
    const std::string w(who);
    try {
        clear_error();
        if (!X || !qz) return fail(AQR_ERR_INVALID_ARG, w + ": null pointer");
        if (n < 1 || d < 1) return fail(AQR_ERR_INVALID_ARG, w + ": n and d must be >= 1");
        if (!all_finite(X, n * (int64_t)d))
            return fail(AQR_ERR_INVALID_ARG, w + ": non-finite input value");
        aqr_quantizer* q = *qz;
        bool created = false;
        if (!q) {
            if (!p) return fail(AQR_ERR_INVALID_ARG, w + ": params required to train");
            if (p->k_rho < 1 || p->n_sample < 1 || !(p->eps > 0) || p->p_max < 0 ||
                p->p_max > 0.5 || p->M0 < 2 || p->efc0 < 1 || p->weights < 0 ||
                p->weights > 1)
                return fail(AQR_ERR_INVALID_ARG, w + ": parameter out of range");
            q = new aqr_quantizer();
            created = true;
            aqr_status st = train(X, n, d, *p, host_threads(p->threads), device, *q);
            if (st != AQR_OK) {
                delete q;
                return st;
            }
        } else if (q->info.d != d) {
            return fail(AQR_ERR_INVALID_ARG, w + ": d does not match the quantiser");
        }
        if (codes_out)
            encode_rows(X, n, d, q->info.d_pad, *q, codes_out, host_threads(p ? p->threads : 0));
        if (created) *qz = q;
        return AQR_OK;
    } catch (const std::bad_alloc&) {
        return fail(AQR_ERR_OOM, w + ": out of host memory");
    } catch (...) {
        return fail(AQR_ERR_STATE, w + ": unexpected failure");
    }
}

}  // namespace

extern "C" aqr_status aqr_quantize(const float* X, int64_t n, int32_t d, const aqr_qparams* p,
                                   aqr_quantizer** qz, uint8_t* codes_out) {
    return quantize(X, n, d, p, qz, codes_out, false, "aqr_quantize");
}

extern "C" aqr_status aqr_quantize_device(const float* X, int64_t n, int32_t d,
                                          const aqr_qparams* p, aqr_quantizer** qz,
                                          uint8_t* codes_out) {
    return quantize(X, n, d, p, qz, codes_out, true, "aqr_quantize_device");
}

extern "C" aqr_status aqr_density(const float* X, int64_t n, int32_t d, const aqr_qparams* p,
                                  int32_t device, double* rho) {
    try {
        clear_error();
        if (!X || !p || !rho) return fail(AQR_ERR_INVALID_ARG, "aqr_density: null pointer");
        if (n < 1 || d < 1) return fail(AQR_ERR_INVALID_ARG, "aqr_density: n and d must be >= 1");
        if (p->k_rho < 1 || p->n_sample < 1 || !(p->eps > 0))
            return fail(AQR_ERR_INVALID_ARG, "aqr_density: parameter out of range");
        if (!all_finite(X, n * (int64_t)d))
            return fail(AQR_ERR_INVALID_ARG, "aqr_density: non-finite input value");
        std::vector<double> r;
        aqr_status st = densities(X, n, d, *p, host_threads(p->threads), device != 0, r);
        if (st != AQR_OK) return st;
        std::memcpy(rho, r.data(), sizeof(double) * (size_t)n);
        return AQR_OK;
    } catch (const std::bad_alloc&) {
        return fail(AQR_ERR_OOM, "aqr_density: out of host memory");
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_density: unexpected failure");
    }
}

extern "C" aqr_status aqr_quantizer_info(const aqr_quantizer* qz, aqr_qinfo* info, float* mn,
                                         float* mx, float* scale) {
    clear_error();
    if (!qz) return fail(AQR_ERR_INVALID_ARG, "aqr_quantizer_info: null quantiser");
    if (info) *info = qz->info;
    const size_t b = sizeof(float) * (size_t)qz->info.d;
    if (mn) std::memcpy(mn, qz->mn.data(), b);
    if (mx) std::memcpy(mx, qz->mx.data(), b);
    if (scale) std::memcpy(scale, qz->scale.data(), b);
    return AQR_OK;
}

extern "C" aqr_status aqr_quantizer_create(const aqr_qinfo* info, const float* mn,
                                           const float* mx, const float* scale,
                                           aqr_quantizer** out) {
    try {
        clear_error();
        if (!info || !mn || !mx || !scale || !out)
            return fail(AQR_ERR_INVALID_ARG, "aqr_quantizer_create: null pointer");
        if (info->d < 1 || info->M < 2 || info->efc < 1)
            return fail(AQR_ERR_INVALID_ARG, "aqr_quantizer_create: d, M or efc out of range");
        for (int32_t j = 0; j < info->d; ++j)
            if (!std::isfinite(mn[j]) || !std::isfinite(mx[j]) || !std::isfinite(scale[j]) ||
                !(scale[j] > 0))
                return fail(AQR_ERR_INVALID_ARG, "aqr_quantizer_create: bad range or scale");
        aqr_quantizer* q = new aqr_quantizer();
        q->info = *info;
        q->info.d_pad = round_up(info->d, 16);
        q->mn.assign(mn, mn + info->d);
        q->mx.assign(mx, mx + info->d);
        q->scale.assign(scale, scale + info->d);
        *out = q;
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_OOM, "aqr_quantizer_create: out of host memory");
    }
}

extern "C" void aqr_quantizer_free(aqr_quantizer* qz) { delete qz; }
