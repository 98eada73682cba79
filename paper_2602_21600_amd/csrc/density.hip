// density.hip -- the quantiser's density search on the device (Section 3.1,
// Stage 1; Alg. 1, density step).
//
// For every sample point x_i the k smallest squared L2 distances to the other
// base points, whose mean gives rho_i = 1 / (mean + eps).  Each distance is
// summed over the dimensions in order, in FP64, with one rounding for every
// subtraction, product and sum (this library is compiled without
// floating-point contraction), so it equals the host's value bit for bit; the
// k smallest values of a sample form one multiset whichever order they are
// found in, and the host sums them in ascending order, as the host quantiser
// does.  The densities are therefore those of the host quantiser exactly.
//
// Work split: one wave scores a tile of 32 sample points against one
// partition of the base rows, 64 rows at a time with one row per lane.  The
// tile's values sit in a [tile][dim][32] FP64 table that every lane reads at
// the same address (scalar loads); each lane converts its own row value once
// per dimension and reuses it for the 32 samples, so the inner loop is three
// FP64 vector operations per (sample, row, dimension): the vector FP64 rate
// bounds the kernel.  Distances are not reshaped into matrix products: the
// |a|^2 + |b|^2 - 2ab form rounds differently and would change the densities.
//
// Per sample the wave keeps the k smallest distances of its partition as an
// ascending list in LDS (element i held by lane i); lane s of a register
// holds list s's last value.  A ballot over the 64 rows finds the distances
// below that bound; each is inserted by a rank count over the list, which
// leaves the list unchanged when an earlier insertion of the same ballot has
// already lowered the bound below it.  The partition lists go to the host,
// which takes the k smallest of each sample's lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "internal.hpp"

namespace aqr {

namespace {

constexpr int kWave = 64;
constexpr int kTileS = 32;   // samples per wave
constexpr int kWaves = 4;    // waves per block
constexpr int kMaxK = 64;    // list length limit: one list element per lane

__device__ __forceinline__ double readlane_f64(double v, int l) {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    u = ((uint64_t)hi << 32) | lo;
    double r;
    __builtin_memcpy(&r, &u, 8);
    return r;
}

// SV: [tiles][d][32] sample values (FP64); SI: [tiles*32] sample row ids
// (-1 for the padding of the last tile); out: [tiles*32][parts][k].
template <bool VEC4>
__global__ __launch_bounds__(kWaves * kWave) void k_density(
    const float* __restrict__ X, int64_t n, int32_t d, const double* __restrict__ SV,
    const int64_t* __restrict__ SI, int32_t tiles, int32_t parts, int64_t part_rows, int32_t k,
    double* __restrict__ out) {
    extern __shared__ double lists[];  // [wave][32][k]
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t gw = (int64_t)blockIdx.x * kWaves + wv;
    if (gw >= (int64_t)tiles * parts) return;  // the whole wave leaves together
    const int32_t tile = (int32_t)(gw / parts);
    const int32_t part = (int32_t)(gw % parts);
    const int64_t r0 = (int64_t)part * part_rows;
    const int64_t r1 = std::min<int64_t>(n, r0 + part_rows);
    double* L = lists + (size_t)wv * kTileS * k;
    const double inf = __builtin_huge_val();
    for (int s = 0; s < kTileS; ++s)
        if (lane < k) L[s * k + lane] = inf;
    double bound = inf;  // lane s: last value of the list of sample s
    const int64_t self = lane < kTileS ? SI[(int64_t)tile * kTileS + lane] : -1;
    const double* sv = SV + (size_t)tile * d * kTileS;
    for (int64_t rb = r0; rb < r1; rb += kWave) {
        const int64_t r = rb + lane;
        const bool live = r < r1;
        const float* xr = X + (live ? r : r1 - 1) * (int64_t)d;
        double acc[kTileS];
#pragma unroll
        for (int u = 0; u < kTileS; ++u) acc[u] = 0.0;
        if (VEC4) {
            const float4* x4 = reinterpret_cast<const float4*>(xr);
            for (int32_t j4 = 0; j4 < d / 4; ++j4) {
                const float4 xv4 = x4[j4];
                const float xs[4] = {xv4.x, xv4.y, xv4.z, xv4.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double xv = (double)xs[c];
                    const double* sj = sv + (size_t)(j4 * 4 + c) * kTileS;
#pragma unroll
                    for (int u = 0; u < kTileS; ++u) {
                        const double df = sj[u] - xv;
                        acc[u] += df * df;
                    }
                }
            }
        } else {
            for (int32_t j = 0; j < d; ++j) {
                const double xv = (double)xr[j];
                const double* sj = sv + (size_t)j * kTileS;
#pragma unroll
                for (int u = 0; u < kTileS; ++u) {
                    const double df = sj[u] - xv;
                    acc[u] += df * df;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kTileS; ++u) {
            const double b = readlane_f64(bound, u);
            const int64_t su = (int64_t)__builtin_amdgcn_readlane((int)(uint32_t)self, u) |
                               ((int64_t)__builtin_amdgcn_readlane((int)(self >> 32), u) << 32);
            uint64_t mask = __ballot(live && r != su && acc[u] < b);
            double* Ls = L + u * k;
            while (mask) {
                const int src = __builtin_ctzll(mask);
                mask &= mask - 1;
                const double v = readlane_f64(acc[u], src);
                const double cur = lane < k ? Ls[lane] : inf;
                const double prev = __shfl_up(cur, 1, kWave);
                const int pos = __popcll(__ballot(lane < k && cur <= v));
                const double nv = lane < pos ? cur : (lane == pos ? v : prev);
                if (lane < k) Ls[lane] = nv;
                const double last = readlane_f64(nv, k - 1);
                bound = lane == u ? last : bound;
            }
        }
    }
    for (int s = 0; s < kTileS; ++s)
        if (lane < k)
            out[(((int64_t)tile * kTileS + s) * parts + part) * k + lane] = L[s * k + lane];
}

aqr_status density_hip_fail(hipError_t e, const char* what) {
    return fail(AQR_ERR_DEVICE, std::string("aqr_quantize_device: ") + what + ": " +
                                    hipGetErrorString(e));
}

}  // namespace

aqr_status device_density_sums(const float* X, int64_t n, int32_t d, const int64_t* S, int64_t m,
                               int32_t k, int T, double* sums) {
    if (k < 1 || k > kMaxK) return fail(AQR_ERR_INVALID_ARG, "aqr_quantize_device: k_rho out of range");
    if (m < 1) return AQR_OK;
    const int64_t tiles64 = (m + kTileS - 1) / kTileS;
    if (tiles64 > std::numeric_limits<int32_t>::max() / 2)
        return fail(AQR_ERR_INVALID_ARG, "aqr_quantize_device: too many sample points");
    const int32_t tiles = (int32_t)tiles64;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return density_hip_fail(e, "hipGetDevice");
    int num_cu = 0;
    e = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return density_hip_fail(e, "device attribute");
    // enough waves for about 16 on every compute unit, no partition below 256 rows
    const int64_t want = std::max<int64_t>(1, ((int64_t)num_cu * 16 + tiles - 1) / tiles);
    const int32_t parts = (int32_t)std::max<int64_t>(1, std::min<int64_t>(want, (n + 255) / 256));
    const int64_t part_rows = (n + parts - 1) / parts;
    const int64_t waves = (int64_t)tiles * parts;

    std::vector<double> sv((size_t)tiles * kTileS * d);
    std::vector<int64_t> si((size_t)tiles * kTileS, -1);
    for (int64_t s = 0; s < (int64_t)tiles * kTileS; ++s) {
        const int64_t src = S[std::min(s, m - 1)];  // the padding repeats the last sample
        if (s < m) si[s] = src;
        const int64_t t = s / kTileS, u = s % kTileS;
        for (int32_t j = 0; j < d; ++j)
            sv[((size_t)t * d + j) * kTileS + u] = (double)X[src * d + j];
    }
    const size_t out_n = (size_t)tiles * kTileS * parts * k;
    float* dX = nullptr;
    double* dSV = nullptr;
    int64_t* dSI = nullptr;
    double* dOut = nullptr;
    auto release = [&]() {
        if (dX) (void)hipFree(dX);
        if (dSV) (void)hipFree(dSV);
        if (dSI) (void)hipFree(dSI);
        if (dOut) (void)hipFree(dOut);
    };
    auto step = [&](hipError_t err, const char* what) -> aqr_status {
        if (err == hipSuccess) return AQR_OK;
        release();
        return density_hip_fail(err, what);
    };
    aqr_status st;
    if ((st = step(hipMalloc(&dX, sizeof(float) * (size_t)n * d), "device memory")) != AQR_OK ||
        (st = step(hipMalloc(&dSV, sizeof(double) * sv.size()), "device memory")) != AQR_OK ||
        (st = step(hipMalloc(&dSI, sizeof(int64_t) * si.size()), "device memory")) != AQR_OK ||
        (st = step(hipMalloc(&dOut, sizeof(double) * out_n), "device memory")) != AQR_OK)
        return st;
    if ((st = step(hipMemcpy(dX, X, sizeof(float) * (size_t)n * d, hipMemcpyHostToDevice),
                   "copy")) != AQR_OK ||
        (st = step(hipMemcpy(dSV, sv.data(), sizeof(double) * sv.size(), hipMemcpyHostToDevice),
                   "copy")) != AQR_OK ||
        (st = step(hipMemcpy(dSI, si.data(), sizeof(int64_t) * si.size(), hipMemcpyHostToDevice),
                   "copy")) != AQR_OK)
        return st;
    const size_t lds = sizeof(double) * kWaves * kTileS * (size_t)k;
    const dim3 grid((unsigned)((waves + kWaves - 1) / kWaves)), block(kWaves * kWave);
    if (d % 4 == 0)
        hipLaunchKernelGGL(k_density<true>, grid, block, lds, 0, dX, n, d, dSV, dSI, tiles, parts,
                           part_rows, k, dOut);
    else
        hipLaunchKernelGGL(k_density<false>, grid, block, lds, 0, dX, n, d, dSV, dSI, tiles,
                           parts, part_rows, k, dOut);
    if ((st = step(hipGetLastError(), "launch")) != AQR_OK) return st;
    std::vector<double> lists(out_n);
    if ((st = step(hipMemcpy(lists.data(), dOut, sizeof(double) * out_n, hipMemcpyDeviceToHost),
                   "copy back")) != AQR_OK)
        return st;
    release();
    // per sample: the k smallest of its partition lists, summed in ascending order
    std::atomic<int64_t> next{0};
    parallel_for_threads(T, [&](int) {
        std::vector<double> v((size_t)parts * k);
        for (;;) {
            const int64_t s = next.fetch_add(64);
            if (s >= m) break;
            for (int64_t i = s; i < std::min(m, s + 64); ++i) {
                std::memcpy(v.data(), &lists[(size_t)i * parts * k], sizeof(double) * v.size());
                std::partial_sort(v.begin(), v.begin() + k, v.end());
                double sum = 0.0;
                for (int32_t u = 0; u < k; ++u) sum += v[u];
                sums[i] = sum;
            }
        }
    });
    return AQR_OK;
}

}  // namespace aqr
