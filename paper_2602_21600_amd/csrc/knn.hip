// knn.hip -- exact k nearest neighbours by brute force on gfx950: the truth
// against which recall@k is measured (squared L2, ties by id).
//
// Two kernels.
//
// k_knn_screen: a dense product Q X^T on the matrix cores.  A block holds 64
// queries and walks one partition of the base rows in tiles of 64 rows; each
// of its four waves accumulates a 32 x 32 block of q.x with the FP32 32x32x2
// MFMA, staging 32 dimensions of both operands at a time through LDS.  The
// screening score of (q, x) is s = |x|^2 - 2 q.x (|q|^2 is the same for every
// x of a query and is left out).  Each query keeps the KC = k + 32 (rounded up
// to 16) smallest keys (ordered FP32 score, id) of its partition in an LDS
// buffer: a tile appends the scores below the query's current bound, and
// once the buffer could overflow in the next tile it is cut back to the KC
// smallest, which lowers the bound.
//
// k_knn_finish: one wave per query merges the partitions' lists, keeps the KC
// smallest screening keys, re-scores those candidates exactly, in FP64 with
// the direct differences summed over the dimensions in order (one rounding per
// subtraction, product and sum, as the exact definition is written), sorts
// them by (distance, id) and writes the first k.
//
// Exactness.  FP32 screening can misorder rows whose distances differ by less
// than its rounding error, so the finish kernel certifies each query: every
// row outside the candidate set has a screening key above the cut (the
// largest kept key), so its exact distance is at least |q|^2 + s_cut - B,
// where B bounds the FP32 error of any row's score (from the largest |x|^2
// seen and |q|).  When that bound exceeds the k-th re-scored distance, no
// outside row can enter the top k and the result is exact; the optional
// certified[q] output records this.  With 32 spare candidates it holds on
// every workload here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace aqr {
namespace knn {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWave = 64;
constexpr int QB = 64;        // queries per block
constexpr int XB = 64;        // base rows per tile
constexpr int KCH = 32;       // dimensions per staged chunk
constexpr int LDR = KCH + 4;  // LDS row stride in floats (16-byte aligned rows)
constexpr int kMaxK = 128;
constexpr int kMaxParts = 8;
constexpr uint64_t kEmpty = ~0ull;

struct Header {
    uint32_t xmax2;  // bits of the largest |x|^2 seen (non-negative floats order as integers)
    uint32_t pad[63];
};

struct ScreenArgs {
    const float* X;
    int64_t n;
    int32_t d;
    const float* Q;
    int64_t nq;
    int32_t kc;       // candidates kept per query and partition
    int32_t cap;      // LDS buffer entries per query (kc + XB)
    int32_t parts;
    int64_t part_rows;
    uint64_t* keys;   // [nq][parts][kc]
    Header* hdr;
};

// Order-preserving map of a float to an unsigned integer.
__device__ __forceinline__ uint32_t ord(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void k_knn_init(Header* h) {
    if (threadIdx.x == 0 && blockIdx.x == 0) h->xmax2 = 0u;
}

// Cut query i's buffer back to its kc smallest keys (one wave; cnt > kc).
__device__ __forceinline__ void compact(uint64_t* buf, int cnt, int kc, uint64_t* tmp,
                                        uint64_t* thr, int* cntp, int lane) {
    for (int m = lane; m < cnt; m += kWave) {
        const uint64_t v = buf[m];
        int r = 0;
        for (int u = 0; u < cnt; ++u) r += buf[u] < v ? 1 : 0;
        if (r < kc) tmp[r] = v;  // keys are distinct (one per row)
    }
    wsync();
    for (int m = lane; m < kc; m += kWave) buf[m] = tmp[m];
    wsync();
    if (lane == 0) {
        *thr = tmp[kc - 1];
        *cntp = kc;
    }
    wsync();
}

__global__ __launch_bounds__(256) void k_knn_screen(ScreenArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* Qs = reinterpret_cast<float*>(smem);               // [QB][LDR]
    float* Xs = Qs + QB * LDR;                                 // [XB][LDR]
    float* xn = Xs + XB * LDR;                                 // [XB]
    uint64_t* thr = reinterpret_cast<uint64_t*>(xn + XB);      // [QB]
    int* cnt = reinterpret_cast<int*>(thr + QB);               // [QB]
    uint64_t* tmp = reinterpret_cast<uint64_t*>(cnt + QB);     // [4][kc]
    uint64_t* buf = tmp + 4 * a.kc;                            // [QB][cap]

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * QB;
    const int p = blockIdx.y;
    const int64_t x_begin = (int64_t)p * a.part_rows;
    const int64_t x_end = min(a.n, x_begin + a.part_rows);
    const int nqb = (int)min((int64_t)QB, a.nq - q0);
    const int d = a.d;
    const int nchunk = (d + KCH - 1) / KCH;

    for (int i = t; i < QB; i += 256) {
        thr[i] = kEmpty;
        cnt[i] = 0;
    }
    __syncthreads();

    // operand roles of this wave: queries [qh*32, +32) x rows [xh*32, +32)
    const int qh = wave & 1, xh = wave >> 1;
    const int hl = lane >> 5;    // which 4 of each 8 staged dimensions this lane feeds
    const int rl = lane & 31;
    float xpart = 0.0f;          // |x|^2 partial of staged row (t >> 2)

    for (int64_t x0 = x_begin; x0 < x_end; x0 += XB) {
        const int nxb = (int)min((int64_t)XB, x_end - x0);
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
        xpart = 0.0f;
        for (int c = 0; c < nchunk; ++c) {
            const int col = c * KCH + (t & 31);
            // stage 32 dimensions of the 64 queries and 64 rows: instruction e
            // of thread t reads row (t >> 5) + 8e, one 128-byte segment per row
            float qv[8], xv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = (t >> 5) + 8 * e;
                const bool cq = col < d && r < nqb;
                const bool cx = col < d && r < nxb;
                qv[e] = cq ? a.Q[(q0 + r) * d + col] : 0.0f;
                xv[e] = cx ? a.X[(x0 + r) * d + col] : 0.0f;
            }
            __syncthreads();  // the previous chunk's operands have been read
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = (t >> 5) + 8 * e;
                Qs[r * LDR + (t & 31)] = qv[e];
                Xs[r * LDR + (t & 31)] = xv[e];
            }
            __syncthreads();
            {
                // |x|^2 of staged row t >> 2 over its 8-dimension slice
                const float* xr = Xs + (t >> 2) * LDR + (t & 3) * 8;
#pragma unroll
                for (int e = 0; e < 8; ++e) xpart += xr[e] * xr[e];
            }
            // Each MFMA step sums over two dimensions, one per half-wave.  A
            // lane reads four consecutive dimensions (one 16-byte load) and
            // feeds them to four steps; the other half-wave feeds the four
            // after them, so the eight dimensions of a group go in once each.
            const float* qa = Qs + (qh * 32 + rl) * LDR + 4 * hl;
            const float* xb = Xs + (xh * 32 + rl) * LDR + 4 * hl;
#pragma unroll
            for (int g = 0; g < KCH / 8; ++g) {
                const float4 av = *reinterpret_cast<const float4*>(qa + 8 * g);
                const float4 bv = *reinterpret_cast<const float4*>(xb + 8 * g);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv.y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, bv.z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, bv.w, acc, 0, 0, 0);
            }
        }
        // |x|^2 of each staged row: four threads per row
        xpart += __shfl_xor(xpart, 1, kWave);
        xpart += __shfl_xor(xpart, 2, kWave);
        if ((t & 3) == 0) {
            xn[t >> 2] = xpart;
            if ((t >> 2) < nxb) atomicMax(&a.hdr->xmax2, __float_as_uint(xpart));
        }
        __syncthreads();
        // Output block of the 32x32x2 MFMA: lane l holds column l mod 32 and,
        // in register r, row 8 (r / 4) + 4 (l / 32) + r mod 4.
        const int j = xh * 32 + rl;
        const bool jv = j < nxb;
        const float xj = xn[j];
        const uint32_t id = (uint32_t)(x0 + j);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = qh * 32 + 8 * (r >> 2) + 4 * hl + (r & 3);
            const uint64_t key = ((uint64_t)ord(xj - 2.0f * acc[r]) << 32) | id;
            if (jv && i < nqb && key < thr[i]) {
                const int pos = atomicAdd(&cnt[i], 1);
                buf[i * a.cap + pos] = key;
            }
        }
        __syncthreads();
        // a buffer that could overflow in the next tile is cut back to kc
        for (int i = wave; i < nqb; i += 4) {
            const int c = __builtin_amdgcn_readfirstlane(cnt[i]);
            if (c > a.cap - XB) compact(buf + i * a.cap, c, a.kc, tmp + wave * a.kc, &thr[i], &cnt[i], lane);
        }
        __syncthreads();
    }
    // the partition's list of each query: its kc smallest keys (padded)
    for (int i = wave; i < nqb; i += 4) {
        const int c = __builtin_amdgcn_readfirstlane(cnt[i]);
        if (c > a.kc) compact(buf + i * a.cap, c, a.kc, tmp + wave * a.kc, &thr[i], &cnt[i], lane);
        const int cc = min(c, a.kc);
        uint64_t* out = a.keys + ((q0 + i) * a.parts + p) * (int64_t)a.kc;
        for (int m = lane; m < a.kc; m += kWave) out[m] = m < cc ? buf[i * a.cap + m] : kEmpty;
    }
}

struct FinishArgs {
    const float* X;
    int64_t n;
    int32_t d;
    const float* Q;
    int64_t nq;
    int32_t k, kc, parts;
    const uint64_t* keys;
    const Header* hdr;
    int32_t* out_id;
    double* out_dist;
    uint8_t* certified;
};

__global__ __launch_bounds__(256) void k_knn_finish(FinishArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * 4 + wave;
    if (q >= a.nq) return;
    const int m_all = a.parts * a.kc;
    uint64_t* all = reinterpret_cast<uint64_t*>(smem) + (size_t)wave * (m_all + 2 * a.kc);
    uint64_t* sel = all + m_all;          // kc smallest screening keys
    uint64_t* ex = sel + a.kc;            // (ordered exact distance, id)... see below
    double* dist = reinterpret_cast<double*>(ex);  // exact distances of sel, in sel's order
    for (int m = lane; m < m_all; m += kWave) all[m] = a.keys[q * m_all + m];
    wsync();
    // the kc smallest keys of the partitions' lists.  Row keys are distinct;
    // the padding of short lists repeats one value, so equal keys are ranked
    // by position and every rank below kc is written exactly once.
    for (int m = lane; m < m_all; m += kWave) {
        const uint64_t v = all[m];
        int r = 0;
        for (int u = 0; u < m_all; ++u) r += (all[u] < v || (all[u] == v && u < m)) ? 1 : 0;
        if (r < a.kc) sel[r] = v;
    }
    wsync();
    // exact FP64 distances of the candidates, dimensions in order
    const float* qr = a.Q + q * a.d;
    for (int m = lane; m < a.kc; m += kWave) {
        const uint64_t v = sel[m];
        double s = __builtin_huge_val();
        if (v != kEmpty && (int64_t)(uint32_t)v < a.n) {
            const float* xr = a.X + (int64_t)(uint32_t)v * a.d;
            s = 0.0;
            for (int j = 0; j < a.d; ++j) {
                const double df = (double)qr[j] - (double)xr[j];
                s = s + df * df;
            }
        }
        dist[m] = s;
    }
    wsync();
    // rank by (distance, id); write the first k
    int valid = 0;
    for (int m = 0; m < a.kc; ++m) valid += sel[m] != kEmpty ? 1 : 0;
    double dk = __builtin_huge_val();
    for (int m = lane; m < a.kc; m += kWave) {
        const double dm = dist[m];
        const uint32_t im = (uint32_t)sel[m];
        const bool vm = sel[m] != kEmpty;
        int r = 0;
        for (int u = 0; u < a.kc; ++u) {
            const bool vu = sel[u] != kEmpty;
            const double du = dist[u];
            const uint32_t iu = (uint32_t)sel[u];
            // valid entries first, then by (distance, id)
            const bool lt = vu && (!vm || du < dm || (du == dm && iu < im));
            r += lt ? 1 : 0;
        }
        if (r < a.k) {
            a.out_id[q * a.k + r] = vm ? (int32_t)im : -1;
            a.out_dist[q * a.k + r] = vm ? dm : __builtin_huge_val();
        }
        if (vm && r == a.k - 1) dk = dm;
    }
    for (int m = valid + lane; m < a.k; m += kWave) {  // fewer rows than k
        a.out_id[q * a.k + m] = -1;
        a.out_dist[q * a.k + m] = __builtin_huge_val();
    }
    if (a.certified) {
        // the k-th exact distance (every lane takes the minimum over lanes:
        // one lane holds it)
        for (int o = 32; o >= 1; o >>= 1) dk = fmin(dk, __shfl_xor(dk, o, kWave));
        uint8_t ok = 1;
        if (valid >= a.kc && a.n > a.kc) {
            // some rows stayed outside the candidates: bound their distance
            const uint64_t cut = sel[a.kc - 1];
            const double s_cut = (double)unord((uint32_t)(cut >> 32));
            double qn = 0.0;
            for (int j = 0; j < a.d; ++j) qn += (double)qr[j] * (double)qr[j];
            const double x2 = (double)__uint_as_float(a.hdr->xmax2);
            const double u = 1.0 / 16777216.0;  // FP32 unit roundoff
            const double B = 1.01 * (a.d + 4) * u * (x2 * (1.0 + 2.0 * (a.d + 4) * u) +
                                                     2.0 * sqrt(qn) * sqrt(x2));
            ok = (qn + s_cut - B > dk) ? 1 : 0;
        }
        if (lane == 0) a.certified[q] = ok;
    }
}

int kc_for(int k) { return (k + 32 + 15) / 16 * 16; }

int parts_for(int64_t n, int64_t nq) {
    const int64_t qblocks = (nq + QB - 1) / QB;
    int64_t p = (512 + qblocks - 1) / qblocks;
    p = std::min<int64_t>(p, std::max<int64_t>(1, n / 4096));
    return (int)std::max<int64_t>(1, std::min<int64_t>(p, kMaxParts));
}

}  // namespace knn
}  // namespace aqr

using namespace aqr;

extern "C" size_t aqr_knn_workspace_size(int64_t n, int64_t nq, int32_t k) {
    if (n < 1 || nq < 0 || k < 1 || k > knn::kMaxK) return 0;
    const int kc = knn::kc_for(k), parts = knn::parts_for(n, nq);
    return sizeof(knn::Header) + (size_t)std::max<int64_t>(nq, 1) * parts * kc * 8;
}

namespace {

aqr_status knn_run(const char* who, const float* X, int64_t n, int32_t d, const float* Q,
                   int64_t nq, int32_t k, int32_t* out_id, double* out_dist, uint8_t* certified,
                   void* ws, size_t ws_bytes, void* stream) {
    try {
        clear_error();
        if (nq < 0) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": nq < 0");
        if (n < 1 || n > (int64_t)0x7FFFFFFF)
            return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": n must be in [1, 2^31-1]");
        if (d < 1 || d > 4096) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": d must be in [1, 4096]");
        if (k < 1 || k > knn::kMaxK)
            return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": k must be in [1, 128]");
        if (nq == 0) return AQR_OK;
        if (!X || !Q || !out_id || !out_dist || !ws)
            return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": null pointer");
        if (ws_bytes < aqr_knn_workspace_size(n, nq, k))
            return fail(AQR_ERR_OOM, std::string(who) + ": workspace smaller than aqr_knn_workspace_size()");
        if (((uintptr_t)ws & 15) != 0)
            return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": workspace must be 16-byte aligned");
        const int kc = knn::kc_for(k), parts = knn::parts_for(n, nq);
        knn::Header* hdr = reinterpret_cast<knn::Header*>(ws);
        uint64_t* keys = reinterpret_cast<uint64_t*>(reinterpret_cast<unsigned char*>(ws) +
                                                     sizeof(knn::Header));
        int64_t part_rows = (n + parts - 1) / parts;
        part_rows = (part_rows + knn::XB - 1) / knn::XB * knn::XB;
        knn::ScreenArgs sa{X, n, d, Q, nq, kc, kc + knn::XB, parts, part_rows, keys, hdr};
        const size_t lds_screen = (size_t)(knn::QB + knn::XB) * knn::LDR * 4 + knn::XB * 4 +
                                  knn::QB * 8 + knn::QB * 4 + 4 * (size_t)kc * 8 +
                                  (size_t)knn::QB * (kc + knn::XB) * 8;
        knn::FinishArgs fa{X, n, d, Q, nq, k, kc, parts, keys, hdr, out_id, out_dist, certified};
        const size_t lds_finish = 4 * ((size_t)parts * kc + 2 * kc) * 8;
        hipDevice_t dv = 0;
        hipError_t e = hipGetDevice(&dv);
        int max_lds = 0;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dv);
        if (e != hipSuccess) return fail(AQR_ERR_DEVICE, std::string(who) + ": " + hipGetErrorString(e));
        if (lds_screen > (size_t)max_lds || lds_finish > (size_t)max_lds)
            return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": LDS per block exceeds the device limit");
        static std::atomic<int> set_s{0}, set_f{0};
        if ((int)lds_screen > set_s.load()) {
            e = hipFuncSetAttribute((const void*)knn::k_knn_screen,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_screen);
            if (e != hipSuccess) return fail(AQR_ERR_DEVICE, std::string(who) + ": " + hipGetErrorString(e));
            set_s.store((int)lds_screen);
        }
        if ((int)lds_finish > set_f.load()) {
            e = hipFuncSetAttribute((const void*)knn::k_knn_finish,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_finish);
            if (e != hipSuccess) return fail(AQR_ERR_DEVICE, std::string(who) + ": " + hipGetErrorString(e));
            set_f.store((int)lds_finish);
        }
        hipStream_t s = (hipStream_t)stream;
        hipLaunchKernelGGL(knn::k_knn_init, dim3(1), dim3(64), 0, s, hdr);
        const int64_t qblocks = (nq + knn::QB - 1) / knn::QB;
        if (qblocks > 0x7FFFFFFF) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": nq too large");
        hipLaunchKernelGGL(knn::k_knn_screen, dim3((unsigned)qblocks, (unsigned)parts), dim3(256),
                           lds_screen, s, sa);
        hipLaunchKernelGGL(knn::k_knn_finish, dim3((unsigned)((nq + 3) / 4)), dim3(256), lds_finish,
                           s, fa);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(AQR_ERR_DEVICE, std::string(who) + ": " + hipGetErrorString(e));
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_STATE, std::string(who) + ": unexpected failure");
    }
}

}  // namespace

extern "C" aqr_status aqr_knn_bruteforce(const float* X, int64_t n, int32_t d, const float* Q,
                                         int64_t nq, int32_t k, int32_t* out_id,
                                         double* out_dist, uint8_t* certified, void* ws,
                                         size_t ws_bytes, void* stream) {
    return knn_run("aqr_knn_bruteforce", X, n, d, Q, nq, k, out_id, out_dist, certified, ws,
                   ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// The same without a caller workspace, for callers that cannot allocate
// device memory: the partition lists and the header live in a file-scope
// device array (one copy per device, held until the process ends).  Its
// device address is looked up once per device and kept; host code never
// passes the array's name itself to a kernel.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)16 << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

aqr_status scratch_for_current_device(const char* who, void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(AQR_ERR_DEVICE, std::string(who) + ": " + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(AQR_ERR_DEVICE, std::string(who) + ": device index out of range");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(AQR_ERR_DEVICE, std::string(who) + ": hipGetSymbolAddress: " +
                                            hipGetErrorString(e));
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return AQR_OK;
}

}  // namespace

extern "C" size_t aqr_knn_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" aqr_status aqr_knn_bruteforce_noalloc(const float* X, int64_t n, int32_t d,
                                                 const float* Q, int64_t nq, int32_t k,
                                                 int32_t* out_id, double* out_dist,
                                                 uint8_t* certified, void* stream) {
    const char* who = "aqr_knn_bruteforce_noalloc";
    try {
        clear_error();
        if (nq == 0) return AQR_OK;
        const size_t need = aqr_knn_workspace_size(n, nq, k);
        if (need == 0)
            return knn_run(who, X, n, d, Q, nq, k, out_id, out_dist, certified, nullptr, 0,
                           stream);  // reports the argument error
        if (need > kScratchBytes)
            return fail(AQR_ERR_INVALID_ARG,
                        std::string(who) + ": needs " + std::to_string(need) +
                            " bytes of scratch, above its fixed " + std::to_string(kScratchBytes) +
                            " (split the queries into smaller calls)");
        void* ws = nullptr;
        aqr_status st = scratch_for_current_device(who, &ws);
        if (st != AQR_OK) return st;
        return knn_run(who, X, n, d, Q, nq, k, out_id, out_dist, certified, ws, kScratchBytes,
                       stream);
    } catch (...) {
        return fail(AQR_ERR_STATE, std::string(who) + ": unexpected failure");
    }
}
