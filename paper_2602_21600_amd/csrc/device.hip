// device.hip -- gfx950 kernels and device-side entry points of libaqr.
//
// Query path of AQR-HNSW (Section 3.2, Algorithm 2) on an MI355X:
//   * k_search: one wavefront per query in a persistent loop (queries are
//     pulled from an atomic counter).  Per query: encode the FP32 query to
//     8-bit codes, greedy descent through the upper layers, then the layer-0
//     search with width ef (Stage 1).  The same kernel instantiated on FP32
//     rows is the baseline HNSW search.
//   * k_rerank: one wavefront per query: asymmetric distances on decoded
//     codes, sort, early termination, exact FP32 distances on the survivors
//     and assembly of the top k (Stages 2 and 3).
//   * k_serve: the same per-query code in a resident kernel fed from a ring
//     of requests in pinned host memory.
//
// Layer-0 search form.  The result list W is one sorted array of (D, id)
// keys in LDS whose low bit is an "expanded" flag; the next node to expand
// is the nearest unexpanded entry and the search ends when none is left.
// All unvisited neighbours of one expansion are scored together and merged
// into W as one batch (keys below the current bound, W kept at ef entries).
// The visited set is an LDS cache that may forget ids but never reports an
// id it has not seen.  Under the strict (D, id) order these choices give
// the same expansions, the same distinct visited set and the same result
// as the two-heap search of HNSW: a node scored again after being
// forgotten has the same key, so it is either in W already (dropped on key
// equality) or not below the bound.
//
// Distances.  Code rows are read 16 bytes per lane; a row is spread over G
// lanes (G = 16-byte chunks of the row, rounded up to a power of two, at
// least 4 and at most 64) so one wave reads 64/G rows per pass, each row one
// contiguous segment.  The 8-bit squared distance is exact in uint32 as
// |q|^2 + sum(x*x - 2 q*x) with the 4 x u8 dot product instruction, reduced
// across the G lanes by DPP lane permutes.  FP32 rows use fused
// multiply-add on direct differences.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <new>
#include <vector>

#include "internal.hpp"

namespace aqr {
namespace dev {

constexpr uint32_t kNone = 0xFFFFFFFFu;
// Spare bytes after the code rows and after the FP32 rows of an index arena:
// the search reads whole chunk slots of a row without clamping them to the
// row, at most CPL * 2^LG = 1,024 slots of 16 bytes (FP32 rows of up to
// kMaxD floats: 16 chunks per lane on 64 lanes) from the row start.
constexpr size_t kRowSlack = 16384;
constexpr int kWave = 64;
constexpr int kMaxD = 4096;

struct Idx {
    const uint8_t* codes;    // n x dp bytes
    const float* X;          // n x xs floats
    const uint32_t* adj0;    // n x s0
    const int32_t* ubase;    // n: first upper row of the node (level >= 1) or -1
    const uint32_t* uadj;    // rows x s1
    const float* qmin;       // dp (padding 0)
    const float* qscale;     // dp (padding 1)
    int64_t n;
    int32_t d, dp, xs, s0, s1;
    int32_t cs;              // code row stride in bytes (>= dp, whole 128-byte lines)
    int32_t nrm;             // 1: |x^|^2 of each code row (uint32) sits at byte dp of the row
    int32_t xst;             // FP32 row stride in floats (>= xs, whole 128-byte lines)
    uint32_t ep;
    int32_t L;
    int32_t idbits;          // ceil(log2(n)), at least 1
};

struct Taps {
    int32_t cap;
    uint32_t* expanded;
    uint32_t* evaluated;
    uint32_t* counts;
};

struct RTaps {
    uint32_t* a_id;
    float* a_dist;
    uint8_t* et;
    int32_t* nrr;
};

// ---------------------------------------------------------------------------
// wave primitives
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// number of set bits of m below this lane
__device__ __forceinline__ int below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t v, int m) {
    return (uint32_t)__shfl_xor((int)v, m, kWave);
}
__device__ __forceinline__ float shfl_xor_f32(float v, int m) { return __shfl_xor(v, m, kWave); }
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    for (int m = 32; m >= 1; m >>= 1) {
        uint32_t lo = shfl_xor_u32((uint32_t)v, m);
        uint32_t hi = shfl_xor_u32((uint32_t)(v >> 32), m);
        uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_u32(v, m);
    return v;
}

// Sum over aligned groups of G lanes (G a power of two <= 64), result in
// every lane of the group.  Steps inside a row of 16 lanes use DPP lane
// permutes (quad swaps, then the half-row and row mirrors); wider groups
// finish with LDS-routed permutes.  Every step pairs lanes symmetrically, so
// all lanes of a group hold the same value, also in floating point.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_t(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i in each group of 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i in each row of 16

__device__ __forceinline__ float group_sum_f32(float v, int G) {
    if (G >= 2) v += __uint_as_float(dpp_t<kDppXor1>(__float_as_uint(v)));
    if (G >= 4) v += __uint_as_float(dpp_t<kDppXor2>(__float_as_uint(v)));
    if (G >= 8) v += __uint_as_float(dpp_t<kDppHalfMirror>(__float_as_uint(v)));
    if (G >= 16) v += __uint_as_float(dpp_t<kDppMirror>(__float_as_uint(v)));
    for (int m = 16; m < G; m <<= 1) v += shfl_xor_f32(v, m);
    return v;
}

// Sum over aligned groups of 2^LG lanes, known at compile time; the sum is
// complete in the last lane of each group (lanes G-1, 2G-1, ...).  Inside a
// row of 16 the butterfly above leaves it in every lane; across rows the
// row broadcasts add row 0 into row 1 and row 2 into row 3, then rows 0-1
// into row 3.
constexpr int kDppBcast15 = 0x142;    // lane 15 of each row to the next row
constexpr int kDppBcast31 = 0x143;    // lane 31 to rows 2 and 3
template <int LG>
__device__ __forceinline__ uint32_t gsum_u32(uint32_t v) {
    if constexpr (LG >= 1) v += dpp_t<kDppXor1>(v);
    if constexpr (LG >= 2) v += dpp_t<kDppXor2>(v);
    if constexpr (LG >= 3) v += dpp_t<kDppHalfMirror>(v);
    if constexpr (LG >= 4) v += dpp_t<kDppMirror>(v);
    if constexpr (LG >= 5)
        v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppBcast15, 0xA, 0xF, false);
    if constexpr (LG >= 6)
        v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppBcast31, 0xC, 0xF, false);
    return v;
}
template <int LG>
__device__ __forceinline__ float gsum_f32(float v) {
    if constexpr (LG >= 1) v += __uint_as_float(dpp_t<kDppXor1>(__float_as_uint(v)));
    if constexpr (LG >= 2) v += __uint_as_float(dpp_t<kDppXor2>(__float_as_uint(v)));
    if constexpr (LG >= 3) v += __uint_as_float(dpp_t<kDppHalfMirror>(__float_as_uint(v)));
    if constexpr (LG >= 4) v += __uint_as_float(dpp_t<kDppMirror>(__float_as_uint(v)));
    if constexpr (LG >= 5)
        v += __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(
            0, (int)__float_as_uint(v), kDppBcast15, 0xA, 0xF, false));
    if constexpr (LG >= 6)
        v += __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(
            0, (int)__float_as_uint(v), kDppBcast31, 0xC, 0xF, false));
    return v;
}

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_udot4(a, b, c, false);
}

// ---------------------------------------------------------------------------
// row distances
// ---------------------------------------------------------------------------

// Query encoding, Section 3.2: clamp(rint(fl32(fl32(q - min) * scale)), 0, 255).
// The build compiles with -ffp-contract=off, so the two FP32 operations stay
// separate and correctly rounded.
__device__ __forceinline__ uint32_t encode1(float v, float mn, float sc) {
    float t = v - mn;
    float u = t * sc;
    float r = __builtin_rintf(u);
    r = r < 0.0f ? 0.0f : (r > 255.0f ? 255.0f : r);
    return (uint32_t)r;
}

template <bool F32>
struct Rows;

// 8-bit code rows: chunk = 16 codes; partial = sum(x*x - 2 q*x) (mod 2^32)
template <>
struct Rows<false> {
    using Acc = uint32_t;
    __device__ static __forceinline__ uint4 load(const Idx& ix, uint32_t id, int ch) {
        return reinterpret_cast<const uint4*>(ix.codes + (uint64_t)id * (uint32_t)ix.cs)[ch];
    }
    __device__ static __forceinline__ uint32_t part(uint4 x, uint4 q) {
        uint32_t xx = dot4(x.x, x.x, 0u);
        xx = dot4(x.y, x.y, xx);
        xx = dot4(x.z, x.z, xx);
        xx = dot4(x.w, x.w, xx);
        uint32_t xq = dot4(x.x, q.x, 0u);
        xq = dot4(x.y, q.y, xq);
        xq = dot4(x.z, q.z, xq);
        xq = dot4(x.w, q.w, xq);
        return xx - 2u * xq;
    }
    __device__ static __forceinline__ uint32_t zero() { return 0u; }
    __device__ static __forceinline__ uint32_t add(uint32_t a, uint32_t b) { return a + b; }
    template <int LG>
    __device__ static __forceinline__ uint32_t gsum(uint32_t v) {
        return gsum_u32<LG>(v);
    }
    // key distance bits from the reduced partial and |q|^2
    __device__ static __forceinline__ uint32_t dbits(uint32_t s, uint32_t qq) { return qq + s; }
};

// FP32 rows: chunk = 4 floats; partial = sum (q - x)^2 by fused multiply-add
template <>
struct Rows<true> {
    using Acc = float;
    __device__ static __forceinline__ uint4 load(const Idx& ix, uint32_t id, int ch) {
        return reinterpret_cast<const uint4*>(ix.X + (uint64_t)id * (uint32_t)ix.xst)[ch];
    }
    __device__ static __forceinline__ float part(uint4 x, uint4 q) {
        float acc = 0.0f;
        float d0 = __uint_as_float(q.x) - __uint_as_float(x.x);
        acc = __builtin_fmaf(d0, d0, acc);
        float d1 = __uint_as_float(q.y) - __uint_as_float(x.y);
        acc = __builtin_fmaf(d1, d1, acc);
        float d2 = __uint_as_float(q.z) - __uint_as_float(x.z);
        acc = __builtin_fmaf(d2, d2, acc);
        float d3 = __uint_as_float(q.w) - __uint_as_float(x.w);
        acc = __builtin_fmaf(d3, d3, acc);
        return acc;
    }
    __device__ static __forceinline__ float zero() { return 0.0f; }
    __device__ static __forceinline__ float add(float a, float b) { return a + b; }
    template <int LG>
    __device__ static __forceinline__ float gsum(float v) {
        return gsum_f32<LG>(v);
    }
    __device__ static __forceinline__ uint32_t dbits(float s, uint32_t) { return __float_as_uint(s); }
};

struct Geo {
    int G, lg, rpp, nch, sub, grp;
};

__device__ __forceinline__ Geo make_geo(int lg, int nch, int lane) {
    Geo g;
    g.lg = lg;
    g.G = 1 << lg;
    g.rpp = kWave >> lg;
    g.nch = nch;
    g.sub = lane & (g.G - 1);
    g.grp = lane >> lg;
    return g;
}

// Score rows ids[r0 .. r0 + US * RPP) that lie below nn (ids in LDS); keys[r] =
// (dist bits << 32) | (id << 1): the low bit is left free for the expanded
// flag of W, and keys still order by (distance, id).  Rows are spread over
// groups of 2^LG lanes, one 16-byte chunk per lane and CPL chunks per lane;
// the US row sets of a pass are loaded before any is scored.  There are no
// divergent branches: rows past nn read row 0, and chunk slots past the row
// read whatever follows it (the row sections of the index arena end with
// kRowSlack spare bytes, more than any geometry's CPL * 2^LG chunks), and
// both are masked out of the sum.
//
// NRM (8-bit rows whose padding holds |x^|^2 at byte dp, and a row geometry
// with a spare chunk slot): the slot after the row's last chunk loads the
// chunk that starts with |x^|^2, and the data chunks need only q.x, so each
// row costs half the dot products.  The query chunks past the row are zero,
// so the slots past the row add nothing to q.x.  The sum |x|^2 - 2 q.x is the
// same integer either way.
template <bool F32, int CPL, int US, int LG, bool NRM = false>
__device__ __forceinline__ void eval_pass(const Idx& ix, const uint32_t* ids, int nn, int r0,
                                          uint64_t* keys, const uint4 (&qv)[CPL], uint32_t qq,
                                          const int sub, const int grp, const int nch) {
    using R = Rows<F32>;
    constexpr int G = 1 << LG, RPP = kWave >> LG;
    uint4 x[US][CPL];
    uint32_t id[US];
#pragma unroll
    for (int u = 0; u < US; ++u) {
        const int r = r0 + u * RPP + grp;
        id[u] = r < nn ? ids[r] : 0u;
#pragma unroll
        for (int c = 0; c < CPL; ++c) x[u][c] = R::load(ix, id[u], sub + c * G);
    }
#pragma unroll
    for (int u = 0; u < US; ++u) {
        typename R::Acc s = R::zero();
        if constexpr (NRM && !F32) {
            uint32_t xq = 0u, nr = 0u;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                xq = dot4(x[u][c].x, qv[c].x, xq);
                xq = dot4(x[u][c].y, qv[c].y, xq);
                xq = dot4(x[u][c].z, qv[c].z, xq);
                xq = dot4(x[u][c].w, qv[c].w, xq);
                nr += sub + c * G == nch ? x[u][c].x : 0u;
            }
            s = nr - 2u * xq;
        } else {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int ch = sub + c * G;
                const typename R::Acc t = R::part(x[u][c], qv[c]);
                s = R::add(s, ch < nch ? t : R::zero());
            }
        }
        s = R::template gsum<LG>(s);
        const int r = r0 + u * RPP + grp;
        if (sub == G - 1 && r < nn)
            keys[r] = ((uint64_t)R::dbits(s, qq) << 32) | ((uint64_t)id[u] << 1);
    }
}

// Score nn rows in passes of as many row sets as the remaining rows need, at
// most U, so a short list costs as many sets as it fills, not U.
template <bool F32, int CPL, int U, int LG, bool NRM = false>
__device__ __forceinline__ void eval_rows(const Idx& ix, const uint32_t* ids, int nn,
                                          uint64_t* keys, const uint4 (&qv)[CPL], uint32_t qq,
                                          const int lane, const int nch) {
    constexpr int G = 1 << LG, RPP = kWave >> LG;
    const int sub = lane & (G - 1), grp = lane >> LG;
    for (int r0 = 0; r0 < nn;) {
        const int sets = min(U, (nn - r0 + RPP - 1) / RPP);  // wave-uniform
        if constexpr (U >= 4) {
            if (sets == 4) {
                eval_pass<F32, CPL, (U >= 4 ? 4 : 1), LG, NRM>(ix, ids, nn, r0, keys, qv, qq, sub, grp, nch);
                r0 += 4 * RPP;
                continue;
            }
        }
        if constexpr (U >= 3) {
            if (sets == 3) {
                eval_pass<F32, CPL, (U >= 3 ? 3 : 1), LG, NRM>(ix, ids, nn, r0, keys, qv, qq, sub, grp, nch);
                r0 += 3 * RPP;
                continue;
            }
        }
        if constexpr (U >= 2) {
            if (sets == 2) {
                eval_pass<F32, CPL, (U >= 2 ? 2 : 1), LG, NRM>(ix, ids, nn, r0, keys, qv, qq, sub, grp, nch);
                r0 += 2 * RPP;
                continue;
            }
        }
        eval_pass<F32, CPL, 1, LG, NRM>(ix, ids, nn, r0, keys, qv, qq, sub, grp, nch);
        r0 += RPP;
    }
}

// ---------------------------------------------------------------------------
// forgetful visited cache: buckets of four 16-bit entries
// ---------------------------------------------------------------------------
// h = id * C mod 2^B is a bijection of [0, 2^B) (C odd).  With nb buckets,
// 2^vb <= nb < 2^(vb+1), the bucket is floor(h * nb / 2^B), and the entry is
// h's place in its bucket, r = h * nb mod 2^B, scaled to 1 + floor(r * 65535
// / 2^B) in [1, 65535] (0 marks an empty place).  Two values of h in one
// bucket have places at least nb apart, so their entries differ whenever
// nb * 65535 >= 2^B: always when B - vb <= 15, and with B - vb = 16 when
// nb > 2^vb.  (bucket, entry) then identifies the id exactly.  With hs =
// h * 2^(32 - B), one 32 x 32-bit product gives both: the bucket is the high
// word of hs * nb and r * 2^(32 - B) = lo its low word, and 1 + floor(lo *
// 65535 / 2^32) = q + [m > q or lo = 0] with q = lo >> 16, m = lo & 0xFFFF
// (65535 m - 65536 q >= 0 exactly then), all full-rate operations.  A
// bucket keeps its four most recent entries.
struct VisCache {
    uint64_t* b;
    int vb;      // floor(log2 nb)
    int B;       // hash width
    uint32_t nb;  // buckets
    // bucket and entry of hs = h * 2^(32 - B)
    __device__ __forceinline__ void place(uint32_t hs, uint32_t& bucket, uint32_t& e) const {
        const uint64_t p = (uint64_t)hs * nb;
        bucket = (uint32_t)(p >> 32);
        const uint32_t lo = (uint32_t)p, q = lo >> 16;
        e = q + (((lo & 0xFFFFu) > q || lo == 0u) ? 1u : 0u);
    }
    __device__ __forceinline__ bool test_insert(uint32_t id) const {
        uint32_t bucket, e;
        place((id * 0x9E3779B1u) << (32 - B), bucket, e);
        const uint64_t w = b[bucket];
        const bool hit = ((uint32_t)(w & 0xFFFFu) == e) | ((uint32_t)((w >> 16) & 0xFFFFu) == e) |
                         ((uint32_t)((w >> 32) & 0xFFFFu) == e) | ((uint32_t)(w >> 48) == e);
        if (!hit) b[bucket] = (w << 16) | e;
        return hit;
    }
    // Whole-wave form: lanes with nothing to insert (an invalid id, or a
    // hit) write the spare bucket nb instead of branching around the store.
    __device__ __forceinline__ bool test_insert_if(uint32_t id, bool valid) const {
        uint32_t bucket, e;
        place(((valid ? id : 0u) * 0x9E3779B1u) << (32 - B), bucket, e);
        const uint64_t w = b[bucket];
        const bool hit = ((uint32_t)(w & 0xFFFFu) == e) | ((uint32_t)((w >> 16) & 0xFFFFu) == e) |
                         ((uint32_t)((w >> 32) & 0xFFFFu) == e) | ((uint32_t)(w >> 48) == e);
        b[valid && !hit ? bucket : nb] = (w << 16) | e;
        return hit;
    }
};

// ---------------------------------------------------------------------------
// LDS layout of one wave in the search kernel
// ---------------------------------------------------------------------------
struct SearchLds {
    int ef_cap, st_cap, vb, xs, dp;
    bool own_w = true;   // false: W lives elsewhere; the layout keeps its spare entry only
    int xb = 0;          // visited buckets beyond 2^vb (fewer than 2^vb)
    bool w_last = false; // W after the visited buckets (the batch kernel)
    // Layout of one wave: [FP32 query | query codes | W | neighbour ids |
    // their keys | visited buckets], or with w_last [FP32 query | query
    // codes | neighbour ids | their keys | visited buckets | W].  W holds
    // keys whose low bit is the expanded flag.  Each array has one spare
    // entry past its end (W: index ef_cap; the neighbour ids: index st_cap,
    // which is the first key slot; the visited buckets: index 2^vb + xb):
    // lanes with nothing to store write there, so stores need no divergent
    // branch.  The query comes first so that the serving kernel can reuse
    // everything after it for Stages 2-3, from W on.  With W last, only W's
    // size depends on ef_cap, so waves with lists of two sizes share every
    // other offset; between the buckets and W lie two words of the wave's
    // work claims (off_claim) and a free word just below W.
    __host__ __device__ static size_t r16(size_t o) { return (o + 15) & ~(size_t)15; }
    __host__ __device__ size_t off_qf() const { return 0; }
    __host__ __device__ size_t off_qc() const { return (size_t)xs * 4; }
    __host__ __device__ size_t w_bytes() const { return own_w ? (size_t)(ef_cap + 1) * 8 : (size_t)8; }
    __host__ __device__ size_t off_st() const {
        return w_last ? r16(off_qc() + (size_t)dp) : r16(off_mk() + w_bytes());
    }
    __host__ __device__ size_t off_sk() const { return off_st() + (size_t)st_cap * 4; }
    __host__ __device__ size_t off_vis() const { return off_sk() + (size_t)st_cap * 8; }
    __host__ __device__ size_t vis_end() const {
        return r16(off_vis() + (size_t)8 * (((size_t)1 << vb) + xb) + 16);
    }
    __host__ __device__ size_t off_claim() const {
        return r16(off_vis() + (size_t)8 * (((size_t)1 << vb) + xb) + 8);
    }
    __host__ __device__ size_t off_mk() const {
        return w_last ? off_claim() + 16 : r16(off_qc() + (size_t)dp);
    }
    __host__ __device__ size_t bytes() const {
        return w_last ? r16(off_mk() + w_bytes()) : vis_end();
    }
};

__device__ __forceinline__ int st_cap_of(int s0, int s1) {
    return max(s0, s1) <= 64 ? 64 : ((max(s0, s1) + 63) / 64) * 64;
}

struct SearchArgs {
    Idx ix;
    const float* Q;
    int64_t nq;
    const int32_t* kq;
    const int32_t* efq;
    const int32_t* ncq;
    const int32_t* order;
    int32_t m_ef;
    int32_t ef_cap;
    int32_t out_stride;
    int32_t vb;
    int32_t xb;         // visited buckets beyond 2^vb
    int32_t nsw;        // waves per block with lists of ef_cap2 (the last nsw; 0: none)
    int32_t ef_cap2;
    size_t wave_lds2;   // LDS of such a wave
    int32_t mode;       // 0: Stage-1 candidates; 1: FP32 baseline top-k
    int32_t lg, nch;    // row geometry
    size_t wave_lds;
    uint32_t* out_id;
    uint32_t* out_D;    // mode 0: integer D; mode 1: FP32 distance bits
    int32_t* out_cnt;
    int32_t* counter;   // [0]: claims of positions [0, c); [1]: c; [2]: claims of [c, nq)
    Taps taps;
};

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Stage 1 of one valid query, run by the whole wave.
//
// The result list W (at most ef_cap keys, sorted, expanded flag in the low
// bit) lives in LDS.  A merge finds each admitted key's place in W by
// bisection (one lane per key), drops keys already in W, ranks the admitted
// keys among themselves, then shifts the W entries above the lowest insertion point
// slot by slot (64 entries per slot, last slot first) and writes the
// admitted keys into the gaps.  Only the slots at or above the lowest
// insertion point are touched, and W is never held in registers.
//
// Every branch that steers a loop is on a wave-uniform value (a ballot, a
// popcount or a readfirstlane), and every single-lane block is closed by a
// wave barrier before the next loop control, so all lanes stay converged at
// each cross-lane operation.
template <bool F32, int CPL, int U, int LG, bool TAPS, bool NRM = false>
__device__ __forceinline__ void search_query(const SearchArgs& a, const int64_t q, const int efe,
                                             const int nc, const int lane,
                                             const VisCache& vis, uint64_t* mk, uint64_t* spare,
                                             uint32_t* st_id, uint64_t* st_key, uint64_t* visb,
                                             float* qf, uint8_t* qc) {
    const Idx& ix = a.ix;
    const int st_cap = st_cap_of(ix.s0, ix.s1);  // index of the spare neighbour-id entry
    uint32_t qq = 0;
    if (!F32) {
        uint32_t part = 0;
        for (int j = lane; j < ix.dp; j += kWave) {
            uint32_t c = j < ix.d ? encode1(qf[j], ix.qmin[j], ix.qscale[j]) : 0u;
            qc[j] = (uint8_t)c;
            part += c * c;
        }
        qq = wave_sum_u32(part);
    }
    wsync();
    uint4 qv[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int ch = (lane & ((1 << LG) - 1)) + (c << LG);
        if (ch < a.nch)
            qv[c] = F32 ? reinterpret_cast<const uint4*>(qf)[ch]
                        : reinterpret_cast<const uint4*>(qc)[ch];
        else
            qv[c] = make_uint4(0u, 0u, 0u, 0u);
    }

    uint32_t n_exp = 0, n_eval = 0, n_up = 0, n_adm = 0, n_upx = 0;
    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();

    // ---- greedy descent through the upper layers (search width 1) ----
    uint32_t cur = ix.ep;
    if (lane == 0) st_id[0] = cur;
    wsync();
    eval_rows<F32, CPL, U, LG, NRM>(ix, st_id, 1, st_key, qv, qq, lane, a.nch);
    wsync();
    uint64_t curkey = uni64(st_key[0]);
    for (int l = ix.L; l >= 1; --l) {
        for (;;) {
            const uint32_t* row = ix.uadj + ((int64_t)ix.ubase[cur] + (l - 1)) * ix.s1;
            int cnt = 0;
            for (int b0 = 0; b0 < ix.s1; b0 += kWave) {
                uint32_t e = (b0 + lane < ix.s1) ? row[b0 + lane] : kNone;
                uint64_t m = ballot(e != kNone);
                st_id[e != kNone ? cnt + below(m) : st_cap] = e;
                cnt += __popcll(m);
            }
            wsync();
            eval_rows<F32, CPL, U, LG, NRM>(ix, st_id, cnt, st_key, qv, qq, lane, a.nch);
            wsync();
            n_up += cnt;
            ++n_upx;
            uint64_t best = ~0ull;
            for (int j = lane; j < cnt; j += kWave) best = min(best, st_key[j]);
            best = uni64(wave_min_u64(best));
            if (best < curkey) {
                curkey = best;
                cur = (uint32_t)best >> 1;
            } else {
                break;
            }
        }
    }


    // ---- layer-0 search with width efe ----
    for (int i = lane; i < (int)vis.nb; i += kWave) visb[i] = 0ull;
    wsync();
    if (lane == 0) {
        vis.test_insert((uint32_t)curkey >> 1);
        mk[0] = curkey;
    }
    wsync();
    int wsize = 1;
    int first = 0;
    const int nad = (ix.s0 + kWave - 1) / kWave;  // 64-entry chunks of an adjacency row (<= 4)
    // Speculative adjacency (rows of at most 128 entries): each pop also loads
    // the row of the next unexpanded entry of W after the popped one, and
    // parks it in the neighbour-id array once the expansion no longer needs
    // that array.  When no admitted key lands before that entry, it is the
    // next pop and its row is read from LDS, so the expansion waits for one
    // dependent global round trip (the code rows) instead of two.  Adjacency
    // rows never change during a search, so the results are the same either
    // way.
    uint32_t spec = kNone;
    for (;;) {
        // nearest unexpanded entry of W, and the one after it
        int idx = -1, sidx = -1;
        uint64_t kc = 0, ks = 0;
        for (int b0 = first & ~(kWave - 1); b0 < wsize; b0 += kWave) {
            const int i = b0 + lane;
            const uint64_t w = mk[i];  // inside W's capacity (whole 64-entry slots)
            uint64_t m = ballot(i >= first && i < wsize && (w & 1ull) == 0);
            if (m) {
                const int t = (int)__builtin_ctzll(m);
                idx = b0 + t;
                kc = readlane64(w, t);
                m &= m - 1;
                if (m) {
                    const int t2 = (int)__builtin_ctzll(m);
                    sidx = b0 + t2;
                    ks = readlane64(w, t2);
                } else if (b0 + kWave < wsize) {
                    // b0 + kWave < wsize <= ef_cap, a multiple of 64: this
                    // slot lies inside W's capacity too
                    const int i2 = b0 + kWave + lane;
                    const uint64_t w2 = mk[i2];
                    const uint64_t m2 = ballot(i2 < wsize && (w2 & 1ull) == 0);
                    if (m2) {
                        const int t2 = (int)__builtin_ctzll(m2);
                        sidx = b0 + kWave + t2;
                        ks = readlane64(w2, t2);
                    }
                }
                break;
            }
        }
        idx = uni(idx);
        if (idx < 0) break;
        sidx = uni(sidx);
        const uint32_t c = (uint32_t)kc >> 1;
        const uint32_t cn = sidx >= 0 ? (uint32_t)ks >> 1 : kNone;
        first = idx + 1;
        wsync();
        mk[idx] = kc | 1ull;  // expanded; every lane stores the same value
        if (TAPS && lane == 0 && a.taps.expanded && (int)n_exp < a.taps.cap)
            a.taps.expanded[q * a.taps.cap + n_exp] = c;
        wsync();
        ++n_exp;
        // unvisited neighbours of c
        const uint32_t* row = ix.adj0 + (int64_t)c * ix.s0;
        uint32_t e[4];
        uint32_t nxt = kNone, nxt1 = kNone;  // the speculative row, in flight
        if (nad == 1) {
            const int j = lane < ix.s0 ? lane : 0;
            // (the parked row is stored masked, so the two paths differ and
            // are not folded into one flat load, which would wait for both)
            if (uni(spec == c ? 1 : 0))
                e[0] = st_id[lane];  // parked by the previous expansion
            else
                e[0] = lane < ix.s0 ? row[j] : kNone;
            // issued after c's row on both paths (c's own row again when W
            // holds no further unexpanded entry): waiting for c's row leaves
            // this load outstanding
            nxt = ix.adj0[(int64_t)(cn != kNone ? cn : c) * ix.s0 + j];
            spec = cn;
            e[1] = e[2] = e[3] = kNone;
        } else if (nad == 2) {
            // rows of 65..128 entries: the same in two 64-entry chunks; every
            // lane's first-chunk entry lies inside the row
            const int j1 = kWave + lane;
            const int j1c = j1 < ix.s0 ? j1 : 0;
            if (uni(spec == c ? 1 : 0)) {
                e[0] = st_id[lane];
                e[1] = st_id[j1];
            } else {
                e[0] = lane < ix.s0 ? row[lane] : kNone;
                e[1] = j1 < ix.s0 ? row[j1c] : kNone;
            }
            const uint32_t* nrow = ix.adj0 + (int64_t)(cn != kNone ? cn : c) * ix.s0;
            nxt = nrow[lane];
            nxt1 = nrow[j1c];
            spec = cn;
            e[2] = e[3] = kNone;
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = b * kWave + lane;
                const uint32_t v = b < nad ? row[j < ix.s0 ? j : 0] : kNone;
                e[b] = j < ix.s0 ? v : kNone;
            }
        }
        int nn = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (b < nad) {
                const bool valid = e[b] != kNone;
                const bool isnew = !vis.test_insert_if(e[b], valid) && valid;
                const uint64_t m = ballot(isnew);
                st_id[isnew ? nn + below(m) : st_cap] = e[b];
                nn += __popcll(m);
            }
        }
        wsync();
        nn = uni(nn);
        // park the speculative row in the neighbour-id array (st_cap >= 64 *
        // nad), masked past the row
        auto park = [&]() {
            if (nad <= 2) st_id[lane] = lane < ix.s0 ? nxt : kNone;
            if (nad == 2) st_id[kWave + lane] = kWave + lane < ix.s0 ? nxt1 : kNone;
        };
        if (nn == 0) {
            park();
            wsync();
            continue;
        }
        if (TAPS && a.taps.evaluated) {
            for (int j = lane; j < nn; j += kWave) {
                const int p = (int)n_eval + j;
                if (p < a.taps.cap) a.taps.evaluated[q * a.taps.cap + p] = st_id[j];
            }
        }
        n_eval += nn;
        eval_rows<F32, CPL, U, LG, NRM>(ix, st_id, nn, st_key, qv, qq, lane, a.nch);
        wsync();
        // the neighbour ids are consumed: park the speculative row there (the
        // code rows were issued after it, so it has arrived)
        park();
        // merge the scored neighbours, 64 at a time
        for (int b0 = 0; b0 < nn; b0 += kWave) {
            const uint64_t bound = wsize == efe ? uni64(mk[efe - 1]) : ~0ull;
            const int j = b0 + lane;
            const uint64_t key = j < nn ? st_key[j] : ~0ull;
            uint64_t A = ballot(key < bound);
            if (A == 0) continue;
            // entries of W below the key, by bisection of the sorted list:
            // the key's count lies in [lo, lo + n] and n shrinks by its
            // half each step (the same on every lane), so every read is
            // inside W and no lane branches.  (Narrowing to a 64-entry slot
            // first, by the slot heads, or a 4-way search with independent
            // reads, cost more issue slots than the dependent reads they
            // saved: the merge is bound by the instructions the waves of a
            // SIMD share, not by the latency of one chain.)
            int lo = 0;
            for (int n = wsize; n > 1;) {
                const int half = n >> 1;
                lo = mk[lo + half] < key ? lo + half : lo;
                n -= half;
            }
            // The last step reads W[lo] and W[lo + 1] together (lo + 1 <=
            // wsize: inside W, or the LDS word just past W's capacity, whose
            // value is not used since lo + 1 == wsize leaves lo == wsize).
            // The entry at the key's place shows whether the key is already
            // in W (a node the visited cache forgot); such a key is dropped.
            const uint64_t w0 = mk[lo], w1 = mk[lo + 1];
            const bool past = w0 < key;
            lo += past ? 1 : 0;
            const uint64_t wl = past ? w1 : w0;
            A &= ~ballot(lo < wsize && (wl | 1ull) == (key | 1ull));
            const int m_adm = __popcll(A);
            if (m_adm == 0) continue;
            n_adm += m_adm;
            const bool mine = ((A >> lane) & 1ull) != 0;
            int rankA = 0;
            int lo_min = INT_MAX, lo_max = -1;
            for (uint64_t it = A; it != 0; it &= it - 1) {
                const int t = (int)__builtin_ctzll(it);
                rankA += readlane64(key, t) < key ? 1 : 0;
                const int lt = __builtin_amdgcn_readlane(lo, t);
                lo_min = min(lo_min, lt);
                lo_max = max(lo_max, lt);
            }
            const int pos = lo + rankA;
            // W entry i moves up by the number of admitted keys with lower
            // bound <= i.  Slots are moved from the last one down: an entry
            // only moves up and past the slots already moved.  Each slot is
            // read whole before it is written, and the slot below is read
            // before this one is written (this slot's entries land at or
            // above its own start, so the slot below is not overwritten).
            wsync();
            const int sl_lo = lo_min >> 6;
            int sl = (wsize - 1) >> 6;
            uint64_t wn = mk[sl * kWave + lane];  // inside W's capacity
            for (; sl >= sl_lo; --sl) {
                const int i = sl * kWave + lane;
                const bool v = i < wsize && i >= lo_min;
                const uint64_t w = wn;
                if (sl > sl_lo) wn = mk[i - kWave];
                // a slot wholly above every insertion point moves by m_adm;
                // otherwise: the keys placed below the slot, then those of
                // the keys placed inside it that lie at or below the entry
                int sh = m_adm;
                if (lo_max > sl * kWave) {
                    sh = __popcll(ballot(mine && lo < sl * kWave));
                    for (uint64_t it = ballot(mine && (lo >> 6) == sl); it != 0; it &= it - 1)
                        sh += __builtin_amdgcn_readlane(lo, (int)__builtin_ctzll(it)) <= i ? 1 : 0;
                }
                const int p = i + sh;
                uint64_t* dst = v && p < efe ? mk + p : spare;  // others write the spare entry
                *dst = w;
            }
            uint64_t* dst = mine && pos < efe ? mk + pos : spare;
            *dst = key;
            // the smallest admitted key has rank 0: its position is lo_min
            first = min(first, lo_min);
            wsize = min(efe, wsize + m_adm);
            wsync();
        }
    }

    // ---- outputs ----
    const int cnt = min(nc, wsize);
    if (a.mode == 2) {
        // serving: the caller reads the first cnt keys of W from LDS
        wsync();
        if (lane == 0) *reinterpret_cast<int*>(st_id) = cnt;
        wsync();
    } else if (a.mode == 0) {
        for (int i = lane; i < cnt; i += kWave) {
            const uint64_t key = mk[i];
            a.out_id[q * a.out_stride + i] = (uint32_t)key >> 1;
            a.out_D[q * a.out_stride + i] = (uint32_t)(key >> 32);
        }
        if (lane == 0) a.out_cnt[q] = cnt;
    } else {
        for (int i = lane; i < a.out_stride; i += kWave) {
            const bool v = i < cnt;
            const uint64_t key = v ? mk[i] : ~0ull;
            a.out_id[q * a.out_stride + i] = v ? (uint32_t)key >> 1 : kNone;
            a.out_D[q * a.out_stride + i] = v ? (uint32_t)(key >> 32) : 0x7F800000u;
        }
    }
    if (TAPS && a.taps.counts && lane == 0) {
        const uint64_t t_end = __builtin_amdgcn_s_memrealtime();
        uint32_t* cq = a.taps.counts + q * 8;
        cq[0] = n_exp;
        cq[1] = n_eval;
        cq[2] = n_up;
        cq[3] = n_adm;
        cq[4] = n_upx;
        cq[5] = (uint32_t)(t_end - t_start);
        cq[6] = (uint32_t)t_start;
        cq[7] = (uint32_t)(t_start >> 32);
    }
}

// Register budget: seven waves per SIMD for code rows of up to 16 chunks (a
// few spilled values cost less than the lost wave), five when four row sets
// are in flight; wider rows and the FP32 rows keep the compiler's choice.
template <bool F32, int CPL, int U, int LG>
constexpr int search_waves_per_eu() { return !F32 && (CPL << LG) <= 16 ? (U >= 4 ? 5 : 7) : 1; }

template <bool F32, int CPL, int U, int LG, bool TAPS, bool NRM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(search_waves_per_eu<F32, CPL, U, LG>())))
void k_search(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const Idx& ix = a.ix;
    // With two list sizes the block's last nsw waves hold lists of ef_cap2
    // and follow the others in LDS.
    const int nbw = (int)(blockDim.x / kWave) - a.nsw;
    const bool small = wave >= nbw;
    const int ef_cap = small ? a.ef_cap2 : a.ef_cap;
    // The 8-bit search encodes the query straight from global memory, so its
    // layout has no FP32 query (xs 0); the FP32 search keeps it in LDS.
    const SearchLds L{ef_cap, st_cap_of(ix.s0, ix.s1), a.vb, F32 ? ix.xs : 0, ix.dp, true, a.xb, true};
    unsigned char* base = smem + (small ? (size_t)nbw * a.wave_lds + (size_t)(wave - nbw) * a.wave_lds2
                                        : (size_t)wave * a.wave_lds);
    uint64_t* mk = reinterpret_cast<uint64_t*>(base + L.off_mk());
    uint32_t* st_id = reinterpret_cast<uint32_t*>(base + L.off_st());
    uint64_t* st_key = reinterpret_cast<uint64_t*>(base + L.off_sk());
    uint64_t* visb = reinterpret_cast<uint64_t*>(base + L.off_vis());
    float* qlds = reinterpret_cast<float*>(base + L.off_qf());
    uint8_t* qc = base + L.off_qc();

    VisCache vis{visb, a.vb, max(ix.idbits, a.vb + 1), (1u << a.vb) + (uint32_t)a.xb};

    // Work: positions [0, c) of the order (the queries with lists above
    // ef_cap2) go to the waves with lists of ef_cap, from counter[0]; the
    // rest, [c, nq), to every wave once it has no other work, from
    // counter[2].  Without two sizes, or when the order is not split at c
    // (c < 0), the ef_cap waves take everything from counter[0] and the
    // others leave.  The claim state lives in two LDS words of the wave, so
    // that no register carries it across the search: claim[0] = r >= 0
    // while claiming [0, r) from counter[0], -(c + 1) once claiming [c, nq)
    // from counter[2]; claim[1] = the wave's list capacity.  Every lane
    // stores the same values.
    int* claim = reinterpret_cast<int*>(base + L.off_claim());
    {
        int r0 = (int)a.nq;
        if (a.nsw > 0) {
            const int cs = uni(a.counter[1]);
            if (cs < 0 && small) return;  // the whole wave
            r0 = cs < 0 ? (int)a.nq : small ? -(cs + 1) : cs;
        }
        claim[0] = r0;
        claim[1] = ef_cap;
        wsync();
    }
    for (;;) {
        // Every lane takes part in the work-counter atomic (only lane 0 adds
        // one) and lane 0's old value is read with readfirstlane: no divergent
        // branch precedes this cross-lane read, and the branches below that
        // steer the loop are on wave-uniform values.
        const int r = uni(claim[0]);
        int w;
        if (r >= 0) {
            w = uni(atomicAdd(a.counter, lane == 0 ? 1 : 0));
            if (w >= r) {
                if (a.nsw == 0 || r == (int)a.nq) break;
                claim[0] = -(r + 1);
                wsync();
                continue;
            }
        } else {
            w = -r - 1 + uni(atomicAdd(a.counter + 2, lane == 0 ? 1 : 0));
            if ((int64_t)w >= a.nq) break;
        }
        const int64_t q = a.order ? (int64_t)a.order[w] : (int64_t)w;
        if (uni((q >= 0 && q < a.nq) ? 1 : 0)) {  // skip entries outside [0, nq)
            const int k = a.kq[q];
            const int ef = a.efq[q];
            const int efe = max(ef, k);
            int nc;
            if (a.mode == 0) {
                if (a.ncq)
                    nc = a.ncq[q];
                else
                    nc = min(max(efe / a.m_ef, k), efe);
            } else {
                nc = k;
            }
            const int cap = uni(claim[1]);
            int bad =
                uni((k < 1 || efe > cap || nc < 1 || nc > a.out_stride || nc > efe) ? 1 : 0);
            float* qf = F32 ? qlds : const_cast<float*>(a.Q + q * ix.d);
            if (!bad) {
                // reject non-finite values; the FP32 search copies the query
                // into LDS (zero padded)
                bool nonfinite = false;
                for (int j = lane; j < ix.xs; j += kWave) {
                    const float v = j < ix.d ? a.Q[q * ix.d + j] : 0.0f;
                    nonfinite |= !__builtin_isfinite(v);
                    if (F32) qf[j] = v;
                }
                bad = uni(ballot(nonfinite) != 0 ? 1 : 0);
            }
            if (bad) {
                if (a.mode == 0) {
                    if (lane == 0) a.out_cnt[q] = -1;
                } else {
                    for (int t = lane; t < a.out_stride; t += kWave) {
                        a.out_id[q * a.out_stride + t] = kNone;
                        a.out_D[q * a.out_stride + t] = 0x7F800000u;
                    }
                }
            } else {
                // lanes with nothing to store in W write the free word below it
                search_query<F32, CPL, U, LG, TAPS, NRM>(a, q, efe, nc, lane, vis, mk, mk - 1,
                                                    st_id, st_key, visb, qf, qc);
            }
        }
        wsync();
    }
}

// Batched build: write changed layer-0 rows (width entries each) into the
// device adjacency (row stride s0); rows[] are node ids below n, checked on
// the host.
__global__ void k_scatter_rows(uint32_t* adj0, int32_t s0, const uint32_t* rows,
                               const uint32_t* data, int32_t nrows, int32_t width) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nrows * width) return;
    const int64_t r = i / width, c = i - r * width;
    adj0[(int64_t)rows[r] * s0 + c] = data[i];
}

// Batched build: the neighbour heuristic of the insertion step (Alg. 1's
// HNSW construction) for every point of a chunk, one wave per point.  The
// candidates of point b are cand_id / cand_D[b * stride + t], t < cnt[b]:
// ascending keys (D, id), D = |x - x_b|^2 over the codes.  Candidate e is
// kept when no point s kept before it has |x_e - x_s|^2 < D_e, until M are
// kept.  Lane t holds the t-th kept id and computes |x_e - x_s|^2 over the
// d_pad code bytes as |x_e|^2 + |x_s|^2 - 2 x_e.x_s, the integer the host
// heuristic computes (below 2^32 for d_pad <= 66,000).  M <= 64.
__global__ __launch_bounds__(256) void k_select(Idx ix, const uint32_t* cand_id,
                                                const uint32_t* cand_D, const int32_t* cnt,
                                                int32_t nb, int32_t stride, int32_t M,
                                                uint32_t* sel, int32_t* nsel) {
    const int lane = lane_id();
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (b >= nb) return;  // the whole wave
    const int nch = ix.dp / 16;
    const int c = min(max(cnt[b], 0), stride);
    uint32_t s = kNone;  // this lane's kept id (lanes below r)
    uint32_t ss = 0;     // its |x_s|^2
    int r = 0;
    for (int i = 0; i < c && r < M; ++i) {
        const uint32_t e = cand_id[b * stride + i];  // one address on every lane
        const uint32_t de = cand_D[b * stride + i];
        const uint4* xe = reinterpret_cast<const uint4*>(ix.codes + (uint64_t)e * (uint32_t)ix.cs);
        const uint4* xs =
            reinterpret_cast<const uint4*>(ix.codes + (uint64_t)(lane < r ? s : e) * (uint32_t)ix.cs);
        uint32_t ee = 0u, es = 0u;
        for (int ch = 0; ch < nch; ++ch) {
            const uint4 a = xe[ch], q = xs[ch];
            ee = dot4(a.x, a.x, ee);
            ee = dot4(a.y, a.y, ee);
            ee = dot4(a.z, a.z, ee);
            ee = dot4(a.w, a.w, ee);
            es = dot4(a.x, q.x, es);
            es = dot4(a.y, q.y, es);
            es = dot4(a.z, q.z, es);
            es = dot4(a.w, q.w, es);
        }
        const bool closer = lane < r && ee + ss - 2u * es < de;
        if (ballot(closer) == 0) {  // wave-uniform
            if (lane == r) {
                s = e;
                ss = ee;
            }
            ++r;
        }
    }
    if (lane < M) sel[b * M + lane] = lane < r ? s : kNone;
    if (lane == 0) nsel[b] = r;
}

__global__ void k_reset(int32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Two list sizes: c = the number of queries with ef_eff = max(ef, k) above
// ef_small; counter[1] = c when the order lists exactly those queries first
// (positions [0, c)), else -1; both claim counters start at zero.  One block.
__global__ __launch_bounds__(1024) void k_split(const int32_t* kq, const int32_t* efq,
                                                 const int32_t* order, int64_t nq,
                                                 int32_t ef_small, int32_t* counter) {
    __shared__ int32_t cnt[2];
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    int big = 0;
    for (int64_t q = threadIdx.x; q < nq; q += blockDim.x)
        big += max(efq[q], kq[q]) > ef_small ? 1 : 0;
    atomicAdd(&cnt[0], big);
    __syncthreads();
    const int64_t c = cnt[0];
    int placed = 0;  // positions below c that hold such a query
    for (int64_t w = threadIdx.x; w < c; w += blockDim.x) {
        const int64_t q = order ? (int64_t)order[w] : w;
        placed += (q >= 0 && q < nq && max(efq[q], kq[q]) > ef_small) ? 1 : 0;
    }
    atomicAdd(&cnt[1], placed);
    __syncthreads();
    if (threadIdx.x == 0) {
        counter[0] = 0;
        counter[1] = cnt[1] == cnt[0] ? cnt[0] : -1;
        counter[2] = 0;
    }
}

// ---------------------------------------------------------------------------
// Batched build, reverse links on the device (lists of 2M <= 63 entries)
// ---------------------------------------------------------------------------
// Chunk point b takes its own layer-0 list (its nsel[b] selections, the rest
// empty), and every link x <- ids[b] of its selections is listed as key x,
// value b * M + t: in the order the links are made.  Unused entries get key
// kNone and sort last.
__global__ void k_link_prep(uint32_t* adj0, int32_t s0, int32_t cap, const uint32_t* ids,
                            const uint32_t* sel, const int32_t* nsel, int32_t nb, int32_t M,
                            uint32_t* lkey, uint32_t* lval) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)nb * M) {
        const int64_t b = i / M;
        const int t = (int)(i - b * M);
        lkey[i] = t < nsel[b] ? sel[i] : kNone;
        lval[i] = (uint32_t)i;
    }
    if (i < (int64_t)nb * cap) {
        const int64_t b = i / cap;
        const int j = (int)(i - b * cap);
        adj0[(int64_t)ids[b] * s0 + j] = (j < M && j < nsel[b]) ? sel[b * M + j] : kNone;
    }
}

// Start of each run of equal targets in the sorted link keys (any order).
__global__ void k_link_heads(const uint32_t* key, int64_t N, int32_t* seg, int32_t* nseg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t x = key[i];
    if (x != kNone && (i == 0 || key[i - 1] != x)) seg[atomicAdd(nseg, 1)] = (int32_t)i;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = shfl_xor_u32((uint32_t)v, m), hi = shfl_xor_u32((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of one 64-bit key per lane, ascending by lane.
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t k, int lane) {
    for (int size = 2; size <= kWave; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint64_t o = shfl_xor_u64(k, stride);
            const bool up = (lane & size) == 0, low = (lane & stride) == 0;
            k = (low == up) ? (o < k ? o : k) : (o > k ? o : k);
        }
    return k;
}

// |x_a|^2 and x_a.x_b over the d_pad code bytes (rows at stride cs).
__device__ __forceinline__ void code_dots(const Idx& ix, uint32_t a, uint32_t b, uint32_t& aa,
                                          uint32_t& ab) {
    const uint4* xa = reinterpret_cast<const uint4*>(ix.codes + (uint64_t)a * (uint32_t)ix.cs);
    const uint4* xb = reinterpret_cast<const uint4*>(ix.codes + (uint64_t)b * (uint32_t)ix.cs);
    aa = 0u;
    ab = 0u;
    for (int ch = 0; ch < ix.dp / 16; ++ch) {
        const uint4 p = xa[ch], q = xb[ch];
        aa = dot4(p.x, p.x, aa);
        aa = dot4(p.y, p.y, aa);
        aa = dot4(p.z, p.z, aa);
        aa = dot4(p.w, p.w, aa);
        ab = dot4(p.x, q.x, ab);
        ab = dot4(p.y, q.y, ab);
        ab = dot4(p.z, q.z, ab);
        ab = dot4(p.w, q.w, ab);
    }
}

// One wave per target x (the runs found by k_link_heads, taken from a work
// counter): lane j holds entry j of x's list; the links into x are applied
// in the order they were made, as the host does one by one: a self link or
// an id already listed is skipped, a list with room takes the id at its end,
// and a full list of cap entries is shrunk with the heuristic over its
// entries and the new id, keyed (|x_e - x_x|^2, e) ascending.
__global__ __launch_bounds__(256) void k_link(Idx ix, uint32_t* adj0, int32_t s0, int32_t cap,
                                              const uint32_t* ids, int32_t M,
                                              const uint32_t* key, const uint32_t* val, int64_t N,
                                              const int32_t* seg, const int32_t* nseg,
                                              int32_t* counter) {
    const int lane = lane_id();
    const int ns = uni(*nseg);
    for (;;) {
        const int got = atomicAdd(counter, lane == 0 ? 1 : 0);
        const int s = uni(got);
        if (s >= ns) break;
        const int64_t i0 = seg[s];
        const uint32_t x = (uint32_t)uni((int)key[i0]);
        uint32_t r = lane < cap ? adj0[(int64_t)x * s0 + lane] : kNone;
        int cnt = __popcll(ballot(r != kNone));
        uint32_t xx, unused;
        code_dots(ix, x, x, xx, unused);
        for (int64_t i = i0; i < N; ++i) {
            if (uni(key[i] != x ? 1 : 0)) break;
            const uint32_t y = (uint32_t)uni((int)ids[val[i] / (uint32_t)M]);
            if (y == x) continue;
            if (ballot(r == y) != 0) continue;
            if (cnt < cap) {
                if (lane == cnt) r = y;
                ++cnt;
                continue;
            }
            // full: the cap entries and y (lane cap), keyed by distance to x
            const uint32_t e = lane < cap ? r : (lane == cap ? y : x);
            uint32_t ee, ex;
            code_dots(ix, e, x, ee, ex);
            uint64_t k = lane <= cap ? ((uint64_t)(ee + xx - 2u * ex) << 32) | e : ~0ull;
            k = wave_sort_u64(k, lane);
            uint32_t kept = kNone, kn = 0u;
            int rr = 0;
            for (int c = 0; c <= cap && rr < cap; ++c) {
                const uint64_t kc = readlane64(k, c);
                const uint32_t ec = (uint32_t)kc, dc = (uint32_t)(kc >> 32);
                uint32_t cc, cs;
                code_dots(ix, ec, lane < rr ? kept : ec, cc, cs);
                const bool closer = lane < rr && cc + kn - 2u * cs < dc;
                if (ballot(closer) == 0) {
                    if (lane == rr) {
                        kept = ec;
                        kn = cc;
                    }
                    ++rr;
                }
            }
            r = lane < rr ? kept : kNone;
            cnt = rr;
        }
        if (lane < cap) adj0[(int64_t)x * s0 + lane] = r;
    }
}

constexpr int kOrderMaxEf = 1024;

// Work order of a batch, longest first: queries sorted by ef_eff = max(ef, k)
// descending (a counting sort over ef_eff clamped to [0, 1024], one block).
// The order inside one ef_eff value follows the slot claims; no result
// depends on it.
__global__ __launch_bounds__(1024) void k_order(const int32_t* kq, const int32_t* efq,
                                                 int64_t nq, int32_t* order) {
    __shared__ int32_t bin[kOrderMaxEf + 1];
    for (int i = threadIdx.x; i <= kOrderMaxEf; i += blockDim.x) bin[i] = 0;
    __syncthreads();
    for (int64_t q = threadIdx.x; q < nq; q += blockDim.x) {
        const int e = min(max(max(efq[q], kq[q]), 0), kOrderMaxEf);
        atomicAdd(&bin[kOrderMaxEf - e], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i <= kOrderMaxEf; ++i) {
            const int c = bin[i];
            bin[i] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int64_t q = threadIdx.x; q < nq; q += blockDim.x) {
        const int e = min(max(max(efq[q], kq[q]), 0), kOrderMaxEf);
        const int slot = atomicAdd(&bin[kOrderMaxEf - e], 1);
        order[slot] = (int32_t)q;
    }
}

__global__ void k_encode(Idx ix, const float* Q, int64_t nq, uint8_t* out) {
    const int64_t q = blockIdx.x;
    if (q >= nq) return;
    for (int j = threadIdx.x; j < ix.dp; j += blockDim.x) {
        uint32_t c = 0;
        if (j < ix.d) c = encode1(Q[q * ix.d + j], ix.qmin[j], ix.qscale[j]);
        out[q * ix.dp + j] = (uint8_t)c;
    }
}

// ---------------------------------------------------------------------------
// re-rank: Stage 2 (asymmetric), early termination, Stage 3 (exact), assembly
// ---------------------------------------------------------------------------

struct RerankArgs {
    Idx ix;
    const float* Q;
    int64_t nq;
    const uint32_t* cid;
    const int32_t* ccnt;
    int32_t nc_stride;
    int32_t nc_cap;
    int32_t r_cap;
    const int32_t* kq;
    int32_t n_rerank;
    int32_t out_stride;
    float tau_gap, tau_ratio, eps;
    int32_t force_et;
    int32_t assembly;    // 0: fill from A while fewer than k; 1: union with the rest of A
    int32_t lg8, nch8;   // geometry of code rows
    int32_t lgf, nchf;   // geometry of FP32 rows
    size_t wave_lds;
    int32_t* out_id;
    float* out_dist;
    uint8_t* out_kind;
    RTaps taps;
};

struct RerankLds {
    int nc_cap, r_cap, xs;
    __host__ __device__ size_t bytes() const {
        size_t o = 0;
        o += (size_t)nc_cap * 8 * 2;   // A keys, sorted A
        o += (size_t)r_cap * 8 * 2;    // R keys, sorted R
        o += (size_t)r_cap * 2;        // kinds
        o += (size_t)nc_cap * 4;       // ids staging
        o = (o + 15) & ~(size_t)15;
        o += (size_t)xs * 4;           // FP32 query
        return (o + 15) & ~(size_t)15;
    }
};

// Asymmetric partial over one 16-code chunk: decode x~ = fl32(code / scale) + min
// (IEEE division), then sum (q - x~)^2 by fused multiply-add.
__device__ __forceinline__ float asym_chunk(uint4 x, const float (&qr)[16], const float (&mr)[16],
                                            const float (&sr)[16]) {
    float acc = 0.0f;
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const float code = (float)((w[t >> 2] >> (8 * (t & 3))) & 0xFFu);
        const float xt = code / sr[t] + mr[t];
        const float df = qr[t] - xt;
        acc = __builtin_fmaf(df, df, acc);
    }
    return acc;
}

// Stages 2-3, early termination and assembly for one query, run by the
// whole wave.  qf: the FP32 query (xs floats, LDS); ids: the nc Stage-1
// candidates (LDS); A, As, Rk, Rs, kind, kinds: LDS scratch; outputs are
// the query's rows (out_stride entries) and optional taps.
template <int CPL8, int CPLF, bool SYS = false>
__device__ __forceinline__ void rerank_query(const RerankArgs& a, const int lane, const int k,
                                             int nc, const float* qf, const uint32_t* ids,
                                             uint64_t* A, uint64_t* As, uint64_t* Rk,
                                             uint64_t* Rs, uint8_t* kind, uint8_t* kinds,
                                             int32_t* out_id, float* out_dist, uint8_t* out_kind,
                                             const int out_stride, uint32_t* a_id_out,
                                             float* a_dist_out, uint8_t* et_out,
                                             int32_t* nrr_out) {
    const Idx& ix = a.ix;
    // Stage 2: d^a on decoded codes, G8 lanes per code row
    {
        const Geo g = make_geo(a.lg8, a.nch8, lane);
        float qr[CPL8][16], mr[CPL8][16], sr[CPL8][16];
#pragma unroll
        for (int c = 0; c < CPL8; ++c) {
            const int ch = g.sub + c * g.G;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = ch * 16 + t;
                // padded dimensions (d <= j < d_pad) contribute exactly zero:
                // code 0 decodes to 0 with min 0, against a query value of 0
                const bool in = ch < g.nch && j < ix.d;
                qr[c][t] = in ? qf[j] : 0.0f;
                mr[c][t] = in ? ix.qmin[j] : 0.0f;
                sr[c][t] = in ? ix.qscale[j] : 1.0f;
            }
        }
        for (int r0 = 0; r0 < nc; r0 += g.rpp) {
            const int r = r0 + g.grp;
            const uint32_t id = r < nc ? ids[r] : kNone;
            float s = 0.0f;
#pragma unroll
            for (int c = 0; c < CPL8; ++c) {
                const int ch = g.sub + c * g.G;
                if (id != kNone && ch < g.nch) {
                    const uint4 x =
                        reinterpret_cast<const uint4*>(ix.codes + (int64_t)id * ix.cs)[ch];
                    s += asym_chunk(x, qr[c], mr[c], sr[c]);
                }
            }
            s = group_sum_f32(s, g.G);
            if (g.sub == 0 && r < nc) A[r] = ((uint64_t)__float_as_uint(s) << 32) | id;
        }
    }
    wsync();
    // sort A by (d^a, id): rank by counting
    for (int i = lane; i < nc; i += kWave) {
        const uint64_t v = A[i];
        int r = 0;
        for (int t = 0; t < nc; ++t) r += A[t] < v ? 1 : 0;
        As[r] = v;
    }
    wsync();
    // early termination (Section 3.2, Algorithm 2)
    int et = 0;
    if (nc > k) {
        const float dk = __uint_as_float((uint32_t)(As[k - 1] >> 32));
        const float dk1 = __uint_as_float((uint32_t)(As[k] >> 32));
        const float gap = (dk1 - dk) / (dk + a.eps);
        const float ratio = dk1 / (dk + a.eps);
        et = (gap > a.tau_gap) || (ratio > a.tau_ratio);
    }
    if (a.force_et >= 0) et = a.force_et != 0;
    et = uni(et);
    const int want = et ? k : max(a.n_rerank, k);
    const int nrr = uni(min(nc, want));
    // Stage 3: exact FP32 distances on A[0..nrr), GF lanes per row
    {
        const Geo g = make_geo(a.lgf, a.nchf, lane);
        uint4 qv[CPLF];
#pragma unroll
        for (int c = 0; c < CPLF; ++c) {
            const int ch = g.sub + c * g.G;
            qv[c] = ch < g.nch ? reinterpret_cast<const uint4*>(qf)[ch] : make_uint4(0, 0, 0, 0);
        }
        for (int r0 = 0; r0 < nrr; r0 += g.rpp) {
            const int r = r0 + g.grp;
            const uint32_t id = r < nrr ? (uint32_t)As[r] : kNone;
            float s = 0.0f;
#pragma unroll
            for (int c = 0; c < CPLF; ++c) {
                const int ch = g.sub + c * g.G;
                if (id != kNone && ch < g.nch)
                    s += Rows<true>::part(Rows<true>::load(ix, id, ch), qv[c]);
            }
            s = group_sum_f32(s, g.G);
            if (g.sub == 0 && r < nrr) {
                Rk[r] = ((uint64_t)__float_as_uint(s) << 32) | id;
                kind[r] = 1;
            }
        }
    }
    // assembly: fill from A while fewer than k, or (union) join every
    // remaining candidate of A with its d^a; R holds at most nc entries
    const int fill = a.assembly == 1 ? nc - nrr : max(0, min(nc - nrr, k - nrr));
    for (int t = lane; t < fill; t += kWave) {
        Rk[nrr + t] = As[nrr + t];
        kind[nrr + t] = 2;
    }
    const int nr = nrr + fill;
    wsync();
    for (int i = lane; i < nr; i += kWave) {
        const uint64_t v = Rk[i];
        int r = 0;
        for (int t = 0; t < nr; ++t) r += Rk[t] < v ? 1 : 0;
        Rs[r] = v;
        kinds[r] = kind[i];
    }
    wsync();
    for (int t = lane; t < out_stride; t += kWave) {
        const bool v = t < k && t < nr;
        const int32_t oi = v ? (int32_t)(uint32_t)Rs[t] : -1;
        const uint32_t od = v ? (uint32_t)(Rs[t] >> 32) : 0x7F800000u;
        if constexpr (SYS) {
            // pinned host memory: write through the GPU caches
            __hip_atomic_store(out_id + t, oi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(reinterpret_cast<uint32_t*>(out_dist) + t, od, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        } else {
            out_id[t] = oi;
            out_dist[t] = __uint_as_float(od);
        }
        if (out_kind) out_kind[t] = v ? kinds[t] : 0;
    }
    if (a_id_out) {
        for (int t = lane; t < nc; t += kWave) {
            a_id_out[t] = (uint32_t)As[t];
            a_dist_out[t] = __uint_as_float((uint32_t)(As[t] >> 32));
        }
    }
    if (lane == 0) {
        if (et_out) *et_out = (uint8_t)et;
        if (nrr_out) *nrr_out = nrr;
    }
}

template <int CPL8, int CPLF>
__global__ __launch_bounds__(256) void k_rerank(RerankArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    if (q >= a.nq) return;
    const Idx& ix = a.ix;
    const int nc_cap = a.nc_cap;
    const int r_cap = a.r_cap;
    unsigned char* base = smem + (size_t)wave * a.wave_lds;
    uint64_t* A = reinterpret_cast<uint64_t*>(base);
    uint64_t* As = A + nc_cap;
    uint64_t* Rk = As + nc_cap;
    uint64_t* Rs = Rk + r_cap;
    uint8_t* kind = reinterpret_cast<uint8_t*>(Rs + r_cap);
    uint8_t* kinds = kind + r_cap;
    uint32_t* ids = reinterpret_cast<uint32_t*>(kinds + r_cap);
    size_t off = (size_t)nc_cap * 16 + (size_t)r_cap * 18 + (size_t)nc_cap * 4;
    off = (off + 15) & ~(size_t)15;
    float* qf = reinterpret_cast<float*>(base + off);

    const int k = a.kq[q];
    int nc = a.ccnt[q];
    const bool bad = nc < 0 || nc > a.nc_stride || k < 1 || k > a.out_stride;
    if (bad) {
        for (int t = lane; t < a.out_stride; t += kWave) {
            a.out_id[q * a.out_stride + t] = -1;
            a.out_dist[q * a.out_stride + t] = __builtin_huge_valf();
            if (a.out_kind) a.out_kind[q * a.out_stride + t] = 0;
        }
        if (lane == 0) {
            if (a.taps.et) a.taps.et[q] = 0;
            if (a.taps.nrr) a.taps.nrr[q] = 0;
        }
        return;
    }
    for (int j = lane; j < ix.xs; j += kWave) qf[j] = j < ix.d ? a.Q[q * ix.d + j] : 0.0f;
    // candidate ids outside [0, n) are dropped (they cannot come from aqr_search)
    int ncv = 0;
    for (int b0 = 0; b0 < nc; b0 += kWave) {
        const int j = b0 + lane;
        const uint32_t id = j < nc ? a.cid[q * a.nc_stride + j] : kNone;
        const bool ok = j < nc && (int64_t)id < ix.n;
        const uint64_t m = ballot(ok);
        if (ok) ids[ncv + below(m)] = id;
        ncv += __popcll(m);
    }
    nc = ncv;
    wsync();

    rerank_query<CPL8, CPLF>(a, lane, k, nc, qf, ids, A, As, Rk, Rs, kind, kinds,
                             a.out_id + q * a.out_stride, a.out_dist + q * a.out_stride,
                             a.out_kind ? a.out_kind + q * a.out_stride : nullptr, a.out_stride,
                             a.taps.a_id ? a.taps.a_id + q * a.nc_stride : nullptr,
                             a.taps.a_dist ? a.taps.a_dist + q * a.nc_stride : nullptr,
                             a.taps.et ? a.taps.et + q : nullptr,
                             a.taps.nrr ? a.taps.nrr + q : nullptr);
}


// ---------------------------------------------------------------------------
// serving: a persistent kernel fed through a ring in pinned host memory
// ---------------------------------------------------------------------------
// Host side publishes request t (slot t % ring: k, ef, query) and then
// releases ctl->tail = t + 1 (system scope).  Wave 0 of block 0 is the
// dispatcher: it mirrors ctl->tail into device memory and raises the device
// stop flag when the host asks to stop or after idle_ticks of the 100 MHz
// clock with no unclaimed request.  Every other wave is a worker: it claims
// the next published request with a compare-and-swap on the device head,
// runs Stage 1 and Stages 2-3 with the same code as the batch kernels,
// writes the result rows into the ring and releases done[slot] = t + 1.
// Workers leave once the stop flag is up and no request is left unclaimed,
// so every wave of the grid exits.
struct ServeDev {
    uint64_t head;      // next request to claim
    uint64_t tail;      // mirror of the host's tail
    uint32_t stop;      // raised by the dispatcher
    uint32_t pad;
};

struct ServeCtl {       // pinned host memory
    uint64_t tail;      // requests published by the host
    uint32_t stop;      // host asks the kernel to leave
    uint32_t pad;
    uint64_t exited;    // epoch of the last launch whose dispatcher has left
};

struct ServeArgs {
    SearchArgs s;       // Idx, m_ef, ef_cap, vb (largest visited cache), geometry, wave_lds
    RerankArgs r;       // geometry and thresholds of the re-rank part
    int32_t ring;
    int32_t k_max;
    int32_t nc_max;
    int32_t vb_lo;      // smallest visited cache a request gets (log2 buckets)
    size_t run_bytes;   // per-wave region for one request's arrays (the largest request)
    uint64_t idle_ticks;
    uint64_t epoch;
    const int32_t* req_slot;  // [ring]: slot of ticket t at t mod ring
    uint64_t* consumed;       // [ring]: 1 + the last ticket whose entry a worker has read
    const int32_t* req_k;     // [slots]
    const int32_t* req_ef;    // [slots]
    const int64_t* req_off;   // [slots]: byte offset of the request's state in the arena
    unsigned char* arena;     // request state: query (d floats, 64-byte aligned), then
                              // k ids and k distances
    uint64_t* done;           // [slots]
    uint32_t* svc;            // [slots]: device service time of the request (100 MHz ticks)
    ServeCtl* ctl;
    ServeDev* dev;
};

// LDS arrays of one request in the serving kernel: the Stage-1 arrays [W |
// neighbour ids | their keys | visited buckets] sized by the request's own ef
// (W: ef_eff rounded up to 64 keys; visited buckets 2^vb with vb growing with
// ef_eff), overlaid after Stage 1 by the Stage 2-3 arrays [candidate ids | A
// | sorted A | R | sorted R | kinds] sized by its N_c, counted in 512-byte
// pages.  Each wave holds a region for the largest request; the host charges
// every request its own page count against the server's LDS budget.
__host__ __device__ inline int serve_vb(int efe, int vb_lo, int vb_hi) {
    int lg = 0;
    while ((1 << lg) < efe) ++lg;
    return max(vb_lo, min(vb_hi, lg + 1));
}
__host__ __device__ inline size_t serve_rr_bytes(int nc) {
    const size_t c = (size_t)((nc + 15) / 16 * 16);
    return c * 4 + c * 16 + c * 18;
}
__host__ __device__ inline int serve_pages(int efe, int nc, int st_cap, int vb_lo, int vb_hi) {
    const SearchLds run{(efe + 63) / 64 * 64, st_cap, serve_vb(efe, vb_lo, vb_hi), 0, 0, true};
    const size_t b = max(run.bytes(), serve_rr_bytes(nc));
    return (int)((b + 511) / 512);
}

// Synchronisation of the serving loop.  The spin loops use relaxed atomics
// only: acquire and release at agent or system scope maintain the per-XCD L2
// caches (invalidate / write back), and thousands of spinning waves doing that
// would starve the searching ones.  Ordering comes from dependencies instead:
//  - request data in pinned host memory is read with system-scope relaxed
//    loads (they bypass the GPU caches), at addresses that depend on the
//    claimed sequence number, which depends on the mirrored tail, which was
//    read after the host published the data;
//  - results are written with system-scope relaxed stores (write-through),
//    and the wave waits for every store to complete before it writes the done
//    flag.
__device__ __forceinline__ uint64_t ld_sys(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_sys32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_sys(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// wait until every memory operation this wave issued has completed
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Register budget for four waves per SIMD: the search and re-rank phases of
// a worker are never live at once; without the hint the compiler keeps more
// registers than three waves allow (a few values spill at four).
template <int CPL, int U, int LG, int CPL8, int CPLF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_serve(ServeArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const SearchArgs& sa = a.s;
    const Idx& ix = sa.ix;
    ServeDev* dv = a.dev;

    if (blockIdx.x == 0 && wave == 0) {
        // dispatcher: mirror the host's publication counter into device memory
        if (lane == 0) {
            uint64_t last = ld_agent(&dv->tail);
            uint64_t since = __builtin_amdgcn_s_memrealtime();
            for (;;) {
                const uint64_t t = ld_sys(&a.ctl->tail);
                if (t > last) {
                    __hip_atomic_store(&dv->tail, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    last = t;
                }
                const uint32_t stop = ld_sys32(&a.ctl->stop);
                const uint64_t h = ld_agent(&dv->head);
                const uint64_t now = __builtin_amdgcn_s_memrealtime();
                if (h < last) since = now;  // unclaimed work: not idle
                if (stop != 0u || now - since > a.idle_ticks) {
                    // the final tail is visible before the stop flag
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    __hip_atomic_store(&dv->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    // tell the host: requests published from now on need a relaunch
                    st_sys(&a.ctl->exited, a.epoch);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        return;
    }

    // worker LDS: [FP32 query | its codes | W's spare entry | request run],
    // the run laid out per request by its ef and N_c
    unsigned char* base = smem + (size_t)wave * sa.wave_lds;
    const int st_cap = st_cap_of(ix.s0, ix.s1);
    const SearchLds L{0, st_cap, 0, ix.xs, ix.dp, false};
    float* qf = reinterpret_cast<float*>(base + L.off_qf());
    uint8_t* qc = base + L.off_qc();
    uint64_t* spare = reinterpret_cast<uint64_t*>(base + L.off_mk());
    unsigned char* run = base + L.off_st();

    for (;;) {
        // take the next sequence number (one atomic add per request; lane 0
        // adds, every lane reads the old value after the branch has joined),
        // then wait until the host has published it
        uint64_t t = 0;
        if (lane == 0)
            t = __hip_atomic_fetch_add(&dv->head, (uint64_t)1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        wsync();
        const uint64_t tk = uni64(t);
        int quit = 0;
        int backoff = 1;
        for (;;) {
            uint64_t tl = 0;
            uint32_t st = 0;
            if (lane == 0) {
                tl = ld_agent(&dv->tail);
                if (tl <= tk) {
                    st = __hip_atomic_load(&dv->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (st != 0u) {
                        // the dispatcher published its final tail before raising stop
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        tl = ld_agent(&dv->tail);
                    }
                }
            }
            wsync();
            const uint64_t tlu = uni64(tl);
            if (tlu > tk) break;           // published: serve it
            if (uni((int)st) != 0) {       // never published: leave
                quit = 1;
                break;
            }
            for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(16);
            backoff = min(backoff * 2, 8);  // about 0.4 to 3.4 us
        }
        if (quit) break;
        const uint64_t t_claim = __builtin_amdgcn_s_memrealtime();
        const int slot =
            uni((int)ld_sys32(reinterpret_cast<const uint32_t*>(a.req_slot) + tk % a.ring));
        // the queue entry has been read: the host may reuse it for ticket tk + ring
        wait_mem();  // the entry's load has completed before the release below
        if (lane == 0) st_sys(a.consumed + tk % a.ring, (uint64_t)tk + 1);
        if (slot < 0 || slot >= a.ring) continue;  // not written by aqr_server_submit
        const int k = uni((int)ld_sys32(reinterpret_cast<const uint32_t*>(a.req_k) + slot));
        const int ef = uni((int)ld_sys32(reinterpret_cast<const uint32_t*>(a.req_ef) + slot));
        const int64_t off = (int64_t)ld_sys(reinterpret_cast<const uint64_t*>(a.req_off) + slot);
        const int efe = max(ef, k);
        const int nc = min(max(efe / sa.m_ef, k), efe);
        int bad = uni((k < 1 || k > a.k_max || efe > sa.ef_cap || nc > a.nc_max) ? 1 : 0);
        const int64_t qbytes = ((int64_t)ix.d * 4 + 63) / 64 * 64;
        const uint32_t* rq = reinterpret_cast<const uint32_t*>(a.arena + off);
        int32_t* oid = reinterpret_cast<int32_t*>(a.arena + off + qbytes);
        float* od = reinterpret_cast<float*>(a.arena + off + qbytes + (int64_t)max(k, 1) * 4);
        if (!bad) {
            bool nonfinite = false;
            for (int j = lane; j < ix.xs; j += kWave) {
                const float v = j < ix.d ? __uint_as_float(ld_sys32(rq + j)) : 0.0f;
                nonfinite |= !__builtin_isfinite(v);
                qf[j] = v;
            }
            bad = uni(ballot(nonfinite) != 0 ? 1 : 0);
        }
        // the row is k entries long (the host pads it to k_max)
        if (bad) {
            for (int j = lane; j < max(1, min(k, a.k_max)); j += kWave) {
                st_sys(oid + j, -1);
                st_sys(reinterpret_cast<uint32_t*>(od) + j, 0x7F800000u);
            }
        } else {
            // the request's arrays, laid out by its ef and N_c
            const int vbq = serve_vb(efe, a.vb_lo, sa.vb);
            const SearchLds R{(efe + 63) / 64 * 64, st_cap, vbq, 0, 0, true};
            uint64_t* mk = reinterpret_cast<uint64_t*>(run + R.off_mk());
            uint32_t* st_id = reinterpret_cast<uint32_t*>(run + R.off_st());
            uint64_t* st_key = reinterpret_cast<uint64_t*>(run + R.off_sk());
            uint64_t* visb = reinterpret_cast<uint64_t*>(run + R.off_vis());
            const VisCache vis{visb, vbq, max(ix.idbits, vbq + 1), 1u << vbq};
            SearchArgs sq = sa;
            sq.vb = vbq;
            sq.xb = 0;
            // Stage 1 writes its N_c candidates into the search part; the
            // re-rank reads them from there
            search_query<false, CPL, U, LG, false, false>(sq, 0, efe, nc, lane, vis, mk, spare, st_id,
                                                   st_key, visb, qf, qc);
            const int cnt = uni(*reinterpret_cast<const int*>(st_id));
            // Stages 2-3 overlay the run from its start: the candidate ids are
            // copied out of W (each 64-id chunk is read before it is written,
            // and the id array starts where W starts, so no unread key is
            // overwritten)
            const int c16 = (nc + 15) / 16 * 16;
            uint32_t* rids = reinterpret_cast<uint32_t*>(run);
            uint64_t* A = reinterpret_cast<uint64_t*>(run + (size_t)c16 * 4);
            uint64_t* As = A + c16;
            uint64_t* Rk = As + c16;
            uint64_t* Rs = Rk + c16;
            uint8_t* kind = reinterpret_cast<uint8_t*>(Rs + c16);
            uint8_t* kinds = kind + c16;
            for (int j = lane; j < cnt; j += kWave) rids[j] = (uint32_t)mk[j] >> 1;
            wsync();
            rerank_query<CPL8, CPLF, true>(a.r, lane, k, cnt, qf, rids, A, As, Rk, Rs, kind,
                                           kinds, oid, od, nullptr, k, nullptr, nullptr,
                                           nullptr, nullptr);
        }
        if (lane == 0)
            st_sys(a.svc + slot, (uint32_t)(__builtin_amdgcn_s_memrealtime() - t_claim));
        wait_mem();  // the row is in host memory before the flag
        wsync();
        if (lane == 0) st_sys(a.done + slot, (uint64_t)tk + 1);
        wsync();
    }
}

// Before a (re)launch: every request below the mirrored tail has been
// served, and sequence numbers taken beyond it by workers that left were
// never published, so numbering restarts at the tail.
__global__ void k_serve_reset(ServeDev* dv) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        dv->stop = 0u;
        dv->head = dv->tail;
    }
}

}  // namespace dev
}  // namespace aqr

// ===========================================================================
// host side
// ===========================================================================

using namespace aqr;
using aqr::dev::Idx;

struct aqr_index {
    Idx v;
    int device;
    int32_t M;
    int num_cu;
    size_t max_lds;     // per block
    size_t cu_lds;      // per compute unit
};

namespace {

struct Layout {
    size_t codes, X, adj0, ubase, uadj, qmin, qscale, total;
    int32_t dp, xs, s0, s1, cs, xst;
    int64_t rows;
};

// Row stride of a gathered row of b bytes: the next power of two up to 128,
// whole 128-byte lines beyond.  A row then never straddles more cache lines
// than its length needs (a 96-byte row at a 96-byte stride touches 1.5
// lines on average, at a 128-byte stride one).
int64_t line_stride(int64_t b) {
    if (b <= 128) {
        int64_t p = 16;
        while (p < b) p <<= 1;
        return p;
    }
    return (b + 127) / 128 * 128;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout_of(const aqr_quantizer* qz, const aqr_graph* g) {
    Layout L{};
    const int64_t n = g->n;
    L.dp = qz->info.d_pad;
    L.xs = round_up(qz->info.d, 4);
    L.cs = (int32_t)line_stride(L.dp);
    L.xst = (int32_t)(line_stride((int64_t)L.xs * 4) / 4);
    L.s0 = round_up(2 * g->M, 16);
    L.s1 = round_up(g->M, 16);
    L.rows = std::max<int64_t>(g->upper_off[n], 1);
    size_t o = 0;
    L.codes = o;
    o = align256(o + (size_t)n * L.cs + dev::kRowSlack);
    L.X = o;
    o = align256(o + (size_t)n * L.xst * 4 + dev::kRowSlack);
    L.adj0 = o;
    o = align256(o + (size_t)n * L.s0 * 4);
    L.ubase = o;
    o = align256(o + (size_t)n * 4);
    L.uadj = o;
    o = align256(o + (size_t)L.rows * L.s1 * 4);
    L.qmin = o;
    o = align256(o + (size_t)L.dp * 4);
    L.qscale = o;
    o = align256(o + (size_t)L.dp * 4);
    L.total = o;
    return L;
}

aqr_status hip_fail(hipError_t e, const char* what) {
    return fail(AQR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int ilog2_ceil(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b;
}

int pow2_lg_for(int nch) {
    // smallest lg with 2^lg >= min(nch, 64)
    int lg = 0;
    while ((1 << lg) < std::min(nch, 64)) ++lg;
    return lg;
}

}  // namespace

extern "C" aqr_status aqr_index_bytes(const aqr_quantizer* qz, const aqr_graph* g, size_t* bytes) {
    clear_error();
    if (!qz || !g || !bytes) return fail(AQR_ERR_INVALID_ARG, "aqr_index_bytes: null pointer");
    *bytes = layout_of(qz, g).total;
    return AQR_OK;
}

extern "C" aqr_status aqr_index_bind(const aqr_quantizer* qz, const aqr_graph* g,
                                     const uint8_t* codes, const float* X, void* dev_arena,
                                     size_t arena_bytes, void* stream, aqr_index** out) {
    try {
        clear_error();
        if (!qz || !g || !codes || !X || !dev_arena || !out)
            return fail(AQR_ERR_INVALID_ARG, "aqr_index_bind: null pointer");
        if (qz->info.d > dev::kMaxD)
            return fail(AQR_ERR_INVALID_ARG, "aqr_index_bind: d above 4096 is not supported");
        if (g->n > (int64_t)0x7FFFFFFF)
            return fail(AQR_ERR_INVALID_ARG, "aqr_index_bind: n above 2^31-1 is not supported");
        const Layout L = layout_of(qz, g);
        if (arena_bytes < L.total)
            return fail(AQR_ERR_OOM, "aqr_index_bind: arena smaller than aqr_index_bytes()");
        if (((uintptr_t)dev_arena & 255) != 0)
            return fail(AQR_ERR_INVALID_ARG, "aqr_index_bind: arena must be 256-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = g->n;
        const int32_t d = qz->info.d, M = g->M;
        unsigned char* A = (unsigned char*)dev_arena;
        hipError_t e;
        // host staging in the device layout
        std::vector<float> xs;
        const float* Xsrc = X;
        if (L.xst != d) {
            xs.assign((size_t)n * L.xst, 0.0f);
            for (int64_t i = 0; i < n; ++i)
                std::memcpy(&xs[(size_t)i * L.xst], X + i * d, sizeof(float) * d);
            Xsrc = xs.data();
        }
        // code rows at the line stride; when the padding has room, the row's
        // |x^|^2 (exact, uint32) follows its d_pad codes, so the search needs
        // only q.x per row
        std::vector<uint8_t> cst;
        const uint8_t* Csrc = codes;
        const bool nrm = L.cs >= L.dp + 4;
        if (L.cs != L.dp) {
            cst.assign((size_t)n * L.cs, 0);
            parallel_for_threads(std::max(1, std::min(16, (int)(n / 65536))), [&](int t) {
                const int T = std::max(1, std::min(16, (int)(n / 65536)));
                const int64_t i0 = n * t / T, i1 = n * (t + 1) / T;
                for (int64_t i = i0; i < i1; ++i) {
                    const uint8_t* src = codes + i * L.dp;
                    uint8_t* dst = &cst[(size_t)i * L.cs];
                    std::memcpy(dst, src, (size_t)L.dp);
                    if (nrm) {
                        uint32_t xx = 0;
                        for (int32_t j = 0; j < L.dp; ++j) xx += (uint32_t)src[j] * src[j];
                        std::memcpy(dst + L.dp, &xx, 4);
                    }
                }
            });
            Csrc = cst.data();
        }
        std::vector<uint32_t> a0((size_t)n * L.s0, AQR_NONE);
        for (int64_t i = 0; i < n; ++i)
            std::memcpy(&a0[(size_t)i * L.s0], &g->adj0[(size_t)i * 2 * M], sizeof(uint32_t) * 2 * M);
        std::vector<int32_t> ub(n, -1);
        for (int64_t i = 0; i < n; ++i)
            if (g->level[i] > 0) ub[i] = (int32_t)g->upper_off[i];
        std::vector<uint32_t> ua((size_t)L.rows * L.s1, AQR_NONE);
        for (int64_t r = 0; r < g->upper_off[n]; ++r)
            std::memcpy(&ua[(size_t)r * L.s1], &g->upper_adj[(size_t)r * M], sizeof(uint32_t) * M);
        std::vector<float> qmin(L.dp, 0.0f), qsc(L.dp, 1.0f);
        for (int32_t j = 0; j < d; ++j) {
            qmin[j] = qz->mn[j];
            qsc[j] = qz->scale[j];
        }
        struct Cp {
            size_t off;
            const void* src;
            size_t bytes;
        } cps[] = {
            {L.codes, Csrc, (size_t)n * L.cs},
            {L.X, Xsrc, (size_t)n * L.xst * 4},
            {L.adj0, a0.data(), a0.size() * 4},
            {L.ubase, ub.data(), ub.size() * 4},
            {L.uadj, ua.data(), ua.size() * 4},
            {L.qmin, qmin.data(), qmin.size() * 4},
            {L.qscale, qsc.data(), qsc.size() * 4},
        };
        for (const Cp& c : cps) {
            e = hipMemcpyAsync(A + c.off, c.src, c.bytes, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "aqr_index_bind: copy");
        }
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "aqr_index_bind: synchronize");
        aqr_index* ix = new aqr_index();
        Idx& v = ix->v;
        v.codes = A + L.codes;
        v.X = reinterpret_cast<const float*>(A + L.X);
        v.adj0 = reinterpret_cast<const uint32_t*>(A + L.adj0);
        v.ubase = reinterpret_cast<const int32_t*>(A + L.ubase);
        v.uadj = reinterpret_cast<const uint32_t*>(A + L.uadj);
        v.qmin = reinterpret_cast<const float*>(A + L.qmin);
        v.qscale = reinterpret_cast<const float*>(A + L.qscale);
        v.n = n;
        v.d = d;
        v.dp = L.dp;
        v.xs = L.xs;
        v.cs = L.cs;
        v.xst = L.xst;
        v.nrm = (L.cs >= L.dp + 4) ? 1 : 0;
        v.s0 = L.s0;
        v.s1 = L.s1;
        v.ep = g->ep;
        v.L = g->L;
        v.idbits = std::max(1, ilog2_ceil(n));
        ix->M = M;
        e = hipGetDevice(&ix->device);
        if (e != hipSuccess) {
            delete ix;
            return hip_fail(e, "aqr_index_bind: hipGetDevice");
        }
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, ix->device);
        if (e != hipSuccess) {
            delete ix;
            return hip_fail(e, "aqr_index_bind: hipGetDeviceProperties");
        }
        ix->num_cu = prop.multiProcessorCount;
        ix->max_lds = prop.sharedMemPerBlock;
        ix->cu_lds = std::max(prop.maxSharedMemoryPerMultiProcessor, prop.sharedMemPerBlock);
        *out = ix;
        return AQR_OK;
    } catch (const std::bad_alloc&) {
        return fail(AQR_ERR_OOM, "aqr_index_bind: out of host memory");
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_index_bind: unexpected failure");
    }
}

extern "C" void aqr_index_free(aqr_index* ix) { delete ix; }

extern "C" size_t aqr_search_workspace_size(void) { return 256; }

namespace {

// Blocks per CU that the LDS holds.  gfx950 allocates a block's LDS in
// 1,280-byte units (160 KB / 128): five blocks of 32,000 bytes are resident
// on a CU, five of 32,256 bytes are not.  The runtime's occupancy query
// counts in smaller units and reports five for the latter, so its answer is
// capped by this one.
constexpr size_t kLdsUnit = 1280;
inline size_t lds_alloc(size_t bytes) { return (bytes + kLdsUnit - 1) / kLdsUnit * kLdsUnit; }
inline int lds_blocks_per_cu(size_t cu_lds, size_t block_lds) {
    return block_lds == 0 ? INT_MAX : (int)(cu_lds / lds_alloc(block_lds));
}

template <bool F32, int CPL, int U, int LG>
hipError_t launch_search_k(dev::SearchArgs& a, int blocks, int wpb, size_t lds, int ncu,
                           size_t cu_lds, hipStream_t s) {
    const bool taps = a.taps.expanded || a.taps.evaluated || a.taps.counts;
    // rows with |x|^2 in their padding, and a spare chunk slot to read it
    const bool nrm = !F32 && a.ix.nrm && a.nch < (CPL << LG);
    const int kv = (taps ? 1 : 0) + (nrm ? 2 : 0);
    auto kern = nrm ? (taps ? dev::k_search<F32, CPL, U, LG, true, true>
                            : dev::k_search<F32, CPL, U, LG, false, true>)
                    : (taps ? dev::k_search<F32, CPL, U, LG, true, false>
                            : dev::k_search<F32, CPL, U, LG, false, false>);
    // the dynamic-LDS limit is raised once per size and kernel, outside any stream capture
    static std::atomic<int> lds_set[4] = {0, 0, 0, 0};
    std::atomic<int>& ls = lds_set[kv];
    hipError_t e = hipSuccess;
    if ((int)lds > ls.load()) {
        e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        if (e != hipSuccess) return e;
        ls.store((int)lds);
    }
    if (blocks <= 0) {
        // Resident blocks per CU for this kernel, block size and LDS size,
        // asked of the runtime once and kept: the query is not free, and a
        // launch that waits on it leaves the device idle.
        static std::mutex occ_mu;
        static std::map<std::pair<int, int>, int> occ[4];
        const std::pair<int, int> key{wpb, (int)lds};
        int per_cu = 0;
        {
            std::lock_guard<std::mutex> lk(occ_mu);
            auto it = occ[kv].find(key);
            if (it != occ[kv].end()) per_cu = it->second;
        }
        if (per_cu == 0) {
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, wpb * dev::kWave, lds);
            if (e != hipSuccess) return e;
            if (cu_lds > 0) per_cu = std::min(per_cu, lds_blocks_per_cu(cu_lds, lds));
            per_cu = std::max(1, per_cu);
            std::lock_guard<std::mutex> lk(occ_mu);
            occ[kv][key] = per_cu;
        }
        blocks = per_cu * std::max(1, ncu);
        const int64_t need = (a.nq + wpb - 1) / wpb;
        if ((int64_t)blocks > need) blocks = (int)std::max<int64_t>(1, need);
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(wpb * dev::kWave), lds, s, a);
    return hipGetLastError();
}

// Row geometry by row width (nch 16-byte chunks): CPL chunks per lane on
// groups of 2^LG lanes (CPL * 2^LG >= nch), U rows per group in flight.
// Short rows take two chunks per lane on narrow groups; wide rows take four
// or eight chunks per lane, so that a pass of the wave still scores several
// rows: one wave works on one query, and with few queries in
// a batch the number of rows in flight per wave sets the latency.  A batch
// of at most one wave per SIMD (lat) leaves registers to spare, so wide
// rows then keep four row sets in flight instead of two (128 VGPRs of rows).
// Short code rows keep four sets in flight (a whole 64-entry adjacency row
// scored in one pass instead of two dependent ones) when registers are not
// what limits the waves per SIMD: with lat, or when the LDS of one wave
// leaves room for at most five waves per SIMD (lds_few).
template <bool F32>
hipError_t launch_search(dev::SearchArgs& a, int nch, int blocks, int wpb, size_t lds, int ncu,
                         size_t cu_lds, hipStream_t s, bool lat, bool lds_few) {
    auto lg_for = [](int groups) {  // smallest lg with 2^lg >= groups, at least 2
        int lg = 2;
        while ((1 << lg) < groups) ++lg;
        return lg;
    };
    if constexpr (!F32) {
        if (nch <= 16) {  // up to 256 bytes: 2 chunks per lane, 2 (4) rows in flight
            const bool u4 = lat || lds_few;
            switch (lg_for((nch + 1) / 2)) {
                case 2:
                    return u4 ? launch_search_k<F32, 2, 4, 2>(a, blocks, wpb, lds, ncu, cu_lds, s)
                              : launch_search_k<F32, 2, 2, 2>(a, blocks, wpb, lds, ncu, cu_lds, s);
                default:
                    return u4 ? launch_search_k<F32, 2, 4, 3>(a, blocks, wpb, lds, ncu, cu_lds, s)
                              : launch_search_k<F32, 2, 2, 3>(a, blocks, wpb, lds, ncu, cu_lds, s);
            }
        }
        if (nch <= 32)  // up to 512 bytes: 4 chunks per lane, 2 rows in flight
            return launch_search_k<F32, 4, 2, 3>(a, blocks, wpb, lds, ncu, cu_lds, s);
        if (nch <= 64)  // up to 1 KB: 8 chunks per lane, 2 (lat: 4) rows in flight
            return lat ? launch_search_k<F32, 8, 4, 3>(a, blocks, wpb, lds, ncu, cu_lds, s)
                       : launch_search_k<F32, 8, 2, 3>(a, blocks, wpb, lds, ncu, cu_lds, s);
        if (nch <= 128) return launch_search_k<F32, 8, 1, 4>(a, blocks, wpb, lds, ncu, cu_lds, s);
        return launch_search_k<F32, 8, 1, 5>(a, blocks, wpb, lds, ncu, cu_lds, s);
    } else {
        if (nch <= 16) {  // up to 64 floats: 2 chunks per lane
            switch (lg_for((nch + 1) / 2)) {
                case 2: return launch_search_k<F32, 2, 2, 2>(a, blocks, wpb, lds, ncu, cu_lds, s);
                default: return launch_search_k<F32, 2, 2, 3>(a, blocks, wpb, lds, ncu, cu_lds, s);
            }
        }
        if (nch <= 64) {  // up to 256 floats: 2 chunks per lane on up to 32 lanes
            switch (lg_for((nch + 1) / 2)) {
                case 4: return launch_search_k<F32, 2, 2, 4>(a, blocks, wpb, lds, ncu, cu_lds, s);
                default: return launch_search_k<F32, 2, 2, 5>(a, blocks, wpb, lds, ncu, cu_lds, s);
            }
        }
        if (nch <= 256) {  // up to 1,024 floats: 8 chunks per lane on up to 32 lanes
            switch (lg_for((nch + 7) / 8)) {
                case 2:
                case 3:
                case 4:
                    return lat ? launch_search_k<F32, 8, 4, 4>(a, blocks, wpb, lds, ncu, cu_lds, s)
                               : launch_search_k<F32, 8, 2, 4>(a, blocks, wpb, lds, ncu, cu_lds, s);
                default:
                    return lat ? launch_search_k<F32, 8, 4, 5>(a, blocks, wpb, lds, ncu, cu_lds, s)
                               : launch_search_k<F32, 8, 2, 5>(a, blocks, wpb, lds, ncu, cu_lds, s);
            }
        }
        if (nch <= 512) return launch_search_k<F32, 8, 1, 6>(a, blocks, wpb, lds, ncu, cu_lds, s);
        return launch_search_k<F32, 16, 1, 6>(a, blocks, wpb, lds, ncu, cu_lds, s);
    }
}

int cpl_for(int nch) {
    int cpl = 1;
    while (cpl * 64 < nch) cpl <<= 1;
    return cpl;
}

aqr_status run_search(const aqr_index* ix, const float* Q, int64_t nq, const int32_t* k,
                      const int32_t* ef, const int32_t* nc, const aqr_sparams* sp,
                      uint32_t* out_id, uint32_t* out_D, int32_t* out_cnt, void* ws,
                      size_t ws_bytes, const aqr_taps* taps, void* stream, bool f32,
                      const char* who) {
    clear_error();
    if (!ix || !sp) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": null pointer");
    if (nq < 0) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": nq < 0");
    if (nq == 0) return AQR_OK;  // an empty batch needs no buffers
    if (!k || !ef || !out_id || !out_D || !ws || (!f32 && !out_cnt))
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": null pointer");
    if (!Q) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": null queries");
    if (nq > (int64_t)INT32_MAX) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": nq too large");
    if (sp->ef_max < 1 || sp->ef_max > 1024)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": ef_max must be in [1, 1024]");
    if (sp->out_stride < 1)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": out_stride must be >= 1");
    if (!f32 && !nc && sp->m_ef < 1)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": m_ef must be >= 1");
    if (ws_bytes < aqr_search_workspace_size())
        return fail(AQR_ERR_OOM, std::string(who) + ": workspace too small");
    if (taps && (taps->expanded || taps->evaluated) && taps->cap < 1)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": taps->cap must be >= 1");
    const Idx& v = ix->v;
    int vb = sp->visited_log2 > 0 ? sp->visited_log2 : 7;
    if (vb < 4 || vb > 14) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": visited_log2 out of [4, 14]");
    // at most 16 stored bits per id (16 only with more than 2^vb buckets)
    if (std::max(v.idbits, vb + 1) - vb > 16) vb = v.idbits - 16;
    const int wpb = sp->waves_per_block > 0 ? sp->waves_per_block : 4;
    if (wpb != 1 && wpb != 2 && wpb != 4)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": waves_per_block must be 1, 2 or 4");
    if (v.s0 > 256)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": layer-0 rows above 256 entries are not supported");
    const int nsw = sp->small_waves;
    if (nsw < 0 || nsw >= wpb)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": small_waves must be in [0, waves_per_block)");
    if (nsw > 0 && (sp->ef_small < 1 || sp->ef_small >= sp->ef_max))
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": ef_small must be in [1, ef_max)");
    const int ef_cap = (sp->ef_max + 63) / 64 * 64;  // W capacity: whole 64-entry slots
    const int st_cap = std::max(v.s0, v.s1) <= 64 ? 64 : (std::max(v.s0, v.s1) + 63) / 64 * 64;
    // the 8-bit search keeps no FP32 query in LDS
    dev::SearchLds sl{ef_cap, st_cap, vb, f32 ? v.xs : 0, v.dp, true, 0, true};
    dev::SearchLds sl2{nsw > 0 ? (sp->ef_small + 63) / 64 * 64 : 0, st_cap, vb, f32 ? v.xs : 0, v.dp,
                       true, 0, true};
    auto block_bytes = [&]() { return sl.bytes() * (wpb - nsw) + (nsw > 0 ? sl2.bytes() * nsw : 0); };
    // The LDS that the blocks resident per CU leave unused holds more visited
    // buckets (fewer than 2^vb more): the same blocks stay resident, and the
    // cache forgets fewer of the nodes a query meets.
    size_t blk0 = 0, per_cu = 0;
    auto fill = [&]() {
        sl.vb = sl2.vb = vb;
        sl.xb = sl2.xb = 0;
        blk0 = block_bytes();
        per_cu = (size_t)lds_blocks_per_cu(ix->cu_lds, blk0);
        if (per_cu >= 1) {
            const size_t room = std::min(ix->cu_lds / per_cu / kLdsUnit * kLdsUnit, (size_t)ix->max_lds);
            size_t xb = room > blk0 ? (room - blk0) / (8 * (size_t)wpb) : 0;
            sl.xb = sl2.xb = (int)std::min(xb, ((size_t)1 << vb) - 1);
            while (sl.xb > 0 && block_bytes() > room) sl.xb = sl2.xb = sl.xb - 1;
        }
    };
    fill();
    // 16 stored bits need more than 2^vb buckets; without room for one more,
    // the cache doubles instead (15 stored bits)
    if (std::max(v.idbits, vb + 1) - vb == 16 && sl.xb == 0) {
        ++vb;
        fill();
    }
    if (blk0 > ix->max_lds)
        return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": LDS per block exceeds the device limit (lower ef_max, visited_log2 or waves_per_block)");
    const size_t wl = sl.bytes();
    const size_t lds = block_bytes();
    dev::SearchArgs a{};
    a.ix = v;
    a.Q = Q;
    a.nq = nq;
    a.kq = k;
    a.efq = ef;
    a.ncq = f32 ? nullptr : nc;
    a.order = sp->order;
    a.m_ef = std::max(1, sp->m_ef);
    a.ef_cap = sl.ef_cap;
    a.out_stride = sp->out_stride;
    a.vb = vb;
    a.xb = sl.xb;
    a.nsw = nsw;
    a.ef_cap2 = sl2.ef_cap;
    a.wave_lds2 = nsw > 0 ? sl2.bytes() : 0;
    a.mode = f32 ? 1 : 0;
    const int nch = f32 ? v.xs / 4 : v.dp / 16;
    a.nch = nch;
    a.lg = std::max(2, pow2_lg_for(nch));
    a.wave_lds = wl;
    a.out_id = out_id;
    a.out_D = out_D;
    a.out_cnt = out_cnt;
    a.counter = reinterpret_cast<int32_t*>(ws);
    if (taps) {
        a.taps.cap = taps->cap;
        a.taps.expanded = taps->expanded;
        a.taps.evaluated = taps->evaluated;
        a.taps.counts = taps->counts;
    }
    hipStream_t s = (hipStream_t)stream;
    if (nsw > 0)
        hipLaunchKernelGGL(dev::k_split, dim3(1), dim3(1024), 0, s, k, ef, sp->order, nq,
                           sp->ef_small, a.counter);
    else
        hipLaunchKernelGGL(dev::k_reset, dim3(1), dim3(64), 0, s, a.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, who);
    const int cpl = cpl_for(nch);
    if (cpl > 16) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": row too wide");
    if (!f32 && cpl > 4) return fail(AQR_ERR_INVALID_ARG, std::string(who) + ": code row too wide");
    const bool lat = nq <= (int64_t)ix->num_cu * 4;  // at most one wave per SIMD
    // LDS leaves at most five waves per SIMD (counted in whole blocks)
    const bool lds_few = per_cu * (size_t)wpb <= 20;
    e = f32 ? launch_search<true>(a, nch, sp->blocks, wpb, lds, ix->num_cu, ix->cu_lds, s, lat, lds_few)
            : launch_search<false>(a, nch, sp->blocks, wpb, lds, ix->num_cu, ix->cu_lds, s, lat, lds_few);
    if (e != hipSuccess) return hip_fail(e, who);
    return AQR_OK;
}

}  // namespace

extern "C" aqr_status aqr_search(const aqr_index* ix, const float* Q, int64_t nq,
                                 const int32_t* k, const int32_t* ef, const int32_t* nc,
                                 const aqr_sparams* sp, uint32_t* cand_id, uint32_t* cand_D,
                                 int32_t* cand_cnt, void* ws, size_t ws_bytes,
                                 const aqr_taps* taps, void* stream) {
    try {
        return run_search(ix, Q, nq, k, ef, nc, sp, cand_id, cand_D, cand_cnt, ws, ws_bytes, taps,
                          stream, false, "aqr_search");
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_search: unexpected failure");
    }
}

extern "C" aqr_status aqr_search_fp32(const aqr_index* ix, const float* Q, int64_t nq,
                                      const int32_t* k, const int32_t* ef, const aqr_sparams* sp,
                                      int32_t* out_id, float* out_dist, void* ws, size_t ws_bytes,
                                      const aqr_taps* taps, void* stream) {
    try {
        return run_search(ix, Q, nq, k, ef, nullptr, sp, reinterpret_cast<uint32_t*>(out_id),
                          reinterpret_cast<uint32_t*>(out_dist), nullptr, ws, ws_bytes, taps,
                          stream, true, "aqr_search_fp32");
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_search_fp32: unexpected failure");
    }
}

extern "C" aqr_status aqr_encode_queries(const aqr_index* ix, const float* Q, int64_t nq,
                                         uint8_t* qcodes, void* stream) {
    clear_error();
    if (!ix) return fail(AQR_ERR_INVALID_ARG, "aqr_encode_queries: null pointer");
    if (nq < 0) return fail(AQR_ERR_INVALID_ARG, "aqr_encode_queries: nq < 0");
    if (nq == 0) return AQR_OK;
    if (!qcodes) return fail(AQR_ERR_INVALID_ARG, "aqr_encode_queries: null pointer");
    if (!Q) return fail(AQR_ERR_INVALID_ARG, "aqr_encode_queries: null queries");
    hipLaunchKernelGGL(dev::k_encode, dim3((unsigned)nq), dim3(128), 0, (hipStream_t)stream,
                       ix->v, Q, nq, qcodes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "aqr_encode_queries");
    return AQR_OK;
}

namespace {

template <int C8, int CF>
hipError_t launch_rerank_cf(dev::RerankArgs& a, int wpb, size_t lds, hipStream_t s) {
    auto kern = dev::k_rerank<C8, CF>;
    static std::atomic<int> lds_set{0};
    if ((int)lds > lds_set.load()) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set.store((int)lds);
    }
    const int64_t blocks = (a.nq + wpb - 1) / wpb;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(wpb * dev::kWave), lds, s, a);
    return hipGetLastError();
}

template <int C8>
hipError_t launch_rerank_c8(dev::RerankArgs& a, int cf, int wpb, size_t lds, hipStream_t s) {
    switch (cf) {
        case 1: return launch_rerank_cf<C8, 1>(a, wpb, lds, s);
        case 2: return launch_rerank_cf<C8, 2>(a, wpb, lds, s);
        case 4: return launch_rerank_cf<C8, 4>(a, wpb, lds, s);
        case 8: return launch_rerank_cf<C8, 8>(a, wpb, lds, s);
        default: return launch_rerank_cf<C8, 16>(a, wpb, lds, s);
    }
}

}  // namespace

extern "C" aqr_status aqr_rerank(const aqr_index* ix, const float* Q, int64_t nq,
                                 const uint32_t* cand_id, const int32_t* cand_cnt,
                                 int32_t nc_stride, const int32_t* k, const aqr_rparams* rp,
                                 int32_t* out_id, float* out_dist, uint8_t* out_kind,
                                 const aqr_rtaps* taps, void* stream) {
    try {
        clear_error();
        if (!ix || !rp) return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: null pointer");
        if (nq < 0) return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: nq < 0");
        if (nq == 0) return AQR_OK;  // an empty batch needs no buffers
        if (!cand_id || !cand_cnt || !k || !out_id || !out_dist)
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: null pointer");
        if (!Q) return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: null queries");
        if (nc_stride < 1 || nc_stride > 1024)
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: nc_stride must be in [1, 1024]");
        if (rp->out_stride < 1 || rp->out_stride > 1024)
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: out_stride must be in [1, 1024]");
        if (rp->n_rerank < 0) return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: n_rerank < 0");
        if (rp->assembly != 0 && rp->assembly != 1)
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: assembly must be 0 (fill) or 1 (union)");
        if (!(rp->eps >= 0.0f) || std::isnan(rp->tau_gap) || std::isnan(rp->tau_ratio))
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: bad thresholds");
        if (taps && ((taps->a_id == nullptr) != (taps->a_dist == nullptr)))
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: a_id and a_dist go together");
        const Idx& v = ix->v;
        const int wpb = rp->waves_per_block > 0 ? rp->waves_per_block : 4;
        if (wpb != 1 && wpb != 2 && wpb != 4)
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: waves_per_block must be 1, 2 or 4");
        dev::RerankArgs a{};
        a.ix = v;
        a.Q = Q;
        a.nq = nq;
        a.cid = cand_id;
        a.ccnt = cand_cnt;
        a.nc_stride = nc_stride;
        a.nc_cap = (nc_stride + 15) / 16 * 16;
        // R holds the exact entries plus the fill from A: at most nc entries
        a.r_cap = a.nc_cap;
        a.kq = k;
        a.n_rerank = rp->n_rerank;
        a.out_stride = rp->out_stride;
        a.tau_gap = rp->tau_gap;
        a.tau_ratio = rp->tau_ratio;
        a.eps = rp->eps;
        a.force_et = rp->force_et < 0 ? -1 : (rp->force_et ? 1 : 0);
        a.assembly = rp->assembly;
        a.nch8 = v.dp / 16;
        a.lg8 = pow2_lg_for(a.nch8);
        a.nchf = v.xs / 4;
        a.lgf = pow2_lg_for(a.nchf);
        dev::RerankLds rl{a.nc_cap, a.r_cap, v.xs};
        a.wave_lds = rl.bytes();
        const size_t lds = a.wave_lds * wpb;
        if (lds > ix->max_lds)
            return fail(AQR_ERR_INVALID_ARG, "aqr_rerank: LDS per block exceeds the device limit");
        a.out_id = out_id;
        a.out_dist = out_dist;
        a.out_kind = out_kind;
        if (taps) {
            a.taps.a_id = taps->a_id;
            a.taps.a_dist = taps->a_dist;
            a.taps.et = taps->et;
            a.taps.nrr = taps->nrr;
        }
        const int c8 = cpl_for(a.nch8), cf = cpl_for(a.nchf);
        hipStream_t s = (hipStream_t)stream;
        hipError_t e;
        switch (c8) {
            case 1: e = launch_rerank_c8<1>(a, cf, wpb, lds, s); break;
            case 2: e = launch_rerank_c8<2>(a, cf, wpb, lds, s); break;
            default: e = launch_rerank_c8<4>(a, cf, wpb, lds, s); break;
        }
        if (e != hipSuccess) return hip_fail(e, "aqr_rerank");
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_rerank: unexpected failure");
    }
}

// ===========================================================================
// batch plans: order + Stage 1 + Stages 2-3 as one captured graph
// ===========================================================================

struct aqr_plan {
    const aqr_index* ix = nullptr;
    aqr_sparams sp{};
    aqr_rparams rp{};
    aqr_batch_buffers b{};
    int32_t use_graph = 0;
    hipGraphExec_t exec = nullptr;
    int64_t graph_nq = -1;
    hipStream_t capture_stream = nullptr;  // private, default priority; only records
};

namespace {

aqr_status plan_enqueue(aqr_plan* p, int64_t nq, hipStream_t s) {
    const aqr_batch_buffers& b = p->b;
    aqr_sparams sp = p->sp;
    if (b.order) {
        hipLaunchKernelGGL(dev::k_order, dim3(1), dim3(1024), 0, s, b.k, b.ef, nq, b.order);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "aqr_plan_launch: order");
        sp.order = b.order;
    }
    aqr_taps taps{};
    taps.counts = b.counts;
    aqr_status st = aqr_search(p->ix, b.Q, nq, b.k, b.ef, nullptr, &sp, b.cand_id, b.cand_D,
                               b.cand_cnt, b.ws, b.ws_bytes, b.counts ? &taps : nullptr, s);
    if (st != AQR_OK) return st;
    return aqr_rerank(p->ix, b.Q, nq, b.cand_id, b.cand_cnt, sp.out_stride, b.k, &p->rp,
                      b.out_id, b.out_dist, b.out_kind, nullptr, s);
}

}  // namespace

extern "C" aqr_status aqr_plan_create(const aqr_index* ix, const aqr_sparams* sp,
                                      const aqr_rparams* rp, const aqr_batch_buffers* b,
                                      int32_t use_graph, aqr_plan** out) {
    try {
        clear_error();
        if (!ix || !sp || !rp || !b || !out)
            return fail(AQR_ERR_INVALID_ARG, "aqr_plan_create: null pointer");
        if (!b->Q || !b->k || !b->ef || !b->cand_id || !b->cand_D || !b->cand_cnt ||
            !b->out_id || !b->out_dist || !b->ws)
            return fail(AQR_ERR_INVALID_ARG, "aqr_plan_create: null buffer");
        if (b->nq_max < 1 || b->nq_max > (int64_t)INT32_MAX)
            return fail(AQR_ERR_INVALID_ARG, "aqr_plan_create: nq_max out of range");
        if (sp->order)
            return fail(AQR_ERR_INVALID_ARG,
                        "aqr_plan_create: the work order comes from buffers->order");
        if (sp->ef_max > dev::kOrderMaxEf)
            return fail(AQR_ERR_INVALID_ARG, "aqr_plan_create: ef_max above 1024");
        aqr_plan* p = new aqr_plan();
        p->ix = ix;
        p->sp = *sp;
        p->rp = *rp;
        p->b = *b;
        p->use_graph = use_graph;
        *out = p;
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_OOM, "aqr_plan_create: out of host memory");
    }
}

extern "C" aqr_status aqr_plan_launch(aqr_plan* p, int64_t nq, void* stream) {
    try {
        clear_error();
        if (!p) return fail(AQR_ERR_INVALID_ARG, "aqr_plan_launch: null plan");
        if (nq < 0 || nq > p->b.nq_max)
            return fail(AQR_ERR_INVALID_ARG, "aqr_plan_launch: nq outside [0, nq_max]");
        if (nq == 0) return AQR_OK;
        hipStream_t s = (hipStream_t)stream;
        if (!p->use_graph) return plan_enqueue(p, nq, s);
        if (!p->exec || p->graph_nq != nq) {
            if (p->exec) {
                (void)hipGraphExecDestroy(p->exec);
                p->exec = nullptr;
            }
            // one eager pass on the caller's stream sets every launch
            // attribute outside the capture and produces this batch's results
            aqr_status st = plan_enqueue(p, nq, s);
            if (st != AQR_OK) return st;
            // the sequence is recorded on a private stream (the caller's stream
            // may be the legacy default stream, which cannot be captured) and
            // the graph is launched on the caller's stream from then on
            hipError_t e = hipSuccess;
            if (!p->capture_stream) {
                e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
                if (e != hipSuccess) {
                    p->capture_stream = nullptr;
                    return hip_fail(e, "aqr_plan_launch: capture stream");
                }
            }
            hipStream_t cs = p->capture_stream;
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "aqr_plan_launch: begin capture");
            st = plan_enqueue(p, nq, cs);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(cs, &graph);
            if (st != AQR_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "aqr_plan_launch: end capture");
            e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                p->exec = nullptr;
                return hip_fail(e, "aqr_plan_launch: instantiate");
            }
            p->graph_nq = nq;
            return AQR_OK;
        }
        hipError_t e = hipGraphLaunch(p->exec, s);
        if (e != hipSuccess) return hip_fail(e, "aqr_plan_launch: graph launch");
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_plan_launch: unexpected failure");
    }
}

extern "C" void aqr_plan_free(aqr_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
}

// ===========================================================================
// serving
// ===========================================================================

// Request state (query, result ids and distances) lives in one arena of
// pinned host memory, mapped to the device; requests take byte ranges of it,
// first fit, and return them when their result is collected.
struct ArenaAlloc {
    std::map<int64_t, int64_t> free_;  // offset -> length, coalesced
    int64_t total = 0, used = 0;
    void init(int64_t bytes) {
        free_.clear();
        total = bytes;
        used = 0;
        if (bytes > 0) free_[0] = bytes;
    }
    int64_t alloc(int64_t len) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                const int64_t off = it->first, rest = it->second - len;
                free_.erase(it);
                if (rest > 0) free_[off + len] = rest;
                used += len;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t len) {
        used -= len;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + len == nx->first) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return;
            }
        }
        free_[off] = len;
    }
};

struct aqr_server {
    const aqr_index* ix = nullptr;
    aqr_server_params prm{};
    dev::ServeArgs args{};
    int blocks = 0, wpb = 4;
    size_t lds = 0;
    int st_cap = 64, vb_lo = 4, vb_hi = 9;
    int64_t lds_budget = 0, lds_used = 0;  // pages of outstanding requests
    hipStream_t stream = nullptr;
    dev::ServeCtl* ctl = nullptr;  // pinned, coherent
    int32_t* req_slot = nullptr;
    uint64_t* consumed = nullptr;
    int32_t* req_k = nullptr;
    int32_t* req_ef = nullptr;
    int64_t* req_off = nullptr;
    unsigned char* arena = nullptr;
    uint64_t* done = nullptr;
    uint32_t* svc = nullptr;
    ArenaAlloc arena_alloc;
    uint64_t next_ticket = 0;
    std::vector<uint64_t> slot_ticket;  // sequence number in the slot, or ~0 when free
    std::vector<int32_t> free_slots;
    std::vector<int32_t> slot_k;        // k of the request in the slot
    std::vector<int64_t> slot_bytes;    // its state bytes
    std::vector<int32_t> slot_pages;    // its LDS pages
    bool launched = false;
    std::mutex mu;
    hipError_t (*launch_fn)(aqr_server*) = nullptr;
    hipError_t (*occ_fn)(aqr_server*, int*) = nullptr;
};

namespace {

constexpr uint64_t kFree = ~0ull;
constexpr int kSlotBits = 22;  // ticket = sequence << 22 | slot

// Row sets in flight of the serving worker: four for short code rows (the
// worker runs at four waves per SIMD, so registers allow them), else two.
template <int CPL, int LG>
constexpr int serve_u() { return (CPL << LG) <= 16 ? 4 : 2; }

template <int CPL, int LG, int C8, int CF>
hipError_t serve_occ_t(aqr_server* sv, int* per_cu) {
    constexpr int U = serve_u<CPL, LG>();
    auto kern = dev::k_serve<CPL, U, LG, C8, CF>;
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sv->lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, sv->wpb * dev::kWave,
                                                        sv->lds);
}

template <int CPL, int LG, int C8, int CF>
hipError_t serve_launch_t(aqr_server* sv) {
    constexpr int U = serve_u<CPL, LG>();
    auto kern = dev::k_serve<CPL, U, LG, C8, CF>;
    hipLaunchKernelGGL(dev::k_serve_reset, dim3(1), dim3(64), 0, sv->stream, sv->args.dev);
    hipLaunchKernelGGL(kern, dim3(sv->blocks), dim3(sv->wpb * dev::kWave), sv->lds, sv->stream,
                       sv->args);
    return hipGetLastError();
}

using ServeFns = std::pair<hipError_t (*)(aqr_server*), hipError_t (*)(aqr_server*, int*)>;

template <int CPL, int LG>
ServeFns pick_serve_cf(int cf) {
    switch (cf) {
        case 1: return {serve_launch_t<CPL, LG, 1, 1>, serve_occ_t<CPL, LG, 1, 1>};
        case 2: return {serve_launch_t<CPL, LG, 1, 2>, serve_occ_t<CPL, LG, 1, 2>};
        case 4: return {serve_launch_t<CPL, LG, 1, 4>, serve_occ_t<CPL, LG, 1, 4>};
        default: return {nullptr, nullptr};
    }
}

// Code-row geometry of the serving worker's Stage 1, by row width (nch
// 16-byte chunks, at most 64): the batch kernel's rule with at most four
// chunks per lane.
ServeFns pick_serve(int nch, int cf) {
    if (nch <= 8) return pick_serve_cf<2, 2>(cf);
    if (nch <= 16) return pick_serve_cf<2, 3>(cf);
    if (nch <= 32) return pick_serve_cf<4, 3>(cf);
    if (nch <= 64) return pick_serve_cf<4, 4>(cf);
    return {nullptr, nullptr};
}

// (Re)launch the persistent kernel when it is not running.  A running
// kernel's dispatcher writes its epoch into ctl->exited when it leaves; a
// request published after that is picked up by the relaunch made here on the
// next submit or poll.
aqr_status serve_ensure_running(aqr_server* sv) {
    if (sv->launched) {
        if (__atomic_load_n(&sv->ctl->exited, __ATOMIC_ACQUIRE) != sv->args.epoch) return AQR_OK;
        const hipError_t q = hipStreamSynchronize(sv->stream);  // workers drain
        if (q != hipSuccess) return hip_fail(q, "aqr_server: kernel");
        sv->launched = false;
    }
    sv->args.epoch += 1;
    const hipError_t e = sv->launch_fn(sv);
    if (e != hipSuccess) return hip_fail(e, "aqr_server: launch");
    sv->launched = true;
    return AQR_OK;
}

// Costs a request is charged at admission (and returned when collected).
void serve_cost(const aqr_server* sv, int32_t k, int32_t ef, int32_t* pages, int64_t* bytes) {
    const int efe = std::max(ef, k);
    const int nc = std::min(std::max(efe / sv->prm.m_ef, k), efe);
    *pages = dev::serve_pages(efe, nc, sv->st_cap, sv->vb_lo, sv->vb_hi);
    const int64_t qb = ((int64_t)sv->ix->v.d * 4 + 63) / 64 * 64;
    *bytes = qb + ((int64_t)k * 8 + 63) / 64 * 64;
}

// Both below run with sv->mu held.
aqr_status serve_submit_locked(aqr_server* sv, const float* q, int32_t k, int32_t ef,
                               uint64_t* ticket) {
    if (k < 1 || k > sv->prm.k_max || ef < 1 ||
        std::max(ef, k) > std::max(sv->prm.ef_max, sv->prm.k_max))
        return fail(AQR_ERR_INVALID_ARG, "aqr_server_submit: k or ef outside the server's limits");
    if (sv->free_slots.empty()) return fail(AQR_ERR_BUSY, "aqr_server_submit: no free request slot");
    // The queue entry of sequence t (t mod ring) held sequence t - ring; it
    // may be reused only once a worker has read it.
    const uint64_t t = sv->next_ticket;
    const uint64_t R = (uint64_t)sv->prm.ring;
    if (t >= R && __atomic_load_n(&sv->consumed[t % R], __ATOMIC_ACQUIRE) != t - R + 1)
        return fail(AQR_ERR_BUSY, "aqr_server_submit: queue entry not yet read by a worker");
    int32_t pages = 0;
    int64_t bytes = 0;
    serve_cost(sv, k, ef, &pages, &bytes);
    if (sv->lds_used + pages > sv->lds_budget)
        return fail(AQR_ERR_BUSY, "aqr_server_submit: LDS budget exhausted");
    const int64_t off = sv->arena_alloc.alloc(bytes);
    if (off < 0) return fail(AQR_ERR_BUSY, "aqr_server_submit: request-state budget exhausted");
    const int32_t slot = sv->free_slots.back();
    sv->free_slots.pop_back();
    sv->lds_used += pages;
    const int32_t d = sv->ix->v.d;
    std::memcpy(sv->arena + off, q, sizeof(float) * d);
    sv->req_k[slot] = k;
    sv->req_ef[slot] = ef;
    sv->req_off[slot] = off;
    sv->slot_k[slot] = k;
    sv->slot_bytes[slot] = bytes;
    sv->slot_pages[slot] = pages;
    sv->req_slot[t % R] = slot;
    sv->slot_ticket[slot] = t;
    sv->next_ticket = t + 1;
    __atomic_store_n(&sv->ctl->tail, t + 1, __ATOMIC_RELEASE);
    *ticket = (t << kSlotBits) | (uint64_t)slot;
    return serve_ensure_running(sv);
}

aqr_status serve_poll_locked(aqr_server* sv, uint64_t ticket, int32_t* out_id, float* out_dist,
                             int32_t* is_done, uint32_t* svc_ticks = nullptr,
                             bool relaunch = true) {
    const uint64_t slot = ticket & ((1ull << kSlotBits) - 1);
    const uint64_t seq = ticket >> kSlotBits;
    if (slot >= (uint64_t)sv->prm.ring || sv->slot_ticket[slot] != seq)
        return fail(AQR_ERR_STATE, "aqr_server_poll: unknown or already collected ticket");
    if (__atomic_load_n(&sv->done[slot], __ATOMIC_ACQUIRE) != seq + 1) {
        *is_done = 0;
        return relaunch ? serve_ensure_running(sv) : AQR_OK;
    }
    // the device wrote the first k entries of the row; pad the rest
    const int32_t km = sv->prm.k_max, k = sv->slot_k[slot];
    const int64_t qb = ((int64_t)sv->ix->v.d * 4 + 63) / 64 * 64;
    const unsigned char* st = sv->arena + sv->req_off[slot] + qb;
    if (out_id) {
        std::memcpy(out_id, st, sizeof(int32_t) * k);
        for (int32_t j = k; j < km; ++j) out_id[j] = -1;
    }
    if (out_dist) {
        std::memcpy(out_dist, st + (size_t)k * 4, sizeof(float) * k);
        for (int32_t j = k; j < km; ++j) out_dist[j] = std::numeric_limits<float>::infinity();
    }
    if (svc_ticks) *svc_ticks = sv->svc[slot];
    sv->arena_alloc.release(sv->req_off[slot], sv->slot_bytes[slot]);
    sv->lds_used -= sv->slot_pages[slot];
    sv->slot_ticket[slot] = kFree;
    sv->free_slots.push_back((int32_t)slot);
    *is_done = 1;
    return AQR_OK;
}

}  // namespace

extern "C" size_t aqr_server_workspace_size(void) { return 256; }

extern "C" aqr_status aqr_server_create(const aqr_index* ix, const aqr_server_params* prm,
                                        void* ws, size_t ws_bytes, aqr_server** out) {
    try {
        clear_error();
        if (!ix || !prm || !ws || !out) return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: null pointer");
        if (ws_bytes < aqr_server_workspace_size())
            return fail(AQR_ERR_OOM, "aqr_server_create: workspace too small");
        if (prm->ring < 1 || prm->ring > (1 << 22) || prm->k_max < 1 || prm->k_max > 1024 ||
            prm->ef_max < 1 || prm->ef_max > 1024 || prm->m_ef < 1 || prm->n_rerank < 0 ||
            prm->state_budget < 0 ||
            prm->lds_budget_pages < 0)
            return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: parameter out of range");
        const Idx& v = ix->v;
        const int nch8 = v.dp / 16, nchf = v.xs / 4;
        const int c8 = cpl_for(nch8), cf = cpl_for(nchf);
        if (c8 != 1 || cf > 4)
            return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: serving supports d <= 1024");
        if (v.s0 > 256) return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: rows above 256 entries");
        const int efm = std::max(prm->ef_max, prm->k_max);
        const int ef_cap = (efm + 63) / 64 * 64;
        // visited caches: 2^vb buckets growing with a request's ef, between the
        // smallest that keeps the stored id remainder within 15 bits and the
        // server's largest (visited_log2, default 9)
        int vb_hi = prm->visited_log2 > 0 ? prm->visited_log2 : 9;
        if (vb_hi < 4 || vb_hi > 14)
            return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: visited_log2 out of [4, 14]");
        const int vb_lo = std::max(4, v.idbits - 15);
        vb_hi = std::max(vb_hi, vb_lo);
        const int nc_max = std::min(efm, std::max(prm->k_max, efm / prm->m_ef));
        aqr_server* sv = new aqr_server();
        sv->ix = ix;
        sv->prm = *prm;
        sv->wpb = prm->waves_per_block > 0 ? prm->waves_per_block : 4;
        if (sv->wpb > 4) {
            delete sv;
            return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: waves_per_block above 4");
        }
        sv->st_cap = std::max(v.s0, v.s1) <= 64 ? 64 : (std::max(v.s0, v.s1) + 63) / 64 * 64;
        sv->vb_lo = vb_lo;
        sv->vb_hi = vb_hi;
        // the largest request the kernel accepts: ef_eff up to ef_cap (the
        // host admits at most max(ef_max, k_max)), with k = 1 or k_max
        int32_t max_pages = 0;
        for (int32_t kk : {1, prm->k_max}) {
            int32_t pg = 0;
            int64_t by = 0;
            serve_cost(sv, kk, ef_cap, &pg, &by);
            max_pages = std::max(max_pages, pg);
        }
        // per wave: the query, its codes, W's spare entry and a region for
        // the largest request
        const dev::SearchLds wl{0, sv->st_cap, 0, v.xs, v.dp, false};
        const size_t run_bytes = (size_t)max_pages * 512;
        const size_t wave_lds = dev::SearchLds::r16(wl.off_st() + run_bytes);
        sv->lds = wave_lds * sv->wpb;
        if (sv->lds > ix->max_lds) {
            delete sv;
            return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: LDS per block exceeds the device limit");
        }
        dev::RerankArgs& r = sv->args.r;
        r.ix = v;
        r.nc_cap = (nc_max + 15) / 16 * 16;
        r.r_cap = r.nc_cap;  // R never exceeds the candidate count
        r.n_rerank = prm->n_rerank;
        r.out_stride = prm->k_max;
        r.tau_gap = prm->tau_gap;
        r.tau_ratio = prm->tau_ratio;
        r.eps = prm->eps;
        r.force_et = -1;
        r.assembly = 0;  // the server fills from A (the default reading)
        r.nch8 = nch8;
        r.lg8 = pow2_lg_for(nch8);
        r.nchf = nchf;
        r.lgf = pow2_lg_for(nchf);
        dev::SearchArgs& sa = sv->args.s;
        sa.ix = v;
        sa.m_ef = prm->m_ef;
        sa.ef_cap = ef_cap;
        sa.out_stride = nc_max;
        sa.vb = vb_hi;
        sa.mode = 2;
        sa.nch = nch8;
        sa.lg = std::max(2, pow2_lg_for(nch8));
        sa.wave_lds = wave_lds;
        sv->args.ring = prm->ring;
        sv->args.k_max = prm->k_max;
        sv->args.nc_max = nc_max;
        sv->args.vb_lo = vb_lo;
        sv->args.run_bytes = run_bytes;
        sv->args.idle_ticks = (uint64_t)std::max(1, prm->idle_ms) * 100000ull;
        const ServeFns fns = c8 == 1 ? pick_serve(nch8, cf) : ServeFns{nullptr, nullptr};
        sv->launch_fn = fns.first;
        sv->occ_fn = fns.second;
        if (!sv->launch_fn || !sv->occ_fn) {
            delete sv;
            return fail(AQR_ERR_INVALID_ARG, "aqr_server_create: unsupported row geometry");
        }
        // every block must be resident at once: workers only leave after the
        // dispatcher (block 0) raises the stop flag
        int per_cu = 0;
        hipError_t e = sv->occ_fn(sv, &per_cu);
        if (e != hipSuccess) {
            delete sv;
            return hip_fail(e, "aqr_server_create: occupancy");
        }
        per_cu = std::min(per_cu, lds_blocks_per_cu(ix->cu_lds, sv->lds));
        sv->blocks = std::max(1, per_cu) * std::max(1, ix->num_cu);
        // admission budgets: LDS pages of outstanding requests (default: the
        // resident waves' regions, one largest request each) and
        // request-state bytes (default: every slot at k_max)
        int32_t pg_max = 0;
        int64_t by_max = 0;
        serve_cost(sv, prm->k_max, efm, &pg_max, &by_max);
        sv->lds_budget = prm->lds_budget_pages > 0 ? prm->lds_budget_pages
                                                   : (int64_t)sv->blocks * sv->wpb * max_pages;
        const int64_t state = prm->state_budget > 0 ? prm->state_budget
                                                    : (int64_t)prm->ring * by_max;
        if (sv->lds_budget < max_pages || state < by_max) {
            delete sv;
            return fail(AQR_ERR_INVALID_ARG,
                        "aqr_server_create: a budget below the largest request's cost");
        }
        // pinned, coherent host memory for the ring, the request state and
        // the control block
        const size_t R = (size_t)prm->ring;
        struct Alloc {
            void** p;
            size_t bytes;
        } al[] = {
            {(void**)&sv->ctl, sizeof(dev::ServeCtl)},
            {(void**)&sv->req_slot, R * sizeof(int32_t)},
            {(void**)&sv->consumed, R * sizeof(uint64_t)},
            {(void**)&sv->req_k, R * sizeof(int32_t)},
            {(void**)&sv->req_ef, R * sizeof(int32_t)},
            {(void**)&sv->req_off, R * sizeof(int64_t)},
            {(void**)&sv->arena, (size_t)state},
            {(void**)&sv->done, R * sizeof(uint64_t)},
            {(void**)&sv->svc, R * sizeof(uint32_t)},
        };
        for (const Alloc& x : al) {
            e = hipHostMalloc(x.p, x.bytes, hipHostMallocCoherent | hipHostMallocMapped);
            if (e != hipSuccess) {
                *x.p = nullptr;
                aqr_server_destroy(sv);
                return hip_fail(e, "aqr_server_create: pinned host memory");
            }
            std::memset(*x.p, 0, x.bytes);
        }
        for (size_t i = 0; i < R; ++i) sv->req_slot[i] = -1;
        sv->arena_alloc.init(state);
        sv->args.ctl = sv->ctl;
        sv->args.req_slot = sv->req_slot;
        sv->args.consumed = sv->consumed;
        sv->args.req_k = sv->req_k;
        sv->args.req_ef = sv->req_ef;
        sv->args.req_off = sv->req_off;
        sv->args.arena = sv->arena;
        sv->args.done = sv->done;
        sv->args.svc = sv->svc;
        sv->args.dev = reinterpret_cast<dev::ServeDev*>(ws);
        sv->slot_ticket.assign(R, kFree);
        sv->slot_k.assign(R, 0);
        sv->slot_bytes.assign(R, 0);
        sv->slot_pages.assign(R, 0);
        sv->free_slots.resize(R);
        for (size_t i = 0; i < R; ++i) sv->free_slots[i] = (int32_t)(R - 1 - i);
        e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            sv->stream = nullptr;
            aqr_server_destroy(sv);
            return hip_fail(e, "aqr_server_create: stream");
        }
        dev::ServeDev zero{};
        e = hipMemcpyAsync(ws, &zero, sizeof(zero), hipMemcpyHostToDevice, sv->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(sv->stream);
        if (e != hipSuccess) {
            aqr_server_destroy(sv);
            return hip_fail(e, "aqr_server_create: workspace init");
        }
        *out = sv;
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_OOM, "aqr_server_create: out of host memory");
    }
}

extern "C" aqr_status aqr_server_submit(aqr_server* sv, const float* q, int32_t k, int32_t ef,
                                        uint64_t* ticket) {
    try {
        clear_error();
        if (!sv || !q || !ticket) return fail(AQR_ERR_INVALID_ARG, "aqr_server_submit: null pointer");
        std::lock_guard<std::mutex> lk(sv->mu);
        return serve_submit_locked(sv, q, k, ef, ticket);
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_server_submit: unexpected failure");
    }
}

extern "C" aqr_status aqr_server_poll(aqr_server* sv, uint64_t ticket, int32_t* out_id,
                                      float* out_dist, int32_t* is_done) {
    try {
        clear_error();
        if (!sv || !is_done) return fail(AQR_ERR_INVALID_ARG, "aqr_server_poll: null pointer");
        std::lock_guard<std::mutex> lk(sv->mu);
        return serve_poll_locked(sv, ticket, out_id, out_dist, is_done);
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_server_poll: unexpected failure");
    }
}

extern "C" aqr_status aqr_server_request_cost(const aqr_server* sv, int32_t k, int32_t ef,
                                              int32_t* lds_pages, int64_t* state_bytes) {
    clear_error();
    if (!sv || !lds_pages || !state_bytes)
        return fail(AQR_ERR_INVALID_ARG, "aqr_server_request_cost: null pointer");
    if (k < 1 || k > sv->prm.k_max || ef < 1 ||
        std::max(ef, k) > std::max(sv->prm.ef_max, sv->prm.k_max))
        return fail(AQR_ERR_INVALID_ARG, "aqr_server_request_cost: k or ef outside the server's limits");
    serve_cost(sv, k, ef, lds_pages, state_bytes);
    return AQR_OK;
}

extern "C" aqr_status aqr_server_usage(aqr_server* sv, aqr_server_usage_t* u) {
    clear_error();
    if (!sv || !u) return fail(AQR_ERR_INVALID_ARG, "aqr_server_usage: null pointer");
    std::lock_guard<std::mutex> lk(sv->mu);
    u->ring = sv->prm.ring;
    u->slots_used = sv->prm.ring - (int32_t)sv->free_slots.size();
    u->lds_budget_pages = sv->lds_budget;
    u->lds_used_pages = sv->lds_used;
    u->state_budget = sv->arena_alloc.total;
    u->state_used = sv->arena_alloc.used;
    u->blocks = sv->blocks;
    u->run_pages = (int32_t)(sv->args.run_bytes / 512);
    return AQR_OK;
}

extern "C" aqr_status aqr_server_stop(aqr_server* sv) {
    clear_error();
    if (!sv) return fail(AQR_ERR_INVALID_ARG, "aqr_server_stop: null server");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->launched) return AQR_OK;
    __atomic_store_n(&sv->ctl->stop, 1u, __ATOMIC_RELEASE);
    const hipError_t e = hipStreamSynchronize(sv->stream);
    __atomic_store_n(&sv->ctl->stop, 0u, __ATOMIC_RELEASE);
    sv->launched = false;
    if (e != hipSuccess) return hip_fail(e, "aqr_server_stop");
    return AQR_OK;
}

extern "C" void aqr_server_destroy(aqr_server* sv) {
    if (!sv) return;
    if (sv->launched) (void)aqr_server_stop(sv);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    void* ptrs[] = {sv->ctl,     sv->req_slot, sv->consumed, sv->req_k, sv->req_ef,
                    sv->req_off, sv->arena,    sv->done,     sv->svc};
    for (void* p : ptrs)
        if (p) (void)hipHostFree(p);
    delete sv;
}

// Native trace replay: request i arrives at arrival_s[i] (seconds from the
// start); it is submitted at that time (or as soon as the server admits it)
// and its latency runs from its arrival to the poll that finds it done.  A
// replay that sees no request complete for timeout_s seconds stops with
// AQR_ERR_STATE.
extern "C" aqr_status aqr_server_replay(aqr_server* sv, int64_t n, const double* arrival_s,
                                        const float* Q, const int32_t* k, const int32_t* ef,
                                        int32_t* out_id, float* out_dist, double* latency_s,
                                        double* service_s, double* wall_s) {
    try {
        clear_error();
        if (!sv || !arrival_s || !Q || !k || !ef || !latency_s)
            return fail(AQR_ERR_INVALID_ARG, "aqr_server_replay: null pointer");
        if (n < 0) return fail(AQR_ERR_INVALID_ARG, "aqr_server_replay: negative count");
        std::lock_guard<std::mutex> lk(sv->mu);
        const int32_t d = sv->ix->v.d, km = sv->prm.k_max;
        const double timeout_s = 60.0;
        using clk = std::chrono::steady_clock;
        const auto t0 = clk::now();
        auto now_s = [&] { return std::chrono::duration<double>(clk::now() - t0).count(); };
        std::vector<uint64_t> tick((size_t)n, kFree);
        std::vector<int64_t> pending;  // submitted, not yet done
        pending.reserve(sv->prm.ring);
        int64_t next = 0, finished = 0;
        double last_progress = 0.0;
        std::vector<int32_t> ids(km);
        std::vector<float> dd(km);
        while (finished < n) {
            const double t = now_s();
            while (next < n && arrival_s[next] <= t) {
                uint64_t tk = 0;
                const aqr_status st = serve_submit_locked(sv, Q + next * d, k[next], ef[next], &tk);
                if (st == AQR_ERR_BUSY) break;
                if (st != AQR_OK) return st;
                tick[next] = tk;
                pending.push_back(next);
                ++next;
            }
            bool waiting = false;
            for (size_t i = 0; i < pending.size();) {
                const int64_t r = pending[i];
                int32_t ok = 0;
                uint32_t ticks = 0;
                const aqr_status st =
                    serve_poll_locked(sv, tick[r], out_id ? out_id + r * km : ids.data(),
                                      out_dist ? out_dist + r * km : dd.data(), &ok, &ticks, false);
                if (st != AQR_OK) return st;
                if (ok) {
                    latency_s[r] = now_s() - arrival_s[r];
                    if (service_s) service_s[r] = ticks * 1e-8;  // 100 MHz
                    ++finished;
                    last_progress = now_s();
                    pending[i] = pending.back();
                    pending.pop_back();
                } else {
                    waiting = true;
                    ++i;
                }
            }
            if (waiting) {
                if (now_s() - last_progress > timeout_s)
                    return fail(AQR_ERR_STATE, "aqr_server_replay: no request completed for 60 s");
                const aqr_status st = serve_ensure_running(sv);
                if (st != AQR_OK) return st;
            } else if (next < n) {
                // nothing in flight: wait for the next arrival (spin for the last 50 us)
                const double wait = arrival_s[next] - now_s() - 50e-6;
                if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
                last_progress = now_s();
            }
        }
        if (wall_s) *wall_s = now_s();
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_server_replay: unexpected failure");
    }
}

// ---------------------------------------------------------------------------
// Batched graph construction with the layer-0 searches on the device
// ---------------------------------------------------------------------------
extern "C" aqr_status aqr_build_batched(const uint8_t* codes, const float* X, int64_t n, int32_t d,
                                        const aqr_quantizer* qz, const aqr_bparams* p,
                                        const double* level_u, int64_t seed_n,
                                        int32_t seed_batch, int32_t batch, aqr_graph** out) {
    const char* who = "aqr_build_batched";
    void* arena = nullptr;
    std::vector<void*> bufs, hbufs;  // device buffers, pinned host staging
    aqr_index* ix = nullptr;
    auto release = [&]() {
        if (ix) aqr_index_free(ix);
        for (void* b : bufs) (void)hipFree(b);
        for (void* b : hbufs) (void)hipHostFree(b);
        if (arena) (void)hipFree(arena);
    };
    try {
        clear_error();
        if (!X || !out) return fail(AQR_ERR_INVALID_ARG, "aqr_build_batched: null pointer");
        if (seed_n < 1 || seed_batch < 1 || batch < 1)
            return fail(AQR_ERR_INVALID_ARG,
                        "aqr_build_batched: seed_n, seed_batch and batch must be >= 1");
        aqr_graph* g0 = nullptr;
        aqr_status st =
            build_seeded(codes, n, d, qz, p, level_u, std::min(seed_n, n),
                         std::min(seed_batch, batch), who, &g0);
        if (st != AQR_OK) return st;
        std::unique_ptr<aqr_graph> g(g0);
        const int32_t M = g->M, efc = g->efc;
        if (efc > 1024) return fail(AQR_ERR_INVALID_ARG, "aqr_build_batched: efc above 1024");
        std::vector<uint32_t> R;  // level-0 points left for the chunks, in id order
        for (int64_t i = seed_n; i < n; ++i)
            if (g->level[i] == 0) R.push_back((uint32_t)i);
        if (R.empty()) {
            *out = g.release();
            return AQR_OK;
        }
        const int T = host_threads(p->threads);
        hipError_t e;
        size_t bytes = 0;
        if ((st = aqr_index_bytes(qz, g.get(), &bytes)) != AQR_OK) return st;
        if ((e = hipMalloc(&arena, bytes)) != hipSuccess) {
            release();
            return hip_fail(e, "aqr_build_batched: device memory for the index");
        }
        if ((st = aqr_index_bind(qz, g.get(), codes, X, arena, bytes, nullptr, &ix)) != AQR_OK) {
            release();
            return st;
        }
        const int32_t B = (int32_t)std::min<int64_t>(batch, (int64_t)R.size());
        const int64_t max_dirty = std::min<int64_t>((int64_t)B * (1 + M), n);
        const int32_t s0 = ix->v.s0, W = 2 * M;
        auto dalloc = [&](size_t b) -> void* {
            void* ptr = nullptr;
            if (hipMalloc(&ptr, std::max<size_t>(b, 256)) != hipSuccess) return nullptr;
            bufs.push_back(ptr);
            return ptr;
        };
        float* Qd = (float*)dalloc((size_t)B * d * 4);
        int32_t* kd = (int32_t*)dalloc((size_t)B * 4);
        int32_t* efd = (int32_t*)dalloc((size_t)B * 4);
        int32_t* ncd = (int32_t*)dalloc((size_t)B * 4);
        int32_t* cntd = (int32_t*)dalloc((size_t)B * 4);
        uint32_t* cidd = (uint32_t*)dalloc((size_t)B * efc * 4);
        uint32_t* cDd = (uint32_t*)dalloc((size_t)B * efc * 4);
        void* ws = dalloc(aqr_search_workspace_size());
        // the heuristic's selections on the device (one wave per point, M <= 64)
        const bool dev_select = M <= 64;
        uint32_t* seld = (uint32_t*)dalloc((size_t)B * M * 4);
        int32_t* nseld = (int32_t*)dalloc((size_t)B * 4);
        // the reverse links on the device too when a full list and its new
        // entry fit one wave (2M + 1 <= 64): links sorted by target, one wave
        // per target; the host graph is read back after the last chunk
        const bool dev_link = dev_select && 2 * M + 1 <= dev::kWave;
        const int32_t cap = 2 * M;
        const int64_t NL = (int64_t)B * M;  // links of a full chunk
        uint32_t* idsd = (uint32_t*)dalloc((size_t)B * 4);
        uint32_t* lkey = (uint32_t*)dalloc((size_t)NL * 4);
        uint32_t* lval = (uint32_t*)dalloc((size_t)NL * 4);
        uint32_t* lkey_s = (uint32_t*)dalloc((size_t)NL * 4);
        uint32_t* lval_s = (uint32_t*)dalloc((size_t)NL * 4);
        int32_t* segd = (int32_t*)dalloc((size_t)NL * 4);
        int32_t* ctrd = (int32_t*)dalloc(2 * 4);  // run count, work counter
        size_t sort_bytes = 0;
        if ((e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, lkey, lkey_s, lval, lval_s,
                                                    (int)NL)) != hipSuccess) {
            release();
            return hip_fail(e, "aqr_build_batched: link sort size");
        }
        void* sort_tmp = dalloc(sort_bytes);
        uint32_t* rowd = (uint32_t*)dalloc((size_t)max_dirty * 4);
        uint32_t* datd = (uint32_t*)dalloc((size_t)max_dirty * W * 4);
        for (void* b : bufs)
            if (!b) {
                release();
                return fail(AQR_ERR_OOM, "aqr_build_batched: device memory for the chunks");
            }
        // pinned staging for the per-chunk copies (queries in, candidates out,
        // changed rows in)
        auto halloc = [&](size_t b) -> void* {
            void* ptr = nullptr;
            if (hipHostMalloc(&ptr, std::max<size_t>(b, 256)) != hipSuccess) return nullptr;
            hbufs.push_back(ptr);
            return ptr;
        };
        float* hq = (float*)halloc((size_t)B * d * 4);
        uint32_t* hid = (uint32_t*)halloc((size_t)B * efc * 4);
        uint32_t* hD = (uint32_t*)halloc((size_t)B * efc * 4);
        int32_t* hcnt = (int32_t*)halloc((size_t)B * 4);
        uint32_t* hsel = (uint32_t*)halloc((size_t)B * M * 4);
        int32_t* hnsel = (int32_t*)halloc((size_t)B * 4);
        uint32_t* hrow = (uint32_t*)halloc((size_t)max_dirty * 4);
        uint32_t* hdat = (uint32_t*)halloc((size_t)max_dirty * W * 4);
        for (void* b : hbufs)
            if (!b) {
                release();
                return fail(AQR_ERR_OOM, "aqr_build_batched: pinned host memory for the chunks");
            }
        {
            std::vector<int32_t> one(B, 1), wide(B, efc);
            if ((e = hipMemcpy(kd, one.data(), (size_t)B * 4, hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(efd, wide.data(), (size_t)B * 4, hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(ncd, wide.data(), (size_t)B * 4, hipMemcpyHostToDevice)) != hipSuccess) {
                release();
                return hip_fail(e, "aqr_build_batched: copy");
            }
        }
        aqr_sparams sp{};
        sp.ef_max = efc;
        sp.out_stride = efc;
        sp.m_ef = 1;
        std::vector<uint32_t> dirty;
        std::vector<uint64_t> keys((size_t)B * efc);
        std::vector<uint8_t> mark((size_t)n, 0);  // scratch of link_chunk
        int64_t inserted = n - (int64_t)R.size();
        const int32_t dp = qz->info.d_pad;
        size_t pos = 0;
        const auto t0 = std::chrono::steady_clock::now();
        int64_t next_report = 0;
        double t_search = 0.0, t_link = 0.0, t_rows = 0.0;  // seconds, for the progress report
        auto now = [] { return std::chrono::steady_clock::now(); };
        auto secs = [](std::chrono::steady_clock::time_point a,
                       std::chrono::steady_clock::time_point b) {
            return std::chrono::duration<double>(b - a).count();
        };
        while (pos < R.size()) {
            const int32_t nb = (int32_t)std::min<int64_t>(
                std::min<int64_t>(batch, std::max<int64_t>(1, inserted / 8)),
                (int64_t)(R.size() - pos));
            const uint32_t* ids = R.data() + pos;
            const auto ta = now();
            for (int32_t b = 0; b < nb; ++b)
                std::memcpy(&hq[(size_t)b * d], X + (int64_t)ids[b] * d, sizeof(float) * d);
            if ((e = hipMemcpy(Qd, hq, (size_t)nb * d * 4, hipMemcpyHostToDevice)) != hipSuccess) {
                release();
                return hip_fail(e, "aqr_build_batched: copy");
            }
            st = run_search(ix, Qd, nb, kd, efd, ncd, &sp, cidd, cDd, cntd, ws,
                            aqr_search_workspace_size(), nullptr, nullptr, false, who);
            if (st != AQR_OK) {
                release();
                return st;
            }
            if (dev_select) {
                hipLaunchKernelGGL(dev::k_select, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0,
                                   nullptr, ix->v, cidd, cDd, cntd, nb, efc, M, seld, nseld);
                if ((e = hipGetLastError()) != hipSuccess ||
                    (e = hipMemcpy(hcnt, cntd, (size_t)nb * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
                    (e = hipMemcpy(hsel, seld, (size_t)nb * M * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
                    (e = hipMemcpy(hnsel, nseld, (size_t)nb * 4, hipMemcpyDeviceToHost)) != hipSuccess) {
                    release();
                    return hip_fail(e, "aqr_build_batched: selection");
                }
            } else if ((e = hipMemcpy(hid, cidd, (size_t)nb * efc * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
                       (e = hipMemcpy(hD, cDd, (size_t)nb * efc * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
                       (e = hipMemcpy(hcnt, cntd, (size_t)nb * 4, hipMemcpyDeviceToHost)) != hipSuccess) {
                release();
                return hip_fail(e, "aqr_build_batched: copy");
            }
            for (int32_t b = 0; b < nb; ++b) {
                if (hcnt[b] < 1 || hcnt[b] > efc) {
                    release();
                    return fail(AQR_ERR_STATE, "aqr_build_batched: a chunk search returned no candidates");
                }
                if (dev_select) {
                    if (hnsel[b] < 0 || hnsel[b] > M) {
                        release();
                        return fail(AQR_ERR_STATE, "aqr_build_batched: selection count out of range");
                    }
                    for (int32_t t = 0; t < hnsel[b]; ++t)
                        if ((int64_t)hsel[(size_t)b * M + t] >= n) {
                            release();
                            return fail(AQR_ERR_STATE, "aqr_build_batched: selected id out of range");
                        }
                    continue;
                }
                for (int32_t t = 0; t < hcnt[b]; ++t) {
                    const size_t o = (size_t)b * efc + t;
                    keys[o] = ((uint64_t)hD[o] << 32) | hid[o];
                }
            }
            const auto tb = now();
            if (dev_link) {
                const int64_t nl = (int64_t)nb * M;
                uint32_t* adj0d = const_cast<uint32_t*>(ix->v.adj0);
                if ((e = hipMemcpy(idsd, ids, (size_t)nb * 4, hipMemcpyHostToDevice)) != hipSuccess) {
                    release();
                    return hip_fail(e, "aqr_build_batched: copy");
                }
                hipLaunchKernelGGL(dev::k_link_prep, dim3((unsigned)(((int64_t)nb * cap + 255) / 256)),
                                   dim3(256), 0, nullptr, adj0d, s0, cap, idsd, seld, nseld, nb, M,
                                   lkey, lval);
                size_t sb = sort_bytes;
                if ((e = hipGetLastError()) != hipSuccess ||
                    (e = hipcub::DeviceRadixSort::SortPairs(sort_tmp, sb, lkey, lkey_s, lval, lval_s,
                                                            (int)nl)) != hipSuccess) {
                    release();
                    return hip_fail(e, "aqr_build_batched: link sort");
                }
                hipLaunchKernelGGL(dev::k_reset, dim3(1), dim3(64), 0, nullptr, ctrd);
                hipLaunchKernelGGL(dev::k_reset, dim3(1), dim3(64), 0, nullptr, ctrd + 1);
                hipLaunchKernelGGL(dev::k_link_heads, dim3((unsigned)((nl + 255) / 256)), dim3(256),
                                   0, nullptr, lkey_s, nl, segd, ctrd);
                const int64_t lb = std::max<int64_t>(
                    1, std::min<int64_t>((nl + 3) / 4, (int64_t)std::max(1, ix->num_cu) * 8));
                hipLaunchKernelGGL(dev::k_link, dim3((unsigned)lb), dim3(256), 0, nullptr, ix->v,
                                   adj0d, s0, cap, idsd, M, lkey_s, lval_s, nl, segd, ctrd,
                                   ctrd + 1);
                if ((e = hipGetLastError()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
                    release();
                    return hip_fail(e, "aqr_build_batched: device links");
                }
                t_search += secs(ta, tb);
                t_link += secs(tb, now());
            } else {
                link_chunk(g.get(), codes, dp, ids, nb, keys.data(), efc, hcnt,
                           dev_select ? hsel : nullptr, dev_select ? hnsel : nullptr, T, dirty, mark);
                const auto tc = now();
                const int32_t nr = (int32_t)dirty.size();
                if ((int64_t)nr > max_dirty) {
                    release();
                    return fail(AQR_ERR_STATE, "aqr_build_batched: more changed rows than staged");
                }
                for (int32_t r = 0; r < nr; ++r) {
                    if ((int64_t)dirty[r] >= n) {
                        release();
                        return fail(AQR_ERR_STATE, "aqr_build_batched: row id out of range");
                    }
                    hrow[r] = dirty[r];
                }
                // gather the changed rows into the staging buffer, in parallel
                const int TG = (int)std::max<int64_t>(1, std::min<int64_t>(T, nr / 4096));
                const uint32_t* adj = g->adj0.data();
                parallel_for_threads(TG, [&](int t) {
                    const int32_t r0 = (int32_t)((int64_t)nr * t / TG);
                    const int32_t r1 = (int32_t)((int64_t)nr * (t + 1) / TG);
                    for (int32_t r = r0; r < r1; ++r)
                        std::memcpy(&hdat[(size_t)r * W], &adj[(size_t)hrow[r] * W],
                                    sizeof(uint32_t) * W);
                });
                if ((e = hipMemcpy(rowd, hrow, (size_t)nr * 4, hipMemcpyHostToDevice)) != hipSuccess ||
                    (e = hipMemcpy(datd, hdat, (size_t)nr * W * 4, hipMemcpyHostToDevice)) != hipSuccess) {
                    release();
                    return hip_fail(e, "aqr_build_batched: copy");
                }
                const int64_t tot = (int64_t)nr * W;
                hipLaunchKernelGGL(dev::k_scatter_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                                   nullptr, const_cast<uint32_t*>(ix->v.adj0), s0, rowd, datd, nr, W);
                if ((e = hipGetLastError()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
                    release();
                    return hip_fail(e, "aqr_build_batched: row update");
                }
                t_search += secs(ta, tb);
                t_link += secs(tb, tc);
                t_rows += secs(tc, now());
            }
            pos += nb;
            inserted += nb;
            if (p->progress > 0 && ((int64_t)pos >= next_report || pos == R.size())) {
                std::fprintf(stderr,
                             "[%s] %lld / %lld chunked points linked, %.1f s (device search "
                             "and selection %.1f s, linking %.1f s, row upload %.1f s)\n",
                             who, (long long)pos, (long long)R.size(), secs(t0, now()), t_search,
                             t_link, t_rows);
                std::fflush(stderr);
                next_report = (int64_t)pos + std::max<int64_t>(1, (int64_t)R.size() / p->progress);
            }
        }
        if (dev_link) {
            // the device adjacency is the graph's layer 0 now (rows at stride
            // s0): read back in blocks of rows through pinned staging, each
            // block repacked to 2M entries per row on the host threads
            const int64_t rb = std::max<int64_t>(1, ((int64_t)64 << 20) / ((int64_t)s0 * 4));
            uint32_t* stage = (uint32_t*)halloc((size_t)rb * s0 * 4);
            if (!stage) {
                release();
                return fail(AQR_ERR_OOM, "aqr_build_batched: pinned host memory for the read back");
            }
            for (int64_t r0 = 0; r0 < n; r0 += rb) {
                const int64_t nr = std::min<int64_t>(rb, n - r0);
                if ((e = hipMemcpy(stage, ix->v.adj0 + r0 * s0, (size_t)nr * s0 * 4,
                                   hipMemcpyDeviceToHost)) != hipSuccess) {
                    release();
                    return hip_fail(e, "aqr_build_batched: read back");
                }
                const int TR = (int)std::max<int64_t>(1, std::min<int64_t>(T, nr / 4096));
                uint32_t* dst = g->adj0.data();
                parallel_for_threads(TR, [&](int t) {
                    const int64_t a = nr * t / TR, z = nr * (t + 1) / TR;
                    for (int64_t r = a; r < z; ++r)
                        std::memcpy(&dst[(size_t)(r0 + r) * W], &stage[(size_t)r * s0],
                                    sizeof(uint32_t) * W);
                });
            }
        }
        release();
        *out = g.release();
        return AQR_OK;
    } catch (const std::bad_alloc&) {
        release();
        return fail(AQR_ERR_OOM, "aqr_build_batched: out of host memory");
    } catch (...) {
        release();
        return fail(AQR_ERR_STATE, "aqr_build_batched: unexpected failure");
    }
}
