// internal.hpp -- host-side structures shared by the translation units of
// libaqr (quantiser, graph builder, device index).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/aqr.h"

namespace aqr {

// Thread-local error message; returns the status for one-line use.
aqr_status fail(aqr_status st, const std::string& msg);
void clear_error();

inline int32_t round_up(int32_t x, int32_t m) { return (x + m - 1) / m * m; }

// Number of host worker threads for a request (0 = all hardware threads).
int host_threads(int32_t requested);

// Run fn(t) for t in [0, T) on T threads (T >= 1) and join.
template <class F>
void parallel_for_threads(int T, F fn);

struct Quantizer {
    aqr_qinfo info{};
    std::vector<float> mn, mx, scale;  // d each
};

// Graph in the exchange layout (see aqr_graph_export).
struct Graph {
    int64_t n = 0;
    int32_t M = 0, efc = 0;
    int32_t L = 0;
    uint32_t ep = 0;
    std::vector<int32_t> level;
    std::vector<uint32_t> adj0;      // n * 2M
    std::vector<int64_t> upper_off;  // n + 1
    std::vector<uint32_t> upper_adj; // rows * M
};

}  // namespace aqr

struct aqr_quantizer : aqr::Quantizer {};
struct aqr_graph : aqr::Graph {};

namespace aqr {
// Graph construction pieces shared with the device build (build.cpp).
// chunk_max 0: the seed is inserted one point at a time (concurrently when
// p->threads > 1); chunk_max >= 1: in chunks (see build.cpp), the same graph
// for every thread count.
aqr_status build_seeded(const uint8_t* codes, int64_t n, int32_t d, const aqr_quantizer* qz,
                        const aqr_bparams* p, const double* level_u, int64_t seed_n,
                        int32_t chunk_max, const char* who, aqr_graph** out);
// sel / nsel (nb x M, nb), when given, are the heuristic's selections made
// elsewhere (the device); otherwise link_chunk selects from cand / cnt.
void link_chunk(aqr_graph* g, const uint8_t* codes, int32_t dp, const uint32_t* ids, int32_t nb,
                const uint64_t* cand, int32_t stride, const int32_t* cnt,
                const uint32_t* sel_in, const int32_t* nsel_in, int threads,
                std::vector<uint32_t>& dirty, std::vector<uint8_t>& mark);
// Stage-1 densities on the current device (density.hip): for each of the m
// sample rows S[s] of X (host, n x d), the FP64 sum in ascending order of the
// k smallest squared distances to the other rows, into sums[s].
aqr_status device_density_sums(const float* X, int64_t n, int32_t d, const int64_t* S, int64_t m,
                               int32_t k, int T, double* sums);
}  // namespace aqr

#include <thread>

namespace aqr {
template <class F>
void parallel_for_threads(int T, F fn) {
    if (T <= 1) {
        fn(0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 0; t < T; ++t) th.emplace_back(fn, t);
    for (auto& x : th) x.join();
}
}  // namespace aqr
