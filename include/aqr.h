/*
 * aqr.h -- C-ABI of libaqr, the MI355X (gfx950) AQR-HNSW query path.
 *
 * AQR-HNSW (arXiv 2602.21600) searches an HNSW graph with density-aware
 * 8-bit codes and re-ranks the result in stages.  This library provides:
 *   aqr_quantize   Alg. 1 stages 1-2 (density, percentile ranges, scales,
 *                  codes, Eq. 1), host
 *   aqr_build      Alg. 1 stage 3 (HNSW over the codes), host
 *   aqr_search     Alg. 2 stage 1 (query encoding + coarse quantised graph
 *                  search), device
 *   aqr_rerank     Alg. 2 stages 2-3 (asymmetric distances, early
 *                  termination, exact FP32 re-rank, assembly), device
 * plus the baseline FP32 HNSW search on the same graph, batch plans (one
 * captured launch of uneven queries) and a serving loop (a resident kernel
 * with continuous admission).
 *
 * Conventions
 *   - Every call returns an aqr_status; aqr_last_error() gives a message for
 *     the calling thread.  No C++ exception crosses this interface and the
 *     library never aborts.
 *   - Host pointers are read during the call only.  Device pointers are
 *     allocated and owned by the caller; the query path allocates no device
 *     memory (only the build-time calls aqr_build_batched,
 *     aqr_quantize_device and aqr_density with device != 0 allocate device
 *     memory of their own, and free it before they return).  Handles
 *     (aqr_quantizer, aqr_graph, aqr_index) are created and freed by the
 *     library.
 *   - Device calls are asynchronous on the given stream (a hipStream_t passed
 *     as void*, NULL = default stream).  Arguments are validated on the host
 *     before any launch; a device fault surfaces at the caller's next
 *     synchronisation.
 *   - A batch call with nq = 0 returns AQR_OK without launching anything;
 *     its buffers may then be NULL.
 *   - Keys: every ordering is by (distance, id), id ascending on ties.
 *   - A bound index is read-only; concurrent calls on different streams are
 *     allowed when each call has its own workspace and outputs.
 */
#ifndef AQR_H
#define AQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AQR_VERSION 1
#define AQR_NONE 0xFFFFFFFFu

typedef enum aqr_status {
    AQR_OK = 0,
    AQR_ERR_INVALID_ARG = 1, /* a null pointer, a size out of range, a non-finite value */
    AQR_ERR_OOM = 2,         /* host allocation failed, or a caller buffer is too small */
    AQR_ERR_DEVICE = 3,      /* a HIP call failed */
    AQR_ERR_BUSY = 4,        /* serving: no slot or budget for the request */
    AQR_ERR_CORRUPT = 5,     /* an index blob failed its checks */
    AQR_ERR_STATE = 6        /* a handle is used in the wrong state */
} aqr_status;

/* Message of the last failing call on this thread (never NULL). */
const char* aqr_last_error(void);
int32_t aqr_version(void);

/* ------------------------------------------------------------------------ */
/* Alg. 1 stages 1-2: quantiser (host)                                       */
/* ------------------------------------------------------------------------ */

typedef struct aqr_qparams {
    int32_t k_rho;            /* neighbours of the local density (Section 3.1: 10) */
    int32_t threads;          /* host threads, 0 = all hardware threads */
    int64_t n_sample;         /* density sample size n_s (5000) */
    int64_t sample_threshold; /* densities are sampled when n > this (10000) */
    double eps;               /* epsilon of density, delta and scales (1e-6) */
    double p_max;             /* maximum percentile width P_max, fraction (0.01) */
    int32_t M0;               /* base connectivity M_0 */
    int32_t efc0;             /* base construction depth ef_0 */
    int32_t weights;          /* density weights w_j of Alg. 1 (Eq. 1, eta): 0 = the
                                 printed formula, every w_j the mean density, so
                                 eta = 0; 1 = per-dimension weights, w_j the mean
                                 one-dimensional k_rho-NN density along dimension j
                                 over the measured points (eta > 0) */
} aqr_qparams;

typedef struct aqr_qinfo {
    int32_t d;      /* dimension */
    int32_t d_pad;  /* bytes per code row: d rounded up to 16 */
    int32_t M;      /* M_i = floor(M_0 (1 + delta (1 + eta)))  (Alg. 1) */
    int32_t efc;    /* ef^construction = floor(ef_0 / (1 + delta eta))  (Alg. 1) */
    double delta;   /* global heterogeneity (Alg. 1) */
    double p_lo;    /* lower percentile, fraction: delta * P_max */
    double p_hi;    /* upper percentile, fraction: 1 - delta * P_max */
    double s_dist;  /* distance scale of Eq. 1 */
    double eta;     /* dimension heterogeneity sigma_w / mean_w */
    double w_mean;  /* mean density weight */
} aqr_qinfo;

typedef struct aqr_quantizer aqr_quantizer;

/*
 * Train the quantiser on X (host, n x d FP32, row-major) and encode it.
 * Section 3.1 Stage 1 (densities from the k_rho nearest neighbours, sampled
 * for large n; delta) and Stage 2 (percentile bounds, min_j/max_j/scale_j,
 * density weights, Eq. 1, eta; Alg. 1), and the vector encoding
 * code = clamp(rint(fl32(fl32(x - min_j) * scale_j)), 0, 255).
 * If *qz is NULL a quantiser is trained and returned in *qz (free with
 * aqr_quantizer_free); if *qz is an existing quantiser, X is only encoded.
 * codes_out (host, n x d_pad bytes, may be NULL) receives the codes, padding
 * bytes 0.  Non-finite input values give AQR_ERR_INVALID_ARG.
 */
aqr_status aqr_quantize(const float* X, int64_t n, int32_t d, const aqr_qparams* p,
                        aqr_quantizer** qz, uint8_t* codes_out);

/*
 * aqr_quantize with the density search of Section 3.1 Stage 1 (the k_rho
 * nearest neighbours of every sample point over all n points) on the current
 * device; the rest of the training and the encoding run on the host.  Every
 * distance is summed in the same FP64 order as on the host and the k smallest
 * are summed in ascending order, so the quantiser and the codes are those of
 * aqr_quantize bit for bit.  X stays a host array: the call copies it to
 * device memory it allocates (n x d floats, hipMalloc) and frees before it
 * returns, and waits for its work.  k_rho <= 64.  HIP failures give
 * AQR_ERR_DEVICE; the other errors are those of aqr_quantize.
 */
aqr_status aqr_quantize_device(const float* X, int64_t n, int32_t d, const aqr_qparams* p,
                               aqr_quantizer** qz, uint8_t* codes_out);

/*
 * The densities rho_i of Section 3.1 Stage 1 into rho (host, n doubles):
 * 1 / (mean of the k_rho smallest squared L2 distances to the other points
 * + eps), FP64; with n > p->sample_threshold only the points
 * floor(s n / n_s), s < n_s = min(p->n_sample, n), are measured and every
 * other point gets their mean.  device != 0 runs the neighbour search on the
 * current device (as aqr_quantize_device), 0 on p->threads host threads;
 * both give the same values.  Only p->k_rho (<= 64), n_sample,
 * sample_threshold, eps and threads are read.
 */
aqr_status aqr_density(const float* X, int64_t n, int32_t d, const aqr_qparams* p,
                       int32_t device, double* rho);

/* Copy out the scalars and the per-dimension min_j, max_j, scale_j (each d
 * floats; any array pointer may be NULL). */
aqr_status aqr_quantizer_info(const aqr_quantizer* qz, aqr_qinfo* info, float* min_out,
                              float* max_out, float* scale_out);

/* Create a quantiser from stored parameters (info->d, M, efc and the
 * scalars are taken as given). */
aqr_status aqr_quantizer_create(const aqr_qinfo* info, const float* mn, const float* mx,
                                const float* scale, aqr_quantizer** out);
void aqr_quantizer_free(aqr_quantizer* qz);

/* ------------------------------------------------------------------------ */
/* Alg. 1 stage 3: HNSW graph over the codes (host)                          */
/* ------------------------------------------------------------------------ */

typedef struct aqr_bparams {
    int32_t M;             /* connectivity; <= 0 takes M_i of the quantiser */
    int32_t efc;           /* construction depth; <= 0 takes ef^c of the quantiser */
    int32_t threads;       /* 1 = sequential and deterministic, 0 = all hardware threads */
    int32_t progress;      /* > 0: a line on stderr after each 1/progress of the points */
    uint64_t seed;         /* level draws when level_u is NULL (SplitMix64) */
} aqr_bparams;

typedef struct aqr_ginfo {
    int64_t n;
    int32_t M;          /* layer cap M on layers >= 1, 2M on layer 0 */
    int32_t efc;
    int32_t L;          /* top level */
    uint32_t ep;        /* entry point */
    int64_t upper_rows; /* sum of levels: rows of the upper-layer table */
} aqr_ginfo;

typedef struct aqr_graph aqr_graph;

/*
 * Build the HNSW graph over codes (host, n x d_pad bytes) by inserting the
 * points in index order (Alg. 1: G.Insert(q_i, i, M_i, ef^c)).  Levels are
 * floor(-ln(u_i) / ln(M)) with u_i = level_u[i] in (0, 1] (host, n doubles),
 * or drawn from SplitMix64(seed) when level_u is NULL.  With threads == 1
 * the build is sequential and deterministic; otherwise points are inserted
 * concurrently (the graph then depends on thread timing).
 */
aqr_status aqr_build(const uint8_t* codes, int64_t n, int32_t d, const aqr_quantizer* qz,
                     const aqr_bparams* p, const double* level_u, aqr_graph** g);

aqr_status aqr_graph_info(const aqr_graph* g, aqr_ginfo* info);

/*
 * Export / import the graph as plain arrays (host):
 *   level[n]                int32
 *   adj0[n][2M]             uint32, layer-0 neighbours, unused = AQR_NONE
 *   upper_off[n+1]          int64, node i owns rows upper_off[i]..upper_off[i+1]-1,
 *                           row upper_off[i]+l-1 is layer l
 *   upper_adj[rows][M]      uint32, unused = AQR_NONE
 */
aqr_status aqr_graph_export(const aqr_graph* g, int32_t* level, uint32_t* adj0,
                            int64_t* upper_off, uint32_t* upper_adj);
aqr_status aqr_graph_import(int64_t n, int32_t M, const int32_t* level, const uint32_t* adj0,
                            const int64_t* upper_off, const uint32_t* upper_adj, uint32_t ep,
                            aqr_graph** g);
void aqr_graph_free(aqr_graph* g);

/*
 * Batched construction with the layer-0 searches on the current device
 * (the insertion step of Alg. 1 and HNSW, reordered so that many insertions
 * search at once).  Points are inserted in id order in chunks of
 * min(cap, max(1, floor(m / 8))) points, m = points already in the graph:
 * first the seed (every point below seed_n and every point with level >= 1)
 * with cap = min(seed_batch, batch), then the other points with cap = batch.  Every point of a chunk searches the graph as it
 * stood before the chunk and selects its neighbours with the heuristic: a
 * seed point on every level it occupies (on the host, chunk points in
 * parallel), any other point on layer 0 (search and selection on the
 * device; the selection on the host when M > 64).  Then each point takes
 * its lists, the reverse links are added in id order per target (for the
 * other points on the device when 2M + 1 <= 64, else on the host, different
 * target nodes in parallel) and, for the seed, the entry point moves to
 * each point above the top level, in id order.  The graph does not
 * depend on threads; batch = 1 is sequential insertion, and seed_batch = 1
 * with seed_n >= n is aqr_build with threads == 1 (with seed_n >= n no
 * device is used).  Small seed chunks keep the upper layers close to those
 * of sequential insertion (64 is a good default).
 * codes: host, n x d_pad; X: host FP32 n x d, the vectors the codes encode
 * (the device search encodes them again).  The call allocates and frees
 * device memory for the index and the chunks (hipMalloc) and pinned host
 * staging for the chunk copies (hipHostMalloc), and waits for its work.
 * Levels and p as in aqr_build; efc <= 1024.
 */
aqr_status aqr_build_batched(const uint8_t* codes, const float* X, int64_t n, int32_t d,
                             const aqr_quantizer* qz, const aqr_bparams* p, const double* level_u,
                             int64_t seed_n, int32_t seed_batch, int32_t batch,
                             aqr_graph** out);

/* ------------------------------------------------------------------------ */
/* index file: quantiser, codes, FP32 rows and graph in one checksummed file */
/* ------------------------------------------------------------------------ */

typedef struct aqr_index_header {
    int64_t n;
    int32_t d;
    int32_t d_pad;
    int32_t M;
    int32_t reserved;
    int64_t upper_rows;
    uint64_t file_bytes;
} aqr_index_header;

/*
 * Write a built index (host): the quantiser of Section 3.1 (min_j, max_j,
 * scale_j and the scalars of Alg. 1), the codes (n x d_pad bytes), the FP32
 * rows X (n x d) that Stage 3 re-ranks with, and the HNSW graph, with a
 * CRC-32C (Castagnoli, RFC 3720) per 64 MiB block.  n is the graph's; the
 * file is replaced if it exists.  I/O failures give AQR_ERR_STATE.
 */
aqr_status aqr_index_save(const char* path, const aqr_quantizer* qz, const aqr_graph* g,
                          const uint8_t* codes, const float* X);
/* Read and check the header of an index file (shapes, section table, file
 * length): AQR_ERR_CORRUPT on a mismatch or a truncated file. */
aqr_status aqr_index_file_info(const char* path, aqr_index_header* info);
/*
 * Load an index file: *qz and *g receive new handles (free with
 * aqr_quantizer_free / aqr_graph_free); codes_out (host, n x d_pad bytes)
 * and X_out (host, n x d floats) are caller buffers sized from
 * aqr_index_file_info.  Every block checksum, the zero padding of the code
 * rows and the graph's structure are verified; any mismatch, a truncated
 * file or trailing bytes give AQR_ERR_CORRUPT, and no handle is returned.
 */
aqr_status aqr_index_load(const char* path, aqr_quantizer** qz, aqr_graph** g,
                          uint8_t* codes_out, float* X_out);

/* ------------------------------------------------------------------------ */
/* device index                                                              */
/* ------------------------------------------------------------------------ */

typedef struct aqr_index aqr_index;

/* Bytes of the device arena aqr_index_bind needs for this quantiser/graph. */
aqr_status aqr_index_bytes(const aqr_quantizer* qz, const aqr_graph* g, size_t* bytes);

/*
 * Copy the index into a caller-owned device arena (dev_arena, arena_bytes
 * >= aqr_index_bytes) on stream s and wait for the copy: codes (host,
 * n x d_pad), FP32 originals X (host, n x d, kept for the exact re-rank,
 * Alg. 1), the graph and the quantiser.  The returned handle refers to the
 * arena; it does not own it.  The arena must outlive the handle.
 */
aqr_status aqr_index_bind(const aqr_quantizer* qz, const aqr_graph* g, const uint8_t* codes,
                          const float* X, void* dev_arena, size_t arena_bytes, void* stream,
                          aqr_index** ix);
void aqr_index_free(aqr_index* ix);

/* ------------------------------------------------------------------------ */
/* Alg. 2 stage 1: coarse quantised search (device)                          */
/* ------------------------------------------------------------------------ */

typedef struct aqr_sparams {
    int32_t ef_max;       /* >= every ef_eff = max(ef, k) of the batch (<= 1024) */
    int32_t out_stride;   /* row stride of the per-query outputs (N_c or k) */
    int32_t m_ef;         /* ef multiplier when nc is not given (Table 3: 2 or 3) */
    int32_t waves_per_block; /* 0 = library default */
    int32_t blocks;       /* persistent grid size, 0 = fill the device */
    int32_t visited_log2; /* log2 of visited-cache buckets (4 ids each), 0 = 7, in [4, 14];
                             raised to (id bits - 16) when smaller.  The launch
                             adds the buckets (fewer than 2^visited_log2) that
                             fit in the LDS its resident blocks leave unused;
                             with 16 stored bits it needs at least one, else it
                             takes the next size.  No result depends on it. */
    const int32_t* order; /* device, nullable: work order of the queries (a permutation) */
    /* Two list sizes in one launch (0 = off): small_waves of the
     * waves_per_block waves of each block (0 <= small_waves < waves_per_block)
     * keep LDS for lists of ef_small (1 <= ef_small < ef_max) instead of
     * ef_max, so more waves fit on a CU.  Queries with ef_eff > ef_small go
     * to the other waves, which take the rest once those are done.  The
     * split expects order to list the queries with ef_eff > ef_small first
     * (as a longest-first order does); if it does not, only the ef_max waves
     * search.  No result depends on these fields. */
    int32_t ef_small;
    int32_t small_waves;
} aqr_sparams;

typedef struct aqr_taps {
    int32_t cap;          /* ids recorded per query in the lists below */
    uint32_t* expanded;   /* device [nq][cap], nullable: layer-0 expansion order */
    uint32_t* evaluated;  /* device [nq][cap], nullable: layer-0 evaluated ids, in
                             order, re-evaluations after cache evictions included */
    uint32_t* counts;     /* device [nq][8], nullable: layer-0 expansions,
                             layer-0 evaluations, upper-layer evaluations,
                             admissions to W, upper-layer expansions, query
                             duration and start time (low, high word) in ticks
                             of the 100 MHz device real-time clock */
} aqr_taps;

/* Workspace bytes for aqr_search / aqr_search_fp32. */
size_t aqr_search_workspace_size(void);

/*
 * Stage 1 for nq queries Q (device, nq x d FP32).  Per query (device arrays
 * of nq int32): k, ef, and optionally nc (NULL derives
 * N_c = clamp(floor(ef_eff / m_ef), k, ef_eff), ef_eff = max(ef, k)).
 * Each query is encoded (Section 3.2, same rounding as aqr_quantize),
 * descends the upper layers greedily and searches layer 0 with ef_eff
 * (Section 3.2 Stage 1, Algorithm 2).  Outputs (device): cand_id and cand_D [nq][out_stride]
 * hold the first N_c entries of the result list, ascending by (D, id), where
 * D = sum_j (q^_j - x^_j)^2 is the exact integer code distance (the paper's
 * d^q is s_dist * D); cand_cnt[nq] = number written, or -1 for a query with
 * invalid parameters (k < 1, ef_eff > ef_max, N_c > out_stride) or a
 * non-finite value.  ws: device workspace of aqr_search_workspace_size()
 * bytes.  taps may be NULL.
 */
aqr_status aqr_search(const aqr_index* ix, const float* Q, int64_t nq, const int32_t* k,
                      const int32_t* ef, const int32_t* nc, const aqr_sparams* sp,
                      uint32_t* cand_id, uint32_t* cand_D, int32_t* cand_cnt, void* ws,
                      size_t ws_bytes, const aqr_taps* taps, void* stream);

/* Query encoding alone (device): qcodes [nq][d_pad] bytes, padding 0. */
aqr_status aqr_encode_queries(const aqr_index* ix, const float* Q, int64_t nq, uint8_t* qcodes,
                              void* stream);

/* ------------------------------------------------------------------------ */
/* Alg. 2 stages 2-3: re-rank (device)                                       */
/* ------------------------------------------------------------------------ */

typedef struct aqr_rparams {
    int32_t n_rerank;     /* N_rerank (Table 3: 12..28) */
    int32_t out_stride;   /* row stride of out_id/out_dist/out_kind (>= every k) */
    float tau_gap;        /* gap threshold (Table 3) */
    float tau_ratio;      /* ratio threshold (Table 3) */
    float eps;            /* epsilon of gap and ratio (1e-6) */
    int32_t force_et;     /* -1 automatic, 0 never, 1 always */
    int32_t waves_per_block; /* 0 = library default */
    int32_t assembly;     /* Alg. 2 assembly, two readings: 0 fills R with the next
                             candidates of A (with their d^a) only while it holds fewer
                             than k results; 1 joins every candidate of A not re-ranked
                             to the exact results and keeps the k smallest.  Other
                             values: AQR_ERR_INVALID_ARG */
} aqr_rparams;

typedef struct aqr_rtaps {
    uint32_t* a_id;   /* device [nq][nc_stride], nullable: the A list (Stage 2 order) */
    float* a_dist;    /* device [nq][nc_stride], nullable: its d^a */
    uint8_t* et;      /* device [nq], nullable: early-termination decision */
    int32_t* nrr;     /* device [nq], nullable: candidates re-ranked exactly */
} aqr_rtaps;

/*
 * Stages 2-3 for nq queries (Section 3.2, Algorithm 2), on the Stage-1 lists
 * cand_id/cand_cnt (device, stride nc_stride) and the FP32 queries Q:
 *   d^a = sum_j (q_j - x~_j)^2 with x~_j = fl32(fl32(x^_j / scale_j) + min_j),
 *   A = candidates sorted by (d^a, id);
 *   early termination when |A| > k: gap = (d_{k+1}-d_k)/(d_k+eps) > tau_gap or
 *   ratio = d_{k+1}/(d_k+eps) > tau_ratio;
 *   n_rr = min(|A|, k) under early termination, else min(|A|, max(n_rerank, k));
 *   exact d^e = sum_j (q_j - x_j)^2 (FP32, fused multiply-add) on A[0..n_rr);
 *   R = the exact entries, then A[n_rr..] with their d^a while |R| < k;
 *   top k of R by (distance, id), padded with (-1, +inf).
 * Outputs (device, [nq][out_stride]): out_id int32, out_dist float,
 * out_kind uint8 (nullable; 1 exact, 2 asymmetric, 0 padding).  A query
 * with cand_cnt < 0 or k outside [1, out_stride] is all padding.
 */
aqr_status aqr_rerank(const aqr_index* ix, const float* Q, int64_t nq, const uint32_t* cand_id,
                      const int32_t* cand_cnt, int32_t nc_stride, const int32_t* k,
                      const aqr_rparams* rp, int32_t* out_id, float* out_dist, uint8_t* out_kind,
                      const aqr_rtaps* taps, void* stream);

/* ------------------------------------------------------------------------ */
/* baseline: HNSW on FP32 vectors over the same graph (device)               */
/* ------------------------------------------------------------------------ */

/*
 * Baseline HNSW search (Section 4.1 "Baseline HNSW") on the FP32 originals
 * of the index, same graph and same search as aqr_search with FP32 squared
 * L2 distances (fused multiply-add).  Per query k and ef (device); outputs
 * (device) out_id/out_dist [nq][sp->out_stride]: the first k of the result
 * list, padded with (-1, +inf); a query with invalid parameters is all
 * padding.
 */
aqr_status aqr_search_fp32(const aqr_index* ix, const float* Q, int64_t nq, const int32_t* k,
                           const int32_t* ef, const aqr_sparams* sp, int32_t* out_id,
                           float* out_dist, void* ws, size_t ws_bytes, const aqr_taps* taps,
                           void* stream);

/* ------------------------------------------------------------------------ */
/* exact k nearest neighbours by brute force (device)                        */
/* ------------------------------------------------------------------------ */

/*
 * The exact truth of the recall measure (Section 4.1: recall@k against the
 * true k nearest neighbours under L2): for each of the nq queries Q (device,
 * nq x d FP32, row stride d) the k rows of X (device, n x d FP32, row stride
 * d) with the smallest squared L2 distance, ordered by (distance, id).
 * Rows are screened with FP32 matrix products on the matrix cores
 * (|x|^2 - 2 q.x); the k + 32 best screened rows (rounded up to 16) are
 * re-scored exactly in FP64, summing (q_j - x_j)^2 over j in order, so the
 * distances are those of the FP64 definition bit for bit.
 * Outputs (device): out_id [nq][k] (int32, -1 past n), out_dist [nq][k]
 * (FP64, +inf past n); certified [nq] (nullable): 1 when an error bound of
 * the FP32 screening proves that no row outside the re-scored candidates
 * can enter the top k, else 0.
 * ws: device workspace of at least aqr_knn_workspace_size(n, nq, k) bytes,
 * 16-byte aligned, owned by the caller; it is overwritten.  1 <= k <= 128,
 * 1 <= d <= 4096, 1 <= n < 2^31.  Inputs must be finite (non-finite values
 * give unspecified ids, never an out-of-bounds access).  Asynchronous on
 * stream; nq = 0 launches nothing.
 */
size_t aqr_knn_workspace_size(int64_t n, int64_t nq, int32_t k);
aqr_status aqr_knn_bruteforce(const float* X, int64_t n, int32_t d, const float* Q, int64_t nq,
                              int32_t k, int32_t* out_id, double* out_dist, uint8_t* certified,
                              void* ws, size_t ws_bytes, void* stream);

/*
 * aqr_knn_bruteforce without a caller workspace, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a fixed array of
 * aqr_knn_noalloc_max_bytes() bytes in device memory that the library holds
 * on each device until the process ends; a call needing more
 * (aqr_knn_workspace_size(n, nq, k) above it) fails with
 * AQR_ERR_INVALID_ARG, and the caller splits the queries.  The call
 * allocates nothing.  Every call on one device shares that device's array:
 * calls that overlap on one device (other streams, other threads) race and
 * must be serialised by the caller.  Results equal aqr_knn_bruteforce's.
 */
size_t aqr_knn_noalloc_max_bytes(void);
aqr_status aqr_knn_bruteforce_noalloc(const float* X, int64_t n, int32_t d, const float* Q,
                                      int64_t nq, int32_t k, int32_t* out_id, double* out_dist,
                                      uint8_t* certified, void* stream);

/* ------------------------------------------------------------------------ */
/* batch plans: one captured launch sequence for uneven batches (device)     */
/* ------------------------------------------------------------------------ */

typedef struct aqr_batch_buffers {
    const float* Q;       /* device [nq_max][d] queries */
    int64_t nq_max;
    const int32_t* k;     /* device [nq_max] per-query k */
    const int32_t* ef;    /* device [nq_max] per-query ef */
    uint32_t* cand_id;    /* device [nq_max][sp->out_stride] Stage-1 ids */
    uint32_t* cand_D;     /* device [nq_max][sp->out_stride] Stage-1 distances */
    int32_t* cand_cnt;    /* device [nq_max] */
    int32_t* out_id;      /* device [nq_max][rp->out_stride] */
    float* out_dist;      /* device [nq_max][rp->out_stride] */
    uint8_t* out_kind;    /* device [nq_max][rp->out_stride], nullable */
    int32_t* order;       /* device [nq_max], nullable: work order scratch; when given,
                             queries run longest first (ef_eff descending) */
    void* ws;             /* device workspace of aqr_search_workspace_size() bytes */
    size_t ws_bytes;
    uint32_t* counts;     /* device [nq_max][8], nullable: per-query counters (aqr_taps) */
} aqr_batch_buffers;

typedef struct aqr_plan aqr_plan;

/*
 * A plan binds an index, search and re-rank parameters and caller-owned
 * device buffers (none of which may move while the plan lives).  Launching
 * it runs, on the given stream: the longest-first work order (when
 * buffers->order is given), aqr_search over the batch with per-query k and
 * ef (N_c derived with sp->m_ef), and aqr_rerank.  With use_graph != 0 the
 * first launch for a given nq runs the sequence once on the given stream and
 * records it into a hipGraph on a private stream of the plan; later launches
 * with the same nq replay the graph on the given stream (one graph launch).
 * Results are identical either way.  sp->order must be NULL (the plan owns
 * the order).  A plan is not thread-safe; use one plan per stream.
 */
aqr_status aqr_plan_create(const aqr_index* ix, const aqr_sparams* sp, const aqr_rparams* rp,
                           const aqr_batch_buffers* buffers, int32_t use_graph, aqr_plan** plan);
/* Run the plan on the first nq queries of the buffers (0 <= nq <= nq_max). */
aqr_status aqr_plan_launch(aqr_plan* plan, int64_t nq, void* stream);
void aqr_plan_free(aqr_plan* plan);

/* ------------------------------------------------------------------------ */
/* serving: continuous admission into a resident persistent kernel           */
/* ------------------------------------------------------------------------ */

typedef struct aqr_server_params {
    int32_t ring;         /* request slots: requests admitted and not yet collected */
    int32_t k_max;        /* largest k accepted (row length of a result) */
    int32_t ef_max;       /* largest ef accepted (<= 1024) */
    int32_t m_ef;         /* ef multiplier of N_c */
    int32_t n_rerank;     /* N_rerank */
    float tau_gap, tau_ratio, eps;  /* early termination (Table 3 row "0.97+": 0.010, 1.008) */
    int32_t waves_per_block;        /* 0 = 4 */
    int32_t visited_log2;           /* largest visited cache of a request (log2 buckets of
                                       four ids), 0 = 9; a request gets
                                       2^clamp(ceil(log2 ef_eff) + 1, lo, this), lo = the
                                       smallest that keeps the stored id remainder within
                                       15 bits (idbits - 15, at least 4) */
    int32_t idle_ms;      /* the kernel exits after this long without unclaimed requests */
    int32_t reserved;
    int64_t state_budget; /* bytes of request state (query, result ids and distances) in
                             pinned host memory; 0 = ring requests at k_max */
    int64_t lds_budget_pages; /* admission limit on the LDS pages of requests admitted and
                                 not yet collected; 0 = what the resident waves hold at
                                 once, one largest request each */
} aqr_server_params;

typedef struct aqr_server_usage_t {
    int32_t ring;
    int32_t slots_used;
    int64_t lds_budget_pages;
    int64_t lds_used_pages;
    int64_t state_budget;
    int64_t state_used;
    int32_t blocks;       /* resident blocks of the server kernel */
    int32_t run_pages;    /* LDS pages each resident wave holds for a request */
} aqr_server_usage_t;

typedef struct aqr_server aqr_server;

size_t aqr_server_workspace_size(void);

/*
 * A server keeps the index resident and runs one persistent kernel on a
 * private stream, sized to the device (every block resident).  Requests go
 * into a ring in pinned host memory; each wave takes the next published
 * request as soon as it is free, so requests that arrive while others run
 * start on the next free wave.  One wave mirrors the host's publication
 * counter into device memory; the kernel leaves after idle_ms without
 * unclaimed requests or on aqr_server_stop, and submit/poll relaunch it when
 * needed.  While the kernel runs, its blocks hold most of the device; other
 * work on the device runs in what they leave free, and aqr_server_stop (or
 * idle_ms of quiet) releases it.  ws: caller-owned device workspace
 * (aqr_server_workspace_size() bytes) for the claim counters.
 *
 * Memory per request, sized by its own k and ef (not k_max and ef_max):
 * LDS pages (of the region each resident wave holds for one request) for the
 * result list W (ef_eff keys), the neighbour staging and a visited cache that
 * grows with ef_eff, overlaid after Stage 1 by the Stage 2-3 arrays for its
 * N_c candidates; and request state in pinned host memory (the query and k
 * ids and distances).
 * Admission charges both against the server's budgets
 * (aqr_server_request_cost) and returns them when the result is collected.
 * Each request runs Stage 1 and Stages 2-3 with the same code as
 * aqr_search/aqr_rerank, so its result equals the batch result for the same
 * query, k and ef, whatever else is in flight.
 */
aqr_status aqr_server_create(const aqr_index* ix, const aqr_server_params* p, void* ws,
                             size_t ws_bytes, aqr_server** server);
/* Admit one request (host query of d floats); *ticket is an opaque handle
 * for aqr_server_poll.  AQR_ERR_BUSY when the request does not fit: no free
 * slot, its queue entry not yet read by a worker, or its LDS pages or state
 * bytes beyond what the budgets have left; it fits again once earlier
 * results are collected.  AQR_ERR_INVALID_ARG when k or ef exceed the
 * server limits. */
aqr_status aqr_server_submit(aqr_server* s, const float* q, int32_t k, int32_t ef,
                             uint64_t* ticket);
/* *done = 1 and the result row (k_max entries, padded with (-1, +inf)) is
 * copied when the request is complete; the slot is then free again. */
aqr_status aqr_server_poll(aqr_server* s, uint64_t ticket, int32_t* out_id, float* out_dist,
                           int32_t* done);
/* The LDS pages and state bytes a request of this k and ef is charged. */
aqr_status aqr_server_request_cost(const aqr_server* s, int32_t k, int32_t ef,
                                   int32_t* lds_pages, int64_t* state_bytes);
/* Budgets and what is in use. */
aqr_status aqr_server_usage(aqr_server* s, aqr_server_usage_t* usage);
aqr_status aqr_server_stop(aqr_server* s);
void aqr_server_destroy(aqr_server* s);
/*
 * Replay an arrival trace from the host: request i (query Q[i], k[i], ef[i])
 * arrives at arrival_s[i] seconds after the start and is submitted then, or
 * as soon as the server admits it; latency_s[i] runs from its arrival to the
 * poll that finds it complete; service_s[i] (nullable) is the device time
 * from the wave's claim of the request to its completion.  out_id/out_dist
 * (nullable): [n][k_max].  AQR_ERR_STATE when no request completes for 60 s.
 */
aqr_status aqr_server_replay(aqr_server* s, int64_t n, const double* arrival_s, const float* Q,
                             const int32_t* k, const int32_t* ef, int32_t* out_id,
                             float* out_dist, double* latency_s, double* service_s,
                             double* wall_s);

#ifdef __cplusplus
}
#endif

#endif /* AQR_H */
