/*
 * aqr_oracle.c -- plain CPU oracle of the AQR-HNSW method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product library
 * (libaqr) shares no code, header or table with it.
 *
 * Every function follows the paper's definitions step by step, in the
 * paper's order, without blocking, fusion or reordering.  Floating point is
 * FP64 except where the method itself produces FP32 values that later
 * decide an integer (quantizer ranges, scales, codes, decoded values); those
 * are computed in FP32 with IEEE operations, exactly as stated per function.
 * Build with -ffp-contract=off so that no multiply-add is fused.
 *
 * Keys.  Every ordering in the search uses the strict lexicographic key
 * (distance, id).  Integer code distances are at most d*255^2 < 2^53, so
 * they are held exactly in a double, and one key type serves both the
 * 8-bit code search and the FP32 baseline search.
 *
 * Graph exchange format (plain arrays, shared by value only):
 *   level[n]                      int32, layer of each node
 *   adj0[n][cap0]                 uint32, layer-0 neighbours, cap0 = 2*M,
 *                                 unused slots = 0xFFFFFFFF
 *   upper_off[n+1]                int64, node i owns rows upper_off[i] ..
 *                                 upper_off[i+1]-1, one row per layer
 *                                 1..level[i] (row upper_off[i]+l-1 is
 *                                 layer l)
 *   upper_adj[rows][cap1]         uint32, cap1 = M, padded with 0xFFFFFFFF
 *   entry point ep, top level L
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NONE 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* keys and sorted lists                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double dist;
    uint32_t id;
} okey;

static int okey_lt(okey a, okey b) {
    return a.dist < b.dist || (a.dist == b.dist && a.id < b.id);
}

/* Growable list kept sorted ascending by key. */
typedef struct {
    okey* a;
    int64_t n;
    int64_t cap;
} olist;

static int ol_init(olist* L, int64_t cap) {
    L->n = 0;
    L->cap = cap > 4 ? cap : 4;
    L->a = (okey*)malloc((size_t)L->cap * sizeof(okey));
    return L->a ? 0 : -1;
}

static void ol_free(olist* L) {
    free(L->a);
    L->a = NULL;
    L->n = L->cap = 0;
}

static int ol_insert(olist* L, okey k) {
    if (L->n == L->cap) {
        int64_t nc = L->cap * 2;
        okey* na = (okey*)realloc(L->a, (size_t)nc * sizeof(okey));
        if (!na) return -1;
        L->a = na;
        L->cap = nc;
    }
    int64_t i = L->n;
    while (i > 0 && okey_lt(k, L->a[i - 1])) {
        L->a[i] = L->a[i - 1];
        i--;
    }
    L->a[i] = k;
    L->n++;
    return 0;
}

static okey ol_pop_min(olist* L) {
    okey k = L->a[0];
    memmove(L->a, L->a + 1, (size_t)(L->n - 1) * sizeof(okey));
    L->n--;
    return k;
}

/* Plain insertion sort of an array of keys. */
static void okey_sort(okey* a, int64_t n) {
    for (int64_t i = 1; i < n; i++) {
        okey k = a[i];
        int64_t j = i;
        while (j > 0 && okey_lt(k, a[j - 1])) {
            a[j] = a[j - 1];
            j--;
        }
        a[j] = k;
    }
}

/* ------------------------------------------------------------------------ */
/* threads                                                                   */
/* ------------------------------------------------------------------------ */

void orc_set_threads(int32_t t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int32_t orc_get_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Section 3.1, Stage 1: density characterisation (Alg. 1, density and delta) */
/* ------------------------------------------------------------------------ */

/* Squared L2 in FP64 between two FP32 vectors. */
static double sq_l2_f64(const float* a, const float* b, int32_t d) {
    double s = 0.0;
    for (int32_t j = 0; j < d; j++) {
        double t = (double)a[j] - (double)b[j];
        s += t * t;
    }
    return s;
}

/*
 * Local density rho_i = 1 / (mean of the k smallest squared L2 distances
 * from x_i to the other points + eps).  Self is excluded; the neighbours
 * are taken over the whole dataset.  With n > threshold only the sample
 * S = { floor(s*n/n_s) : s = 0..n_s-1 }, n_s = min(n_s, n), is measured and
 * every other point receives the mean density of the sample.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int32_t orc_density(const float* X, int64_t n, int32_t d, int32_t k_rho, double eps,
                    int64_t n_s, int64_t threshold, double* rho) {
    if (!X || !rho || n < 1 || d < 1 || k_rho < 1 || n_s < 1) return -1;
    int64_t ns = n_s < n ? n_s : n;
    int sampled = n > threshold;
    int64_t m = sampled ? ns : n;
    int32_t k = (int64_t)k_rho < n - 1 ? k_rho : (int32_t)(n - 1);
    unsigned char* in_s = (unsigned char*)calloc((size_t)n, 1);
    if (!in_s) return -1;
    for (int64_t s = 0; s < m; s++) {
        int64_t i = sampled ? (int64_t)((s * n) / ns) : s;
        in_s[i] = 1;
    }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < m; s++) {
        int64_t i = sampled ? (int64_t)((s * n) / ns) : s;
        double best[64];
        double* kb = k <= 64 ? best : (double*)malloc((size_t)k * sizeof(double));
        if (!kb) {
            err = 1;
            continue;
        }
        int32_t cnt = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dij = sq_l2_f64(X + i * d, X + j * d, d);
            if (cnt < k) {
                int32_t p = cnt++;
                while (p > 0 && kb[p - 1] > dij) {
                    kb[p] = kb[p - 1];
                    p--;
                }
                kb[p] = dij;
            } else if (k > 0 && dij < kb[k - 1]) {
                int32_t p = k - 1;
                while (p > 0 && kb[p - 1] > dij) {
                    kb[p] = kb[p - 1];
                    p--;
                }
                kb[p] = dij;
            }
        }
        double mean = 0.0;
        if (k > 0) {
            double sum = 0.0;
            for (int32_t t = 0; t < k; t++) sum += kb[t];
            mean = sum / (double)k;
        }
        rho[i] = 1.0 / (mean + eps);
        if (kb != best) free(kb);
    }
    if (err) {
        free(in_s);
        return -1;
    }
    if (sampled) {
        double sum = 0.0;
        for (int64_t s = 0; s < m; s++) sum += rho[(s * n) / ns];
        double mean = sum / (double)m;
        for (int64_t i = 0; i < n; i++)
            if (!in_s[i]) rho[i] = mean;
    }
    free(in_s);
    return 0;
}

/* Alg. 1 heterogeneity: delta = (max rho - min rho) / (max rho + eps). */
double orc_delta(const double* rho, int64_t n, double eps) {
    double mx = rho[0], mn = rho[0];
    for (int64_t i = 1; i < n; i++) {
        if (rho[i] > mx) mx = rho[i];
        if (rho[i] < mn) mn = rho[i];
    }
    return (mx - mn) / (mx + eps);
}

/* ------------------------------------------------------------------------ */
/* Section 3.1, Stage 2: adaptive quantisation training                      */
/* ------------------------------------------------------------------------ */

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/*
 * Percentile of a sorted array with linear interpolation between order
 * statistics at h = p*(n-1) (the "linear" estimator), in FP64.
 */
double orc_percentile_sorted(const double* v, int64_t n, double p) {
    if (n == 1) return v[0];
    double h = p * (double)(n - 1);
    if (h <= 0.0) return v[0];
    if (h >= (double)(n - 1)) return v[n - 1];
    int64_t lo = (int64_t)floor(h);
    double f = h - (double)lo;
    return v[lo] + f * (v[lo + 1] - v[lo]);
}

/*
 * Per-dimension density weights: the reading of Algorithm 1's w_j in which
 * each dimension has a density of its own.  For dimension j, point i has the
 * one-dimensional density rho_i^(j) = 1 / (mean of the k smallest squared
 * differences (x_ij - x_lj)^2 over the other points l + eps), k as in
 * orc_density; w_j is the mean of rho_i^(j) over the measured points (all n,
 * or the sample of orc_density when n > threshold), summed in point order.
 * Each point's k smallest values are summed in ascending order.
 * Brute force over all pairs.  Returns 0, or -1 on bad arguments.
 */
int32_t orc_dim_weights(const float* X, int64_t n, int32_t d, int32_t k_rho, double eps,
                        int64_t n_s, int64_t threshold, double* w) {
    if (!X || !w || n < 1 || d < 1 || k_rho < 1 || k_rho > 64 || n_s < 1) return -1;
    int64_t ns = n_s < n ? n_s : n;
    int sampled = n > threshold;
    int64_t m = sampled ? ns : n;
    int32_t k = (int64_t)k_rho < n - 1 ? k_rho : (int32_t)(n - 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < d; j++) {
        double sum = 0.0;
        for (int64_t s = 0; s < m; s++) {
            int64_t i = sampled ? (int64_t)((s * n) / ns) : s;
            double best[64];
            int32_t cnt = 0;
            double xi = (double)X[i * d + j];
            for (int64_t l = 0; l < n; l++) {
                if (l == i) continue;
                double t = xi - (double)X[l * d + j];
                double v = t * t;
                if (cnt < k) {
                    int32_t p = cnt++;
                    while (p > 0 && best[p - 1] > v) {
                        best[p] = best[p - 1];
                        p--;
                    }
                    best[p] = v;
                } else if (k > 0 && v < best[k - 1]) {
                    int32_t p = k - 1;
                    while (p > 0 && best[p - 1] > v) {
                        best[p] = best[p - 1];
                        p--;
                    }
                    best[p] = v;
                }
            }
            double mean = 0.0;
            if (k > 0) {
                double acc = 0.0;
                for (int32_t t = 0; t < k; t++) acc += best[t];
                mean = acc / (double)k;
            }
            sum += 1.0 / (mean + eps);
        }
        w[j] = sum / (double)m;
    }
    return 0;
}

/*
 * Quantiser training (Alg. 1, Stage 2).
 *   p_lo = delta*p_max, p_hi = 1 - delta*p_max (fractions)
 *   min_j, max_j = FP32 rounding of the p_lo / p_hi percentiles of column j
 *   scale_j = 255 / ((max_j - min_j) + eps), each operation in FP32
 *   w_j = (1/n) sum_i rho_i for every j (the printed formula has no j)
 *   s_dist = sqrt( sum_j (max_j-min_j)^2 w_j / sum_j 255^2 w_j )   (Eq. 1)
 *   eta = sigma_w / mean_w (mean taken as w_0 + mean of (w_j - w_0))
 * scalars_out: [delta, p_lo, p_hi, s_dist, eta, w_mean]
 * w_in (d doubles) gives the weights of the per-dimension reading
 * (orc_dim_weights); NULL takes the literal reading above.
 */
int32_t orc_train_ranges(const float* X, int64_t n, int32_t d, const double* rho, double eps,
                         double p_max, float* mn, float* mx, float* scale,
                         double* scalars_out, const double* w_in) {
    if (!X || !rho || !mn || !mx || !scale || !scalars_out || n < 1 || d < 1) return -1;
    double delta = orc_delta(rho, n, eps);
    double p_lo = delta * p_max;
    double p_hi = 1.0 - delta * p_max;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < d; j++) {
        double* col = (double*)malloc((size_t)n * sizeof(double));
        if (!col) {
            err = 1;
            continue;
        }
        for (int64_t i = 0; i < n; i++) col[i] = (double)X[i * d + j];
        qsort(col, (size_t)n, sizeof(double), cmp_double);
        mn[j] = (float)orc_percentile_sorted(col, n, p_lo);
        mx[j] = (float)orc_percentile_sorted(col, n, p_hi);
        float range = mx[j] - mn[j];
        float denom = range + (float)1e-6;
        scale[j] = 255.0f / denom;
        free(col);
    }
    if (err) return -1;
    /* per-dimension weights, literally (1/n) sum_i rho_i */
    double rsum = 0.0;
    for (int64_t i = 0; i < n; i++) rsum += rho[i];
    double* w = (double*)malloc((size_t)d * sizeof(double));
    if (!w) return -1;
    for (int32_t j = 0; j < d; j++) w[j] = w_in ? w_in[j] : rsum / (double)n;
    double shift = 0.0;
    for (int32_t j = 0; j < d; j++) shift += w[j] - w[0];
    double wbar = w[0] + shift / (double)d;
    double var = 0.0;
    for (int32_t j = 0; j < d; j++) var += (w[j] - wbar) * (w[j] - wbar);
    double sigma = sqrt(var / (double)d);
    double eta = sigma / wbar;
    double num = 0.0, den = 0.0;
    for (int32_t j = 0; j < d; j++) {
        double r = (double)mx[j] - (double)mn[j];
        num += r * r * w[j];
        den += 255.0 * 255.0 * w[j];
    }
    double s_dist = sqrt(num / den);
    free(w);
    scalars_out[0] = delta;
    scalars_out[1] = p_lo;
    scalars_out[2] = p_hi;
    scalars_out[3] = s_dist;
    scalars_out[4] = eta;
    scalars_out[5] = wbar;
    return 0;
}

/* Alg. 1 connectivity and construction depth. out: [M_i, ef_construction] */
void orc_build_params(int32_t M0, int32_t efc0, double delta, double eta, int32_t* out) {
    out[0] = (int32_t)floor((double)M0 * (1.0 + delta * (1.0 + eta)));
    out[1] = (int32_t)floor((double)efc0 * (1.0 / (1.0 + delta * eta)));
}

/*
 * Vector encoding (Section 3.1 "Vector Encoding"; query encoding in Section
 * 3.2): shift by min_j, scale by scale_j, round to nearest (ties to even),
 * clip to [0, 255].  Each step is one FP32 operation:
 *   code = clamp(rint(fl32(fl32(x - min_j) * scale_j)), 0, 255).
 * Rows are written with stride `stride` bytes (>= d); padding bytes are 0.
 * Returns -1 (and writes nothing further) on a non-finite input.
 */
int32_t orc_encode(const float* X, int64_t n, int32_t d, const float* mn, const float* scale,
                   uint8_t* codes, int32_t stride) {
    if (!X || !mn || !scale || !codes || d < 1 || stride < d) return -1;
    for (int64_t i = 0; i < n * (int64_t)d; i++)
        if (!isfinite(X[i])) return -1;
    for (int64_t i = 0; i < n; i++) {
        for (int32_t j = 0; j < d; j++) {
            float t = X[i * d + j] - mn[j];
            float u = t * scale[j];
            float r = rintf(u);
            if (r < 0.0f) r = 0.0f;
            if (r > 255.0f) r = 255.0f;
            codes[i * stride + j] = (uint8_t)r;
        }
        for (int32_t j = d; j < stride; j++) codes[i * stride + j] = 0;
    }
    return 0;
}

/* Stage 2 decode: x~_j = fl32(fl32(code / scale_j) + min_j). */
void orc_decode(const uint8_t* codes, int64_t n, int32_t d, int32_t stride, const float* mn,
                const float* scale, float* out) {
    for (int64_t i = 0; i < n; i++)
        for (int32_t j = 0; j < d; j++) {
            float t = (float)codes[i * stride + j] / scale[j];
            out[i * d + j] = t + mn[j];
        }
}

/* ------------------------------------------------------------------------ */
/* vector spaces: distances used by the graph                                */
/* ------------------------------------------------------------------------ */

enum { SP_CODES = 0, SP_F32 = 1 };

typedef struct {
    int kind;
    int32_t d;
    int32_t stride; /* bytes per code row, or floats per FP32 row */
    const uint8_t* codes;
    const float* X;
} space;

/* Stage 1 distance: sum_j (q_j - x_j)^2 on 8-bit codes, exact integer. */
static double code_dist(const uint8_t* a, const uint8_t* b, int32_t d) {
    uint64_t s = 0;
    for (int32_t j = 0; j < d; j++) {
        int32_t t = (int32_t)a[j] - (int32_t)b[j];
        s += (uint64_t)(t * t);
    }
    return (double)s;
}

/* Distance from a query (codes or FP32, matching the space) to point id. */
static double sp_dist_q(const space* sp, const void* q, uint32_t id) {
    if (sp->kind == SP_CODES)
        return code_dist((const uint8_t*)q, sp->codes + (int64_t)id * sp->stride, sp->d);
    return sq_l2_f64((const float*)q, sp->X + (int64_t)id * sp->stride, sp->d);
}

static double sp_dist_pp(const space* sp, uint32_t a, uint32_t b) {
    if (sp->kind == SP_CODES)
        return code_dist(sp->codes + (int64_t)a * sp->stride, sp->codes + (int64_t)b * sp->stride,
                         sp->d);
    return sq_l2_f64(sp->X + (int64_t)a * sp->stride, sp->X + (int64_t)b * sp->stride, sp->d);
}

static const void* sp_point(const space* sp, uint32_t id) {
    if (sp->kind == SP_CODES) return sp->codes + (int64_t)id * sp->stride;
    return sp->X + (int64_t)id * sp->stride;
}

/* ------------------------------------------------------------------------ */
/* graph                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int32_t M;
    int32_t cap0, cap1;
    int32_t* level;
    uint32_t* adj0;
    int64_t* upper_off;
    uint32_t* upper_adj;
    uint32_t ep;
    int32_t L;
} graph;

static uint32_t* nbr_row(const graph* g, uint32_t x, int32_t layer, int32_t* cap) {
    if (layer == 0) {
        *cap = g->cap0;
        return g->adj0 + (int64_t)x * g->cap0;
    }
    *cap = g->cap1;
    return g->upper_adj + (g->upper_off[x] + layer - 1) * g->cap1;
}

static int32_t row_count(const uint32_t* row, int32_t cap) {
    int32_t c = 0;
    while (c < cap && row[c] != ORC_NONE) c++;
    return c;
}

/* HNSW level: floor(-ln(u) * m_L) with m_L = 1/ln(M); u in (0, 1]. */
int32_t orc_levels(const double* u, int64_t n, int32_t M, int32_t* level) {
    if (!u || !level || M < 2) return -1;
    double mL = 1.0 / log((double)M);
    for (int64_t i = 0; i < n; i++) {
        if (!(u[i] > 0.0 && u[i] <= 1.0)) return -1;
        level[i] = (int32_t)floor(-log(u[i]) * mL);
    }
    return 0;
}

/* Visited marks for one search (byte per node) with the list of marked ids. */
typedef struct {
    unsigned char* mark;
    uint32_t* list;
    int64_t n;
    int64_t cap;
} visited;

static int vis_init(visited* v, int64_t n) {
    v->mark = (unsigned char*)calloc((size_t)n, 1);
    v->cap = 1024;
    v->n = 0;
    v->list = (uint32_t*)malloc((size_t)v->cap * sizeof(uint32_t));
    return (v->mark && v->list) ? 0 : -1;
}

static void vis_free(visited* v) {
    free(v->mark);
    free(v->list);
}

static int vis_add(visited* v, uint32_t id) {
    if (v->n == v->cap) {
        int64_t nc = v->cap * 2;
        uint32_t* nl = (uint32_t*)realloc(v->list, (size_t)nc * sizeof(uint32_t));
        if (!nl) return -1;
        v->list = nl;
        v->cap = nc;
    }
    v->mark[id] = 1;
    v->list[v->n++] = id;
    return 0;
}

static void vis_reset(visited* v) {
    for (int64_t i = 0; i < v->n; i++) v->mark[v->list[i]] = 0;
    v->n = 0;
}

/* Debug taps of one layer search: expansion order and evaluated ids. */
typedef struct {
    uint32_t* expanded;
    int64_t n_expanded;
    int64_t cap_expanded;
} taps;

/*
 * SEARCH-LAYER of HNSW: candidate set C (min-first), result set W
 * (max-first) and visited set v, all under the key (distance, id).
 *   C = W = v = entry points
 *   loop: c = nearest in C, removed; stop if key(c) > furthest key in W;
 *         for each neighbour e of c at this layer not in v: add e to v;
 *           if |W| < ef or key(e) < furthest key in W: add e to C and W,
 *           and drop the furthest of W when |W| > ef.
 * W (ascending) is returned in *W.  v is left filled (the caller resets).
 */
static int search_layer(const graph* g, const space* sp, const void* q, const okey* eps,
                        int32_t n_eps, int32_t ef, int32_t layer, visited* v, olist* W,
                        taps* tp) {
    olist C;
    if (ol_init(&C, 64)) return -1;
    W->n = 0;
    for (int32_t i = 0; i < n_eps; i++) {
        if (v->mark[eps[i].id]) continue;
        if (vis_add(v, eps[i].id) || ol_insert(&C, eps[i]) || ol_insert(W, eps[i])) {
            ol_free(&C);
            return -1;
        }
    }
    while (W->n > ef) W->n--;
    while (C.n > 0) {
        okey c = ol_pop_min(&C);
        if (okey_lt(W->a[W->n - 1], c)) break;
        if (tp) {
            if (tp->n_expanded < tp->cap_expanded) tp->expanded[tp->n_expanded] = c.id;
            tp->n_expanded++;
        }
        int32_t cap;
        const uint32_t* row = nbr_row(g, c.id, layer, &cap);
        for (int32_t t = 0; t < cap && row[t] != ORC_NONE; t++) {
            uint32_t e = row[t];
            if (v->mark[e]) continue;
            if (vis_add(v, e)) {
                ol_free(&C);
                return -1;
            }
            okey ke = {sp_dist_q(sp, q, e), e};
            if (W->n < ef || okey_lt(ke, W->a[W->n - 1])) {
                if (ol_insert(&C, ke) || ol_insert(W, ke)) {
                    ol_free(&C);
                    return -1;
                }
                if (W->n > ef) W->n--;
            }
        }
    }
    ol_free(&C);
    return 0;
}

/*
 * Neighbour selection heuristic of HNSW (no candidate extension, no kept
 * pruned connections): walk the candidates nearest-first (key relative to
 * the base) and keep e unless some already kept r is strictly closer to e
 * than the base is, i.e. dist(e, r) < dist(e, base).  Stops at M kept.
 * cand must be sorted ascending by key relative to the base.
 */
static int32_t select_heuristic(const space* sp, const okey* cand, int64_t nc, int32_t M,
                                uint32_t* out) {
    int32_t r = 0;
    for (int64_t i = 0; i < nc && r < M; i++) {
        int good = 1;
        for (int32_t t = 0; t < r; t++) {
            if (sp_dist_pp(sp, cand[i].id, out[t]) < cand[i].dist) {
                good = 0;
                break;
            }
        }
        if (good) out[r++] = cand[i].id;
    }
    return r;
}

/* Exposed for tests: heuristic on FP32 points, candidates given as ids. */
int32_t orc_select_heuristic_f32(const float* X, int32_t d, uint32_t base, const uint32_t* ids,
                                 int32_t n_ids, int32_t M, uint32_t* out) {
    space sp = {SP_F32, d, d, NULL, X};
    okey* c = (okey*)malloc((size_t)(n_ids > 0 ? n_ids : 1) * sizeof(okey));
    if (!c) return -1;
    for (int32_t i = 0; i < n_ids; i++) {
        c[i].id = ids[i];
        c[i].dist = sp_dist_pp(&sp, base, ids[i]);
    }
    okey_sort(c, n_ids);
    int32_t r = select_heuristic(&sp, c, n_ids, M, out);
    free(c);
    return r;
}

/* Add a link from x to y at a layer, shrinking x's list with the heuristic
 * when it overflows its cap. */
static int add_link(graph* g, const space* sp, uint32_t x, uint32_t y, int32_t layer) {
    int32_t cap;
    uint32_t* row = nbr_row(g, x, layer, &cap);
    int32_t cnt = row_count(row, cap);
    if (cnt < cap) {
        row[cnt] = y;
        return 0;
    }
    okey* c = (okey*)malloc((size_t)(cap + 1) * sizeof(okey));
    uint32_t* sel = (uint32_t*)malloc((size_t)cap * sizeof(uint32_t));
    if (!c || !sel) {
        free(c);
        free(sel);
        return -1;
    }
    for (int32_t t = 0; t < cap; t++) {
        c[t].id = row[t];
        c[t].dist = sp_dist_pp(sp, x, row[t]);
    }
    c[cap].id = y;
    c[cap].dist = sp_dist_pp(sp, x, y);
    okey_sort(c, cap + 1);
    int32_t r = select_heuristic(sp, c, cap + 1, cap, sel);
    for (int32_t t = 0; t < cap; t++) row[t] = t < r ? sel[t] : ORC_NONE;
    free(c);
    free(sel);
    return 0;
}

/*
 * Sequential HNSW construction over the 8-bit codes (Alg. 1, Stage 3):
 * points are inserted in index order with connectivity M (cap M on upper
 * layers, 2M on layer 0) and construction depth efc.  Levels come from the
 * caller (orc_levels).  The caller allocates the exchange arrays; adj0 and
 * upper_adj are filled with 0xFFFFFFFF here before the build.
 * out2: [entry point, top level]
 */
int32_t orc_build(const uint8_t* codes, int64_t n, int32_t d, int32_t stride, int32_t M,
                  int32_t efc, const int32_t* level, uint32_t* adj0, const int64_t* upper_off,
                  uint32_t* upper_adj, int32_t* out2) {
    if (!codes || !level || !adj0 || !upper_off || !out2 || n < 1 || M < 2 || efc < 1)
        return -1;
    graph g;
    g.n = n;
    g.M = M;
    g.cap0 = 2 * M;
    g.cap1 = M;
    g.level = (int32_t*)level;
    g.adj0 = adj0;
    g.upper_off = (int64_t*)upper_off;
    g.upper_adj = upper_adj;
    for (int64_t i = 0; i < n * g.cap0; i++) adj0[i] = ORC_NONE;
    for (int64_t i = 0; i < upper_off[n] * g.cap1; i++) upper_adj[i] = ORC_NONE;
    space sp = {SP_CODES, d, stride, codes, NULL};
    visited v;
    if (vis_init(&v, n)) return -1;
    olist W;
    if (ol_init(&W, efc + 2)) {
        vis_free(&v);
        return -1;
    }
    okey* eps = (okey*)malloc((size_t)(efc + 2) * sizeof(okey));
    uint32_t* sel = (uint32_t*)malloc((size_t)M * sizeof(uint32_t));
    if (!eps || !sel) return -1;
    g.ep = 0;
    g.L = level[0];
    for (int64_t i = 1; i < n; i++) {
        const void* q = sp_point(&sp, (uint32_t)i);
        int32_t li = level[i];
        okey cur = {sp_dist_q(&sp, q, g.ep), g.ep};
        for (int32_t lc = g.L; lc > li; lc--) {
            if (search_layer(&g, &sp, q, &cur, 1, 1, lc, &v, &W, NULL)) return -1;
            vis_reset(&v);
            cur = W.a[0];
        }
        int32_t n_eps = 1;
        eps[0] = cur;
        for (int32_t lc = li < g.L ? li : g.L; lc >= 0; lc--) {
            if (search_layer(&g, &sp, q, eps, n_eps, efc, lc, &v, &W, NULL)) return -1;
            vis_reset(&v);
            int32_t r = select_heuristic(&sp, W.a, W.n, M, sel);
            int32_t cap;
            uint32_t* row = nbr_row(&g, (uint32_t)i, lc, &cap);
            for (int32_t t = 0; t < r; t++) row[t] = sel[t];
            for (int32_t t = 0; t < r; t++)
                if (add_link(&g, &sp, sel[t], (uint32_t)i, lc)) return -1;
            n_eps = (int32_t)W.n;
            for (int32_t t = 0; t < n_eps; t++) eps[t] = W.a[t];
        }
        if (li > g.L) {
            g.L = li;
            g.ep = (uint32_t)i;
        }
    }
    out2[0] = (int32_t)g.ep;
    out2[1] = g.L;
    free(eps);
    free(sel);
    ol_free(&W);
    vis_free(&v);
    return 0;
}

/*
 * Batched construction over the 8-bit codes: the same insertion step as
 * orc_build, in an order that lets many insertions search at once.
 *   Seed: every point below seed_n and every point with level >= 1, in
 *         increasing id order, in consecutive chunks of
 *         min(seed_batch, batch, max(1, floor(inserted / 8))) points, where
 *         inserted counts the points already in the graph.  Every point of a chunk
 *         plans its insertion against the graph as it stood before the
 *         chunk: greedy descent to one level above its own, then on each of
 *         its levels (top first) a search of width efc and the heuristic's
 *         M neighbours.  Then every point takes its lists; then the reverse
 *         links are added in id order, per point from its top level down;
 *         then the entry point moves to each point above the top level, in
 *         id order.
 *   Batches: the other points (level 0) follow in increasing id order, in
 *         chunks of min(batch, max(1, floor(inserted / 8))) points.  Every point of a chunk searches
 *         the graph as it stood before the chunk (greedy descent on the
 *         upper layers, then layer 0 with width efc), selects M neighbours
 *         with the heuristic and takes them as its layer-0 list; then each
 *         adds the reverse links, in id order.
 * With batch = 1 this is orc_build over the points in the order (seed
 * points, then the rest); with seed_batch = 1 and seed_n = n it is
 * orc_build.
 */
int32_t orc_build_batched(const uint8_t* codes, int64_t n, int32_t d, int32_t stride, int32_t M,
                          int32_t efc, const int32_t* level, int64_t seed_n, int32_t seed_batch,
                          int32_t batch, uint32_t* adj0, const int64_t* upper_off,
                          uint32_t* upper_adj, int32_t* out2) {
    if (!codes || !level || !adj0 || !upper_off || !out2 || n < 1 || M < 2 || efc < 1 ||
        seed_n < 1 || seed_batch < 1 || batch < 1)
        return -1;
    if (seed_batch > batch) seed_batch = batch;
    graph g;
    g.n = n;
    g.M = M;
    g.cap0 = 2 * M;
    g.cap1 = M;
    g.level = (int32_t*)level;
    g.adj0 = adj0;
    g.upper_off = (int64_t*)upper_off;
    g.upper_adj = upper_adj;
    for (int64_t i = 0; i < n * g.cap0; i++) adj0[i] = ORC_NONE;
    for (int64_t i = 0; i < upper_off[n] * g.cap1; i++) upper_adj[i] = ORC_NONE;
    space sp = {SP_CODES, d, stride, codes, NULL};
    visited v;
    olist W;
    okey* eps = (okey*)malloc((size_t)(efc + 2) * sizeof(okey));
    uint32_t* sel = (uint32_t*)malloc((size_t)(batch > 0 ? batch : 1) * M * sizeof(uint32_t));
    int32_t* nsel = (int32_t*)malloc((size_t)batch * sizeof(int32_t));
    uint32_t* chunk = (uint32_t*)malloc((size_t)batch * sizeof(uint32_t));
    if (vis_init(&v, n) || ol_init(&W, efc + 2) || !eps || !sel || !nsel || !chunk) return -1;
    g.ep = 0;
    g.L = level[0];
    int64_t inserted = 1;
    /* seed chunks: plans against the graph before the chunk, then lists,
     * reverse links and entry point, each in id order */
    int32_t Lmax = 0;
    for (int64_t i = 0; i < n; i++)
        if (level[i] > Lmax) Lmax = level[i];
    const int64_t nl = (int64_t)Lmax + 1;
    uint32_t* ssel = (uint32_t*)malloc((size_t)batch * nl * M * sizeof(uint32_t));
    int32_t* snsel = (int32_t*)malloc((size_t)batch * nl * sizeof(int32_t));
    int32_t* stop = (int32_t*)malloc((size_t)batch * sizeof(int32_t));
    if (!ssel || !snsel || !stop) return -1;
    int64_t next_seed = 1;
    for (;;) {
        int64_t want = inserted / 8;
        if (want < 1) want = 1;
        if (want > seed_batch) want = seed_batch;
        int32_t nb = 0;
        while (next_seed < n && nb < want) {
            if (next_seed < seed_n || level[next_seed] > 0) chunk[nb++] = (uint32_t)next_seed;
            next_seed++;
        }
        if (nb == 0) break;
        const uint32_t ep0 = g.ep;
        const int32_t L0 = g.L;
        for (int32_t b = 0; b < nb; b++) {
            const void* q = sp_point(&sp, chunk[b]);
            int32_t li = level[chunk[b]];
            okey cur = {sp_dist_q(&sp, q, ep0), ep0};
            for (int32_t lc = L0; lc > li; lc--) {
                if (search_layer(&g, &sp, q, &cur, 1, 1, lc, &v, &W, NULL)) return -1;
                vis_reset(&v);
                cur = W.a[0];
            }
            stop[b] = li < L0 ? li : L0;
            int32_t n_eps = 1;
            eps[0] = cur;
            for (int32_t lc = stop[b]; lc >= 0; lc--) {
                if (search_layer(&g, &sp, q, eps, n_eps, efc, lc, &v, &W, NULL)) return -1;
                vis_reset(&v);
                snsel[(int64_t)b * nl + lc] =
                    select_heuristic(&sp, W.a, W.n, M, ssel + ((int64_t)b * nl + lc) * M);
                n_eps = (int32_t)W.n;
                for (int32_t t = 0; t < n_eps; t++) eps[t] = W.a[t];
            }
        }
        for (int32_t b = 0; b < nb; b++)
            for (int32_t lc = stop[b]; lc >= 0; lc--) {
                int32_t cap;
                uint32_t* row = nbr_row(&g, chunk[b], lc, &cap);
                const uint32_t* sb = ssel + ((int64_t)b * nl + lc) * M;
                for (int32_t t = 0; t < snsel[(int64_t)b * nl + lc]; t++) row[t] = sb[t];
            }
        for (int32_t b = 0; b < nb; b++)
            for (int32_t lc = stop[b]; lc >= 0; lc--) {
                const uint32_t* sb = ssel + ((int64_t)b * nl + lc) * M;
                for (int32_t t = 0; t < snsel[(int64_t)b * nl + lc]; t++)
                    if (add_link(&g, &sp, sb[t], chunk[b], lc)) return -1;
            }
        for (int32_t b = 0; b < nb; b++)
            if (level[chunk[b]] > g.L) {
                g.L = level[chunk[b]];
                g.ep = chunk[b];
            }
        inserted += nb;
    }
    free(ssel);
    free(snsel);
    free(stop);
    /* batches of the remaining level-0 points */
    int64_t next = seed_n;
    for (;;) {
        int64_t want = inserted / 8;
        if (want < 1) want = 1;
        if (want > batch) want = batch;
        int32_t nb = 0;
        while (next < n && nb < want) {
            if (level[next] == 0) chunk[nb++] = (uint32_t)next;
            next++;
        }
        if (nb == 0) break;
        /* search and select against the graph as it stood before the chunk */
        for (int32_t b = 0; b < nb; b++) {
            const void* q = sp_point(&sp, chunk[b]);
            okey cur = {sp_dist_q(&sp, q, g.ep), g.ep};
            for (int32_t lc = g.L; lc > 0; lc--) {
                if (search_layer(&g, &sp, q, &cur, 1, 1, lc, &v, &W, NULL)) return -1;
                vis_reset(&v);
                cur = W.a[0];
            }
            if (search_layer(&g, &sp, q, &cur, 1, efc, 0, &v, &W, NULL)) return -1;
            vis_reset(&v);
            nsel[b] = select_heuristic(&sp, W.a, W.n, M, sel + (size_t)b * M);
        }
        for (int32_t b = 0; b < nb; b++) {
            int32_t cap;
            uint32_t* row = nbr_row(&g, chunk[b], 0, &cap);
            for (int32_t t = 0; t < nsel[b]; t++) row[t] = sel[(size_t)b * M + t];
        }
        for (int32_t b = 0; b < nb; b++)
            for (int32_t t = 0; t < nsel[b]; t++)
                if (add_link(&g, &sp, sel[(size_t)b * M + t], chunk[b], 0)) return -1;
        inserted += nb;
    }
    out2[0] = (int32_t)g.ep;
    out2[1] = g.L;
    free(eps);
    free(sel);
    free(nsel);
    free(chunk);
    ol_free(&W);
    vis_free(&v);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2, Alg. 2: search                                               */
/* ------------------------------------------------------------------------ */

static void make_graph(graph* g, int64_t n, int32_t M, const int32_t* level, const uint32_t* adj0,
                       const int64_t* upper_off, const uint32_t* upper_adj, uint32_t ep,
                       int32_t L) {
    g->n = n;
    g->M = M;
    g->cap0 = 2 * M;
    g->cap1 = M;
    g->level = (int32_t*)level;
    g->adj0 = (uint32_t*)adj0;
    g->upper_off = (int64_t*)upper_off;
    g->upper_adj = (uint32_t*)upper_adj;
    g->ep = ep;
    g->L = L;
}

/*
 * Search parameters (reading of Section 3.2 with Table 3):
 *   ef_eff = max(ef, k); N_c = clamp(floor(ef_eff / m_ef), k, ef_eff).
 * out2: [ef_eff, N_c]
 */
void orc_param_map(int32_t k, int32_t ef, int32_t m_ef, int32_t* out2) {
    int32_t efe = ef > k ? ef : k;
    int32_t nc = efe / m_ef;
    if (nc < k) nc = k;
    if (nc > efe) nc = efe;
    out2[0] = efe;
    out2[1] = nc;
}

/* One query: greedy descent through layers L..1 (search with ef = 1), then
 * the layer-0 search with ef; returns the first `take` entries of W. */
static int query_one(const graph* g, const space* sp, const void* q, int32_t ef, int32_t take,
                     visited* v, olist* W, uint32_t* out_id, double* out_dist, int32_t* out_cnt,
                     taps* tp, uint32_t* vis_out, int64_t vis_cap, int64_t* vis_n) {
    okey cur = {sp_dist_q(sp, q, g->ep), g->ep};
    for (int32_t lc = g->L; lc >= 1; lc--) {
        if (search_layer(g, sp, q, &cur, 1, 1, lc, v, W, NULL)) return -1;
        vis_reset(v);
        cur = W->a[0];
    }
    if (search_layer(g, sp, q, &cur, 1, ef, 0, v, W, tp)) return -1;
    if (vis_out) {
        for (int64_t t = 0; t < v->n && t < vis_cap; t++) vis_out[t] = v->list[t];
    }
    if (vis_n) *vis_n = v->n;
    vis_reset(v);
    int32_t cnt = (int32_t)(W->n < take ? W->n : take);
    for (int32_t t = 0; t < cnt; t++) {
        out_id[t] = W->a[t].id;
        out_dist[t] = W->a[t].dist;
    }
    *out_cnt = cnt;
    return 0;
}

/*
 * Stage 1 (Alg. 2, coarse quantised search) for a batch of encoded
 * queries qcodes[nq][stride].  Per query: ef_eff[q] and nc[q].
 * Outputs: cand_id/cand_D [nq][nc_stride] (D is the exact integer sum of
 * squared code differences; the reported d^q is s_dist * D), cand_cnt[nq].
 * Optional taps (NULL to skip): expanded[nq][tap_cap] with n_expanded[nq]
 * (layer-0 expansion order) and visited[nq][tap_cap] with n_visited[nq]
 * (distinct layer-0 evaluated ids in evaluation order).
 */
int32_t orc_search_codes(const uint8_t* codes, int64_t n, int32_t d, int32_t stride, int32_t M,
                         const int32_t* level, const uint32_t* adj0, const int64_t* upper_off,
                         const uint32_t* upper_adj, uint32_t ep, int32_t L, const uint8_t* qcodes,
                         int64_t nq, const int32_t* ef_eff, const int32_t* nc, int32_t nc_stride,
                         uint32_t* cand_id, uint32_t* cand_D, int32_t* cand_cnt, int32_t tap_cap,
                         uint32_t* expanded, int64_t* n_expanded, uint32_t* vis, int64_t* n_vis) {
    graph g;
    make_graph(&g, n, M, level, adj0, upper_off, upper_adj, ep, L);
    space sp = {SP_CODES, d, stride, codes, NULL};
    int err = 0;
#pragma omp parallel
    {
        visited v;
        olist W;
        double* dd = (double*)malloc((size_t)(nc_stride > 0 ? nc_stride : 1) * sizeof(double));
        int ok = vis_init(&v, n) == 0 && ol_init(&W, 64) == 0 && dd;
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < nq; qi++) {
            if (!ok) {
                err = 1;
                continue;
            }
            taps tp = {expanded ? expanded + qi * tap_cap : NULL, 0, expanded ? tap_cap : 0};
            int64_t vn = 0;
            int32_t take = nc[qi] < nc_stride ? nc[qi] : nc_stride;
            if (query_one(&g, &sp, qcodes + qi * stride, ef_eff[qi], take, &v, &W,
                          cand_id + qi * nc_stride, dd, &cand_cnt[qi], &tp,
                          vis ? vis + qi * tap_cap : NULL, tap_cap, &vn)) {
                err = 1;
                continue;
            }
            for (int32_t t = 0; t < cand_cnt[qi]; t++) cand_D[qi * nc_stride + t] = (uint32_t)dd[t];
            if (n_expanded) n_expanded[qi] = tp.n_expanded;
            if (n_vis) n_vis[qi] = vn;
        }
        if (ok) {
            vis_free(&v);
            ol_free(&W);
        }
        free(dd);
    }
    return err ? -1 : 0;
}

/*
 * Baseline HNSW on FP32 vectors (same graph), distances in FP64.
 * Returns the first k[q] of W per query: out_id/out_dist [nq][k_stride],
 * padded with (-1, +inf).  expanded (optional, [nq][tap_cap]) records the
 * layer-0 expansion order and n_expanded[q] its length, as in
 * orc_search_codes.
 */
int32_t orc_search_f32(const float* X, int64_t n, int32_t d, int32_t M, const int32_t* level,
                       const uint32_t* adj0, const int64_t* upper_off, const uint32_t* upper_adj,
                       uint32_t ep, int32_t L, const float* Q, int64_t nq, const int32_t* ef_eff,
                       const int32_t* k, int32_t k_stride, int32_t* out_id, double* out_dist,
                       int64_t* n_vis, uint32_t* expanded, int32_t tap_cap, int32_t* n_expanded) {
    graph g;
    make_graph(&g, n, M, level, adj0, upper_off, upper_adj, ep, L);
    space sp = {SP_F32, d, d, NULL, X};
    int err = 0;
#pragma omp parallel
    {
        visited v;
        olist W;
        uint32_t* ids = (uint32_t*)malloc((size_t)(k_stride > 0 ? k_stride : 1) * sizeof(uint32_t));
        int ok = vis_init(&v, n) == 0 && ol_init(&W, 64) == 0 && ids;
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < nq; qi++) {
            if (!ok) {
                err = 1;
                continue;
            }
            int32_t cnt = 0;
            int64_t vn = 0;
            int32_t take = k[qi] < k_stride ? k[qi] : k_stride;
            taps tp = {expanded ? expanded + qi * tap_cap : NULL, 0, expanded ? tap_cap : 0};
            if (query_one(&g, &sp, Q + qi * d, ef_eff[qi], take, &v, &W, ids,
                          out_dist + qi * k_stride, &cnt, &tp, NULL, 0, &vn)) {
                err = 1;
                continue;
            }
            if (n_expanded) n_expanded[qi] = tp.n_expanded;
            for (int32_t t = 0; t < k_stride; t++) {
                if (t < cnt) {
                    out_id[qi * k_stride + t] = (int32_t)ids[t];
                } else {
                    out_id[qi * k_stride + t] = -1;
                    out_dist[qi * k_stride + t] = INFINITY;
                }
            }
            if (n_vis) n_vis[qi] = vn;
        }
        if (ok) {
            vis_free(&v);
            ol_free(&W);
        }
        free(ids);
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2, Alg. 2: Stage 2, early termination, Stage 3, assembly         */
/* ------------------------------------------------------------------------ */

/*
 * Re-rank a batch of Stage-1 candidate lists.
 *   Stage 2: decode every candidate (x~ in FP32, IEEE division), d^a =
 *            sum_j (q_j - x~_j)^2 in FP64; A = sort by (d^a, id).
 *   Early termination when |A| > k: with d_k, d_{k+1} the k-th and
 *            (k+1)-th d^a (1-based), gap = (d_{k+1}-d_k)/(d_k+eps),
 *            ratio = d_{k+1}/(d_k+eps); ET = gap > tau_gap or ratio >
 *            tau_ratio.  force_et[q] (NULL = automatic): -1 automatic,
 *            0 never, 1 always.
 *   Stage 3: n_rr = min(|A|, k) under ET, else min(|A|, max(N_rerank, k));
 *            exact d^e = sum_j (q_j - x_j)^2 in FP64 for A[0..n_rr).
 *   Assembly: R = exact entries, then A[n_rr..] with their d^a while
 *            |R| < k (assembly 0, "as needed to ensure at least k"), or
 *            all of A[n_rr..] (assembly 1, the union reading of R_exact
 *            with the remaining candidates); sorted by (distance, id); top
 *            k; padding (-1, +inf).
 * a_order (optional, [nq][nc_stride]): if given, replaces the Stage-2 sort
 * with this externally supplied order of the candidates (must be a
 * permutation of the candidate list).
 * Outputs: out_id/out_dist/out_kind [nq][k_stride] (kind 1 = exact, 2 =
 * asymmetric, 0 = padding); taps (NULL to skip): a_id/a_dist [nq][nc_stride]
 * (the A list), et[nq], nrr[nq].
 */
int32_t orc_rerank(const float* X, const uint8_t* codes, int64_t n, int32_t d, int32_t stride,
                   const float* mn, const float* scale, const float* Q, int64_t nq,
                   const uint32_t* cand_id, const int32_t* cand_cnt, int32_t nc_stride,
                   const int32_t* k, int32_t k_stride, int32_t n_rerank, double tau_gap,
                   double tau_ratio, double eps, const int32_t* force_et, int32_t assembly,
                   const uint32_t* a_order, int32_t* out_id, double* out_dist, uint8_t* out_kind,
                   uint32_t* a_id, double* a_dist, uint8_t* et_out, int32_t* nrr_out) {
    (void)n;
    int err = 0;
#pragma omp parallel
    {
        okey* A = (okey*)malloc((size_t)(nc_stride + 1) * sizeof(okey));
        okey* R = (okey*)malloc((size_t)(nc_stride + k_stride + 1) * sizeof(okey));
        uint8_t* Rk = (uint8_t*)malloc((size_t)(nc_stride + k_stride + 1));
        float* xt = (float*)malloc((size_t)d * sizeof(float));
        int ok = A && R && Rk && xt;
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < nq; qi++) {
            if (!ok) {
                err = 1;
                continue;
            }
            const float* q = Q + qi * d;
            int32_t nc = cand_cnt[qi];
            int32_t kq = k[qi];
            /* Stage 2: asymmetric distances */
            for (int32_t t = 0; t < nc; t++) {
                uint32_t id = cand_id[qi * nc_stride + t];
                orc_decode(codes + (int64_t)id * stride, 1, d, stride, mn, scale, xt);
                double s = 0.0;
                for (int32_t j = 0; j < d; j++) {
                    double diff = (double)q[j] - (double)xt[j];
                    s += diff * diff;
                }
                A[t].id = id;
                A[t].dist = s;
            }
            if (a_order) {
                /* take the supplied order: look each id up in A */
                okey* B = R;
                for (int32_t t = 0; t < nc; t++) {
                    uint32_t id = a_order[qi * nc_stride + t];
                    int32_t f = -1;
                    for (int32_t u = 0; u < nc; u++)
                        if (A[u].id == id) {
                            f = u;
                            break;
                        }
                    if (f < 0) {
                        err = 1;
                        f = 0;
                    }
                    B[t] = A[f];
                }
                memcpy(A, B, (size_t)nc * sizeof(okey));
            } else {
                okey_sort(A, nc);
            }
            /* early termination */
            int et = 0;
            if (nc > kq) {
                double dk = A[kq - 1].dist, dk1 = A[kq].dist;
                double gap = (dk1 - dk) / (dk + eps);
                double ratio = dk1 / (dk + eps);
                et = (gap > tau_gap) || (ratio > tau_ratio);
            }
            if (force_et && force_et[qi] >= 0) et = force_et[qi] != 0;
            int32_t want = et ? kq : (n_rerank > kq ? n_rerank : kq);
            int32_t nrr = nc < want ? nc : want;
            /* Stage 3: exact distances on the first n_rr of A */
            int32_t nr = 0;
            for (int32_t t = 0; t < nrr; t++) {
                const float* x = X + (int64_t)A[t].id * d;
                R[nr].id = A[t].id;
                R[nr].dist = sq_l2_f64(q, x, d);
                Rk[nr] = 1;
                nr++;
            }
            /* assembly: fill from A only while fewer than k results, or
             * (union) take every remaining candidate */
            for (int32_t t = nrr; t < nc && (assembly == 1 || nr < kq); t++) {
                R[nr] = A[t];
                Rk[nr] = 2;
                nr++;
            }
            /* sort R by (dist, id), carrying the kind */
            for (int32_t i = 1; i < nr; i++) {
                okey kk = R[i];
                uint8_t kd = Rk[i];
                int32_t j = i;
                while (j > 0 && okey_lt(kk, R[j - 1])) {
                    R[j] = R[j - 1];
                    Rk[j] = Rk[j - 1];
                    j--;
                }
                R[j] = kk;
                Rk[j] = kd;
            }
            for (int32_t t = 0; t < k_stride; t++) {
                int64_t o = qi * k_stride + t;
                if (t < kq && t < nr) {
                    out_id[o] = (int32_t)R[t].id;
                    out_dist[o] = R[t].dist;
                    if (out_kind) out_kind[o] = Rk[t];
                } else {
                    out_id[o] = -1;
                    out_dist[o] = INFINITY;
                    if (out_kind) out_kind[o] = 0;
                }
            }
            if (a_id)
                for (int32_t t = 0; t < nc; t++) {
                    a_id[qi * nc_stride + t] = A[t].id;
                    a_dist[qi * nc_stride + t] = A[t].dist;
                }
            if (et_out) et_out[qi] = (uint8_t)et;
            if (nrr_out) nrr_out[qi] = nrr;
        }
        free(A);
        free(R);
        free(Rk);
        free(xt);
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* exact k-nearest neighbours by brute force                                 */
/* ------------------------------------------------------------------------ */

/* FP64 squared L2, ties by id; out_id/out_dist [nq][k]. */
int32_t orc_knn_f32(const float* X, int64_t n, int32_t d, const float* Q, int64_t nq, int32_t k,
                    int32_t* out_id, double* out_dist) {
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; qi++) {
        olist W;
        if (ol_init(&W, k + 1)) {
            err = 1;
            continue;
        }
        for (int64_t j = 0; j < n; j++) {
            okey kj = {sq_l2_f64(Q + qi * d, X + j * d, d), (uint32_t)j};
            if (W.n < k || okey_lt(kj, W.a[W.n - 1])) {
                ol_insert(&W, kj);
                if (W.n > k) W.n--;
            }
        }
        for (int32_t t = 0; t < k; t++) {
            out_id[qi * k + t] = t < W.n ? (int32_t)W.a[t].id : -1;
            out_dist[qi * k + t] = t < W.n ? W.a[t].dist : INFINITY;
        }
        ol_free(&W);
    }
    return err ? -1 : 0;
}

/* Integer code distance brute force, ties by id; out [nq][k]. */
int32_t orc_knn_codes(const uint8_t* codes, int64_t n, int32_t d, int32_t stride,
                      const uint8_t* qcodes, int64_t nq, int32_t k, uint32_t* out_id,
                      uint32_t* out_D) {
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; qi++) {
        olist W;
        if (ol_init(&W, k + 1)) {
            err = 1;
            continue;
        }
        for (int64_t j = 0; j < n; j++) {
            okey kj = {code_dist(qcodes + qi * stride, codes + j * stride, d), (uint32_t)j};
            if (W.n < k || okey_lt(kj, W.a[W.n - 1])) {
                ol_insert(&W, kj);
                if (W.n > k) W.n--;
            }
        }
        for (int32_t t = 0; t < k; t++) {
            out_id[qi * k + t] = t < W.n ? W.a[t].id : ORC_NONE;
            out_D[qi * k + t] = t < W.n ? (uint32_t)W.a[t].dist : ORC_NONE;
        }
        ol_free(&W);
    }
    return err ? -1 : 0;
}
