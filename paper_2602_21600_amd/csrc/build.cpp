// build.cpp -- host HNSW construction of libaqr (Alg. 1 stage 3).
//
// Points are inserted in index order (G.Insert(q_i, i, M_i, ef^c)) with the
// HNSW procedure the paper builds on: greedy descent (search width 1) from
// the top level to level l_i + 1, then on each level l_i..0 a layer search
// of width ef^c whose result seeds the next level, M neighbours picked by
// the diversity heuristic (keep a candidate unless an already kept
// neighbour is strictly closer to it than the new point), reverse links,
// and a heuristic shrink of any list that exceeds its cap (M on levels >= 1,
// 2M on level 0).  Distances are the exact integer squared L2 of the 8-bit
// codes; every ordering is by (D, id) packed into one 64-bit key.
//
// threads == 1 inserts sequentially (deterministic).  With more threads the
// points are inserted concurrently: each neighbour list is read and written
// under a striped lock, and an insertion that raises the top level holds
// the entry-point lock for its whole duration.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <queue>
#include <thread>

#include "internal.hpp"

namespace aqr {

namespace {

constexpr uint32_t kNone = AQR_NONE;
constexpr int kLockStripes = 1 << 16;

inline uint32_t l2u8(const uint8_t* __restrict a, const uint8_t* __restrict b, int32_t dp) {
    uint32_t s = 0;
    for (int32_t j = 0; j < dp; ++j) {
        int32_t t = (int32_t)a[j] - (int32_t)b[j];
        s += (uint32_t)(t * t);
    }
    return s;
}

inline uint64_t mk(uint32_t D, uint32_t id) { return ((uint64_t)D << 32) | id; }
inline uint32_t key_id(uint64_t k) { return (uint32_t)k; }
inline uint32_t key_D(uint64_t k) { return (uint32_t)(k >> 32); }

uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Visited {
    std::vector<uint32_t> tag;
    uint32_t epoch = 0;
    explicit Visited(int64_t n) : tag(n, 0) {}
    void next() {
        if (++epoch == 0) {
            std::fill(tag.begin(), tag.end(), 0);
            epoch = 1;
        }
    }
    bool test_set(uint32_t i) {
        if (tag[i] == epoch) return true;
        tag[i] = epoch;
        return false;
    }
};

struct Builder {
    Graph& g;
    const uint8_t* codes;
    int32_t dp;
    int32_t M, cap0, cap1, efc;
    std::vector<std::mutex> locks;
    std::mutex ep_lock;
    bool concurrent;

    Builder(Graph& g_, const uint8_t* c, int32_t dp_, bool conc)
        : g(g_), codes(c), dp(dp_), M(g_.M), cap0(2 * g_.M), cap1(g_.M), efc(g_.efc),
          locks(conc ? kLockStripes : 1), concurrent(conc) {}

    const uint8_t* row_of(uint32_t i) const { return codes + (int64_t)i * dp; }
    uint32_t dist(uint32_t a, uint32_t b) const { return l2u8(row_of(a), row_of(b), dp); }

    uint32_t* nbrs(uint32_t x, int32_t layer, int32_t& cap) {
        if (layer == 0) {
            cap = cap0;
            return g.adj0.data() + (int64_t)x * cap0;
        }
        cap = cap1;
        return g.upper_adj.data() + (g.upper_off[x] + layer - 1) * cap1;
    }
    std::mutex& lock_of(uint32_t x) { return locks[concurrent ? (x & (kLockStripes - 1)) : 0]; }

    // copy x's list at a layer (under its lock when concurrent)
    int32_t read_list(uint32_t x, int32_t layer, uint32_t* out) {
        int32_t cap;
        const uint32_t* r = nbrs(x, layer, cap);
        if (concurrent) {
            std::lock_guard<std::mutex> lk(lock_of(x));
            return copy_list(r, cap, out);
        }
        return copy_list(r, cap, out);
    }
    static int32_t copy_list(const uint32_t* r, int32_t cap, uint32_t* out) {
        int32_t c = 0;
        while (c < cap && r[c] != kNone) {
            out[c] = r[c];
            ++c;
        }
        return c;
    }

    // Layer search of width ef from the given entry keys; result ascending.
    void search_layer(uint32_t q, const std::vector<uint64_t>& eps, int32_t ef, int32_t layer,
                      Visited& vis, std::vector<uint64_t>& out) {
        std::priority_queue<uint64_t, std::vector<uint64_t>, std::greater<uint64_t>> C;
        std::priority_queue<uint64_t> W;
        vis.next();
        // The point being inserted is never its own candidate. A concurrent
        // insert can link it into a list before its own layer-0 search runs;
        // in a sequential build this mark changes nothing.
        vis.test_set(q);
        for (uint64_t e : eps) {
            if (vis.test_set(key_id(e))) continue;
            C.push(e);
            W.push(e);
        }
        while ((int32_t)W.size() > ef) W.pop();
        std::vector<uint32_t> buf(std::max(cap0, cap1));
        const uint8_t* qr = row_of(q);
        while (!C.empty()) {
            uint64_t c = C.top();
            C.pop();
            if (c > W.top()) break;
            int32_t cnt = read_list(key_id(c), layer, buf.data());
            for (int32_t t = 0; t < cnt; ++t) {
                uint32_t e = buf[t];
                if (vis.test_set(e)) continue;
                uint64_t ke = mk(l2u8(qr, row_of(e), dp), e);
                if ((int32_t)W.size() < ef || ke < W.top()) {
                    C.push(ke);
                    W.push(ke);
                    if ((int32_t)W.size() > ef) W.pop();
                }
            }
        }
        out.resize(W.size());
        for (size_t i = out.size(); i-- > 0;) {
            out[i] = W.top();
            W.pop();
        }
    }

    // Diversity heuristic; cand ascending by key relative to base.
    int32_t heuristic(const uint64_t* cand, size_t nc, int32_t m, uint32_t* sel) const {
        int32_t r = 0;
        for (size_t i = 0; i < nc && r < m; ++i) {
            const uint32_t e = key_id(cand[i]);
            const uint32_t de = key_D(cand[i]);
            bool good = true;
            for (int32_t t = 0; t < r; ++t)
                if (dist(e, sel[t]) < de) {
                    good = false;
                    break;
                }
            if (good) sel[r++] = e;
        }
        return r;
    }

    // Link x -> y at a layer; shrink x's list with the heuristic on overflow.
    void add_link(uint32_t x, uint32_t y, int32_t layer) {
        std::unique_lock<std::mutex> lk(lock_of(x), std::defer_lock);
        if (concurrent) lk.lock();
        link_locked(x, y, layer);
    }
    // Caller holds x's lock. Self links and entries already present are
    // skipped; neither occurs in a sequential build.
    void link_locked(uint32_t x, uint32_t y, int32_t layer) {
        if (y == x) return;
        int32_t cap;
        uint32_t* r = nbrs(x, layer, cap);
        int32_t cnt = 0;
        while (cnt < cap && r[cnt] != kNone) {
            if (r[cnt] == y) return;
            ++cnt;
        }
        if (cnt < cap) {
            r[cnt] = y;
            return;
        }
        std::vector<uint64_t> c(cap + 1);
        for (int32_t t = 0; t < cap; ++t) c[t] = mk(dist(x, r[t]), r[t]);
        c[cap] = mk(dist(x, y), y);
        std::sort(c.begin(), c.end());
        std::vector<uint32_t> sel(cap);
        int32_t k = heuristic(c.data(), c.size(), cap, sel.data());
        for (int32_t t = 0; t < cap; ++t) r[t] = t < k ? sel[t] : kNone;
    }

    void insert(uint32_t i, Visited& vis) {
        const int32_t li = g.level[i];
        std::unique_lock<std::mutex> glk(ep_lock);
        uint32_t ep = g.ep;
        int32_t L = g.L;
        if (li <= L) glk.unlock();
        std::vector<uint64_t> eps{mk(dist(i, ep), ep)};
        std::vector<uint64_t> W;
        for (int32_t lc = L; lc > li; --lc) {
            search_layer(i, eps, 1, lc, vis, W);
            eps.assign(1, W[0]);
        }
        std::vector<uint32_t> sel(M);
        for (int32_t lc = std::min(li, L); lc >= 0; --lc) {
            search_layer(i, eps, efc, lc, vis, W);
            int32_t r = heuristic(W.data(), W.size(), M, sel.data());
            {
                std::unique_lock<std::mutex> lk(lock_of(i), std::defer_lock);
                if (concurrent) lk.lock();
                int32_t cap;
                uint32_t* row = nbrs(i, lc, cap);
                // Links that concurrent inserts appended to i's list meanwhile
                // are merged after the selection, not overwritten; the list is
                // empty here in a sequential build.
                std::vector<uint32_t> prior(row, row + cap);
                for (int32_t t = 0; t < cap; ++t) row[t] = t < r ? sel[t] : kNone;
                for (int32_t t = 0; t < cap && prior[t] != kNone; ++t) link_locked(i, prior[t], lc);
            }
            for (int32_t t = 0; t < r; ++t) add_link(sel[t], i, lc);
            eps = W;
        }
        if (li > L) {
            g.L = li;
            g.ep = i;
        }
    }
};

}  // namespace

}  // namespace aqr

using namespace aqr;

namespace aqr {

// Insertion of the points S (ascending ids, none in the graph yet) in
// chunks of min(chunk_max, max(1, floor(m / 8))) points, m = points already
// in the graph.  Every point of a chunk plans its insertion against the
// graph as it stood before the chunk: greedy descent to one level above its
// own, then on each of its levels a search of width efc and the heuristic's
// M neighbours.  Then each point takes its lists, the reverse links are
// added in id order (per point from its top level down), and the entry
// point moves to each point above the top level, in id order.  The plans
// run on T threads; thread t applies the reverse links into the nodes x
// with x % T == t, in the order above, so the graph does not depend on T.
// With chunks of one point this is sequential insertion.
// Barrier of a fixed set of threads that meet many times in a row (a chunk
// takes a millisecond or so, far longer than a spin); a thread that waits
// long yields its core.
class SpinBarrier {
  public:
    explicit SpinBarrier(int n) : n_(n) {}
    void wait() {
        const unsigned gen = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
            count_.store(0, std::memory_order_relaxed);
            gen_.fetch_add(1, std::memory_order_release);
            return;
        }
        for (int spins = 0; gen_.load(std::memory_order_acquire) == gen; ++spins)
            if (spins > 2000) std::this_thread::yield();
    }

  private:
    const int n_;
    std::atomic<int> count_{0};
    std::atomic<unsigned> gen_{0};
};

// The points of S, in order, in chunks of min(chunk_max, max(1, inserted / 8))
// (Alg. 1's insertion, with every point of a chunk searching the graph as it
// stood before the chunk): each chunk point's searches and neighbour
// selection, then its own lists, then the reverse links of every selection
// in (point, level, rank) order.  T threads stay for the whole seed and meet
// at a barrier between the steps: the searches are shared out point by
// point, the own lists by point, and the reverse links by target list, so
// every list receives its links in the same order whatever T is.  A chunk
// point's searches cannot reach another point of its chunk (nothing links
// to it yet), so the lists a chunk's reverse links change are not the
// lists of its own points.
static void insert_chunks(Graph& g, const uint8_t* codes, int32_t dp, const std::vector<uint32_t>& S,
                          int32_t chunk_max, int T, const std::function<void(int64_t)>& report) {
    Builder B(g, codes, dp, false);
    const int32_t M = g.M, efc = g.efc;
    std::vector<Visited> vis;
    vis.reserve(T);
    for (int t = 0; t < T; ++t) vis.emplace_back(g.n);
    std::vector<std::vector<uint32_t>> sel;  // per chunk point: M per level, top level first
    std::vector<std::vector<int32_t>> nsel;  // per chunk point and level: selected count
    // the chunk, published by thread 0 before the first barrier of a round
    const uint32_t* ids = nullptr;
    int32_t nb = 0;
    uint32_t ep = 0;
    int32_t L = 0;
    bool done = false;
    int64_t inserted = 1;  // point 0
    size_t pos = 0;
    std::atomic<int32_t> nx{0};
    SpinBarrier bar(T);
    parallel_for_threads(T, [&](int t) {
        std::vector<uint64_t> eps, W;
        for (;;) {
            if (t == 0) {
                done = pos >= S.size();
                if (!done) {
                    const int64_t want = std::min<int64_t>(chunk_max, std::max<int64_t>(1, inserted / 8));
                    nb = (int32_t)std::min<int64_t>(want, (int64_t)(S.size() - pos));
                    ids = S.data() + pos;
                    ep = g.ep;
                    L = g.L;
                    sel.assign(nb, {});
                    nsel.assign(nb, {});
                    nx.store(0, std::memory_order_relaxed);
                }
            }
            bar.wait();  // the chunk is published
            if (done) return;
            for (;;) {
                const int32_t b = nx.fetch_add(1);
                if (b >= nb) break;
                const uint32_t i = ids[b];
                const int32_t top = std::min(g.level[i], L);
                eps.assign(1, mk(B.dist(i, ep), ep));
                for (int32_t lc = L; lc > g.level[i]; --lc) {
                    B.search_layer(i, eps, 1, lc, vis[t], W);
                    eps.assign(1, W[0]);
                }
                sel[b].assign((size_t)(top + 1) * M, kNone);
                nsel[b].assign(top + 1, 0);
                for (int32_t lc = top; lc >= 0; --lc) {
                    B.search_layer(i, eps, efc, lc, vis[t], W);
                    nsel[b][lc] = B.heuristic(W.data(), W.size(), M, &sel[b][(size_t)lc * M]);
                    eps = W;
                }
            }
            bar.wait();  // every selection is made
            for (int32_t b = t; b < nb; b += T)
                for (int32_t lc = (int32_t)nsel[b].size() - 1; lc >= 0; --lc) {
                    int32_t cap;
                    uint32_t* row = B.nbrs(ids[b], lc, cap);
                    for (int32_t j = 0; j < nsel[b][lc]; ++j) row[j] = sel[b][(size_t)lc * M + j];
                }
            for (int32_t b = 0; b < nb; ++b)
                for (int32_t lc = (int32_t)nsel[b].size() - 1; lc >= 0; --lc)
                    for (int32_t j = 0; j < nsel[b][lc]; ++j) {
                        const uint32_t x = sel[b][(size_t)lc * M + j];
                        if ((int)(x % (uint32_t)T) == t) B.link_locked(x, ids[b], lc);
                    }
            bar.wait();  // the chunk is linked
            if (t == 0) {
                for (int32_t b = 0; b < nb; ++b)
                    if (g.level[ids[b]] > g.L) {
                        g.L = g.level[ids[b]];
                        g.ep = ids[b];
                    }
                pos += nb;
                inserted += nb;
                report((int64_t)pos);
            }
        }
    });
}

// Levels for every point, then insertion of the seed: every point below
// seed_n and every point with level >= 1, in id order (seed_n >= n: all
// points, the plain build), one at a time (chunk_max 0) or in chunks
// (insert_chunks).  Level-0 points at or above seed_n are left unlinked for
// link_chunk.
aqr_status build_seeded(const uint8_t* codes, int64_t n, int32_t d, const aqr_quantizer* qz,
                        const aqr_bparams* p, const double* level_u, int64_t seed_n,
                        int32_t chunk_max, const char* who, aqr_graph** out) {
    const std::string w(who);
    if (!codes || !qz || !p || !out) return fail(AQR_ERR_INVALID_ARG, w + ": null pointer");
    if (n < 1 || n > (int64_t)0xFFFFFFFEu) return fail(AQR_ERR_INVALID_ARG, w + ": n out of range");
    if (d != qz->info.d) return fail(AQR_ERR_INVALID_ARG, w + ": d does not match the quantiser");
    const int32_t M = p->M > 0 ? p->M : qz->info.M;
    const int32_t efc = p->efc > 0 ? p->efc : qz->info.efc;
    if (M < 2 || M > 512 || efc < 1)
        return fail(AQR_ERR_INVALID_ARG, w + ": M must be in [2, 512] and efc >= 1");
    aqr_graph* g = new aqr_graph();
    g->n = n;
    g->M = M;
    g->efc = efc;
    g->level.resize(n);
    const double mL = 1.0 / std::log((double)M);
    uint64_t state = p->seed;
    for (int64_t i = 0; i < n; ++i) {
        double u;
        if (level_u) {
            u = level_u[i];
            if (!(u > 0.0 && u <= 1.0)) {
                delete g;
                return fail(AQR_ERR_INVALID_ARG, w + ": level draws must lie in (0, 1]");
            }
        } else {
            u = (double)((splitmix64(state) >> 11) + 1) * 0x1.0p-53;
        }
        g->level[i] = (int32_t)std::floor(-std::log(u) * mL);
    }
    g->upper_off.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) g->upper_off[i + 1] = g->upper_off[i] + g->level[i];
    g->adj0.assign((size_t)n * 2 * M, AQR_NONE);
    g->upper_adj.assign((size_t)std::max<int64_t>(g->upper_off[n], 1) * M, AQR_NONE);
    g->ep = 0;
    g->L = g->level[0];
    std::vector<uint32_t> S;  // seed points after point 0, in id order
    for (int64_t i = 1; i < n; ++i)
        if (i < seed_n || g->level[i] > 0) S.push_back((uint32_t)i);
    const int T = host_threads(p->threads);
    const int64_t ns = (int64_t)S.size();
    const int64_t step = p->progress > 0 ? std::max<int64_t>(1, ns / p->progress) : 0;
    const auto t0 = std::chrono::steady_clock::now();
    auto report = [&](int64_t i) {
        if (step && i % step == 0) {
            const double sec =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            std::fprintf(stderr, "[%s] %lld / %lld points inserted, %.1f s\n", who,
                         (long long)(i + 1), (long long)(ns + 1), sec);
            std::fflush(stderr);
        }
    };
    if (chunk_max > 0) {
        int64_t next_step = step;
        insert_chunks(*g, codes, qz->info.d_pad, S, chunk_max, T, [&](int64_t done) {
            if (step && (done >= next_step || done == ns)) {
                const double sec =
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                std::fprintf(stderr, "[%s] %lld / %lld points inserted, %.1f s\n", who,
                             (long long)(done + 1), (long long)(ns + 1), sec);
                std::fflush(stderr);
                next_step = (done / step + 1) * step;
            }
        });
        *out = g;
        return AQR_OK;
    }
    Builder B(*g, codes, qz->info.d_pad, T > 1);
    if (T <= 1 || ns < 1) {
        Visited vis(n);
        for (int64_t i = 0; i < ns; ++i) {
            B.insert(S[i], vis);
            report(i);
        }
    } else {
        std::atomic<int64_t> next{0};
        parallel_for_threads(T, [&](int) {
            Visited vis(n);
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= ns) break;
                B.insert(S[i], vis);
                report(i);
            }
        });
    }
    *out = g;
    return AQR_OK;
}

// One chunk of the batched build: ids (ascending) with their layer-0
// candidates (keys (D << 32) | id, ascending, cnt[b] of them at row b of a
// [nb][stride] array), each from a search of the graph as it stood before
// the chunk.  Selects M neighbours per point with the heuristic (or takes
// the selections sel_in / nsel_in made on the device from the same
// candidates), sets the points' layer-0 lists, then adds the reverse links:
// thread t owns the
// target nodes x with x % T == t and applies the links into them in the
// order they were generated (id order, as a sequential pass would), so the
// result does not depend on T.  dirty receives every id whose layer-0 list
// changed; mark (n bytes, all zero) is scratch and left all zero.
void link_chunk(aqr_graph* g, const uint8_t* codes, int32_t dp, const uint32_t* ids, int32_t nb,
                const uint64_t* cand, int32_t stride, const int32_t* cnt,
                const uint32_t* sel_in, const int32_t* nsel_in, int threads,
                std::vector<uint32_t>& dirty, std::vector<uint8_t>& mark) {
    const int32_t M = g->M;
    Builder B(*g, codes, dp, false);
    std::vector<uint32_t> sel((size_t)nb * M);
    std::vector<int32_t> ns(nb, 0);
    const int T = std::max(1, std::min(threads, (int)std::max(1, nb / 64)));
    std::atomic<int32_t> nx{0};
    parallel_for_threads(T, [&](int) {
        for (;;) {
            const int32_t b = nx.fetch_add(1);
            if (b >= nb) break;
            if (sel_in) {
                ns[b] = std::min(std::max(nsel_in[b], 0), M);
                std::memcpy(&sel[(size_t)b * M], &sel_in[(size_t)b * M], sizeof(uint32_t) * M);
            } else {
                ns[b] = B.heuristic(cand + (size_t)b * stride, (size_t)std::max(0, cnt[b]), M,
                                    &sel[(size_t)b * M]);
            }
            uint32_t* row = g->adj0.data() + (int64_t)ids[b] * 2 * M;
            for (int32_t t = 0; t < 2 * M; ++t) row[t] = t < ns[b] ? sel[(size_t)b * M + t] : kNone;
        }
    });
    const int T2 = std::max(1, threads);
    std::vector<std::vector<uint32_t>> owned(T2);
    parallel_for_threads(T2, [&](int t) {
        for (int32_t b = 0; b < nb; ++b)
            for (int32_t j = 0; j < ns[b]; ++j) {
                const uint32_t x = sel[(size_t)b * M + j];
                if ((int)(x % (uint32_t)T2) != t) continue;
                B.link_locked(x, ids[b], 0);
                if (!mark[x]) {
                    mark[x] = 1;
                    owned[t].push_back(x);
                }
            }
    });
    dirty.assign(ids, ids + nb);
    for (auto& o : owned)
        for (uint32_t x : o) {
            dirty.push_back(x);
            mark[x] = 0;
        }
}

}  // namespace aqr

extern "C" aqr_status aqr_build(const uint8_t* codes, int64_t n, int32_t d,
                                const aqr_quantizer* qz, const aqr_bparams* p,
                                const double* level_u, aqr_graph** out) {
    try {
        clear_error();
        return build_seeded(codes, n, d, qz, p, level_u, n, 0, "aqr_build", out);
    } catch (const std::bad_alloc&) {
        return fail(AQR_ERR_OOM, "aqr_build: out of host memory");
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_build: unexpected failure");
    }
}

extern "C" aqr_status aqr_graph_info(const aqr_graph* g, aqr_ginfo* info) {
    clear_error();
    if (!g || !info) return fail(AQR_ERR_INVALID_ARG, "aqr_graph_info: null pointer");
    info->n = g->n;
    info->M = g->M;
    info->efc = g->efc;
    info->L = g->L;
    info->ep = g->ep;
    info->upper_rows = g->upper_off.empty() ? 0 : g->upper_off[g->n];
    return AQR_OK;
}

extern "C" aqr_status aqr_graph_export(const aqr_graph* g, int32_t* level, uint32_t* adj0,
                                       int64_t* upper_off, uint32_t* upper_adj) {
    clear_error();
    if (!g) return fail(AQR_ERR_INVALID_ARG, "aqr_graph_export: null graph");
    if (level) std::memcpy(level, g->level.data(), sizeof(int32_t) * g->n);
    if (adj0) std::memcpy(adj0, g->adj0.data(), sizeof(uint32_t) * g->n * 2 * g->M);
    if (upper_off) std::memcpy(upper_off, g->upper_off.data(), sizeof(int64_t) * (g->n + 1));
    if (upper_adj)
        std::memcpy(upper_adj, g->upper_adj.data(), sizeof(uint32_t) * g->upper_off[g->n] * g->M);
    return AQR_OK;
}

extern "C" aqr_status aqr_graph_import(int64_t n, int32_t M, const int32_t* level,
                                       const uint32_t* adj0, const int64_t* upper_off,
                                       const uint32_t* upper_adj, uint32_t ep, aqr_graph** out) {
    try {
        clear_error();
        if (!level || !adj0 || !upper_off || !out)
            return fail(AQR_ERR_INVALID_ARG, "aqr_graph_import: null pointer");
        if (n < 1 || M < 2 || M > 512 || (int64_t)ep >= n)
            return fail(AQR_ERR_INVALID_ARG, "aqr_graph_import: n, M or ep out of range");
        if (upper_off[0] != 0) return fail(AQR_ERR_CORRUPT, "aqr_graph_import: upper_off[0] != 0");
        int32_t L = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (level[i] < 0 || upper_off[i + 1] - upper_off[i] != level[i])
                return fail(AQR_ERR_CORRUPT, "aqr_graph_import: levels and row offsets disagree");
            L = std::max(L, level[i]);
        }
        if (level[ep] != L) return fail(AQR_ERR_CORRUPT, "aqr_graph_import: entry point is not on the top level");
        const int64_t rows = upper_off[n];
        if (rows > 0 && !upper_adj) return fail(AQR_ERR_INVALID_ARG, "aqr_graph_import: null upper_adj");
        for (int64_t i = 0; i < n * 2 * M; ++i)
            if (adj0[i] != AQR_NONE && (int64_t)adj0[i] >= n)
                return fail(AQR_ERR_CORRUPT, "aqr_graph_import: neighbour id out of range");
        for (int64_t i = 0; i < rows * M; ++i)
            if (upper_adj[i] != AQR_NONE && (int64_t)upper_adj[i] >= n)
                return fail(AQR_ERR_CORRUPT, "aqr_graph_import: neighbour id out of range");
        aqr_graph* g = new aqr_graph();
        g->n = n;
        g->M = M;
        g->efc = 0;
        g->L = L;
        g->ep = ep;
        g->level.assign(level, level + n);
        g->adj0.assign(adj0, adj0 + n * 2 * M);
        g->upper_off.assign(upper_off, upper_off + n + 1);
        if (rows > 0)
            g->upper_adj.assign(upper_adj, upper_adj + rows * M);
        else
            g->upper_adj.assign(M, AQR_NONE);
        *out = g;
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_OOM, "aqr_graph_import: out of host memory");
    }
}

extern "C" void aqr_graph_free(aqr_graph* g) { delete g; }
