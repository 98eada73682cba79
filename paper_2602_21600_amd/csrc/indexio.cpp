// indexio.cpp -- one checksummed file for a built index: the quantiser
// (Section 3.1 Stage 2: min_j, max_j, scale_j and the scalars of Alg. 1),
// the codes, the FP32 rows that Stage 3 re-ranks with, and the HNSW graph.
//
// Layout (little-endian):
//   header      512 bytes: magic, version, shapes, quantiser scalars, the
//               offset and length of each section, the block size, and a
//               CRC of the header itself
//   payload     the sections, each starting on a 64-byte boundary:
//               min[d], max[d], scale[d] (float32), codes[n][d_pad] (uint8),
//               X[n][d] (float32), level[n] (int32), adj0[n][2M] (uint32),
//               upper_off[n+1] (int64), upper_adj[rows][M] (uint32)
//   trailer     one CRC per 64 MiB block of the payload, a CRC of that
//               table, and an end marker
// The checksum is CRC-32C (Castagnoli polynomial, as in RFC 3720), computed
// with the SSE4.2 crc32 instruction.  Loading checks the header, the file
// length, every block's CRC, the zero padding of the code rows and the
// graph's structure, and reports AQR_ERR_CORRUPT on any mismatch.
#include <nmmintrin.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace aqr;

namespace {

constexpr char kMagic[8] = {'A', 'Q', 'R', 'I', 'N', 'D', 'X', '1'};
constexpr char kEnd[8] = {'A', 'Q', 'R', 'E', 'N', 'D', '0', '1'};
constexpr uint32_t kVersion = 1;
constexpr uint64_t kBlock = 64ull << 20;
constexpr int kSections = 9;

struct FileHeader {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    int64_t n;
    int32_t d, d_pad, M, efc;
    int32_t L;
    uint32_t ep;
    int64_t upper_rows;
    int32_t q_M, q_efc;
    double delta, p_lo, p_hi, s_dist, eta, w_mean;
    uint64_t block_bytes;
    uint64_t payload_bytes;
    uint64_t nblocks;
    uint64_t off[kSections];
    uint64_t len[kSections];
    uint32_t header_crc;  // CRC-32C of the 512 header bytes with this field 0
    uint32_t pad0;
    unsigned char reserved[512 - 8 - 4 - 4 - 8 - 5 * 4 - 4 - 8 - 2 * 4 - 6 * 8 - 3 * 8 -
                           2 * kSections * 8 - 2 * 4];
};
static_assert(sizeof(FileHeader) == 512, "index file header is 512 bytes");

uint32_t crc32c_update(uint32_t crc, const unsigned char* p, size_t len) {
    uint64_t c = crc;
    while (len >= 8) {
        uint64_t v;
        std::memcpy(&v, p, 8);
        c = _mm_crc32_u64(c, v);
        p += 8;
        len -= 8;
    }
    uint32_t c32 = (uint32_t)c;
    while (len--) c32 = _mm_crc32_u8(c32, *p++);
    return c32;
}

uint32_t crc32c(const void* p, size_t len) {
    return ~crc32c_update(~0u, static_cast<const unsigned char*>(p), len);
}

// Running CRC over the payload, one value per kBlock bytes.
struct BlockCrc {
    std::vector<uint32_t> crcs;
    uint32_t cur = ~0u;
    uint64_t in_block = 0;
    void add(const void* data, size_t len) {
        const unsigned char* p = static_cast<const unsigned char*>(data);
        while (len > 0) {
            const size_t take = (size_t)std::min<uint64_t>(len, kBlock - in_block);
            cur = crc32c_update(cur, p, take);
            in_block += take;
            p += take;
            len -= take;
            if (in_block == kBlock) finish_block();
        }
    }
    void finish_block() {
        crcs.push_back(~cur);
        cur = ~0u;
        in_block = 0;
    }
    void finish() {
        if (in_block > 0) finish_block();
    }
};

struct File {
    std::FILE* f = nullptr;
    ~File() {
        if (f) std::fclose(f);
    }
};

uint64_t align64(uint64_t x) { return (x + 63) & ~(uint64_t)63; }

}  // namespace

extern "C" aqr_status aqr_index_save(const char* path, const aqr_quantizer* qz,
                                     const aqr_graph* g, const uint8_t* codes, const float* X) {
    try {
        clear_error();
        if (!path || !qz || !g || !codes || !X)
            return fail(AQR_ERR_INVALID_ARG, "aqr_index_save: null pointer");
        const int64_t n = g->n;
        const int32_t d = qz->info.d, dp = qz->info.d_pad, M = g->M;
        const int64_t rows = g->upper_off[n];
        FileHeader h;
        std::memset(&h, 0, sizeof(h));
        std::memcpy(h.magic, kMagic, 8);
        h.version = kVersion;
        h.header_bytes = sizeof(FileHeader);
        h.n = n;
        h.d = d;
        h.d_pad = dp;
        h.M = M;
        h.efc = g->efc;
        h.L = g->L;
        h.ep = g->ep;
        h.upper_rows = rows;
        h.q_M = qz->info.M;
        h.q_efc = qz->info.efc;
        h.delta = qz->info.delta;
        h.p_lo = qz->info.p_lo;
        h.p_hi = qz->info.p_hi;
        h.s_dist = qz->info.s_dist;
        h.eta = qz->info.eta;
        h.w_mean = qz->info.w_mean;
        h.block_bytes = kBlock;
        const void* src[kSections] = {qz->mn.data(),     qz->mx.data(),        qz->scale.data(),
                                      codes,             X,                    g->level.data(),
                                      g->adj0.data(),    g->upper_off.data(),  g->upper_adj.data()};
        const uint64_t len[kSections] = {
            (uint64_t)d * 4, (uint64_t)d * 4, (uint64_t)d * 4, (uint64_t)n * dp,
            (uint64_t)n * d * 4, (uint64_t)n * 4, (uint64_t)n * 2 * M * 4, (uint64_t)(n + 1) * 8,
            (uint64_t)rows * M * 4};
        uint64_t o = 0;
        for (int s = 0; s < kSections; ++s) {
            h.off[s] = o;
            h.len[s] = len[s];
            o = align64(o + len[s]);
        }
        h.payload_bytes = o;
        h.nblocks = (o + kBlock - 1) / kBlock;
        h.header_crc = 0;
        h.header_crc = crc32c(&h, sizeof(h));
        File F;
        F.f = std::fopen(path, "wb");
        if (!F.f) return fail(AQR_ERR_INVALID_ARG, std::string("aqr_index_save: cannot open ") + path);
        if (std::fwrite(&h, sizeof(h), 1, F.f) != 1)
            return fail(AQR_ERR_STATE, "aqr_index_save: write failed");
        BlockCrc bc;
        static const unsigned char zeros[64] = {0};
        uint64_t pos = 0;
        for (int s = 0; s < kSections; ++s) {
            if (len[s] > 0) {
                // write in pieces so the CRC and the write share the cache
                const unsigned char* p = static_cast<const unsigned char*>(src[s]);
                for (uint64_t done = 0; done < len[s];) {
                    const size_t take = (size_t)std::min<uint64_t>(len[s] - done, 8ull << 20);
                    bc.add(p + done, take);
                    if (std::fwrite(p + done, 1, take, F.f) != take)
                        return fail(AQR_ERR_STATE, "aqr_index_save: write failed");
                    done += take;
                }
            }
            pos += len[s];
            const uint64_t padb = align64(pos) - pos;
            if (padb) {
                bc.add(zeros, (size_t)padb);
                if (std::fwrite(zeros, 1, (size_t)padb, F.f) != padb)
                    return fail(AQR_ERR_STATE, "aqr_index_save: write failed");
                pos += padb;
            }
        }
        bc.finish();
        if (bc.crcs.size() != h.nblocks) return fail(AQR_ERR_STATE, "aqr_index_save: block count");
        const uint32_t tcrc = crc32c(bc.crcs.data(), bc.crcs.size() * 4);
        if (std::fwrite(bc.crcs.data(), 4, bc.crcs.size(), F.f) != bc.crcs.size() ||
            std::fwrite(&tcrc, 4, 1, F.f) != 1 || std::fwrite(kEnd, 1, 8, F.f) != 8)
            return fail(AQR_ERR_STATE, "aqr_index_save: write failed");
        if (std::fclose(F.f) != 0) {
            F.f = nullptr;
            return fail(AQR_ERR_STATE, "aqr_index_save: close failed");
        }
        F.f = nullptr;
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_OOM, "aqr_index_save: out of host memory");
    }
}

namespace {

aqr_status read_header(std::FILE* f, const char* who, FileHeader* h, uint64_t* file_bytes) {
    if (std::fseek(f, 0, SEEK_END) != 0) return fail(AQR_ERR_STATE, std::string(who) + ": seek failed");
    const long long sz = std::ftell(f);
    if (sz < 0) return fail(AQR_ERR_STATE, std::string(who) + ": tell failed");
    *file_bytes = (uint64_t)sz;
    std::rewind(f);
    if ((uint64_t)sz < sizeof(FileHeader) || std::fread(h, sizeof(FileHeader), 1, f) != 1)
        return fail(AQR_ERR_CORRUPT, std::string(who) + ": file shorter than its header");
    if (std::memcmp(h->magic, kMagic, 8) != 0)
        return fail(AQR_ERR_CORRUPT, std::string(who) + ": not an index file (bad magic)");
    const uint32_t stored = h->header_crc;
    FileHeader c = *h;
    c.header_crc = 0;
    if (crc32c(&c, sizeof(c)) != stored)
        return fail(AQR_ERR_CORRUPT, std::string(who) + ": header checksum mismatch");
    if (h->version != kVersion || h->header_bytes != sizeof(FileHeader))
        return fail(AQR_ERR_CORRUPT, std::string(who) + ": unsupported version");
    if (h->n < 1 || h->d < 1 || h->d > 65536 || h->d_pad != round_up(h->d, 16) || h->M < 2 ||
        h->M > 512 || h->upper_rows < 0 || h->block_bytes != kBlock)
        return fail(AQR_ERR_CORRUPT, std::string(who) + ": shapes out of range");
    const uint64_t n = (uint64_t)h->n, d = (uint64_t)h->d;
    const uint64_t want[kSections] = {d * 4, d * 4, d * 4, n * (uint64_t)h->d_pad, n * d * 4,
                                      n * 4, n * 2 * (uint64_t)h->M * 4, (n + 1) * 8,
                                      (uint64_t)h->upper_rows * (uint64_t)h->M * 4};
    uint64_t o = 0;
    for (int s = 0; s < kSections; ++s) {
        if (h->off[s] != o || h->len[s] != want[s])
            return fail(AQR_ERR_CORRUPT, std::string(who) + ": section table disagrees with the shapes");
        o = align64(o + want[s]);
    }
    if (h->payload_bytes != o || h->nblocks != (o + kBlock - 1) / kBlock)
        return fail(AQR_ERR_CORRUPT, std::string(who) + ": payload size disagrees with the shapes");
    const uint64_t total = sizeof(FileHeader) + o + h->nblocks * 4 + 4 + 8;
    if (*file_bytes != total)
        return fail(AQR_ERR_CORRUPT, std::string(who) + (*file_bytes < total
                                                             ? ": file truncated"
                                                             : ": trailing bytes after the index"));
    return AQR_OK;
}

}  // namespace

extern "C" aqr_status aqr_index_file_info(const char* path, aqr_index_header* info) {
    try {
        clear_error();
        if (!path || !info) return fail(AQR_ERR_INVALID_ARG, "aqr_index_file_info: null pointer");
        File F;
        F.f = std::fopen(path, "rb");
        if (!F.f) return fail(AQR_ERR_INVALID_ARG, std::string("aqr_index_file_info: cannot open ") + path);
        FileHeader h;
        uint64_t bytes = 0;
        aqr_status st = read_header(F.f, "aqr_index_file_info", &h, &bytes);
        if (st != AQR_OK) return st;
        info->n = h.n;
        info->d = h.d;
        info->d_pad = h.d_pad;
        info->M = h.M;
        info->reserved = 0;
        info->upper_rows = h.upper_rows;
        info->file_bytes = bytes;
        return AQR_OK;
    } catch (...) {
        return fail(AQR_ERR_OOM, "aqr_index_file_info: out of host memory");
    }
}

extern "C" aqr_status aqr_index_load(const char* path, aqr_quantizer** qz_out, aqr_graph** g_out,
                                     uint8_t* codes_out, float* X_out) {
    const char* who = "aqr_index_load";
    try {
        clear_error();
        if (!path || !qz_out || !g_out || !codes_out || !X_out)
            return fail(AQR_ERR_INVALID_ARG, "aqr_index_load: null pointer");
        File F;
        F.f = std::fopen(path, "rb");
        if (!F.f) return fail(AQR_ERR_INVALID_ARG, std::string("aqr_index_load: cannot open ") + path);
        FileHeader h;
        uint64_t bytes = 0;
        aqr_status st = read_header(F.f, who, &h, &bytes);
        if (st != AQR_OK) return st;
        const int64_t n = h.n;
        const int32_t d = h.d, dp = h.d_pad, M = h.M;
        std::vector<float> mn(d), mx(d), sc(d);
        std::vector<int32_t> level(n);
        std::vector<uint32_t> adj0((size_t)n * 2 * M);
        std::vector<int64_t> uoff(n + 1);
        std::vector<uint32_t> uadj((size_t)std::max<int64_t>(h.upper_rows, 0) * M);
        void* dst[kSections] = {mn.data(),    mx.data(),    sc.data(),   codes_out, X_out,
                                level.data(), adj0.data(),  uoff.data(), uadj.data()};
        BlockCrc bc;
        std::vector<unsigned char> padbuf(64);
        uint64_t pos = 0;
        for (int s = 0; s < kSections; ++s) {
            unsigned char* p = static_cast<unsigned char*>(dst[s]);
            for (uint64_t done = 0; done < h.len[s];) {
                const size_t take = (size_t)std::min<uint64_t>(h.len[s] - done, 8ull << 20);
                if (std::fread(p + done, 1, take, F.f) != take)
                    return fail(AQR_ERR_CORRUPT, std::string(who) + ": file truncated");
                bc.add(p + done, take);
                done += take;
            }
            pos += h.len[s];
            const uint64_t padb = align64(pos) - pos;
            if (padb) {
                if (std::fread(padbuf.data(), 1, (size_t)padb, F.f) != padb)
                    return fail(AQR_ERR_CORRUPT, std::string(who) + ": file truncated");
                bc.add(padbuf.data(), (size_t)padb);
                pos += padb;
            }
        }
        bc.finish();
        std::vector<uint32_t> stored(h.nblocks);
        uint32_t tcrc = 0;
        char end[8];
        if (std::fread(stored.data(), 4, stored.size(), F.f) != stored.size() ||
            std::fread(&tcrc, 4, 1, F.f) != 1 || std::fread(end, 1, 8, F.f) != 8)
            return fail(AQR_ERR_CORRUPT, std::string(who) + ": file truncated");
        if (std::memcmp(end, kEnd, 8) != 0)
            return fail(AQR_ERR_CORRUPT, std::string(who) + ": bad end marker");
        if (crc32c(stored.data(), stored.size() * 4) != tcrc)
            return fail(AQR_ERR_CORRUPT, std::string(who) + ": checksum table corrupt");
        if (bc.crcs.size() != stored.size())
            return fail(AQR_ERR_CORRUPT, std::string(who) + ": block count mismatch");
        for (size_t b = 0; b < stored.size(); ++b)
            if (bc.crcs[b] != stored[b])
                return fail(AQR_ERR_CORRUPT, std::string(who) + ": checksum mismatch in block " +
                                                 std::to_string(b));
        // padding bytes of the code rows must be zero: the device sums every
        // byte of a row
        for (int64_t i = 0; i < n && dp > d; ++i)
            for (int32_t j = d; j < dp; ++j)
                if (codes_out[(size_t)i * dp + j] != 0)
                    return fail(AQR_ERR_CORRUPT, std::string(who) + ": non-zero code padding");
        aqr_qinfo qi{};
        qi.d = d;
        qi.d_pad = dp;
        qi.M = h.q_M;
        qi.efc = h.q_efc;
        qi.delta = h.delta;
        qi.p_lo = h.p_lo;
        qi.p_hi = h.p_hi;
        qi.s_dist = h.s_dist;
        qi.eta = h.eta;
        qi.w_mean = h.w_mean;
        aqr_quantizer* qz = nullptr;
        st = aqr_quantizer_create(&qi, mn.data(), mx.data(), sc.data(), &qz);
        if (st != AQR_OK) return fail(AQR_ERR_CORRUPT, std::string(who) + ": " + aqr_last_error());
        std::unique_ptr<aqr_quantizer> qguard(qz);
        aqr_graph* g = nullptr;
        st = aqr_graph_import(n, M, level.data(), adj0.data(), uoff.data(),
                              h.upper_rows > 0 ? uadj.data() : nullptr, h.ep, &g);
        if (st != AQR_OK) return fail(AQR_ERR_CORRUPT, std::string(who) + ": " + aqr_last_error());
        g->efc = h.efc;
        if (g->L != h.L) {
            aqr_graph_free(g);
            return fail(AQR_ERR_CORRUPT, std::string(who) + ": top level disagrees with the levels");
        }
        *qz_out = qguard.release();
        *g_out = g;
        return AQR_OK;
    } catch (const std::bad_alloc&) {
        return fail(AQR_ERR_OOM, "aqr_index_load: out of host memory");
    } catch (...) {
        return fail(AQR_ERR_STATE, "aqr_index_load: unexpected failure");
    }
}
