// Host-code driver for the sanitizer build: the host parts of libaqr
// (quantiser, graph builder, graph exchange, index file) built with
// AddressSanitizer and UndefinedBehaviorSanitizer and driven through their
// C-ABI on small seeded inputs, error paths included.  The device density
// search is replaced by a stub that reports a device error, so the driver
// needs no GPU.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../paper_2602_21600_amd/csrc/internal.hpp"

namespace aqr {
aqr_status device_density_sums(const float*, int64_t, int32_t, const int64_t*, int64_t, int32_t,
                               int, double*) {
    return fail(AQR_ERR_DEVICE, "no device in the sanitizer build");
}
}  // namespace aqr

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "CHECK failed at line %d: %s (%s)\n", __LINE__, #c, \
                         aqr_last_error());                                   \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : "/tmp";
    std::mt19937_64 rng(12345);
    std::normal_distribution<float> nd(0.0f, 1.0f);
    for (int32_t d : {7, 16, 40}) {
        for (int64_t n : {1LL, 2LL, 50LL, 3000LL, 12000LL}) {
            std::vector<float> X((size_t)n * d);
            for (auto& v : X) v = nd(rng);
            if (n > 10) std::memcpy(&X[(size_t)5 * d], &X[0], sizeof(float) * d);  // a duplicate
            aqr_qparams p{};
            p.k_rho = 10;
            p.threads = 3;
            p.n_sample = 500;
            p.sample_threshold = 1000;
            p.eps = 1e-6;
            p.p_max = 0.01;
            p.M0 = 6;
            p.efc0 = 40;
            p.weights = (int32_t)(n % 2);
            aqr_quantizer* qz = nullptr;
            aqr_qinfo qi{};
            const int32_t dp = (d + 15) / 16 * 16;
            std::vector<uint8_t> codes((size_t)n * dp);
            CHECK(aqr_quantize(X.data(), n, d, &p, &qz, codes.data()) == AQR_OK);
            if (!qz) continue;
            std::vector<float> mn(d), mx(d), sc(d);
            CHECK(aqr_quantizer_info(qz, &qi, mn.data(), mx.data(), sc.data()) == AQR_OK);
            // the device path reports the stubbed device error
            aqr_quantizer* q2 = nullptr;
            CHECK(aqr_quantize_device(X.data(), n, d, &p, &q2, nullptr) != AQR_OK || n <= 1);
            if (q2) aqr_quantizer_free(q2);
            for (int32_t threads : {1, 4}) {
                aqr_bparams bp{};
                bp.threads = threads;
                bp.seed = 99;
                aqr_graph* g = nullptr;
                CHECK(aqr_build(codes.data(), n, d, qz, &bp, nullptr, &g) == AQR_OK);
                if (!g) continue;
                aqr_ginfo gi{};
                CHECK(aqr_graph_info(g, &gi) == AQR_OK);
                std::vector<int32_t> level(n);
                std::vector<uint32_t> adj0((size_t)n * 2 * gi.M);
                std::vector<int64_t> off(n + 1);
                std::vector<uint32_t> up((size_t)std::max<int64_t>(gi.upper_rows, 1) * gi.M);
                CHECK(aqr_graph_export(g, level.data(), adj0.data(), off.data(), up.data()) ==
                      AQR_OK);
                aqr_graph* g2 = nullptr;
                CHECK(aqr_graph_import(n, gi.M, level.data(), adj0.data(), off.data(), up.data(),
                                       gi.ep, &g2) == AQR_OK);
                // index file round trip, then a truncated copy
                const std::string f = dir + "/san_" + std::to_string(d) + "_" +
                                      std::to_string(n) + "_" + std::to_string(threads) + ".aqr";
                CHECK(aqr_index_save(f.c_str(), qz, g, codes.data(), X.data()) == AQR_OK);
                aqr_index_header h{};
                CHECK(aqr_index_file_info(f.c_str(), &h) == AQR_OK);
                std::vector<uint8_t> c2((size_t)n * dp);
                std::vector<float> X2((size_t)n * d);
                aqr_quantizer* q3 = nullptr;
                aqr_graph* g3 = nullptr;
                CHECK(aqr_index_load(f.c_str(), &q3, &g3, c2.data(), X2.data()) == AQR_OK);
                CHECK(c2 == codes && X2 == X);
                if (q3) aqr_quantizer_free(q3);
                if (g3) aqr_graph_free(g3);
                if (std::FILE* fp = std::fopen(f.c_str(), "r+b")) {
                    std::fseek(fp, 0, SEEK_END);
                    const long sz = std::ftell(fp);
                    std::fclose(fp);
                    if (sz > 100) {
                        CHECK(truncate(f.c_str(), sz - 13) == 0);
                        aqr_quantizer* q4 = nullptr;
                        aqr_graph* g4 = nullptr;
                        CHECK(aqr_index_load(f.c_str(), &q4, &g4, c2.data(), X2.data()) ==
                              AQR_ERR_CORRUPT);
                        CHECK(q4 == nullptr && g4 == nullptr);
                    }
                }
                std::remove(f.c_str());
                // corruption of exchanged arrays is rejected
                if (n > 2) {
                    std::vector<uint32_t> bad = adj0;
                    bad[1] = (uint32_t)n;
                    aqr_graph* g5 = nullptr;
                    CHECK(aqr_graph_import(n, gi.M, level.data(), bad.data(), off.data(), up.data(),
                                           gi.ep, &g5) == AQR_ERR_CORRUPT);
                }
                aqr_graph_free(g2);
                aqr_graph_free(g);
            }
            aqr_quantizer* q5 = nullptr;
            CHECK(aqr_quantizer_create(&qi, mn.data(), mx.data(), sc.data(), &q5) == AQR_OK);
            aqr_quantizer_free(q5);
            aqr_quantizer_free(qz);
        }
    }
    // error paths: null pointers and non-finite input
    aqr_quantizer* qz = nullptr;
    CHECK(aqr_quantize(nullptr, 10, 4, nullptr, &qz, nullptr) == AQR_ERR_INVALID_ARG);
    std::vector<float> X(40, 1.0f);
    X[7] = NAN;
    aqr_qparams p{};
    p.k_rho = 10;
    p.n_sample = 5000;
    p.sample_threshold = 10000;
    p.eps = 1e-6;
    p.p_max = 0.01;
    p.M0 = 4;
    p.efc0 = 10;
    CHECK(aqr_quantize(X.data(), 10, 4, &p, &qz, nullptr) == AQR_ERR_INVALID_ARG);
    CHECK(aqr_index_load("/nonexistent/file.aqr", nullptr, nullptr, nullptr, nullptr) ==
          AQR_ERR_INVALID_ARG);
    std::printf("host driver: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
