// errors.cpp -- thread-local error messages and small host utilities.
#include <thread>

#include "internal.hpp"

namespace aqr {

namespace {
thread_local std::string g_last_error;
}

aqr_status fail(aqr_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

void clear_error() { g_last_error.clear(); }

int host_threads(int32_t requested) {
    if (requested > 0) return requested;
    unsigned hc = std::thread::hardware_concurrency();
    return hc ? (int)hc : 1;
}

}  // namespace aqr

extern "C" const char* aqr_last_error(void) { return aqr::g_last_error.c_str(); }
extern "C" int32_t aqr_version(void) { return AQR_VERSION; }
