// Status codes, per-thread error messages and launch checks of the C ABI.
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace {
thread_local char g_message[512] = "";
nacc_tuning g_tuning = {4, 4, 16384, 0};
}

namespace nacc {

int set_error(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_message, sizeof(g_message), fmt, ap);
    va_end(ap);
    return status;
}

void clear_error() { g_message[0] = '\0'; }

const nacc_tuning& tuning() { return g_tuning; }

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        return set_error(NACC_EHIP, "%s: %s", what, hipGetErrorString(e));
    }
    return NACC_OK;
}

}  // namespace nacc

extern "C" {

const char* nacc_version(void) { return "nacc 0.1.0 (gfx950)"; }

void nacc_get_tuning(nacc_tuning* out) {
    if (out != nullptr) *out = g_tuning;
}

int nacc_set_tuning(const nacc_tuning* t) {
    nacc::clear_error();
    NACC_REQUIRE(t != nullptr, NACC_EINVAL, "tuning must be non-NULL");
    const int w = t->march_waves_per_group;
    NACC_REQUIRE(w == 1 || w == 2 || w == 4 || w == 8 || w == 16, NACC_EINVAL,
                 "march_waves_per_group = %d not in {1, 2, 4, 8, 16}", w);
    NACC_REQUIRE(t->render_cached_chunks >= 1 && t->render_cached_chunks <= 4, NACC_EINVAL,
                 "render_cached_chunks = %d not in [1, 4]", t->render_cached_chunks);
    NACC_REQUIRE(t->render_mse_max_blocks >= 1 && t->render_mse_max_blocks <= (1 << 20), NACC_EINVAL,
                 "render_mse_max_blocks = %d not in [1, 2^20]", t->render_mse_max_blocks);
    NACC_REQUIRE(t->render_prefetch == 0 || t->render_prefetch == 1, NACC_EINVAL,
                 "render_prefetch = %d not in {0, 1}", t->render_prefetch);
    g_tuning = *t;
    return NACC_OK;
}

const char* nacc_last_error(void) { return g_message; }

const char* nacc_status_str(int status) {
    switch (status) {
        case NACC_OK: return "NACC_OK";
        case NACC_EINVAL: return "NACC_EINVAL";
        case NACC_ESHAPE: return "NACC_ESHAPE";
        case NACC_ECAPACITY: return "NACC_ECAPACITY";
        case NACC_EHIP: return "NACC_EHIP";
        case NACC_ENOTSUP: return "NACC_ENOTSUP";
        default: return "NACC_UNKNOWN";
    }
}

}  // extern "C"
