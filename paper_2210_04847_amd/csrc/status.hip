// Status codes, per-thread error messages and launch checks of the C ABI.
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace {
thread_local char g_message[512] = "";
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
