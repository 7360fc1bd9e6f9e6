// bs_error.cpp -- status codes and the per-thread error message of the C ABI
// (host code only; shared by every entry point).
#include <cstdarg>
#include <cstdio>

#include "../../include/bluesurfels.h"

namespace bs {
namespace {
thread_local char g_msg[512] = "";
}

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

const char* last_error_text() { return g_msg; }

}  // namespace bs

extern "C" {

const char* bs_error_string(int code) {
    switch (code) {
        case BS_OK: return "BS_OK";
        case BS_ERR_INVALID_ARG: return "BS_ERR_INVALID_ARG";
        case BS_ERR_OUT_OF_MEMORY: return "BS_ERR_OUT_OF_MEMORY";
        case BS_ERR_HIP: return "BS_ERR_HIP";
        case BS_ERR_OVER_BUDGET: return "BS_ERR_OVER_BUDGET";
        case BS_ERR_NOT_READY: return "BS_ERR_NOT_READY";
        case BS_ERR_UNSUPPORTED: return "BS_ERR_UNSUPPORTED";
        case BS_ERR_TIMEOUT: return "BS_ERR_TIMEOUT";
        case BS_ERR_DEVICE: return "BS_ERR_DEVICE";
        default: return "BS_ERR_UNKNOWN";
    }
}

const char* bs_last_error_message(void) { return bs::last_error_text(); }

const char* bs_version(void) { return "0.2.0"; }

}  // extern "C"
