// Host-side plumbing of the C ABI: the per-thread error text, status
// strings and the stderr diagnostics (kept apart from the kernel sources).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <atomic>

#include "tdct.h"
#include "tdct_internal.hpp"

namespace tdct {

static thread_local char g_err[256];
static std::atomic<int> g_log_level{-1};

int log_level() {
    int l = g_log_level.load(std::memory_order_relaxed);
    if (l >= 0) return l;
    const char* e = getenv("TDCT_LOG");
    l = e ? atoi(e) : 0;
    l = l < 0 ? 0 : (l > 3 ? 3 : l);
    int unset = -1;
    g_log_level.compare_exchange_strong(unset, l, std::memory_order_relaxed);
    return g_log_level.load(std::memory_order_relaxed);
}

void log_line(int level, const char* fmt, ...) {
    char buf[640];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    fprintf(stderr, "[tdct %d] %s\n", level, buf);  // one write per line
}

void set_error(const char* what, hipError_t e) {
    snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
    TDCT_LOG(1, "error: %s", g_err);
}

void set_error_text(const char* what) {
    snprintf(g_err, sizeof(g_err), "%s", what);
    TDCT_LOG(1, "error: %s", g_err);
}

}  // namespace tdct

extern "C" {

const char* tdct_strerror(int status) {
    switch (status) {
        case TDCT_OK: return "ok";
        case TDCT_EINVAL: return "invalid argument (null pointer, stride, alignment, keep or op)";
        case TDCT_EDIM: return "width/height not a positive multiple of 8 (or above 65536)";
        case TDCT_EQTAB: return "quantisation table entry outside [1, 4095]";
        case TDCT_ENOMEM: return "out of device memory or request larger than the budget";
        case TDCT_EDEVICE: return "HIP runtime error";
        case TDCT_EBUSY: return "not ready";
        case TDCT_ENOTFOUND: return "unknown ticket";
    }
    return "unknown status";
}

const char* tdct_last_error(void) { return tdct::g_err; }

int tdct_log_level(int level) {
    const int prev = tdct::log_level();
    if (level >= 0) tdct::g_log_level.store(level > 3 ? 3 : level, std::memory_order_relaxed);
    return prev;
}

}  // extern "C"
