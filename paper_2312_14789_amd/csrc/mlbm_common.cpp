// Error reporting and version of libmlbm.so.
#include <cstdio>
#include <string>

#include "mlbm.h"
#include "mlbm_internal.h"

namespace {
thread_local std::string g_last_error;
}

namespace mlbm {

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

}  // namespace mlbm

extern "C" const char *mlbm_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *mlbm_version(void) { return "mlbm 0.1 gfx950"; }
