// Status strings and the thread-local error detail of libbf (no HIP).
#include <cstdarg>
#include <cstdio>
#include <string>

#include "bf_status.h"

namespace {

thread_local std::string g_last_error;

}  // namespace

bf_status bf_fail(bf_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

extern "C" const char *bf_status_str(bf_status s)
{
    switch (s) {
    case BF_OK: return "BF_OK";
    case BF_ERR_INVALID: return "BF_ERR_INVALID";
    case BF_ERR_OOM: return "BF_ERR_OOM";
    case BF_ERR_DEVICE: return "BF_ERR_DEVICE";
    case BF_ERR_BUSY: return "BF_ERR_BUSY";
    case BF_ERR_TIMEOUT: return "BF_ERR_TIMEOUT";
    case BF_ERR_UNSUPPORTED: return "BF_ERR_UNSUPPORTED";
    }
    return "BF_ERR_UNKNOWN";
}

extern "C" const char *bf_last_error(void) { return g_last_error.c_str(); }
