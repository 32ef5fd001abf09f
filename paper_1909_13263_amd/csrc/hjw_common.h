// hjw_common.h - constants and error reporting shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "hjw.h"

namespace hjw {

// Thread-local text of the last error (defined in hjw.hip).
std::string& last_error();

inline hjw_status fail(hjw_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    last_error() = buf;
    return code;
}

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace hjw

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::hjw::fail(HJW_EHIP, "%s failed: %s (%d)", #expr, hipGetErrorString(e_), \
                               int(e_));                                                  \
    } while (0)
