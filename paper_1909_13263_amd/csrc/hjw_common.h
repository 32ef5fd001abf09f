// hjw_common.h - constants and error reporting shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "hjw.h"

namespace hjw {

// Tile shapes: 64 x TY nodes per workgroup in 2-D (segments of 8 per thread;
// TY = 16 with 256 threads or TY = 32 with 512 threads), 1024 nodes in 1-D
// (segments of 4).
constexpr int kTX = 64, kSX = 8, kSY = 8;
constexpr int kTX1 = 1024, kS1 = 4;

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

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace hjw

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::hjw::fail(HJW_EHIP, "%s failed: %s (%d)", #expr, hipGetErrorString(e_), \
                               int(e_));                                                  \
    } while (0)
