// Host-side helpers shared by the libflyte entry points: error reporting,
// argument validation and dispatch from a runtime {base, k} to templates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "flyte.h"

namespace flyte {

// Records a detail message for fb_last_error() on this thread and returns st.
fb_status set_error(fb_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

inline bool format_ok(fb_format f)
{
    if (f.round > 2 || f.reserved != 0) return false;
    if (f.base == 32) return f.k >= 2 && f.k <= 4;
    if (f.base == 64) return f.k >= 2 && f.k <= 8;
    return false;
}

template <int R>
using round_tag = std::integral_constant<int, R>;

// Calls fn(round_tag<mode>{}) for the runtime rounding mode of f.
template <class Fn>
auto dispatch_round(fb_format f, Fn&& fn)
{
    switch (f.round) {
        case 1: return fn(round_tag<1>{});
        case 2: return fn(round_tag<2>{});
        default: return fn(round_tag<0>{});
    }
}

inline bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Checks the most recent launch; maps a HIP error to FB_ERR_RUNTIME.
inline fb_status check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FB_ERR_RUNTIME, "%s: %s", what, hipGetErrorString(e));
    return FB_OK;
}

template <int B, int K>
using fmt_tag = std::pair<std::integral_constant<int, B>, std::integral_constant<int, K>>;

// Calls fn(fmt_tag<base, k>{}) for the runtime format f (which must be valid).
template <class Fn>
auto dispatch_format(fb_format f, Fn&& fn)
{
    switch (f.base * 16 + f.k) {
        case 32 * 16 + 2: return fn(fmt_tag<32, 2>{});
        case 32 * 16 + 3: return fn(fmt_tag<32, 3>{});
        case 32 * 16 + 4: return fn(fmt_tag<32, 4>{});
        case 64 * 16 + 2: return fn(fmt_tag<64, 2>{});
        case 64 * 16 + 3: return fn(fmt_tag<64, 3>{});
        case 64 * 16 + 4: return fn(fmt_tag<64, 4>{});
        case 64 * 16 + 5: return fn(fmt_tag<64, 5>{});
        case 64 * 16 + 6: return fn(fmt_tag<64, 6>{});
        case 64 * 16 + 7: return fn(fmt_tag<64, 7>{});
        default: return fn(fmt_tag<64, 8>{});
    }
}

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Device scratch of at least `bytes` for calls on `stream` (one buffer per
// device and stream, kept for the life of the process).  Growing it
// allocates a new buffer and keeps the old one allocated too, so work already
// queued, and graphs captured earlier, still write valid memory.
fb_status stream_workspace(hipStream_t stream, size_t bytes, void** out);

// One GEMV launch with a given tile (yk = 0: native y; else y packed in yk
// bytes with rounding mode ymode).
fb_status gemv_launch_tile(fb_format f, int64_t m, int64_t n, const void* A, int64_t lda, const void* x, void* y,
                           int tile, hipStream_t stream, int yk = 0, int ymode = 0);

// Transposed GEMV y = A^T x with y native or packed in fy (arguments validated).
fb_status gemv_t_launch(fb_format fa, fb_format fy, int64_t m, int64_t n, const void* A, int64_t lda, const void* x,
                        void* y, hipStream_t stream);

}  // namespace flyte
