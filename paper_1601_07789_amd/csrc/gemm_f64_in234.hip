// FP64 matrix-core GEMM instantiations for {64,2|3|4} operands.
#include "gemm_f64_impl.hpp"

namespace flyte {

template fb_status gemm_f64_run<2>(fb_format, unsigned, const void*, int64_t, const void*, int64_t, void*, int64_t,
                                      int, int, int, const uint8_t*, const uint8_t*, hipStream_t);
template fb_status gemm_f64_run<3>(fb_format, unsigned, const void*, int64_t, const void*, int64_t, void*, int64_t,
                                      int, int, int, const uint8_t*, const uint8_t*, hipStream_t);
template fb_status gemm_f64_run<4>(fb_format, unsigned, const void*, int64_t, const void*, int64_t, void*, int64_t,
                                      int, int, int, const uint8_t*, const uint8_t*, hipStream_t);

}  // namespace flyte
