// fb_gemm / fb_gemm_ex: argument checks and dispatch to the BF16 matrix-core
// paths ({32,2}, {32,3}) or the FP64 matrix-core path (binary64 formats).
#include "gemm_f64_impl.hpp"

namespace flyte {

fb_status gemm_bf16_launch(int mode, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                           int64_t ldb, void* C, int64_t ldc, hipStream_t stream);

#define FLYTE_GEMM_F64_EXTERN(KIN)                                                                                 \
    extern template fb_status gemm_f64_run<KIN>(fb_format, unsigned, const void*, int64_t, const void*, int64_t, \
                                                void*, int64_t, int, int, int, hipStream_t);
FLYTE_GEMM_F64_EXTERN(2)
FLYTE_GEMM_F64_EXTERN(3)
FLYTE_GEMM_F64_EXTERN(4)
FLYTE_GEMM_F64_EXTERN(5)
FLYTE_GEMM_F64_EXTERN(6)
FLYTE_GEMM_F64_EXTERN(7)
FLYTE_GEMM_F64_EXTERN(8)
#undef FLYTE_GEMM_F64_EXTERN

__global__ void k_zero_rows(uint8_t* __restrict__ C, int64_t row_bytes, int64_t pitch, int64_t rows)
{
    const int64_t total = row_bytes * rows;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        C[(i / row_bytes) * pitch + i % row_bytes] = 0;
}

}  // namespace flyte

using namespace flyte;

extern "C" fb_status fb_gemm_ex(fb_format fa, fb_format fb, fb_format fc, int64_t M, int64_t N, int64_t K,
                                const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc,
                                uint32_t flags, hipStream_t stream)
{
    if (flags & ~(uint32_t)FB_GEMM_FOUR_PRODUCTS) return set_error(FB_ERR_ARG, "fb_gemm_ex: unknown flags");
    if (!format_ok(fa) || !format_ok(fb) || !format_ok(fc))
        return set_error(FB_ERR_FORMAT, "fb_gemm: invalid format");
    if (M < 0 || N < 0 || K < 0) return set_error(FB_ERR_ARG, "fb_gemm: negative size");
    if (lda < K || ldb < N || ldc < N) return set_error(FB_ERR_ARG, "fb_gemm: leading dimension too small");
    const bool bf16 = fa.base == 32 && fa.k == 2 && fb.base == 32 && fb.k == 2 && fc.base == 32 && fc.k == 4;
    const bool three = fa.base == 32 && fa.k == 3 && fb.base == 32 && fb.k == 3 && fc.base == 32 && fc.k == 4;
    const bool f64 = fa.base == 64 && fb.base == 64 && fb.k == fa.k && fc.base == 64;
    if (!bf16 && !three && !f64)
        return set_error(FB_ERR_UNSUPPORTED,
                         "fb_gemm: supported: {32,2}x{32,2}->{32,4}, {32,3}x{32,3}->{32,4}, "
                         "{64,k}x{64,same k}->{64,any}");
    if (M == 0 || N == 0) return FB_OK;
    if (!A || !B || !C) return set_error(FB_ERR_ARG, "fb_gemm: null pointer");
    if (!aligned4(A) || !aligned4(B) || !aligned4(C) || (lda * fa.k) % 4 || (ldb * fb.k) % 4 || (ldc * fc.k) % 4)
        return set_error(FB_ERR_ALIGN, "fb_gemm: pointers and rows must be 4-byte aligned");
    if (K == 0) {
        // every entry is an empty sum: +0, whose pattern is all zero bytes in every format
        k_zero_rows<<<1024, 256, 0, stream>>>(static_cast<uint8_t*>(C), N * fc.k, ldc * fc.k, M);
        return check_launch("fb_gemm");
    }
    if ((flags & FB_GEMM_FOUR_PRODUCTS) && !three)
        return set_error(FB_ERR_UNSUPPORTED, "fb_gemm_ex: four products apply to {32,3} operands only");
    if (bf16 || three)
        return gemm_bf16_launch(bf16 ? 0 : ((flags & FB_GEMM_FOUR_PRODUCTS) ? 2 : 1), M, N, K, A, lda, B, ldb, C, ldc,
                                stream);
    if (M % GD_BM || N % GD_BN || K % GD_BK)
        return set_error(FB_ERR_UNSUPPORTED, "fb_gemm: binary64 paths need M, N multiples of %d and K of %d", GD_BM,
                         GD_BK);
    const int64_t blocks = (M / GD_BM) * (N / GD_BN);
    if (blocks > INT32_MAX || M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
        return set_error(FB_ERR_ARG, "fb_gemm: sizes too large");
    const unsigned nb = (unsigned)blocks;
    switch (fa.k) {
        case 2: return gemm_f64_run<2>(fc, nb, A, lda, B, ldb, C, ldc, (int)M, (int)N, (int)K, stream);
        case 3: return gemm_f64_run<3>(fc, nb, A, lda, B, ldb, C, ldc, (int)M, (int)N, (int)K, stream);
        case 4: return gemm_f64_run<4>(fc, nb, A, lda, B, ldb, C, ldc, (int)M, (int)N, (int)K, stream);
        case 5: return gemm_f64_run<5>(fc, nb, A, lda, B, ldb, C, ldc, (int)M, (int)N, (int)K, stream);
        case 6: return gemm_f64_run<6>(fc, nb, A, lda, B, ldb, C, ldc, (int)M, (int)N, (int)K, stream);
        case 7: return gemm_f64_run<7>(fc, nb, A, lda, B, ldb, C, ldc, (int)M, (int)N, (int)K, stream);
        default: return gemm_f64_run<8>(fc, nb, A, lda, B, ldb, C, ldc, (int)M, (int)N, (int)K, stream);
    }
}

extern "C" fb_status fb_gemm(fb_format fa, fb_format fb, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t stream)
{
    return fb_gemm_ex(fa, fb, fc, M, N, K, A, lda, B, ldb, C, ldc, 0, stream);
}
