// fb_gemm / fb_gemm_ex: argument checks and dispatch to the BF16 matrix-core
// paths ({32,2} on the bfloat16 kernel; {32,3} and the scaled pieces of
// {64,2..4} on the piece kernel) or the FP64 matrix-core path (binary64
// formats).
#include "gemm_f64_impl.hpp"
#include "gemm_pieces.hpp"

namespace flyte {

fb_status gemm_bf16_launch(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb,
                           void* C, int64_t ldc, hipStream_t stream);

#define FLYTE_GEMM_F64_EXTERN(KIN)                                                                                 \
    extern template fb_status gemm_f64_run<KIN>(fb_format, unsigned, const void*, int64_t, const void*, int64_t, \
                                                void*, int64_t, int, int, int, const uint8_t*, const uint8_t*, \
                                                hipStream_t);
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

static fb_status gemm_f64_dispatch(fb_format fa, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                                   int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const uint8_t* bandA,
                                   const uint8_t* bandB, hipStream_t stream)
{
    const int64_t blocks = ((M + GD_BM - 1) / GD_BM) * ((N + GD_BN - 1) / GD_BN);
    const unsigned nb = (unsigned)blocks;
    const int m = (int)M, n = (int)N, k = (int)K;
    switch (fa.k) {
        case 2: return gemm_f64_run<2>(fc, nb, A, lda, B, ldb, C, ldc, m, n, k, bandA, bandB, stream);
        case 3: return gemm_f64_run<3>(fc, nb, A, lda, B, ldb, C, ldc, m, n, k, bandA, bandB, stream);
        case 4: return gemm_f64_run<4>(fc, nb, A, lda, B, ldb, C, ldc, m, n, k, bandA, bandB, stream);
        case 5: return gemm_f64_run<5>(fc, nb, A, lda, B, ldb, C, ldc, m, n, k, bandA, bandB, stream);
        case 6: return gemm_f64_run<6>(fc, nb, A, lda, B, ldb, C, ldc, m, n, k, bandA, bandB, stream);
        case 7: return gemm_f64_run<7>(fc, nb, A, lda, B, ldb, C, ldc, m, n, k, bandA, bandB, stream);
        default: return gemm_f64_run<8>(fc, nb, A, lda, B, ldb, C, ldc, m, n, k, bandA, bandB, stream);
    }
}

}  // namespace flyte

using namespace flyte;

extern "C" fb_status fb_gemm_ex(fb_format fa, fb_format fb, fb_format fc, int64_t M, int64_t N, int64_t K,
                                const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc,
                                uint32_t flags, hipStream_t stream)
{
    if (flags & ~(uint32_t)(FB_GEMM_ALL_PRODUCTS | FB_GEMM_FP64)) return set_error(FB_ERR_ARG, "fb_gemm_ex: unknown flags");
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
    const bool pieces64 = f64 && fa.k <= 4 && !(flags & FB_GEMM_FP64);
    if ((flags & FB_GEMM_ALL_PRODUCTS) && !three && !pieces64)
        return set_error(FB_ERR_UNSUPPORTED,
                         "fb_gemm_ex: all products apply to split operands ({32,3}, or {64,3..4} without FB_GEMM_FP64)");
    if ((flags & FB_GEMM_FP64) && !f64)
        return set_error(FB_ERR_UNSUPPORTED, "fb_gemm_ex: FB_GEMM_FP64 applies to binary64 operands");
    if (M == 0 || N == 0) return FB_OK;
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
        return set_error(FB_ERR_ARG, "fb_gemm: sizes too large");
    if (((M + 127) / 128) * ((N + 127) / 128) > INT32_MAX)
        return set_error(FB_ERR_ARG, "fb_gemm: too many tiles");
    if (!A || !B || !C) return set_error(FB_ERR_ARG, "fb_gemm: null pointer");
    if (!aligned4(A) || !aligned4(B) || !aligned4(C) || (lda * fa.k) % 4 || (ldb * fb.k) % 4 || (ldc * fc.k) % 4)
        return set_error(FB_ERR_ALIGN, "fb_gemm: pointers and rows must be 4-byte aligned");
    if (K == 0) {
        // every entry is an empty sum: +0, whose pattern is all zero bytes in every format
        k_zero_rows<<<1024, 256, 0, stream>>>(static_cast<uint8_t*>(C), N * fc.k, ldc * fc.k, M);
        return check_launch("fb_gemm");
    }
    const bool all = (flags & FB_GEMM_ALL_PRODUCTS) != 0;
    if (bf16) return gemm_bf16_launch(M, N, K, A, lda, B, ldb, C, ldc, stream);
    if (three) return gemm_pieces_b32(all, M, N, K, A, lda, B, ldb, C, ldc, stream);
    if (pieces64) {
        // scaling pass (shifts and band flags in the stream workspace), the
        // piece GEMM on every tile of scalable bands, then FP64 on the rest
        void* ws = nullptr;
        fb_status st = stream_workspace(stream, gemm_pieces_scale_bytes(M, N), &ws);
        if (st != FB_OK) return st;
        PcScale sc{};
        st = gemm_pieces_scale(fa.k, M, N, K, A, lda, B, ldb, ws, &sc, stream);
        if (st != FB_OK) return st;
        st = gemm_pieces_b64(fa.k, all, fc, M, N, K, A, lda, B, ldb, C, ldc, sc, stream);
        if (st != FB_OK) return st;
        return gemm_f64_dispatch(fa, fc, M, N, K, A, lda, B, ldb, C, ldc, sc.bandA, sc.bandB, stream);
    }
    return gemm_f64_dispatch(fa, fc, M, N, K, A, lda, B, ldb, C, ldc, nullptr, nullptr, stream);
}

extern "C" fb_status fb_gemm(fb_format fa, fb_format fb, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t stream)
{
    return fb_gemm_ex(fa, fb, fc, M, N, K, A, lda, B, ldb, C, ldc, 0, stream);
}
