// Host interface of the bfloat16-piece GEMMs (gemm_pieces.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flyte.h"

namespace flyte {

// Exponent shifts and band flags of scaled (binary64, k <= 4) operands:
// shiftA[i] = (e_i - 127) << 20 for row i of A, shiftB[j] likewise for column
// j of B (e the largest biased exponent of the row's non-zero elements);
// bandA[b] / bandB[b] != 0 when a row (column) of the 128-wide band b cannot
// be scaled exactly, so its tiles belong to the FP64 GEMM.
struct PcScale {
    const int32_t* shiftA;
    const int32_t* shiftB;
    const uint8_t* bandA;
    const uint8_t* bandB;
};

// Row slabs of the column-statistics pass.
constexpr int kPcColSlabs = 16;

// {32,3} operands (all_products adds lo*lo), FP32 C.
fb_status gemm_pieces_b32(bool all_products, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                          const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t stream);

// Device bytes the scaling pass needs for an M x K times K x N product.
size_t gemm_pieces_scale_bytes(int64_t M, int64_t N);

// Scaling pass over {64,k} operands (k = 2..4) into the device buffer ws
// (gemm_pieces_scale_bytes bytes); fills *sc with pointers into ws.
fb_status gemm_pieces_scale(int k, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                            int64_t ldb, void* ws, PcScale* sc, hipStream_t stream);

// {64,k} operands (k = 2..4) as scaled bfloat16 pieces, C in the binary64
// format fc; tiles in flagged bands are skipped (left to the FP64 GEMM).
// all_products: every product of pieces, else those of combined weight
// within the format's precision.
fb_status gemm_pieces_b64(int k, bool all_products, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                          int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc,
                          hipStream_t stream);

// One input k each (gemm_pieces_b64_k2/3/4.hip).
fb_status gemm_pieces_b64_k2(bool all_products, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc,
                             hipStream_t stream);
fb_status gemm_pieces_b64_k3(bool all_products, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc,
                             hipStream_t stream);
fb_status gemm_pieces_b64_k4(bool all_products, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc,
                             hipStream_t stream);

}  // namespace flyte
