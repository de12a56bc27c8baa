// Scaled binary64 operands ({64,K}, K = 2..4) on the bfloat16-piece GEMM:
// output-format and rounding-mode dispatch.  Each K is instantiated in its own
// source file (gemm_pieces_b64_k2/3/4.hip) so they compile in parallel.
#pragma once

#include "gemm_pieces_impl.hpp"

namespace flyte {

template <int K, int PRODS, int OUTK, int RMODE>
fb_status pc_run_b64(int64_t M, int64_t N, int64_t Kd, const void* A, int64_t lda, const void* B, int64_t ldb,
                            void* C, int64_t ldc, const PcScale& sc, hipStream_t stream)
{
    if constexpr (K == 4)   // three pieces: 128 x 256 tiles keep both stages in LDS (144 KiB)
        return pc_run<PcB64<4>, PRODS, 128, 256, 2, 4, OUTK, RMODE>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
    else
        return pc_run<PcB64<K>, PRODS, 256, 256, 2, 4, OUTK, RMODE>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
}

template <int K, int PRODS>
fb_status pc_b64_out(fb_format fc, int64_t M, int64_t N, int64_t Kd, const void* A, int64_t lda,
                            const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc, hipStream_t stream)
{
    return dispatch_round(fc, [&](auto rt) {
        constexpr int RM = decltype(rt)::value;
        switch (fc.k) {
            case 2: return pc_run_b64<K, PRODS, 2, RM>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
            case 3: return pc_run_b64<K, PRODS, 3, RM>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
            case 4: return pc_run_b64<K, PRODS, 4, RM>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
            case 5: return pc_run_b64<K, PRODS, 5, RM>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
            case 6: return pc_run_b64<K, PRODS, 6, RM>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
            case 7: return pc_run_b64<K, PRODS, 7, RM>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
            default: return pc_run_b64<K, PRODS, 8, 0>(M, N, Kd, A, lda, B, ldb, C, ldc, sc, stream);
        }
    });
}

}  // namespace flyte
