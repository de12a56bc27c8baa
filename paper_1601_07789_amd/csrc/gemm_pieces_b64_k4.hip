// Instantiations of the scaled-piece GEMM for {64,4} operands.
#include "gemm_pieces_b64.hpp"

namespace flyte {

fb_status gemm_pieces_b64_k4(bool all_products, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc,
                             hipStream_t stream)
{
    // default pieces (0,0) (0,1) (0,2) (1,0) (1,1) (2,0): bits 0, 1, 2, 3, 4, 6 of the 3 x 3 set
    return all_products ? pc_b64_out<4, 511>(fc, M, N, K, A, lda, B, ldb, C, ldc, sc, stream)
                        : pc_b64_out<4, 0x5F>(fc, M, N, K, A, lda, B, ldb, C, ldc, sc, stream);
}

}  // namespace flyte
