// Instantiations of the scaled-piece GEMM for {64,2} operands.
#include "gemm_pieces_b64.hpp"

namespace flyte {

fb_status gemm_pieces_b64_k2(bool all_products, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc,
                             hipStream_t stream)
{
    (void)all_products;
    return pc_b64_out<2, 1>(fc, M, N, K, A, lda, B, ldb, C, ldc, sc, stream);
}

}  // namespace flyte
