// bfloat16-piece GEMMs: the binary32 entry ({32,3} operands) and
// the scaling pass of the scaled binary64 operands ({64,2..4}).  The kernel
// template and the loaders are in gemm_pieces_impl.hpp; the binary64
// instantiations are in gemm_pieces_b64.hpp, one source file per input k.
#include "gemm_pieces_impl.hpp"

namespace flyte {

// ---------------------------------------------------------------- scaling pass
// Per row of A (one wave per row): the largest biased exponent of its non-zero
// elements, e_max, as the shift (e_max - 127) << 20 (0 for an all-zero row),
// and a flag when the row cannot be scaled exactly: an element with exponent
// below e_max - PC_SPREAD, a binary64 subnormal, an infinity or a NaN.
__device__ __forceinline__ void pc_elem_stats(uint32_t h, int& emax, int& emin, int& bad)
{
    const int e = (int)((h >> 20) & 0x7FF);
    const bool zero = (h & 0x7FFFFFFFu) == 0;
    bad |= (e == 0x7FF) || (e == 0 && !zero);
    if (!zero) {
        emax = pc_max(emax, e);
        emin = pc_min(emin, e);
    }
}

template <int K>
__device__ __forceinline__ void pc_chunk_stats(const uint32_t (&d)[K], int& emax, int& emin, int& bad)
{
    uint64_t x[4];
    unpack_elems<Fmt<64, K>, 4>(d, x);
#pragma unroll
    for (int e = 0; e < 4; ++e) pc_elem_stats((uint32_t)(x[e] >> 32), emax, emin, bad);
}

__device__ __forceinline__ int32_t pc_stats_word(int emax, int emin, int bad)
{
    // 11 bits e_max, 11 bits (2047 - e_min), 1 bit flag: field-wise maxima combine
    return emax | ((2047 - emin) << 11) | (bad << 22);
}

__device__ __forceinline__ int32_t pc_stats_max(int32_t a, int32_t b)
{
    return pc_max(a & 0x7FF, b & 0x7FF) | pc_max(a & (0x7FF << 11), b & (0x7FF << 11)) | ((a | b) & (1 << 22));
}

__device__ __forceinline__ void pc_stats_final(int32_t w, int32_t& shift, uint8_t& flag)
{
    const int emax = w & 0x7FF, emin = 2047 - ((w >> 11) & 0x7FF), bad = (w >> 22) & 1;
    shift = emax ? (emax - 127) * (1 << 20) : 0;
    flag = (uint8_t)(bad || (emax && emax - emin > PC_SPREAD));
}

template <int K>
__global__ void __launch_bounds__(256) k_pc_row_stats(const uint8_t* __restrict__ A, int64_t lda, int M, int Kd,
                                                      int32_t* __restrict__ shift, uint8_t* __restrict__ flag)
{
    const int row = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (row >= M) return;
    int emax = 0, emin = 2047, bad = 0;
    const uint8_t* base = A + (int64_t)row * lda * K;
    for (int kk = lane * 4; kk < Kd; kk += 256) {
        uint32_t d[K];
        const uint8_t* p = base + (int64_t)kk * K;
        if (kk + 4 <= Kd) load_dwords(reinterpret_cast<const uint32_t*>(p), d);
        else pc_load_edge<K>(p, (Kd - kk) * K, d);
        pc_chunk_stats<K>(d, emax, emin, bad);
    }
    int32_t w = pc_stats_word(emax, emin, bad);
#pragma unroll
    for (int o = 32; o >= 1; o /= 2) w = pc_stats_max(w, __shfl_xor(w, o, 64));
    if (lane == 0) pc_stats_final(w, shift[row], flag[row]);
}

// Per column of B: workgroup (x, y) takes 256 columns (64 lanes x 4) over the
// rows y, y + S, y + 2S, ... (4 row lanes per workgroup); the partial
// statistics of each slab go to part[y][column], combined by k_pc_col_final.
template <int K>
__global__ void __launch_bounds__(256) k_pc_col_stats(const uint8_t* __restrict__ B, int64_t ldb, int Kd, int N,
                                                      int32_t* __restrict__ part)
{
    const int cl = threadIdx.x % 64, rl = threadIdx.x / 64;
    const int col = blockIdx.x * 256 + cl * 4;
    const int S = gridDim.y * 4;
    int emax[4] = {0, 0, 0, 0}, emin[4] = {2047, 2047, 2047, 2047}, bad[4] = {0, 0, 0, 0};
    if (col < N) {
        const int nv = pc_min(4, N - col);
        for (int r = blockIdx.y * 4 + rl; r < Kd; r += S) {
            uint32_t d[K];
            const uint8_t* p = B + ((int64_t)r * ldb + col) * K;
            if (nv == 4) load_dwords(reinterpret_cast<const uint32_t*>(p), d);
            else pc_load_edge<K>(p, nv * K, d);
            uint64_t x[4];
            unpack_elems<Fmt<64, K>, 4>(d, x);
#pragma unroll
            for (int e = 0; e < 4; ++e) pc_elem_stats((uint32_t)(x[e] >> 32), emax[e], emin[e], bad[e]);
        }
    }
    __shared__ int32_t red[4][256];
#pragma unroll
    for (int e = 0; e < 4; ++e) red[rl][cl * 4 + e] = pc_stats_word(emax[e], emin[e], bad[e]);
    __syncthreads();
    if (rl == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int32_t w = red[0][cl * 4 + e];
            for (int q = 1; q < 4; ++q) w = pc_stats_max(w, red[q][cl * 4 + e]);
            if (col + e < N) part[(int64_t)blockIdx.y * N + col + e] = w;
        }
    }
}

__global__ void __launch_bounds__(256) k_pc_col_final(const int32_t* __restrict__ part, int slabs, int N,
                                                      int32_t* __restrict__ shift, uint8_t* __restrict__ flag)
{
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= N) return;
    int32_t w = part[col];
    for (int s = 1; s < slabs; ++s) w = pc_stats_max(w, part[(int64_t)s * N + col]);
    pc_stats_final(w, shift[col], flag[col]);
}

// Band flags: band b of A (B) is flagged when any of its 128 rows (columns) is.
__global__ void __launch_bounds__(128) k_pc_bands(const uint8_t* __restrict__ rowflag, int M,
                                                  uint8_t* __restrict__ band)
{
    const int r = blockIdx.x * 128 + threadIdx.x;
    const int f = (r < M) ? rowflag[r] : 0;
    const int any = __syncthreads_or(f);
    if (threadIdx.x == 0) band[blockIdx.x] = (uint8_t)(any != 0);
}

fb_status gemm_pieces_b32(bool all_products, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                          const void* B, int64_t ldb, void* C, int64_t ldc, hipStream_t stream)
{
    const PcScale none{};
    if (all_products) return pc_run<PcB32K3, 15, 256, 256, 2, 4, 0, 0>(M, N, K, A, lda, B, ldb, C, ldc, none, stream);
    return pc_run<PcB32K3, 7, 256, 256, 2, 4, 0, 0>(M, N, K, A, lda, B, ldb, C, ldc, none, stream);
}

size_t gemm_pieces_scale_bytes(int64_t M, int64_t N)
{
    const int64_t slabs = kPcColSlabs;
    return (size_t)(4 * (M + N) + (M + N) + ((M + 127) / 128 + (N + 127) / 128) + 4 * slabs * N + 256);
}

fb_status gemm_pieces_scale(int k, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                            int64_t ldb, void* ws, PcScale* sc, hipStream_t stream)
{
    // layout: shiftA[M], shiftB[N], part[slabs][N] (int32), rowflag[M], colflag[N], bandA, bandB
    int32_t* shiftA = static_cast<int32_t*>(ws);
    int32_t* shiftB = shiftA + M;
    int32_t* part = shiftB + N;
    uint8_t* rowflag = reinterpret_cast<uint8_t*>(part + (int64_t)kPcColSlabs * N);
    uint8_t* colflag = rowflag + M;
    uint8_t* bandA = colflag + N;
    uint8_t* bandB = bandA + (M + 127) / 128;
    const int slabs = (int)(((K + 3) / 4) < kPcColSlabs ? ((K + 3) / 4 > 0 ? (K + 3) / 4 : 1) : kPcColSlabs);
    auto a = static_cast<const uint8_t*>(A);
    auto b = static_cast<const uint8_t*>(B);
    const unsigned rb = (unsigned)((M + 3) / 4);
    const dim3 cg((unsigned)((N + 255) / 256), (unsigned)slabs);
    switch (k) {
        case 2:
            k_pc_row_stats<2><<<rb, 256, 0, stream>>>(a, lda, (int)M, (int)K, shiftA, rowflag);
            k_pc_col_stats<2><<<cg, 256, 0, stream>>>(b, ldb, (int)K, (int)N, part);
            break;
        case 3:
            k_pc_row_stats<3><<<rb, 256, 0, stream>>>(a, lda, (int)M, (int)K, shiftA, rowflag);
            k_pc_col_stats<3><<<cg, 256, 0, stream>>>(b, ldb, (int)K, (int)N, part);
            break;
        default:
            k_pc_row_stats<4><<<rb, 256, 0, stream>>>(a, lda, (int)M, (int)K, shiftA, rowflag);
            k_pc_col_stats<4><<<cg, 256, 0, stream>>>(b, ldb, (int)K, (int)N, part);
            break;
    }
    k_pc_col_final<<<(unsigned)((N + 255) / 256), 256, 0, stream>>>(part, slabs, (int)N, shiftB, colflag);
    k_pc_bands<<<(unsigned)((M + 127) / 128), 128, 0, stream>>>(rowflag, (int)M, bandA);
    k_pc_bands<<<(unsigned)((N + 127) / 128), 128, 0, stream>>>(colflag, (int)N, bandB);
    sc->shiftA = shiftA;
    sc->shiftB = shiftB;
    sc->bandA = bandA;
    sc->bandB = bandB;
    return check_launch("fb_gemm");
}

fb_status gemm_pieces_b64(int k, bool all_products, fb_format fc, int64_t M, int64_t N, int64_t K, const void* A,
                          int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, const PcScale& sc,
                          hipStream_t stream)
{
    switch (k) {
        case 2: return gemm_pieces_b64_k2(all_products, fc, M, N, K, A, lda, B, ldb, C, ldc, sc, stream);
        case 3: return gemm_pieces_b64_k3(all_products, fc, M, N, K, A, lda, B, ldb, C, ldc, sc, stream);
        default: return gemm_pieces_b64_k4(all_products, fc, M, N, K, A, lda, B, ldb, C, ldc, sc, stream);
    }
}

}  // namespace flyte
