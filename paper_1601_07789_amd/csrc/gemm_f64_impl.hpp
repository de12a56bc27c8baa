// FP64 matrix-core GEMM on binary64-derived k-byte operands (k = 2..8), with
// the result rounded to a k-byte format in the epilogue.
//
// C = A B: A M x K and B K x N row-major packed in one binary64 format; C M x N
// row-major in any binary64 format.  Operands are unpacked (Section 3.2) while
// they are copied into LDS as FP64; products and sums run on
// v_mfma_f64_16x16x4_f64 in FP64; each C entry is then rounded once to the
// output format (Section 5.2) -- the double rounding of Section 3.1 (FP64
// accumulation, then the cut) is part of the method.  For k <= 4 (at most
// 21 significant bits) every product is exact in FP64, so only the FP64 sums
// and the final cut round; the 11-bit exponent of these formats is kept whole.
//
// Tiling: a 256-thread workgroup computes 128 x 128 of C, each wave a 64 x 64
// quarter as 4 x 4 MFMA tiles; K moves in steps of 16 through double-buffered
// LDS.  Both operand tiles are stored k-major (A transposed while unpacking)
// with rows padded to 144 doubles, so the 16 lanes that share a k read 16
// consecutive doubles and the two lane halves of a read hit disjoint banks.
// A row of the transposed A is 288 dwords, 32 modulo the 64 banks, so the bank
// of an A store depends on the m index alone: each wave therefore unpacks 32
// consecutive rows of A x 2 adjacent units along k per instruction (not whole
// rows), which puts exactly two lanes on every bank pair.
// Epilogue: lane l holds rows l/16 + 4r (r = 0..3), column l%16, of each
// 16 x 16 tile (the FP64 instruction's output order); the G lanes
// of one dword-aligned group of columns pass their packed values to the
// group's first lane (cross-lane shuffles), which assembles them with
// v_perm_b32 and writes whole dwords, so no two lanes write the same dword.
#pragma once

#include "codec.hpp"
#include "common.hpp"

namespace flyte {

typedef double f64x4_t __attribute__((ext_vector_type(4)));

constexpr int GD_BM = 128, GD_BN = 128, GD_BK = 16, GD_THREADS = 256;
constexpr int GD_ROW = GD_BM + 16;    // doubles per padded LDS row

__device__ __forceinline__ void gemm_tile_coords_f64(int ntm, int ntn, int& tm, int& tn)
{
    const int nb = ntm * ntn;
    int pid = blockIdx.x;
    if (nb % 8 == 0) pid = (pid % 8) * (nb / 8) + pid / 8;
    constexpr int GROUP = 8;
    const int per_group = GROUP * ntn;
    const int group = pid / per_group;
    const int first_m = group * GROUP;
    const int gsize = (ntm - first_m) < GROUP ? (ntm - first_m) : GROUP;
    tm = first_m + (pid % per_group) % gsize;
    tn = (pid % per_group) / gsize;
}

// A unit u of the 128-row tile (A_UPR units per row) -> (row, unit along k):
// chunk u / 64 picks a block of 32 rows and a pair of units, lane u % 64 the
// row in the block and the unit in the pair.
template <int A_UPR>
__device__ __forceinline__ void a_unit_map(int u, int& row, int& uc)
{
    static_assert(A_UPR >= 2 && A_UPR % 2 == 0, "A units per row");
    const int q = u / 64, l = u % 64;
    row = (q % (GD_BM / 32)) * 32 + l % 32;
    uc = (q / (GD_BM / 32)) * 2 + l / 32;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Loads the N dwords of one unit whose first nbytes bytes are valid (0 <=
// nbytes <= 4 N): dwords wholly inside are loaded, a straddling dword is
// assembled from byte loads, the rest are zero.  Nothing past the valid bytes
// is read.
template <int N>
__device__ __forceinline__ void gd_load_edge(const uint8_t* p, int nbytes, uint32_t (&out)[N])
{
#pragma unroll
    for (int w = 0; w < N; ++w) {
        if (4 * w + 4 <= nbytes) {
            out[w] = *reinterpret_cast<const uint32_t*>(p + 4 * w);
        } else {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (4 * w + b < nbytes) v |= (uint32_t)p[4 * w + b] << (8 * b);
            out[w] = v;
        }
    }
}

__device__ __forceinline__ int gd_clamp(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// bandA, bandB (may be null): when given, only the tiles whose 128-row band of
// A or 128-column band of B is flagged are computed (the rest belong to the
// bfloat16-piece GEMM of the same call).  CHECK: loads and stores are bounded
// (any M, N, K); without it M, N are multiples of 128 and K of 16.
template <int KIN, int KOUT, int MODE, bool CHECK>
__global__ void __launch_bounds__(GD_THREADS, 2)
k_gemm_f64(const uint8_t* __restrict__ A, int64_t lda, const uint8_t* __restrict__ B, int64_t ldb,
           uint8_t* __restrict__ C, int64_t ldc, int M, int N, int K, const uint8_t* __restrict__ bandA,
           const uint8_t* __restrict__ bandB)
{
    using FI = Fmt<64, KIN>;
    using FO = Fmt<64, KOUT>;
    constexpr int U = FI::UNIT;                     // elements per loaded unit
    constexpr int A_UNITS = GD_BM * GD_BK / U / GD_THREADS;
    constexpr int B_UNITS = GD_BK * GD_BN / U / GD_THREADS;
    static_assert(A_UNITS >= 1 && B_UNITS >= 1, "tile too small for the unit");
    __shared__ __attribute__((aligned(16))) double lds[2][2][GD_BK * GD_ROW];   // [stage][A^T, B][k][m or n]

    const int ntm = (M + GD_BM - 1) / GD_BM, ntn = (N + GD_BN - 1) / GD_BN;
    int tm, tn;
    gemm_tile_coords_f64(ntm, ntn, tm, tn);
    if (bandA && !bandA[tm] && !bandB[tn]) return;
    const int m0 = tm * GD_BM, n0 = tn * GD_BN;
    const int t = threadIdx.x, lane = t % 64, wid = t / 64;
    const int wm = wid / 2, wn = wid % 2;
    const bool interior = !CHECK || (m0 + GD_BM <= M && n0 + GD_BN <= N);

    uint32_t ra[A_UNITS][FI::UNIT_DW], rb[B_UNITS][FI::UNIT_DW];
    constexpr int A_UPR = GD_BK / U;    // A units per row of the tile
    constexpr int B_UPR = GD_BN / U;    // B units per row of the tile

    // edge tiles and the last K step load with bounds: elements outside the
    // matrix read as +0, and no byte past a row's last element is read
    auto load_tiles = [&](int k0) {
        const bool edge = CHECK && (!interior || k0 + GD_BK > K);
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            int row, uc;
            a_unit_map<A_UPR>(t + GD_THREADS * i, row, uc);
            const uint8_t* p = A + ((int64_t)(m0 + row) * lda + k0 + uc * U) * KIN;
            if (!edge) load_dwords(reinterpret_cast<const uint32_t*>(p), ra[i]);
            else gd_load_edge(p, m0 + row < M ? gd_clamp(K - (k0 + uc * U), U) * KIN : 0, ra[i]);
        }
#pragma unroll
        for (int i = 0; i < B_UNITS; ++i) {
            const int u = t + GD_THREADS * i, row = u / B_UPR, uc = u % B_UPR;
            const uint8_t* p = B + ((int64_t)(k0 + row) * ldb + n0 + uc * U) * KIN;
            if (!edge) load_dwords(reinterpret_cast<const uint32_t*>(p), rb[i]);
            else gd_load_edge(p, k0 + row < K ? gd_clamp(N - (n0 + uc * U), U) * KIN : 0, rb[i]);
        }
    };
    auto store_tiles = [&](int s) {
        double* At = lds[s][0];
        double* Bs = lds[s][1];
#pragma unroll
        for (int i = 0; i < A_UNITS; ++i) {
            int row, uc;
            a_unit_map<A_UPR>(t + GD_THREADS * i, row, uc);
            uint64_t x[U];
            unpack_elems<FI, U>(ra[i], x);
#pragma unroll
            for (int c = 0; c < U; ++c) At[(uc * U + c) * GD_ROW + row] = __longlong_as_double((long long)x[c]);
        }
#pragma unroll
        for (int i = 0; i < B_UNITS; ++i) {
            const int u = t + GD_THREADS * i, row = u / B_UPR, uc = u % B_UPR;
            uint64_t x[U];
            unpack_elems<FI, U>(rb[i], x);
#pragma unroll
            for (int c = 0; c < U; ++c) Bs[row * GD_ROW + uc * U + c] = __longlong_as_double((long long)x[c]);
        }
    };

    f64x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};

    auto compute = [&](int s) {
        const double* At = lds[s][0];
        const double* Bs = lds[s][1];
        const int c16 = lane % 16, kq = lane / 16;
#pragma unroll
        for (int ks = 0; ks < GD_BK / 4; ++ks) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = At[(ks * 4 + kq) * GD_ROW + wm * 64 + i * 16 + c16];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[(ks * 4 + kq) * GD_ROW + wn * 64 + j * 16 + c16];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };

    // the last K step is peeled so the loop body has no branches
    const int KT = (K + GD_BK - 1) / GD_BK;
    load_tiles(0);
    store_tiles(0);
    __syncthreads();
    for (int kt = 0; kt < KT - 1; ++kt) {
        const int s = kt & 1;
        load_tiles((kt + 1) * GD_BK);
        compute(s);
        store_tiles(s ^ 1);
        __syncthreads();
    }
    compute((KT - 1) & 1);

    // ---- epilogue: round to the output format and store whole dword groups
    constexpr int GO = FO::G;
    const int c16 = lane % 16;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + i * 16 + lane / 16 + 4 * r;
                const int col = n0 + wn * 64 + j * 16 + c16;
                const uint64_t q = round_pack<FO, MODE>((uint64_t)__double_as_longlong(acc[i][j][r]));
                uint64_t g[GO];
                g[0] = q;
#pragma unroll
                for (int e = 1; e < GO; ++e) g[e] = shfl_u64(q, (lane + e) % 64);
                if (c16 % GO == 0 && (interior || (row < M && col < N))) {
                    uint8_t* dst = C + ((int64_t)row * ldc + col) * KOUT;
                    if (interior || col + GO <= N) {
                        uint32_t out[GO * KOUT / 4];
                        assemble_elems<FO, GO>(g, out);
                        store_dwords(reinterpret_cast<uint32_t*>(dst), out);
                    } else {
                        // a group cut by the last column: bytes of its valid elements only
#pragma unroll
                        for (int e = 0; e < GO; ++e)
                            if (col + e < N) store_elem_bytes<FO>(dst + e * KOUT, g[e]);
                    }
                }
            }
}

template <int KIN, int MODE>
fb_status launch_f64(int kout, unsigned blocks, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                     int64_t ldc, int M, int N, int K, const uint8_t* bandA, const uint8_t* bandB, hipStream_t stream)
{
    auto a = static_cast<const uint8_t*>(A);
    auto b = static_cast<const uint8_t*>(B);
    auto c = static_cast<uint8_t*>(C);
    // shapes that are tile multiples take the instance without bounds checks
    const bool check = M % GD_BM != 0 || N % GD_BN != 0 || K % GD_BK != 0;
#define FLYTE_F64_LAUNCH(KO, MO)                                                                                   \
    if (check)                                                                                                   \
        k_gemm_f64<KIN, KO, MO, true><<<blocks, GD_THREADS, 0, stream>>>(a, lda, b, ldb, c, ldc, M, N, K, bandA,  \
                                                                        bandB);                                   \
    else                                                                                                         \
        k_gemm_f64<KIN, KO, MO, false><<<blocks, GD_THREADS, 0, stream>>>(a, lda, b, ldb, c, ldc, M, N, K, bandA, \
                                                                         bandB)
    switch (kout) {
        case 2: FLYTE_F64_LAUNCH(2, MODE); break;
        case 3: FLYTE_F64_LAUNCH(3, MODE); break;
        case 4: FLYTE_F64_LAUNCH(4, MODE); break;
        case 5: FLYTE_F64_LAUNCH(5, MODE); break;
        case 6: FLYTE_F64_LAUNCH(6, MODE); break;
        case 7: FLYTE_F64_LAUNCH(7, MODE); break;
        default: FLYTE_F64_LAUNCH(8, 0); break;
    }
#undef FLYTE_F64_LAUNCH
    return check_launch("fb_gemm");
}

// Runs C = A B for operands packed in {64, KIN} with C in the format fc (valid,
// binary64), any M, N, K >= 1 (edge tiles and the K tail are bounded); with
// bandA/bandB only the flagged bands' tiles.  Instantiated per KIN in its own
// source file so the instantiations compile in parallel.
template <int KIN>
fb_status gemm_f64_run(fb_format fc, unsigned blocks, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                       int64_t ldc, int M, int N, int K, const uint8_t* bandA, const uint8_t* bandB,
                       hipStream_t stream)
{
    return dispatch_round(fc, [&](auto rt) {
        constexpr int MODE = decltype(rt)::value;
        return launch_f64<KIN, MODE>(fc.k, blocks, A, lda, B, ldb, C, ldc, M, N, K, bandA, bandB, stream);
    });
}

}  // namespace flyte
