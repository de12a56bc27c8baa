// GEMMs on binary32-derived operands with BF16 matrix cores (gfx950).
//
// C = A B, A M x K and B K x N row-major packed, C FP32 row-major.
//  MODE 0 ({32,2}): the stored 2-byte patterns are bfloat16 operands as they
//    are (the 16-bit flyte of Table 1 is bit-for-bit bfloat16).
//  MODE 1 ({32,3}): the loader unpacks each 3-byte element to binary32 x and
//    splits it into hi = x with its low 16 bits cleared (a bfloat16) and
//    lo = x - hi (exact in binary32, and exactly a bfloat16 for biased
//    exponent >= 9; rounded to nearest otherwise; 0 for Inf/NaN).  The tile
//    product is hi*hi + hi*lo + lo*hi: three BF16 MFMAs per step into the same
//    FP32 accumulators (lo*lo, below 2^-16 relative, is dropped).
//  MODE 2 ({32,3}, four products): MODE 1 plus lo*lo, so every product of the
//    split operands is formed exactly and only the FP32 accumulation rounds.
//
// Tiling: a workgroup computes a BM x BN tile of C with WGM x WGN waves, each
// wave a (BM/WGM) x (BN/WGN) tile of v_mfma_f32_16x16x32_bf16 results.  Large
// wave tiles keep LDS operand traffic below the LDS bandwidth: BF16 uses
// 256 x 256 x 64 tiles with 8 waves of 128 x 64 (about 94 B/clk of LDS reads
// per CU at the MFMA peak, against 128 available); the 3-product uses
// 256 x 128 x 32 with 4 waves of 128 x 64 (three MFMAs per operand pair);
// shapes that are not multiples of those use 128 x 128 x 64.  K is walked in
// BK steps through double-buffered LDS (one barrier per step; the next step's
// global loads are issued before the current step's MFMAs; the last step is
// peeled).  LDS rows are padded by 16 bytes, so the 16-byte operand reads of
// 16 lanes hit distinct banks.  B is stored in LDS transposed (n-major, k contiguous):
// each thread loads KR rows of B and transposes them in registers with
// v_perm_b32, so every MFMA operand is one ds_read_b128.  Workgroups are
// renumbered so that consecutive tiles of C run on the same XCD (sharing its
// L2), grouped 8 tile-rows at a time.
#include "codec.hpp"
#include "common.hpp"

namespace flyte {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Tile index of this workgroup: XCD-aware renumbering, then 8-row groups.
__device__ __forceinline__ void gemm_tile_coords(int ntm, int ntn, int& tm, int& tn)
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

// bfloat16 pattern of a binary32 value, round to nearest even (non-NaN input).
__device__ __forceinline__ uint32_t bf16_rne(uint32_t u)
{
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// hi/lo split of a binary32 pattern (MODE 1).
__device__ __forceinline__ void split_hi_lo(uint32_t u, uint32_t& hi, uint32_t& lo)
{
    hi = u >> 16;
    const float r = __uint_as_float(u) - __uint_as_float(u & 0xFFFF0000u);
    lo = ((u & 0x7F800000u) == 0x7F800000u) ? 0u : bf16_rne(__float_as_uint(r));
}

// Tile configuration: BM x BN x BK workgroup tile, WGM x WGN waves (wave tile
// (BM/WGM) x (BN/WGN) as 16 x 16 MFMA tiles), B loaded in groups of KR rows.
// Stores KR bf16 (KR/2 dwords) at an LDS address: one ds_write_b128 or b64.
template <int KR>
__device__ __forceinline__ void store_row_chunk(uint16_t* dst, const uint32_t (&v)[KR / 2])
{
    if constexpr (KR == 8) {
        *reinterpret_cast<u32x4_t*>(dst) = u32x4_t{v[0], v[1], v[2], v[3]};
    } else {
        typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
        *reinterpret_cast<u32x2_t*>(dst) = u32x2_t{v[0], v[1]};
    }
}

template <int MODE, int BM, int BN, int BK, int WGM, int WGN, int KR>
struct B32Tile {
    static constexpr int THREADS = 64 * WGM * WGN;
    static constexpr int TM = BM / WGM, TN = BN / WGN;
    static constexpr int FM = TM / 16, FN = TN / 16;
    static constexpr int PARTS = MODE ? 2 : 1;          // hi (and lo) operand tiles
    static constexpr int KB = MODE ? 3 : 2;             // stored bytes per element
    static constexpr int ROW = BK + 8;                  // bf16 per padded LDS row
    static constexpr int A_TILE = BM * ROW, B_TILE = BN * ROW;
    static constexpr int STAGE = PARTS * (A_TILE + B_TILE);
    // A: chunks of A_EL consecutive elements of a row (16 or 48 bytes)
    static constexpr int A_EL = MODE ? 16 : 8;
    static constexpr int A_CPR = BK / A_EL;
    static constexpr int A_N = BM * A_CPR / THREADS;
    static constexpr int A_DW = A_EL * KB / 4;
    // B: groups of KR k-rows x BCOL columns (one dword or one 4-element unit per row)
    static constexpr int BCOL = MODE ? 4 : 2;
    static constexpr int B_GPR = BN / BCOL;
    static constexpr int B_G = (BK / KR) * B_GPR / THREADS;
    static constexpr int B_DW = MODE ? 3 : 1;
    static_assert(BK % 32 == 0 && TM % 16 == 0 && TN % 16 == 0, "tile shape");
    static_assert(A_N * THREADS == BM * A_CPR && A_N >= 1, "A staging must divide evenly");
    static_assert(B_G * THREADS == (BK / KR) * B_GPR && B_G >= 1, "B staging must divide evenly");
    static_assert(KR == 4 || KR == 8, "B group rows");
};

template <int MODE, int BM, int BN, int BK, int WGM, int WGN, int KR>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm_b32(const uint8_t* __restrict__ A, int64_t lda, const uint8_t* __restrict__ B, int64_t ldb,
           float* __restrict__ C, int64_t ldc, int M, int N, int K)
{
    using T = B32Tile<MODE, BM, BN, BK, WGM, WGN, KR>;
    constexpr int THREADS = T::THREADS, PARTS = T::PARTS, KB = T::KB, ROW = T::ROW;
    constexpr int FM = T::FM, FN = T::FN;
    // [stage][A hi, (A lo), B hi, (B lo)]
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][T::STAGE];

    const int ntm = M / BM, ntn = N / BN;
    int tm, tn;
    gemm_tile_coords(ntm, ntn, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x, lane = t % 64, wid = t / 64;
    const int wm = wid / WGN, wn = wid % WGN;

    uint32_t ra[T::A_N][T::A_DW];
    uint32_t rb[T::B_G][KR][T::B_DW];

    auto a_tile = [&](int s, int part) { return lds[s] + part * T::A_TILE; };
    auto b_tile = [&](int s, int part) { return lds[s] + PARTS * T::A_TILE + part * T::B_TILE; };

    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int i = 0; i < T::A_N; ++i) {
            const int c = t + THREADS * i, row = c / T::A_CPR, kc = c % T::A_CPR;
            load_dwords(reinterpret_cast<const uint32_t*>(A + ((int64_t)(m0 + row) * lda + k0 + kc * T::A_EL) * KB),
                        ra[i]);
        }
#pragma unroll
        for (int g = 0; g < T::B_G; ++g) {
            const int gi = t + THREADS * g, np = gi % T::B_GPR, kg = gi / T::B_GPR;
#pragma unroll
            for (int r = 0; r < KR; ++r)
                load_dwords(reinterpret_cast<const uint32_t*>(
                                B + ((int64_t)(k0 + kg * KR + r) * ldb + n0 + T::BCOL * np) * KB),
                            rb[g][r]);
        }
    };

    auto store_tiles = [&](int s) {
        uint16_t* Ah = a_tile(s, 0);
        uint16_t* Bh = b_tile(s, 0);
#pragma unroll
        for (int i = 0; i < T::A_N; ++i) {
            const int c = t + THREADS * i, row = c / T::A_CPR, kc = c % T::A_CPR;
            if constexpr (MODE == 0) {
                *reinterpret_cast<u32x4_t*>(Ah + row * ROW + kc * 8) = u32x4_t{ra[i][0], ra[i][1], ra[i][2], ra[i][3]};
            } else {
                using F = Fmt<32, 3>;
                uint16_t* Al = a_tile(s, 1);
                uint32_t x[16];
                unpack_elems<F, 16>(ra[i], x);
                uint32_t hi[8], lo[8];
#pragma unroll
                for (int e = 0; e < 16; e += 2) {
                    uint32_t h0, l0, h1, l1;
                    split_hi_lo(x[e], h0, l0);
                    split_hi_lo(x[e + 1], h1, l1);
                    hi[e / 2] = h0 | (h1 << 16);
                    lo[e / 2] = l0 | (l1 << 16);
                }
                u32x4_t* dh = reinterpret_cast<u32x4_t*>(Ah + row * ROW + kc * 16);
                u32x4_t* dl = reinterpret_cast<u32x4_t*>(Al + row * ROW + kc * 16);
                dh[0] = u32x4_t{hi[0], hi[1], hi[2], hi[3]};
                dh[1] = u32x4_t{hi[4], hi[5], hi[6], hi[7]};
                dl[0] = u32x4_t{lo[0], lo[1], lo[2], lo[3]};
                dl[1] = u32x4_t{lo[4], lo[5], lo[6], lo[7]};
            }
        }
#pragma unroll
        for (int g = 0; g < T::B_G; ++g) {
            const int gi = t + THREADS * g, np = gi % T::B_GPR, kg = gi / T::B_GPR;
            if constexpr (MODE == 0) {
                // row r holds columns (2np, 2np+1) as low/high halves: transpose to k-contiguous columns
                uint32_t c0[KR / 2], c1[KR / 2];
#pragma unroll
                for (int i = 0; i < KR / 2; ++i) {
                    c0[i] = __builtin_amdgcn_perm(rb[g][2 * i + 1][0], rb[g][2 * i][0], 0x05040100u);
                    c1[i] = __builtin_amdgcn_perm(rb[g][2 * i + 1][0], rb[g][2 * i][0], 0x07060302u);
                }
                store_row_chunk<KR>(Bh + (2 * np) * ROW + kg * KR, c0);
                store_row_chunk<KR>(Bh + (2 * np + 1) * ROW + kg * KR, c1);
            } else {
                using F = Fmt<32, 3>;
                uint16_t* Bl = b_tile(s, 1);
                uint32_t hi[KR][4], lo[KR][4];   // [row][column]
#pragma unroll
                for (int r = 0; r < KR; ++r) {
                    uint32_t x[4];
                    unpack_elems<F, 4>(rb[g][r], x);
#pragma unroll
                    for (int c = 0; c < 4; ++c) split_hi_lo(x[c], hi[r][c], lo[r][c]);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint32_t vh[KR / 2], vl[KR / 2];
#pragma unroll
                    for (int i = 0; i < KR / 2; ++i) {
                        vh[i] = hi[2 * i][c] | (hi[2 * i + 1][c] << 16);
                        vl[i] = lo[2 * i][c] | (lo[2 * i + 1][c] << 16);
                    }
                    store_row_chunk<KR>(Bh + (4 * np + c) * ROW + kg * KR, vh);
                    store_row_chunk<KR>(Bl + (4 * np + c) * ROW + kg * KR, vl);
                }
            }
        }
    };

    f32x4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int s) {
        const uint16_t* Ah = a_tile(s, 0);
        const uint16_t* Bh = b_tile(s, 0);
        const int r16 = lane % 16, kq = 8 * (lane / 16);
#pragma unroll
        for (int ks = 0; ks < BK / 32; ++ks) {
            bf16x8_t a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = *reinterpret_cast<const bf16x8_t*>(Ah + (wm * T::TM + i * 16 + r16) * ROW + ks * 32 + kq);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[j] = *reinterpret_cast<const bf16x8_t*>(Bh + (wn * T::TN + j * 16 + r16) * ROW + ks * 32 + kq);
            if constexpr (MODE == 0) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            } else {
                const uint16_t* Al = a_tile(s, 1);
                const uint16_t* Bl = b_tile(s, 1);
                bf16x8_t al[FM], bl[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    al[i] = *reinterpret_cast<const bf16x8_t*>(Al + (wm * T::TM + i * 16 + r16) * ROW + ks * 32 + kq);
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    bl[j] = *reinterpret_cast<const bf16x8_t*>(Bl + (wn * T::TN + j * 16 + r16) * ROW + ks * 32 + kq);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bl[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], b[j], acc[i][j], 0, 0, 0);
                        if constexpr (MODE == 2)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bl[j], acc[i][j], 0, 0, 0);
                    }
            }
        }
    };

    // the last K step is peeled so the loop body has no branches
    const int KT = K / BK;
    load_tiles(0);
    store_tiles(0);
    __syncthreads();
    for (int kt = 0; kt < KT - 1; ++kt) {
        const int s = kt & 1;
        load_tiles((kt + 1) * BK);
        compute(s);
        store_tiles(s ^ 1);
        __syncthreads();
    }
    compute((KT - 1) & 1);

    // ---- epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * T::TM + i * 16 + 4 * (lane / 16) + r;
                const int col = n0 + wn * T::TN + j * 16 + lane % 16;
                C[(int64_t)row * ldc + col] = acc[i][j][r];
            }
}

template <int MODE, int BM, int BN, int BK, int WGM, int WGN, int KR>
static void launch_b32(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                       int64_t ldc, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((M / BM) * (N / BN));
    k_gemm_b32<MODE, BM, BN, BK, WGM, WGN, KR><<<blocks, 64 * WGM * WGN, 0, stream>>>(
        static_cast<const uint8_t*>(A), lda, static_cast<const uint8_t*>(B), ldb, static_cast<float*>(C), ldc, (int)M,
        (int)N, (int)K);
}

fb_status gemm_bf16_launch(int mode, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                           int64_t ldb, void* C, int64_t ldc, hipStream_t stream)
{
    if (M % 128 || N % 128 || K % 64)
        return set_error(FB_ERR_UNSUPPORTED, "fb_gemm: binary32 paths need M, N multiples of 128 and K of 64");
    if (M == 0 || N == 0) return FB_OK;
    if ((M / 128) * (N / 128) > INT32_MAX || M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
        return set_error(FB_ERR_ARG, "fb_gemm: sizes too large");
    if (mode == 0) {
        if (M % 256 == 0 && N % 256 == 0)
            launch_b32<0, 256, 256, 64, 2, 4, 8>(M, N, K, A, lda, B, ldb, C, ldc, stream);
        else
            launch_b32<0, 128, 128, 64, 2, 2, 8>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    } else if (mode == 1) {
        if (M % 256 == 0)
            launch_b32<1, 256, 128, 32, 2, 2, 4>(M, N, K, A, lda, B, ldb, C, ldc, stream);
        else
            launch_b32<1, 128, 128, 64, 2, 2, 8>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    } else {
        if (M % 256 == 0)
            launch_b32<2, 256, 128, 32, 2, 2, 4>(M, N, K, A, lda, B, ldb, C, ldc, stream);
        else
            launch_b32<2, 128, 128, 64, 2, 2, 8>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    }
    return check_launch("fb_gemm");
}

}  // namespace flyte
