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
//
// Tiling: a 256-thread workgroup computes a 128 x 128 tile of C; each of its
// 4 waves a 64 x 64 quarter as 4 x 4 v_mfma_f32_16x16x32_bf16 tiles.  K is
// walked in steps of 64 through double-buffered LDS (one barrier per step;
// the next step's global loads are issued before the current step's MFMAs).
// LDS rows are padded to 144 bytes, so the 16-byte operand reads of 16 lanes
// hit distinct banks.  B is stored in LDS transposed (n-major, k contiguous):
// each thread loads 8 rows of B and transposes them in registers with
// v_perm_b32, so every MFMA operand is one ds_read_b128.  Workgroups are
// renumbered so that consecutive tiles of C run on the same XCD (sharing its
// L2), grouped 8 tile-rows at a time.
#include "codec.hpp"
#include "common.hpp"

namespace flyte {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int GB_BM = 128, GB_BN = 128, GB_BK = 64, GB_THREADS = 256;
constexpr int GB_LDS_ROW = GB_BK + 8;                 // bf16 per padded LDS row (144 bytes)
constexpr int GB_TILE = GB_BM * GB_LDS_ROW;           // bf16 per operand tile

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

template <int MODE>
struct GemmStage {
    static constexpr int PARTS = MODE ? 2 : 1;
};

template <int MODE>
__global__ void __launch_bounds__(GB_THREADS)
k_gemm_bf16(const uint8_t* __restrict__ A, int64_t lda, const uint8_t* __restrict__ B, int64_t ldb,
            float* __restrict__ C, int64_t ldc, int M, int N, int K)
{
    constexpr int PARTS = GemmStage<MODE>::PARTS;
    constexpr int KB = MODE ? 3 : 2;   // stored bytes per element
    // [stage][A parts..., B parts...][tile]
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][2 * PARTS][GB_TILE];

    const int ntm = M / GB_BM, ntn = N / GB_BN;
    int tm, tn;
    gemm_tile_coords(ntm, ntn, tm, tn);
    const int m0 = tm * GB_BM, n0 = tn * GB_BN;
    const int t = threadIdx.x, lane = t % 64, wid = t / 64;
    const int wm = wid / 2, wn = wid % 2;

    // ---- global -> register staging
    // A: MODE 0: 4 chunks of 8 elements (16 B) per thread; MODE 1: 2 units of 16 elements (48 B).
    constexpr int A_N = MODE ? 2 : 4;
    constexpr int A_DW = MODE ? 12 : 4;
    uint32_t ra[A_N][A_DW];
    // B: MODE 0: 2 groups of 8 rows x 2 columns (one dword per row); MODE 1: 1 group of 8 rows x 4 columns (3 dwords per row).
    constexpr int B_G = MODE ? 1 : 2;
    constexpr int B_DW = MODE ? 3 : 1;
    uint32_t rb[B_G][8][B_DW];

    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int i = 0; i < A_N; ++i) {
            if constexpr (MODE == 0) {
                const int c = t + GB_THREADS * i, row = c / 8, kc = c % 8;
                const uint32_t* p = reinterpret_cast<const uint32_t*>(A + ((int64_t)(m0 + row) * lda + k0 + kc * 8) * KB);
                load_dwords(p, ra[i]);
            } else {
                const int u = t + GB_THREADS * i, row = u / 4, uc = u % 4;
                const uint32_t* p = reinterpret_cast<const uint32_t*>(A + ((int64_t)(m0 + row) * lda + k0 + uc * 16) * KB);
                load_dwords(p, ra[i]);
            }
        }
#pragma unroll
        for (int g = 0; g < B_G; ++g) {
            if constexpr (MODE == 0) {
                const int np = t % 64, kg = t / 64 + 4 * g;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const uint32_t* p = reinterpret_cast<const uint32_t*>(
                        B + ((int64_t)(k0 + kg * 8 + r) * ldb + n0 + 2 * np) * KB);
                    rb[g][r][0] = *p;
                }
            } else {
                const int ng = t % 32, kg = t / 32;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const uint32_t* p = reinterpret_cast<const uint32_t*>(
                        B + ((int64_t)(k0 + kg * 8 + r) * ldb + n0 + 4 * ng) * KB);
                    load_dwords(p, rb[g][r]);
                }
            }
        }
    };

    auto store_tiles = [&](int s) {
        uint16_t* As_hi = lds[s][0];
        uint16_t* Bs_hi = lds[s][PARTS];
#pragma unroll
        for (int i = 0; i < A_N; ++i) {
            if constexpr (MODE == 0) {
                const int c = t + GB_THREADS * i, row = c / 8, kc = c % 8;
                *reinterpret_cast<u32x4_t*>(As_hi + row * GB_LDS_ROW + kc * 8) =
                    u32x4_t{ra[i][0], ra[i][1], ra[i][2], ra[i][3]};
            } else {
                using F = Fmt<32, 3>;
                uint16_t* As_lo = lds[s][1];
                const int u = t + GB_THREADS * i, row = u / 4, uc = u % 4;
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
                u32x4_t* dh = reinterpret_cast<u32x4_t*>(As_hi + row * GB_LDS_ROW + uc * 16);
                u32x4_t* dl = reinterpret_cast<u32x4_t*>(As_lo + row * GB_LDS_ROW + uc * 16);
                dh[0] = u32x4_t{hi[0], hi[1], hi[2], hi[3]};
                dh[1] = u32x4_t{hi[4], hi[5], hi[6], hi[7]};
                dl[0] = u32x4_t{lo[0], lo[1], lo[2], lo[3]};
                dl[1] = u32x4_t{lo[4], lo[5], lo[6], lo[7]};
            }
        }
#pragma unroll
        for (int g = 0; g < B_G; ++g) {
            if constexpr (MODE == 0) {
                const int np = t % 64, kg = t / 64 + 4 * g;
                uint32_t c0[4], c1[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // low halves (column 2np) and high halves (column 2np+1) of rows 2i, 2i+1
                    c0[i] = __builtin_amdgcn_perm(rb[g][2 * i + 1][0], rb[g][2 * i][0], 0x05040100u);
                    c1[i] = __builtin_amdgcn_perm(rb[g][2 * i + 1][0], rb[g][2 * i][0], 0x07060302u);
                }
                *reinterpret_cast<u32x4_t*>(Bs_hi + (2 * np) * GB_LDS_ROW + kg * 8) = u32x4_t{c0[0], c0[1], c0[2], c0[3]};
                *reinterpret_cast<u32x4_t*>(Bs_hi + (2 * np + 1) * GB_LDS_ROW + kg * 8) = u32x4_t{c1[0], c1[1], c1[2], c1[3]};
            } else {
                using F = Fmt<32, 3>;
                uint16_t* Bs_lo = lds[s][3];
                const int ng = t % 32, kg = t / 32;
                uint32_t hi[8][4], lo[8][4];   // [row][column]
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    uint32_t x[4];
                    unpack_elems<F, 4>(rb[g][r], x);
#pragma unroll
                    for (int c = 0; c < 4; ++c) split_hi_lo(x[c], hi[r][c], lo[r][c]);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    u32x4_t vh, vl;
                    vh.x = hi[0][c] | (hi[1][c] << 16); vh.y = hi[2][c] | (hi[3][c] << 16);
                    vh.z = hi[4][c] | (hi[5][c] << 16); vh.w = hi[6][c] | (hi[7][c] << 16);
                    vl.x = lo[0][c] | (lo[1][c] << 16); vl.y = lo[2][c] | (lo[3][c] << 16);
                    vl.z = lo[4][c] | (lo[5][c] << 16); vl.w = lo[6][c] | (lo[7][c] << 16);
                    *reinterpret_cast<u32x4_t*>(Bs_hi + (4 * ng + c) * GB_LDS_ROW + kg * 8) = vh;
                    *reinterpret_cast<u32x4_t*>(Bs_lo + (4 * ng + c) * GB_LDS_ROW + kg * 8) = vl;
                }
            }
        }
    };

    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int s) {
        const uint16_t* As_hi = lds[s][0];
        const uint16_t* Bs_hi = lds[s][PARTS];
        const int r16 = lane % 16, kq = 8 * (lane / 16);
#pragma unroll
        for (int ks = 0; ks < GB_BK / 32; ++ks) {
            bf16x8_t a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[i] = *reinterpret_cast<const bf16x8_t*>(As_hi + (wm * 64 + i * 16 + r16) * GB_LDS_ROW + ks * 32 + kq);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = *reinterpret_cast<const bf16x8_t*>(Bs_hi + (wn * 64 + j * 16 + r16) * GB_LDS_ROW + ks * 32 + kq);
            if constexpr (MODE == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            } else {
                const uint16_t* As_lo = lds[s][1];
                const uint16_t* Bs_lo = lds[s][3];
                bf16x8_t al[4], bl[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    al[i] = *reinterpret_cast<const bf16x8_t*>(As_lo + (wm * 64 + i * 16 + r16) * GB_LDS_ROW + ks * 32 + kq);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bl[j] = *reinterpret_cast<const bf16x8_t*>(Bs_lo + (wn * 64 + j * 16 + r16) * GB_LDS_ROW + ks * 32 + kq);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bl[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], b[j], acc[i][j], 0, 0, 0);
                    }
            }
        }
    };

    // the last K step is peeled so the loop body has no branches
    const int KT = K / GB_BK;
    load_tiles(0);
    store_tiles(0);
    __syncthreads();
    for (int kt = 0; kt < KT - 1; ++kt) {
        const int s = kt & 1;
        load_tiles((kt + 1) * GB_BK);
        compute(s);
        store_tiles(s ^ 1);
        __syncthreads();
    }
    compute((KT - 1) & 1);

    // ---- epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + i * 16 + 4 * (lane / 16) + r;
                const int col = n0 + wn * 64 + j * 16 + lane % 16;
                C[(int64_t)row * ldc + col] = acc[i][j][r];
            }
}

fb_status gemm_bf16_launch(int mode, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                           int64_t ldb, void* C, int64_t ldc, hipStream_t stream)
{
    if (M % GB_BM || N % GB_BN || K % GB_BK)
        return set_error(FB_ERR_UNSUPPORTED, "fb_gemm: binary32 paths need M, N multiples of %d and K of %d", GB_BM,
                         GB_BK);
    if (M == 0 || N == 0) return FB_OK;
    const int64_t blocks = (M / GB_BM) * (N / GB_BN);
    if (blocks > INT32_MAX || M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
        return set_error(FB_ERR_ARG, "fb_gemm: sizes too large");
    if (mode == 0)
        k_gemm_bf16<0><<<(unsigned)blocks, GB_THREADS, 0, stream>>>(static_cast<const uint8_t*>(A), lda,
                                                                     static_cast<const uint8_t*>(B), ldb,
                                                                     static_cast<float*>(C), ldc, (int)M, (int)N, (int)K);
    else
        k_gemm_bf16<1><<<(unsigned)blocks, GB_THREADS, 0, stream>>>(static_cast<const uint8_t*>(A), lda,
                                                                     static_cast<const uint8_t*>(B), ldb,
                                                                     static_cast<float*>(C), ldc, (int)M, (int)N, (int)K);
    return check_launch("fb_gemm");
}

}  // namespace flyte
