// GEMMs on binary32-derived operands with BF16 matrix cores (gfx950).
//
// C = A B, A M x K and B K x N row-major packed, C FP32 row-major.
//  MODE 0 ({32,2}): the stored 2-byte patterns are bfloat16 operands as they
//    are (the 16-bit flyte of Table 1 is bit-for-bit bfloat16).
//  MODE 1 ({32,3}): each 3-byte element, unpacked to binary32 x, is split into
//    hi = x with its low 16 bits cleared (a bfloat16) and lo = x - hi (exact
//    in binary32, and exactly a bfloat16 for biased exponent >= 9; rounded to
//    nearest otherwise; 0 for Inf/NaN).  The tile product is hi*hi + hi*lo +
//    lo*hi: three BF16 MFMAs per step into the same FP32 accumulators (lo*lo,
//    below 2^-16 relative, is dropped).
//  MODE 2 ({32,3}, four products): MODE 1 plus lo*lo, so every product of the
//    split operands is formed exactly and only the FP32 accumulation rounds.
//
// The split is done once per element by a streaming pass before the GEMM (A
// into row-major hi/lo planes, B into n-major planes, transposed through LDS),
// in the per-stream workspace; the GEMM loader then copies plane tiles to LDS
// as they are.  Splitting inside the GEMM loader would repeat the split for
// every tile of C that reads the element (N/BN times for A, M/BM for B), which
// makes the split, not the matrix cores, the bound.
//
// Tiling: a workgroup computes a BM x BN tile of C with WGM x WGN waves, each
// wave a (BM/WGM) x (BN/WGN) tile of v_mfma_f32_16x16x32_bf16 results.  Large
// wave tiles keep LDS operand traffic below the LDS bandwidth (a 64 x 128 or
// 128 x 64 wave tile reads about 94 B/clk of LDS per CU at the MFMA peak,
// against 128 available).  8 waves per workgroup, two per SIMD: BF16 in
// 256 x 256 x 64 tiles as 4 x 2 waves of 64 x 128 (144 KiB of LDS), the split
// products in 256 x 256 x 32 tiles as 2 x 4 waves of 128 x 64 (their two
// planes fill the 160 KiB of LDS exactly; the short K step keeps registers
// for two waves per SIMD).  Shapes that are not multiples of 256 use 256 x 128
// x 32 (split products, M a multiple of 256) or 128 x 128 x 64.  K is
// walked in BK steps through double-buffered LDS (one barrier per step; the
// next step's global loads are issued before the current step's MFMAs; the
// last step is peeled).  LDS rows are padded by 16 bytes, so the 16-byte
// operand reads of 16 lanes hit distinct banks.  B is stored in LDS n-major
// (k contiguous): for BF16 each thread loads KR rows of B and transposes them
// in registers with v_perm_b32; the split planes of B are already n-major.
// Every MFMA operand is one ds_read_b128.  Workgroups are renumbered so that
// consecutive tiles of C run on the same XCD (sharing its L2), grouped 8
// tile-rows at a time.
#include <algorithm>

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

// hi/lo split of a binary32 pattern (MODE 1).  A NaN whose payload lies only
// in the bits below hi would leave hi with a zero mantissa, an infinity, so
// hi gets the quiet bit for every NaN: NaN stays NaN.
__device__ __forceinline__ void split_hi_lo(uint32_t u, uint32_t& hi, uint32_t& lo)
{
    hi = u >> 16;
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) hi |= 0x40u;
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
    static constexpr int ROW = BK + 8;                  // bf16 per padded LDS row
    static constexpr int A_TILE = BM * ROW, B_TILE = BN * ROW;
    static constexpr int STAGE = PARTS * (A_TILE + B_TILE);
    // A (and the B planes): chunks of 8 consecutive bf16 of a row (16 bytes)
    static constexpr int CPR = BK / 8;
    static constexpr int A_N = BM * CPR / THREADS;
    static constexpr int BT_N = BN * CPR / THREADS;
    // MODE 0 B: groups of KR k-rows x 2 columns (one dword per row)
    static constexpr int B_GPR = BN / 2;
    static constexpr int B_G = (BK / KR) * B_GPR / THREADS;
    static_assert(BK % 32 == 0 && TM % 16 == 0 && TN % 16 == 0, "tile shape");
    static_assert(A_N * THREADS == BM * CPR && A_N >= 1, "A staging must divide evenly");
    static_assert(MODE == 0 || (BT_N * THREADS == BN * CPR && BT_N >= 1), "B plane staging must divide evenly");
    static_assert(MODE != 0 || (B_G * THREADS == (BK / KR) * B_GPR && B_G >= 1), "B staging must divide evenly");
    static_assert(KR == 4 || KR == 8, "B group rows");
};

template <int MODE, int BM, int BN, int BK, int WGM, int WGN, int KR>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm_b32(const uint8_t* __restrict__ A, int64_t lda, const uint8_t* __restrict__ B, int64_t ldb,
           float* __restrict__ C, int64_t ldc, int M, int N, int K)
{
    // MODE 0: A and B are the packed {32,2} matrices (bfloat16 patterns).
    // MODE 1, 2: A = hi and lo planes [2][M][lda] of bfloat16; B = hi and lo
    // planes [2][N][ldb] of B transposed (n-major).
    using T = B32Tile<MODE, BM, BN, BK, WGM, WGN, KR>;
    // The split products hold hi and lo fragments of both operands; an (empty)
    // statement that clobbers an accumulation register makes the compiler keep
    // the MFMA accumulators in AGPRs, which leaves the fragments room in the
    // VGPRs (no spills at two waves per SIMD).
    if constexpr (MODE != 0) asm volatile("; accumulators in AGPRs" ::: "a0");
    constexpr int THREADS = T::THREADS, PARTS = T::PARTS, ROW = T::ROW;
    constexpr int FM = T::FM, FN = T::FN;
    // [stage][A hi, (A lo), B hi, (B lo)]
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][T::STAGE];

    const int ntm = M / BM, ntn = N / BN;
    int tm, tn;
    gemm_tile_coords(ntm, ntn, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x, lane = t % 64, wid = t / 64;
    const int wm = wid / WGN, wn = wid % WGN;
    const int64_t a_plane = (int64_t)M * lda * 2, b_plane = (int64_t)N * ldb * 2;   // bytes

    uint32_t ra[PARTS][T::A_N][4];
    constexpr int RB_N = MODE ? T::BT_N : 1;
    uint32_t rbt[PARTS][RB_N][4];
    constexpr int RB_G = MODE ? 1 : T::B_G;
    uint32_t rb[RB_G][KR];

    auto a_tile = [&](int s, int part) { return lds[s] + part * T::A_TILE; };
    auto b_tile = [&](int s, int part) { return lds[s] + PARTS * T::A_TILE + part * T::B_TILE; };

    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PARTS; ++p)
#pragma unroll
            for (int i = 0; i < T::A_N; ++i) {
                const int c = t + THREADS * i, row = c / T::CPR, kc = c % T::CPR;
                load_dwords(reinterpret_cast<const uint32_t*>(A + p * a_plane + ((int64_t)(m0 + row) * lda + k0 + kc * 8) * 2),
                            ra[p][i]);
            }
        if constexpr (MODE == 0) {
#pragma unroll
            for (int g = 0; g < T::B_G; ++g) {
                const int gi = t + THREADS * g, np = gi % T::B_GPR, kg = gi / T::B_GPR;
#pragma unroll
                for (int r = 0; r < KR; ++r)
                    rb[g][r] = *reinterpret_cast<const uint32_t*>(B + ((int64_t)(k0 + kg * KR + r) * ldb + n0 + 2 * np) * 2);
            }
        } else {
#pragma unroll
            for (int p = 0; p < PARTS; ++p)
#pragma unroll
                for (int i = 0; i < T::BT_N; ++i) {
                    const int c = t + THREADS * i, row = c / T::CPR, kc = c % T::CPR;
                    load_dwords(reinterpret_cast<const uint32_t*>(B + p * b_plane +
                                                                  ((int64_t)(n0 + row) * ldb + k0 + kc * 8) * 2),
                                rbt[p][i]);
                }
        }
    };

    auto store_tiles = [&](int s) {
#pragma unroll
        for (int p = 0; p < PARTS; ++p)
#pragma unroll
            for (int i = 0; i < T::A_N; ++i) {
                const int c = t + THREADS * i, row = c / T::CPR, kc = c % T::CPR;
                *reinterpret_cast<u32x4_t*>(a_tile(s, p) + row * ROW + kc * 8) =
                    u32x4_t{ra[p][i][0], ra[p][i][1], ra[p][i][2], ra[p][i][3]};
            }
        if constexpr (MODE == 0) {
            uint16_t* Bh = b_tile(s, 0);
#pragma unroll
            for (int g = 0; g < T::B_G; ++g) {
                const int gi = t + THREADS * g, np = gi % T::B_GPR, kg = gi / T::B_GPR;
                // row r holds columns (2np, 2np+1) as low/high halves: transpose to k-contiguous columns
                uint32_t c0[KR / 2], c1[KR / 2];
#pragma unroll
                for (int i = 0; i < KR / 2; ++i) {
                    c0[i] = __builtin_amdgcn_perm(rb[g][2 * i + 1], rb[g][2 * i], 0x05040100u);
                    c1[i] = __builtin_amdgcn_perm(rb[g][2 * i + 1], rb[g][2 * i], 0x07060302u);
                }
                store_row_chunk<KR>(Bh + (2 * np) * ROW + kg * KR, c0);
                store_row_chunk<KR>(Bh + (2 * np + 1) * ROW + kg * KR, c1);
            }
        } else {
#pragma unroll
            for (int p = 0; p < PARTS; ++p)
#pragma unroll
                for (int i = 0; i < T::BT_N; ++i) {
                    const int c = t + THREADS * i, row = c / T::CPR, kc = c % T::CPR;
                    *reinterpret_cast<u32x4_t*>(b_tile(s, p) + row * ROW + kc * 8) =
                        u32x4_t{rbt[p][i][0], rbt[p][i][1], rbt[p][i][2], rbt[p][i][3]};
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
        if constexpr (MODE == 0) {
            // One read-ahead pipeline over the K sub-steps of the stage: each B
            // fragment is read one column block ahead of the MFMAs that use it
            // (the last block reads the next sub-step's first B fragment), and
            // the next sub-step's A fragments are read halfway through the
            // current one, so the wave waits for at most one LDS read before an
            // MFMA group.  The group barriers keep the compiler to this order.
            // The wave raises its issue priority for the block, so the other
            // wave on the SIMD does its staging while this one feeds the
            // matrix core.
            constexpr int KSN = BK / 32, JA = FN / 2;
            auto read_a = [&](int ks, int i) {
                return *reinterpret_cast<const bf16x8_t*>(Ah + (wm * T::TM + i * 16 + r16) * ROW + ks * 32 + kq);
            };
            auto read_b = [&](int ks, int j) {
                return *reinterpret_cast<const bf16x8_t*>(Bh + (wn * T::TN + j * 16 + r16) * ROW + ks * 32 + kq);
            };
            bf16x8_t a[2][FM], b[FN];
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int i = 0; i < FM; ++i) a[0][i] = read_a(0, i);
            b[0] = read_b(0, 0);
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks) {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if (j + 1 < FN) b[j + 1] = read_b(ks, j + 1);
                    else if (ks + 1 < KSN) b[0] = read_b(ks + 1, 0);
                    if (j == JA && ks + 1 < KSN) {
#pragma unroll
                        for (int i = 0; i < FM; ++i) a[(ks + 1) & 1][i] = read_a(ks + 1, i);
                    }
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks & 1][i], b[j], acc[i][j], 0, 0, 0);
                }
            }
            __builtin_amdgcn_sched_group_barrier(0x100, FM + 1, 0);   // LDS reads
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks) {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if (ks < KSN - 1 || j < FN - 1) {
                        if (j == JA && ks + 1 < KSN) __builtin_amdgcn_sched_group_barrier(0x100, 1 + FM, 0);
                        else __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                    }
                    __builtin_amdgcn_sched_group_barrier(0x008, FM, 0);   // MFMAs
                }
            }
            __builtin_amdgcn_s_setprio(0);
        } else {
            const uint16_t* Al = a_tile(s, 1);
            const uint16_t* Bl = b_tile(s, 1);
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int ks = 0; ks < BK / 32; ++ks) {
                bf16x8_t a[FM], b[FN], al[FM], bl[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    a[i] = *reinterpret_cast<const bf16x8_t*>(Ah + (wm * T::TM + i * 16 + r16) * ROW + ks * 32 + kq);
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[j] = *reinterpret_cast<const bf16x8_t*>(Bh + (wn * T::TN + j * 16 + r16) * ROW + ks * 32 + kq);
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
            __builtin_amdgcn_s_setprio(0);
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
        // keep the next step's global loads ahead of this step's MFMAs, so
        // their latency is covered by the whole step
        __builtin_amdgcn_sched_barrier(0);
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

// Split pass for A ({32,3}, rows x cols, leading dimension ld elements): hi and
// lo planes of bfloat16, row-major with leading dimension cols.  One lane per
// 4-element unit (12 bytes in, 8 + 8 bytes out).
__global__ void __launch_bounds__(256)
k_split_rows(const uint8_t* __restrict__ src, int64_t ld, int64_t rows, int64_t cols, uint16_t* __restrict__ hi,
             uint16_t* __restrict__ lo)
{
    using F = Fmt<32, 3>;
    const int64_t upr = cols / 4, total = rows * upr;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = q / upr, c4 = q % upr;
        uint32_t P[3];
        load_dwords(reinterpret_cast<const uint32_t*>(src + (row * ld + c4 * 4) * 3), P);
        uint32_t x[4], h[4], l[4];
        unpack_elems<F, 4>(P, x);
#pragma unroll
        for (int c = 0; c < 4; ++c) split_hi_lo(x[c], h[c], l[c]);
        const int64_t o = row * cols + c4 * 4;
        uint32_t hv[2] = {h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
        uint32_t lv[2] = {l[0] | (l[1] << 16), l[2] | (l[3] << 16)};
        store_dwords(reinterpret_cast<uint32_t*>(hi + o), hv);
        store_dwords(reinterpret_cast<uint32_t*>(lo + o), lv);
    }
}

// Split pass for B ({32,3}, rows x cols, leading dimension ld elements) into
// hi and lo planes of B transposed (cols x rows, leading dimension rows), 64 x
// 64 tiles through LDS (blockIdx.x: tile row, blockIdx.y: tile column): a lane
// reads 4-element units of a row and writes the split halves down LDS columns;
// then 16-byte chunks of the transposed rows go out.  rows and cols are
// multiples of 64.
__global__ void __launch_bounds__(256)
k_split_cols_t(const uint8_t* __restrict__ src, int64_t ld, int64_t rows, int64_t cols, uint16_t* __restrict__ hi,
               uint16_t* __restrict__ lo)
{
    using F = Fmt<32, 3>;
    constexpr int TP = 64 + 8;   // padded LDS row (bf16)
    __shared__ __attribute__((aligned(16))) uint16_t tile[2][64][TP];   // [plane][col][row]
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int u = t + 256 * i, r = u / 16, cu = u % 16;
        uint32_t P[3];
        load_dwords(reinterpret_cast<const uint32_t*>(src + ((r0 + r) * ld + c0 + cu * 4) * 3), P);
        uint32_t x[4];
        unpack_elems<F, 4>(P, x);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint32_t h, l;
            split_hi_lo(x[c], h, l);
            tile[0][cu * 4 + c][r] = (uint16_t)h;
            tile[1][cu * 4 + c][r] = (uint16_t)l;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = t + 256 * i, p = idx / 512, c = (idx % 512) / 8, ch = idx % 8;
        const u32x4_t v = *reinterpret_cast<const u32x4_t*>(&tile[p][c][ch * 8]);
        uint16_t* dst = (p ? lo : hi) + (c0 + c) * rows + r0 + ch * 8;
        *reinterpret_cast<u32x4_t*>(dst) = v;
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
    if (mode != 0 && N / 64 > 65535)   // grid.y of the split pass of B
        return set_error(FB_ERR_UNSUPPORTED, "fb_gemm: {32,3} operands need N <= %d", 65535 * 64);
    if (mode == 0) {
        if (M % 256 == 0 && N % 256 == 0)
            launch_b32<0, 256, 256, 64, 4, 2, 8>(M, N, K, A, lda, B, ldb, C, ldc, stream);
        else
            launch_b32<0, 128, 128, 64, 2, 2, 8>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    } else {
        // split both operands once into bfloat16 planes in the stream workspace
        void* ws = nullptr;
        const size_t bytes = (size_t)(M * K + N * K) * 4;
        fb_status st = stream_workspace(stream, bytes, &ws);
        if (st != FB_OK) return st;
        uint16_t* ap = static_cast<uint16_t*>(ws);
        uint16_t* bp = ap + 2 * M * K;
        const int64_t units = M * (K / 4);
        const unsigned sblocks = (unsigned)std::min<int64_t>((units + 255) / 256, 8192);
        k_split_rows<<<sblocks, 256, 0, stream>>>(static_cast<const uint8_t*>(A), lda, M, K, ap, ap + M * K);
        k_split_cols_t<<<dim3((unsigned)(K / 64), (unsigned)(N / 64)), 256, 0, stream>>>(
            static_cast<const uint8_t*>(B), ldb, K, N, bp, bp + N * K);
        if (mode == 1) {
            if (M % 256 == 0 && N % 256 == 0)
                launch_b32<1, 256, 256, 32, 2, 4, 4>(M, N, K, ap, K, bp, K, C, ldc, stream);
            else if (M % 256 == 0)
                launch_b32<1, 256, 128, 32, 2, 2, 4>(M, N, K, ap, K, bp, K, C, ldc, stream);
            else
                launch_b32<1, 128, 128, 64, 2, 2, 8>(M, N, K, ap, K, bp, K, C, ldc, stream);
        } else {
            if (M % 256 == 0 && N % 256 == 0)
                launch_b32<2, 256, 256, 32, 2, 4, 4>(M, N, K, ap, K, bp, K, C, ldc, stream);
            else if (M % 256 == 0)
                launch_b32<2, 256, 128, 32, 2, 2, 4>(M, N, K, ap, K, bp, K, C, ldc, stream);
            else
                launch_b32<2, 128, 128, 64, 2, 2, 8>(M, N, K, ap, K, bp, K, C, ldc, stream);
        }
    }
    return check_launch("fb_gemm");
}

}  // namespace flyte
