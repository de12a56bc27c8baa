// GEMMs whose operands are split into bfloat16 pieces while they are staged
// into LDS, on BF16 matrix cores with FP32 accumulation.
//
// The loader reads the packed k-byte elements as they are stored (4 elements,
// k dwords, per load), turns each element into P bfloat16 pieces whose sum is
// the element (or, for the default split products, its value to the stated
// precision), and writes piece planes to LDS; the MFMA loop then forms the
// products of pieces that the product set names, all into the same FP32
// accumulators (Section 3.1: compute in the next type that holds the data;
// Section 4.3: conversion is part of the load).
//
//  {32,3}: hi = the top two bytes (a NaN gets the quiet bit, so it stays
//    NaN), lo = x - hi rounded to bfloat16 (exact for biased exponent >= 9;
//    0 for Inf/NaN).  Products hi*hi + hi*lo + lo*hi, or all four.
//  {64,2}, {64,3}, {64,4} (5, 13 and 21 significant bits): the 11-bit
//    exponent does not fit a bfloat16, so every row i of A and column j of B
//    is scaled by an exact power of two, 2^-(e_i - 1023) and 2^-(e_j - 1023)
//    with e the largest biased exponent in it, so its largest element lies in
//    [1, 2); the scaled element is an exact binary32 value, cut into 1, 2 or 3
//    bfloat16 pieces of 8, 8 and 5 bits (exact).  C_ij = 2^(e_i - 1023 + e_j -
//    1023) * acc_ij in FP64, then cut to the output format.  A pass before the GEMM finds e_i, e_j and the rows and
//    columns that cannot be scaled exactly (an element more than 2^40 below
//    the largest, a binary64 subnormal, Inf or NaN); every 128 x 128 tile of C
//    in a 128-row band of A or 128-column band of B holding such a row or
//    column is recomputed by the FP64 matrix-core GEMM, which runs after this
//    one on exactly those tiles.
//
// Tiling: BM x BN x 32 per workgroup, WGM x WGN waves each (BM/WGM) x
// (BN/WGN) of v_mfma_f32_16x16x32_bf16 tiles; double-buffered LDS, one
// barrier per K step, the next step's global loads issued before the current
// step's MFMAs ({64,2}, one product per step: the loads of the step after next
// issued after a step's LDS stores, before its barrier).  A piece planes are m-major (k contiguous, unpadded; 16-byte
// chunk c of row R at c ^ ((R >> 2) & 3)), read with ds_read_b128.  Two B
// layouts, chosen by the loader (KMAJOR_B):
//  - k-major B (the binary64 pieces): B piece planes k-major as B is stored
//    (16-byte chunk c of k-row R at c ^ 2 g(R), g(R) = (R & 3) | ((R >> 1) &
//    4)), a thread forming the pairs of 4 columns of each of its 4 k-rows,
//    and each B operand read with two transposing LDS reads
//    (ds_read_b64_tr_b16).
//  - n-major B ({32,3}): B pairs formed down the group's 4 k-rows (so no
//    separate transposition), every operand one ds_read_b128.  Column n of
//    the tile goes to plane n % 4, row n / 4 (rows padded to 80 bytes, planes
//    64 bytes apart), so the 64 lanes of a store instruction (4 columns apart)
//    write consecutive rows.  The {32,3} loader needs more registers for its
//    special values, and there the k-major layout's extra address registers
//    cost spills (3-product 383 -> 295 TFLOP/s at 8192^3).
// The swizzles and the plane offset put the 16 lanes of a read phase (and the
// 8 k-rows of a transposing read phase) on distinct banks, and the 32 lanes of
// a store phase on 64 distinct banks.
// Shapes need not be tile multiples.  Rows past M load the last row; with N a
// multiple of 4, column groups past N load the last one (whole chunks),
// otherwise the column groups that reach past N load with bounds; a partial
// last K step, peeled out of the loop, loads with bounds (elements outside the
// matrix read as +0, and the bytes past a row's last element are never read).
// C is stored only inside the matrix.
#pragma once

#include "codec.hpp"
#include "common.hpp"
#include "gemm_pieces.hpp"

namespace flyte {

typedef __bf16 pc_bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 pc_bf16x2 __attribute__((ext_vector_type(2)));
typedef float pc_f32x4 __attribute__((ext_vector_type(4)));
typedef float pc_f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t pc_u32x2 __attribute__((ext_vector_type(2)));
typedef short pc_i16x4 __attribute__((ext_vector_type(4)));
typedef short pc_i16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) pc_i16x4 pc_lds_i16x4;

constexpr int PC_BK = 32;            // K per stage: one MFMA
constexpr int PC_ROW = PC_BK + 8;    // bfloat16 per padded LDS row (n-major layout)
constexpr int PC_PLANE_PAD = 32;     // bfloat16 between the four column planes of an n-major B tile
constexpr int PC_SPREAD = 40;        // largest exponent spread a scaled row or column may have

__host__ __device__ constexpr int pc_min(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int pc_max(int a, int b) { return a > b ? a : b; }

// bfloat16 pair from two binary32 values, rounded to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pc_cvt_pair(float a, float b)
{
    const pc_f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, pc_bf16x2));
}

// top halves of two binary32 patterns (the bfloat16 values they are, when exact)
__device__ __forceinline__ uint32_t pc_top_pair(uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_perm(b, a, 0x07060302u);
}

// ---------------------------------------------------------------- loaders
// A loader turns a chunk of 4 packed elements (KB dwords) into the binary32
// patterns x[e] of their (scaled) values, and says how piece p of such a
// value is formed: piece<p, SAFE>(x) is a binary32 pattern whose top half is
// piece p, and ROUND_P (when set) marks the one piece that is paired by
// rounding to nearest even (v_cvt_pk_bf16_f32) instead of taking top halves.
// SAFE selects the handling of infinities and NaNs (only the {32,3} loader
// has any); a wave takes the SAFE forms only when one of its elements of the
// K step is not finite.  shift[e] (scaled formats): (e_ref - 127) << 20 of
// the row or column of element e.

struct PcB32K3 {
    static constexpr int KB = 3, PIECES = 2, ROUND_P = 1;
    static constexpr bool SCALED = false, SPECIALS = true, KMAJOR_B = false, DWORD_PAIRS = false, EARLY_LOADS = false;
    __device__ static void values(const uint32_t (&d)[3], const int32_t (&)[4], uint32_t (&x)[4])
    {
        unpack_elems<Fmt<32, 3>, 4>(d, x);
    }
    // hi = the top two bytes (a NaN keeps its quiet bit set, so it stays NaN);
    // lo = x - hi (exact in binary32), 0 for Inf/NaN
    template <int PC, bool SAFE>
    __device__ static uint32_t piece(uint32_t u)
    {
        if constexpr (PC == 0) {
            if constexpr (SAFE) return ((u & 0x7FFFFFFFu) > 0x7F800000u) ? (u | 0x00400000u) : u;
            return u;
        } else {
            const float lo = __uint_as_float(u) - __uint_as_float(u & 0xFFFF0000u);
            if constexpr (SAFE) return ((u & 0x7F800000u) != 0x7F800000u) ? __float_as_uint(lo) : 0u;
            return __float_as_uint(lo);
        }
    }
};

// {64,K}, K = 2..4: the scaled binary32 value of each element, then P = K - 1
// pieces of it (8, 8 and 5 significant bits), all exact.
template <int K>
struct PcB64 {
    static constexpr int KB = K, PIECES = K - 1, ROUND_P = -1;
    // K = 2: a loaded dword is one bfloat16 pair (see pc_b64k2_pair), and with one product
    // per step the loads of the step after next are issued before each barrier
    static constexpr bool SCALED = true, SPECIALS = false, KMAJOR_B = true, DWORD_PAIRS = (K == 2),
                          EARLY_LOADS = (K == 2);
    __device__ static void values(const uint32_t (&d)[K], const int32_t (&shift)[4], uint32_t (&x)[4])
    {
        uint64_t u[4];
        unpack_elems<Fmt<64, K>, 4>(d, u);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // the element (its low word is zero for K <= 4) times 2^(1023 - e_ref), exact, then
            // to binary32, exact for a row that can be scaled (the scaled value lies in
            // [2^-40, 2) with at most 21 significant bits); zeros stay signed zeros
            const double v = __builtin_amdgcn_ldexp(__longlong_as_double((long long)u[e]), 896 - (shift[e] >> 20));
            x[e] = __float_as_uint((float)v);
        }
    }
    template <int PC, bool SAFE>
    __device__ static uint32_t piece(uint32_t f)
    {
        // the value minus its leading 8 bits, PC times (exact subtractions)
        uint32_t r = f;
#pragma unroll
        for (int q = 0; q < PC; ++q) r = __float_as_uint(__uint_as_float(r) - __uint_as_float(r & 0xFFFF0000u));
        return r;
    }
};

// {64,2}: the dword holding two elements (s, 11-bit e, 4-bit m each, one per half) to
// the bfloat16 pair of their scaled values, s | (e - e_ref + 127) << 7 | m << 3, in
// packed 16-bit arithmetic; sub holds (e_ref - 127) << 7 of each half's row or column,
// mod 2^16.  For a row or column that can be scaled, e - e_ref + 127 lies in [87, 127],
// so the difference needs no wider arithmetic; zeros keep their sign.  The same bits as
// the scaled binary32 value's top half.
typedef unsigned short pc_u16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pc_b64k2_pair(uint32_t d, pc_u16x2_t sub)
{
    const uint32_t magw = d & 0x7FFF7FFFu;
    const pc_u16x2_t mag = __builtin_bit_cast(pc_u16x2_t, magw);
    const uint32_t v = __builtin_bit_cast(uint32_t, (mag << 3) - sub);
    // times min(magnitude, 1): 0 for a zero half, 1 otherwise (packed min and
    // multiply, written as instructions so the compiler keeps the halves packed)
    uint32_t nz, r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(nz) : "v"(magw), "v"(0x00010001u));
    asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(r) : "v"(v), "v"(nz));
    return (d & 0x80008000u) | r;
}

// (e_ref - 127) << 7 mod 2^16 of a row or column, from its shift word (e_ref - 127) << 20
__device__ __forceinline__ unsigned short pc_b64k2_sub(int32_t shift)
{
    return (unsigned short)((shift >> 20) * 128);
}

// piece PC of two values as one bfloat16 pair
template <class LD, int PC, bool SAFE>
__device__ __forceinline__ uint32_t pc_pair(uint32_t a, uint32_t b)
{
    const uint32_t pa = LD::template piece<PC, SAFE>(a), pb = LD::template piece<PC, SAFE>(b);
    if constexpr (PC == LD::ROUND_P) return pc_cvt_pair(__uint_as_float(pa), __uint_as_float(pb));
    return pc_top_pair(pa, pb);
}

// Loads KB dwords of one 4-element chunk whose first nbytes bytes are valid
// (0 <= nbytes <= 4 KB): dwords wholly inside are loaded, a straddling dword
// is assembled from byte loads, the rest are zero.  Nothing past the valid
// bytes is read.
template <int KB>
__device__ __forceinline__ void pc_load_edge(const uint8_t* p, int nbytes, uint32_t (&out)[KB])
{
#pragma unroll
    for (int w = 0; w < KB; ++w) {
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

__device__ __forceinline__ void pc_tile_coords(int ntm, int ntn, int& tm, int& tn)
{
    const int nb = ntm * ntn;
    int pid = blockIdx.x;
    if (nb % 8 == 0) pid = (pid % 8) * (nb / 8) + pid / 8;   // consecutive tiles on one XCD
    constexpr int GROUP = 8;
    const int per_group = GROUP * ntn;
    const int group = pid / per_group;
    const int first_m = group * GROUP;
    const int gsize = (ntm - first_m) < GROUP ? (ntm - first_m) : GROUP;
    tm = first_m + (pid % per_group) % gsize;
    tn = (pid % per_group) / gsize;
}

__device__ __forceinline__ uint64_t pc_shfl_u64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// PRODS: bit (pa * P + pb) set = form the product of A piece pa and B piece pb.
// OUTK = 0: C is FP32 (binary32 operands); else C is packed binary64 in OUTK
// bytes, rounded in mode RMODE (scaled operands).
// EDGE 0: M, N are multiples of BM, BN and K of 32.  EDGE 1: any M, K with N a
// multiple of 4; rows past M and column groups past N load the last row /
// column group (whole chunks, so no element of a valid column moves), a
// partial last K step loads with bounds, and C is stored only inside the
// matrix.  EDGE 2: any M, N, K and leading dimensions; rows past M load the
// last row, B column groups that reach past N and a partial last K step load
// with bounds, addresses in 64 bits.
template <class LD, int PRODS, int BM, int BN, int WGM, int WGN, int OUTK, int RMODE, int EDGE>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm_pc(const uint8_t* __restrict__ A, int64_t lda, const uint8_t* __restrict__ B, int64_t ldb,
          void* __restrict__ Cv, int64_t ldc, int M, int N, int K, PcScale sc)
{
    constexpr int THREADS = 64 * WGM * WGN, P = LD::PIECES, KB = LD::KB;
    constexpr int TM = BM / WGM, TN = BN / WGN, FM = TM / 16, FN = TN / 16;
    constexpr bool KM = LD::KMAJOR_B;
    // n-major B: column n of the tile in plane n % 4, row n / 4, the planes BQ apart
    constexpr int BQ = (BN / 4) * PC_ROW + PC_PLANE_PAD;
    constexpr int A_TILE = BM * PC_BK, B_TILE = KM ? PC_BK * BN : 4 * BQ, STAGE = P * (A_TILE + B_TILE);
    constexpr int A_CH = BM * (PC_BK / 4) / THREADS;            // A chunks (4 elements of a row) per thread
    constexpr int B_GR = (PC_BK / 4) * (BN / 4) / THREADS;      // B groups (4 k-rows x 4 columns) per thread
    static_assert(A_CH * THREADS == BM * (PC_BK / 4) && A_CH >= 1, "A staging must divide evenly");
    static_assert(B_GR * THREADS == (PC_BK / 4) * (BN / 4) && B_GR >= 1, "B staging must divide evenly");
    static_assert(TM % 16 == 0 && TN % 16 == 0, "wave tile");
    static_assert(!KM || BN >= 128, "the B swizzle permutes 8 blocks of 16 columns");
    static_assert(KM || TN % 16 == 0, "n-major B planes hold whole 16-column blocks");
    static_assert(KM || BN % 128 == 0, "n-major B groups: 32 column groups per k-row group pair");
    static_assert(STAGE * 2 * 2 <= 160 * 1024, "LDS");
    static_assert(OUTK == 0 || LD::SCALED, "packed binary64 C comes from scaled operands");
    static_assert(!LD::DWORD_PAIRS || (KM && P == 1 && KB == 2), "dword pairs: one piece of {64,2}, k-major B");
    // The accumulators go to AGPRs (an empty statement that clobbers one makes
    // the compiler place them there), leaving the VGPRs to fragments and loads.
    asm volatile("; accumulators in AGPRs" ::: "a0");
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][STAGE];

    const int ntm = (M + BM - 1) / BM, ntn = (N + BN - 1) / BN;
    int tm, tn;
    pc_tile_coords(ntm, ntn, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    if constexpr (LD::SCALED) {
        // The FP64 GEMM that follows recomputes every 128 x 128 tile whose row
        // band or column band is flagged; this tile is skipped only when all
        // its 128 x 128 parts are such tiles.
        const int b0 = m0 / 128, b1 = (pc_min(m0 + BM, M) - 1) / 128;
        const int c0 = n0 / 128, c1 = (pc_min(n0 + BN, N) - 1) / 128;
        bool rows = true, cols = true;
        for (int b = b0; b <= b1; ++b) rows &= sc.bandA[b] != 0;
        for (int b = c0; b <= c1; ++b) cols &= sc.bandB[b] != 0;
        if (rows || cols) return;
    }
    const int t = threadIdx.x, lane = t % 64, wid = t / 64;
    const int wm = wid / WGN, wn = wid % WGN;
    const bool interior = EDGE == 0 || (m0 + BM <= M && n0 + BN <= N);

    // B group gi (4 k-rows x 4 columns) -> its column group and k-row group.  k-major: the
    // 64 groups of a wave run along the columns of one k-row group.  n-major: each 32-lane
    // phase of a wave takes 16 column groups of each of two k-row groups, so the 8-byte
    // stores of one instruction (a row per column, the k-row group's 8 bytes in it) fall on
    // 64 distinct banks.
    auto b_cg = [](int gi) {
        if constexpr (KM) return gi % (BN / 4);
        return 32 * ((gi / 64) % (BN / 128)) + gi % 16 + 16 * ((gi / 32) % 2);
    };
    auto b_kg = [](int gi) {
        if constexpr (KM) return gi / (BN / 4);
        return 2 * ((gi / 64) / (BN / 128)) + (gi / 16) % 2;
    };

    // tile row of A chunk c and first tile column of B group gi, as loaded (rows clamped
    // in EDGE 1 and 2, column groups in EDGE 1)
    auto a_row = [&](int c) {
        const int r = c / (PC_BK / 4);
        return EDGE >= 1 ? pc_min(m0 + r, M - 1) - m0 : r;
    };
    auto b_col = [&](int gi) {
        const int cc = b_cg(gi) * 4;
        return EDGE == 1 ? pc_min(n0 + cc, N - 4) - n0 : cc;
    };

    // exponent shifts of this thread's A rows and B columns (fixed over K)
    int32_t sa[A_CH][4], sb[B_GR][4];
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
        const int row = m0 + a_row(t + THREADS * i);
        const int32_t v = (LD::SCALED && row < M) ? sc.shiftA[row] : 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) sa[i][e] = v;
    }
#pragma unroll
    for (int g = 0; g < B_GR; ++g) {
        const int col = n0 + b_col(t + THREADS * g);
#pragma unroll
        for (int e = 0; e < 4; ++e) sb[g][e] = (LD::SCALED && col + e < N) ? sc.shiftB[col + e] : 0;
    }

    uint32_t ra[A_CH][KB], rb[B_GR][4][KB];

    // Byte offsets of this thread's chunks from the tile's corner, fixed over
    // K: the per-step address is a wave-uniform base plus these (the host
    // keeps BM * lda * KB and 32 * ldb * KB below 2^31 for EDGE 0 and 1).
    uint32_t aoff[A_CH], boff[B_GR][4];
#pragma unroll
    for (int i = 0; i < A_CH; ++i) {
        const int c = t + THREADS * i;
        aoff[i] = (uint32_t)(a_row(c) * lda * KB + (c % (PC_BK / 4)) * 4 * KB);
    }
#pragma unroll
    for (int g = 0; g < B_GR; ++g) {
        const int gi = t + THREADS * g;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            boff[g][r] = (uint32_t)((b_kg(gi) * 4 + r) * ldb * KB + b_col(gi) * KB);
    }
    const uint8_t* Atile = A + (int64_t)m0 * lda * KB;
    const uint8_t* Btile = B + (int64_t)n0 * KB;

    // a whole K step (k0 + 32 <= K)
    auto load_full = [&](int k0) {
        if constexpr (EDGE == 2) {
            // 64-bit addresses (the leading dimensions need not keep tile offsets
            // within 31 bits); A rows past M load the last row, and only B column
            // groups that reach past N load with bounds (those past it read nothing)
#pragma unroll
            for (int i = 0; i < A_CH; ++i) {
                const int c = t + THREADS * i, row = m0 + a_row(c), kk = k0 + (c % (PC_BK / 4)) * 4;
                load_dwords(reinterpret_cast<const uint32_t*>(A + ((int64_t)row * lda + kk) * KB), ra[i]);
            }
#pragma unroll
            for (int g = 0; g < B_GR; ++g) {
                const int gi = t + THREADS * g, col = n0 + b_cg(gi) * 4, kr = k0 + b_kg(gi) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint8_t* p = B + ((int64_t)(kr + r) * ldb + col) * KB;
                    if (col + 4 <= N) load_dwords(reinterpret_cast<const uint32_t*>(p), rb[g][r]);
                    else pc_load_edge<KB>(p, pc_max(0, N - col) * KB, rb[g][r]);
                }
            }
        } else {
            const uint8_t* Ak = Atile + k0 * KB;
            const uint8_t* Bk = Btile + (int64_t)k0 * ldb * KB;
#pragma unroll
            for (int i = 0; i < A_CH; ++i) load_dwords(reinterpret_cast<const uint32_t*>(Ak + aoff[i]), ra[i]);
#pragma unroll
            for (int g = 0; g < B_GR; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) load_dwords(reinterpret_cast<const uint32_t*>(Bk + boff[g][r]), rb[g][r]);
        }
    };
    // a partial last K step (EDGE 1 and 2): every load bounded
    auto load_bounded = [&](int k0) {
#pragma unroll
        for (int i = 0; i < A_CH; ++i) {
            const int c = t + THREADS * i, row = m0 + c / (PC_BK / 4), kk = k0 + (c % (PC_BK / 4)) * 4;
            const uint8_t* p = A + ((int64_t)row * lda + kk) * KB;
            const int nv = row < M ? pc_max(0, pc_min(4, K - kk)) : 0;
            pc_load_edge<KB>(p, nv * KB, ra[i]);
        }
#pragma unroll
        for (int g = 0; g < B_GR; ++g) {
            const int gi = t + THREADS * g, col = n0 + b_cg(gi) * 4, kr = k0 + b_kg(gi) * 4;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint8_t* p = B + ((int64_t)(kr + r) * ldb + col) * KB;
                const int nv = kr + r < K ? pc_max(0, pc_min(4, N - col)) : 0;
                pc_load_edge<KB>(p, nv * KB, rb[g][r]);
            }
        }
    };

    auto store_tiles = [&](int s) {
        uint16_t* As = lds[s];
        uint16_t* Bs = lds[s] + P * A_TILE;
        if constexpr (LD::DWORD_PAIRS) {
            // one piece, each loaded dword one pair: A along its chunk, B along the columns
#pragma unroll
            for (int i = 0; i < A_CH; ++i) {
                const int c = t + THREADS * i, row = c / (PC_BK / 4), kc = c % (PC_BK / 4);
                const int ao = row * PC_BK + ((kc >> 1) ^ ((row >> 2) & 3)) * 8 + (kc & 1) * 4;
                const unsigned short u = pc_b64k2_sub(sa[i][0]);
                const pc_u16x2_t sub = {u, u};
                *reinterpret_cast<pc_u32x2*>(As + ao) = pc_u32x2{pc_b64k2_pair(ra[i][0], sub), pc_b64k2_pair(ra[i][1], sub)};
            }
#pragma unroll
            for (int g = 0; g < B_GR; ++g) {
                const int gi = t + THREADS * g, nc = b_cg(gi) * 4, kg = b_kg(gi);
                const pc_u16x2_t sub0 = {pc_b64k2_sub(sb[g][0]), pc_b64k2_sub(sb[g][1])};
                const pc_u16x2_t sub1 = {pc_b64k2_sub(sb[g][2]), pc_b64k2_sub(sb[g][3])};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int kr = kg * 4 + r, gr = (kr & 3) | ((kr >> 1) & 4);
                    const int bo = kr * BN + ((nc >> 3) ^ (2 * gr)) * 8 + (nc & 7);
                    *reinterpret_cast<pc_u32x2*>(Bs + bo) =
                        pc_u32x2{pc_b64k2_pair(rb[g][r][0], sub0), pc_b64k2_pair(rb[g][r][1], sub1)};
                }
            }
            return;
        }
        uint32_t xa[A_CH][4], xb[B_GR][4][4];   // values: A [chunk][element], B [group][k-row][column]
#pragma unroll
        for (int i = 0; i < A_CH; ++i) LD::values(ra[i], sa[i], xa[i]);
#pragma unroll
        for (int g = 0; g < B_GR; ++g)
#pragma unroll
            for (int r = 0; r < 4; ++r) LD::values(rb[g][r], sb[g], xb[g][r]);
        // piece pairs: A along its chunk, B down its 4 k-rows
        auto a_pair = [&](auto ip, auto safe, int i, int h) {
            return pc_pair<LD, decltype(ip)::value, decltype(safe)::value>(xa[i][2 * h], xa[i][2 * h + 1]);
        };
        // B pairs: k-major, columns (2h, 2h + 1) of k-row r of the group; n-major, k-rows (2h, 2h + 1)
        // of column r
        auto b_pair = [&](auto ip, auto safe, int g, int r, int h) {
            if constexpr (KM)
                return pc_pair<LD, decltype(ip)::value, decltype(safe)::value>(xb[g][r][2 * h], xb[g][r][2 * h + 1]);
            else
                return pc_pair<LD, decltype(ip)::value, decltype(safe)::value>(xb[g][2 * h][r], xb[g][2 * h + 1][r]);
        };
        auto put = [&](auto safe) {
#pragma unroll
            for (int i = 0; i < A_CH; ++i) {
                const int c = t + THREADS * i, row = c / (PC_BK / 4), kc = c % (PC_BK / 4);
                static_for<P>([&](auto ip) {
                    constexpr int p = decltype(ip)::value;
                    const int ao = row * PC_BK + ((kc >> 1) ^ ((row >> 2) & 3)) * 8 + (kc & 1) * 4;
                    *reinterpret_cast<pc_u32x2*>(As + p * A_TILE + ao) = pc_u32x2{a_pair(ip, safe, i, 0), a_pair(ip, safe, i, 1)};
                });
            }
#pragma unroll
            for (int g = 0; g < B_GR; ++g) {
                const int gi = t + THREADS * g, nc = b_cg(gi) * 4, kg = b_kg(gi);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // k-major: k-row kg * 4 + r, columns nc .. nc + 3; n-major: column nc + r (plane r,
                    // row nc / 4), k-rows kg * 4 ..
                    const int kr = kg * 4 + r, gr = (kr & 3) | ((kr >> 1) & 4);
                    const int bo = KM ? kr * BN + ((nc >> 3) ^ (2 * gr)) * 8 + (nc & 7) : r * BQ + (nc / 4) * PC_ROW + kg * 4;
                    static_for<P>([&](auto ip) {
                        constexpr int p = decltype(ip)::value;
                        *reinterpret_cast<pc_u32x2*>(Bs + p * B_TILE + bo) = pc_u32x2{b_pair(ip, safe, g, r, 0), b_pair(ip, safe, g, r, 1)};
                    });
                }
            }
        };
        if constexpr (LD::SPECIALS) {
            // A wave takes the forms that handle Inf and NaN only when one of
            // its values of this step is one (a wave-uniform branch).  The test
            // runs on the piece-0 pairs (top halves): a half shifted left by one
            // is at least 0xFF00 exactly when its exponent field is all ones.
            typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));
            u16x2_t mx = {0, 0};
#pragma unroll
            for (int i = 0; i < A_CH; ++i)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    mx = __builtin_elementwise_max(
                        mx, __builtin_bit_cast(u16x2_t, a_pair(std::integral_constant<int, 0>{}, std::false_type{}, i, h) << 1));
#pragma unroll
            for (int g = 0; g < B_GR; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        mx = __builtin_elementwise_max(
                            mx, __builtin_bit_cast(u16x2_t,
                                                   b_pair(std::integral_constant<int, 0>{}, std::false_type{}, g, r, h) << 1));
            const bool special = mx.x >= 0xFF00 || mx.y >= 0xFF00;
            if (__builtin_amdgcn_ballot_w64(special)) put(std::true_type{});
            else put(std::false_type{});
        } else {
            put(std::false_type{});
        }
    };

    pc_f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = pc_f32x4{0.f, 0.f, 0.f, 0.f};

    // fragment offsets within a plane: A row r16 of each 16-row block, chunk lane / 16 (swizzled);
    // B transposing reads: lane s of a 16-lane group addresses k-row 8 (lane / 16) + s / 4 (+ 4
    // for the upper half), columns 4 (s % 4) .. + 3 of the 16-column block (swizzled by g of the row)
    // (n-major: column r16 of each 16 block in plane r16 % 4, k offset 8 (lane / 16))
    const int r16 = lane % 16;
    const int a_lane = (wm * TM + r16) * PC_BK + (((lane / 16) ^ ((r16 >> 2) & 3)) * 8);
    const int b_lane = KM ? (8 * (lane / 16) + r16 / 4) * BN + 4 * (r16 % 4)
                          : (r16 % 4) * BQ + ((wn * TN) / 4 + r16 / 4) * PC_ROW + 8 * (lane / 16);
    const int bg = (r16 / 4) | (((lane / 16) & 1) << 2);
    auto compute = [&](int s) {
        pc_bf16x8 a[P][FM], b[P][FN];
        auto read_a = [&](int p, int i) {
            a[p][i] = *reinterpret_cast<const pc_bf16x8*>(lds[s] + p * A_TILE + a_lane + i * 16 * PC_BK);
        };
        __builtin_amdgcn_s_setprio(1);
        // the first row block of A and all of B first, so the MFMAs of row block 0 start
        // after those reads while the rest of A arrives
#pragma unroll
        for (int p = 0; p < P; ++p) read_a(p, 0);
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if constexpr (KM) {
                    const uint16_t* q = lds[s] + P * A_TILE + p * B_TILE + b_lane + ((wn * FN + j) ^ bg) * 16;
                    const pc_i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((pc_lds_i16x4*)(q));
                    const pc_i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((pc_lds_i16x4*)(q + 4 * BN));
                    b[p][j] = __builtin_bit_cast(pc_bf16x8, pc_i16x8(__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7)));
                } else {
                    b[p][j] = *reinterpret_cast<const pc_bf16x8*>(lds[s] + P * A_TILE + p * B_TILE + b_lane + j * 4 * PC_ROW);
                }
            }
#pragma unroll
        for (int i = 1; i < FM; ++i)
#pragma unroll
            for (int p = 0; p < P; ++p) read_a(p, i);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                static_for<P * P>([&](auto iq) {
                    constexpr int q = decltype(iq)::value;
                    if constexpr ((PRODS >> q) & 1)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q / P][i], b[q % P][j], acc[i][j], 0, 0, 0);
                });
        __builtin_amdgcn_s_setprio(0);
    };

    // KF whole K steps, then (EDGE 1 and 2) a partial one; the bounded loads of the
    // partial step stay out of the loop body
    const int KF = K / PC_BK, KT = (K + PC_BK - 1) / PC_BK;
    auto load_step = [&](int kt) {
        if (EDGE == 0 || kt < KF) load_full(kt * PC_BK);
        else load_bounded(kt * PC_BK);
    };
    if constexpr (LD::EARLY_LOADS) {
        load_step(0);
        store_tiles(0);
        if (KT > 1) load_step(1);
        __syncthreads();
        for (int kt = 0; kt < KT - 1; ++kt) {
            const int s = kt & 1;
            compute(s);
            store_tiles(s ^ 1);
            // the loads of the step after next are issued before the barrier
            if (kt + 2 < KT) load_step(kt + 2);
            __syncthreads();
        }
    } else {
        load_step(0);
        store_tiles(0);
        __syncthreads();
        for (int kt = 0; kt < KF - 1; ++kt) {
            const int s = kt & 1;
            load_full((kt + 1) * PC_BK);
            // the next step's global loads stay ahead of this step's MFMAs
            __builtin_amdgcn_sched_barrier(0);
            compute(s);
            store_tiles(s ^ 1);
            __syncthreads();
        }
        if (EDGE != 0 && KT > KF && KF > 0) {
            const int s = (KF - 1) & 1;
            load_bounded(KF * PC_BK);
            __builtin_amdgcn_sched_barrier(0);
            compute(s);
            store_tiles(s ^ 1);
            __syncthreads();
        }
    }
    compute((KT - 1) & 1);

    // ---- epilogue: lane holds rows 4 * (lane / 16) + r, column lane % 16 of each 16 x 16 tile
    if constexpr (OUTK == 0) {
        float* C = static_cast<float*>(Cv);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * TM + i * 16 + 4 * (lane / 16) + r;
                    const int col = n0 + wn * TN + j * 16 + lane % 16;
                    if (interior || (row < M && col < N)) C[(int64_t)row * ldc + col] = acc[i][j][r];
                }
    } else {
        // C_ij = 2^(e_i - 1023 + e_j - 1023) acc_ij in FP64 (exact), cut to OUTK bytes;
        // the G lanes of a dword-aligned group of columns hand their packed
        // values to the group's first lane, which stores whole dwords (or, for a
        // group cut by the last column, the bytes of its valid elements)
        using FO = Fmt<64, OUTK>;
        constexpr int GO = FO::G;
        uint8_t* C = static_cast<uint8_t*>(Cv);
        const int c16 = lane % 16;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn * TN + j * 16 + c16;
            // the scaled value of an element is 2^-(e_ref - 1023) times it
            const int ec = (col < N) ? (sc.shiftB[col] >> 20) - 896 : 0;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm * TM + i * 16 + 4 * (lane / 16) + r;
                    const int er = (row < M) ? (sc.shiftA[row] >> 20) - 896 : 0;
                    const double v = __builtin_amdgcn_ldexp((double)acc[i][j][r], er + ec);
                    const uint64_t q = round_pack<FO, RMODE>((uint64_t)__double_as_longlong(v));
                    uint64_t gq[GO];
                    gq[0] = q;
#pragma unroll
                    for (int e = 1; e < GO; ++e) gq[e] = pc_shfl_u64(q, (lane + e) % 64);
                    if (c16 % GO == 0 && row < M && col < N) {
                        uint8_t* dst = C + ((int64_t)row * ldc + col) * OUTK;
                        if (col + GO <= N) {
                            uint32_t out[GO * OUTK / 4];
                            assemble_elems<FO, GO>(gq, out);
                            store_dwords(reinterpret_cast<uint32_t*>(dst), out);
                        } else {
#pragma unroll
                            for (int e = 0; e < GO; ++e)
                                if (col + e < N) store_elem_bytes<FO>(dst + e * OUTK, gq[e]);
                        }
                    }
                }
        }
    }
}

// ---------------------------------------------------------------- host side
template <class LD, int PRODS, int BM, int BN, int WGM, int WGN, int OUTK, int RMODE>
fb_status pc_run(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb,
                        void* C, int64_t ldc, const PcScale& sc, hipStream_t stream)
{
    const int64_t blocks = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    auto a = static_cast<const uint8_t*>(A);
    auto b = static_cast<const uint8_t*>(B);
    // shapes that are tile multiples take the instance without bounds, those
    // with N a multiple of 4 the clamped one (both need per-tile offsets that
    // fit 31 bits), the rest the bounded one
    constexpr int KB = LD::KB;
    const bool offs = (int64_t)BM * lda * KB < (1ll << 31) && (int64_t)PC_BK * ldb * KB < (1ll << 31);
    const unsigned grid = (unsigned)blocks, threads = 64 * WGM * WGN;
    if (offs && M % BM == 0 && N % BN == 0 && K % PC_BK == 0)
        k_gemm_pc<LD, PRODS, BM, BN, WGM, WGN, OUTK, RMODE, 0><<<grid, threads, 0, stream>>>(
            a, lda, b, ldb, C, ldc, (int)M, (int)N, (int)K, sc);
    else if (offs && N % 4 == 0)
        k_gemm_pc<LD, PRODS, BM, BN, WGM, WGN, OUTK, RMODE, 1><<<grid, threads, 0, stream>>>(
            a, lda, b, ldb, C, ldc, (int)M, (int)N, (int)K, sc);
    else
        k_gemm_pc<LD, PRODS, BM, BN, WGM, WGN, OUTK, RMODE, 2><<<grid, threads, 0, stream>>>(
            a, lda, b, ldb, C, ldc, (int)M, (int)N, (int)K, sc);
    return check_launch("fb_gemm");
}

}  // namespace flyte
