// GEMV y = A x over a packed row-major A (the paper's BLAS level-2 kernel,
// Section 6.2; its 2x unrolled variant is one point of the tile space here).
//
// A workgroup is 4 waves, arranged as 4/KS row groups of KS waves.  Each
// wave splits into 64/LPR lane groups; a lane group owns RPW consecutive rows
// and walks them together with the same lane groups of the other KS-1 waves of
// its row group: in one loop trip the KS*LPR lanes read KS*LPR*U consecutive
// units of every row (U units per lane, each instruction contiguous across the
// wave), unpack them with compile-time v_perm_b32 and accumulate with fma in
// the base type.  KS > 1 puts more lanes on fewer rows, so the workgroups in
// flight sweep a narrower band of A.  x is read directly (it stays in L1/L2:
// one x unit serves RPW rows).  The LPR partial sums of a row are combined by
// a fixed xor butterfly, then the KS wave partials in a fixed order through
// LDS, so every result is a fixed sequence of base-type operations for a
// given tile configuration.  NT marks the A loads non-temporal (A is read
// once; x should stay cached).  PIPE software-pipelines the unit loop: the
// next trip's loads are issued before this trip's FMAs, into a second set of
// registers (the same operations in the same order, so the same results).
#pragma once

#include "codec.hpp"

namespace flyte {

constexpr int kGemvBlock = 256;
constexpr int kGemvWaves = kGemvBlock / 64;

struct GemvArgs {
    const uint8_t* A;      // packed matrix
    int64_t row_bytes;     // lda * k
    const void* x;         // native
    void* y;               // native, or packed in yk bytes
    int32_t m, n;
    int32_t yk;            // 0: y is native; else y is stored in yk bytes per element
    int32_t ymode;         // rounding mode of a packed y
};

template <int LPR, int RPW, int U, int KS = 1, bool NT = false, bool STAGED = false, bool PIPE = false>
struct GemvTile {
    static_assert(KS == 1 || KS == 2 || KS == 4, "waves per row group");
    static_assert(!STAGED || LPR == 64, "staged tiles use whole waves per row group");
    static_assert(!(STAGED && PIPE), "the staged sweep is not pipelined");
    static constexpr int lpr = LPR, rpw = RPW, u = U, ks = KS;
    static constexpr bool nt = NT, staged = STAGED, pipe = PIPE;
    static constexpr int rows_per_wave = (64 / LPR) * RPW;
    static constexpr int rows_per_block = (kGemvWaves / KS) * rows_per_wave;
};

template <int N>
__device__ __forceinline__ void load_dwords_nt(const uint32_t* __restrict__ p, uint32_t (&out)[N])
{
    static_for<(N + 3) / 4>([&](auto iv) {
        constexpr int o = 4 * decltype(iv)::value;
        constexpr int r = N - o < 4 ? N - o : 4;
        if constexpr (r == 4) {
            const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p + o));
            out[o] = v.x; out[o + 1] = v.y; out[o + 2] = v.z; out[o + 3] = v.w;
        } else if constexpr (r == 3) {
            const u32x3 v = __builtin_nontemporal_load(reinterpret_cast<const u32x3*>(p + o));
            out[o] = v.x; out[o + 1] = v.y; out[o + 2] = v.z;
        } else if constexpr (r == 2) {
            const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p + o));
            out[o] = v.x; out[o + 1] = v.y;
        } else {
            out[o] = __builtin_nontemporal_load(p + o);
        }
    });
}

template <class T, int LPR>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int o = LPR / 2; o >= 1; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// Rows [tile_row0, tile_row0 + rows_per_block) of one GEMV.
template <class F, class TILE>
__device__ __forceinline__ void gemv_block(const GemvArgs& a, int64_t tile_row0)
{
    using T = typename F::bits_t;
    using N = typename F::native_t;
    constexpr int LPR = TILE::lpr, RPW = TILE::rpw, U = TILE::u, KS = TILE::ks;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int rgrp = wave / KS, ws = wave % KS;            // row group, wave within it
    const int grp = lane / LPR, gl = lane % LPR;
    const int64_t r0 = tile_row0 + (int64_t)rgrp * TILE::rows_per_wave + (int64_t)grp * RPW;
    const int sl = ws * LPR + gl;                          // lane index within the KS*LPR sweep
    const int64_t nunits = a.n / F::UNIT;
    const uint32_t* xw = static_cast<const uint32_t*>(a.x);

    const uint32_t* rowp[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        int64_t rr = r0 + r;
        if (rr >= a.m) rr = a.m - 1;   // keep loads in bounds; result discarded below
        rowp[r] = reinterpret_cast<const uint32_t*>(a.A + rr * a.row_bytes);
    }
    N acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = N(0);

    int64_t unit0 = 0;   // first unit handled by the per-lane unit loop below
    if constexpr (TILE::staged) {
        // LDS byte staging: a wave's span of 1024 elements of a row (k KiB) is
        // read with lane-contiguous dwordx4 loads (each instruction one
        // contiguous KiB, no cache line shared between instructions), written
        // to the wave's LDS slice, and read back as 16 consecutive elements per
        // lane (lane stride 16k bytes: k*4 dwords, whose start banks differ for
        // the 16 lanes of a read phase because gcd(4k, 64) = 4 for odd k).
        constexpr int SPAN_DW = 16 * F::k * 64 / 4;   // dwords of one row span
        __shared__ __attribute__((aligned(16))) uint32_t stage[kGemvWaves][SPAN_DW];
        const int64_t nspans = a.n / 1024;
        for (int64_t sp = ws; sp < nspans; sp += KS) {
            // all rows' loads first (RPW * k instructions in flight per lane) ...
            uint32_t V[RPW][F::k][4];
#pragma unroll
            for (int r = 0; r < RPW; ++r)
#pragma unroll
                for (int j = 0; j < F::k; ++j)
                    load_dwords_nt<4>(rowp[r] + sp * SPAN_DW + (j * 64 + lane) * 4, V[r][j]);
            const int64_t e0 = sp * 1024 + lane * 16;
            uint32_t X[16 * F::W / 4];
            load_dwords(xw + e0 * (F::W / 4), X);
            T xb[16];
            words_to_bits<F, 16>(X, xb);
            // ... then each row through the wave's LDS slice in turn
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
#pragma unroll
                for (int j = 0; j < F::k; ++j)
                    *reinterpret_cast<u32x4*>(&stage[wave][(j * 64 + lane) * 4]) =
                        u32x4{V[r][j][0], V[r][j][1], V[r][j][2], V[r][j][3]};
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                uint32_t P[4 * F::k];
#pragma unroll
                for (int j = 0; j < F::k; ++j) {
                    const u32x4 v = *reinterpret_cast<const u32x4*>(&stage[wave][lane * 4 * F::k + 4 * j]);
                    P[4 * j] = v.x; P[4 * j + 1] = v.y; P[4 * j + 2] = v.z; P[4 * j + 3] = v.w;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                T ab[16];
                unpack_elems<F, 16>(P, ab);
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[r] = fma_n(as_native<F>(ab[e]), as_native<F>(xb[e]), acc[r]);
            }
        }
        unit0 = nspans * (1024 / F::UNIT);
    }

    // one trip: U units of every row (and of x) per lane
    auto load_trip = [&](int64_t g0, uint32_t (&X)[U][F::UNIT_NW], uint32_t (&P)[RPW][U][F::UNIT_DW]) {
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + (int64_t)u * KS * LPR;
            if (g < nunits) {
                load_dwords(xw + g * F::UNIT_NW, X[u]);
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    if constexpr (TILE::nt) load_dwords_nt(rowp[r] + g * F::UNIT_DW, P[r][u]);
                    else load_dwords(rowp[r] + g * F::UNIT_DW, P[r][u]);
                }
            }
        });
    };
    auto fma_trip = [&](int64_t g0, uint32_t (&X)[U][F::UNIT_NW], uint32_t (&P)[RPW][U][F::UNIT_DW]) {
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + (int64_t)u * KS * LPR;
            if (g < nunits) {
                T xb[F::UNIT];
                words_to_bits<F, F::UNIT>(X[u], xb);
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    T ab[F::UNIT];
                    unpack_elems<F, F::UNIT>(P[r][u], ab);
#pragma unroll
                    for (int e = 0; e < F::UNIT; ++e)
                        acc[r] = fma_n(as_native<F>(ab[e]), as_native<F>(xb[e]), acc[r]);
                }
            }
        });
    };
    constexpr int64_t STEP = (int64_t)KS * LPR * U;
    if constexpr (TILE::pipe) {
        // two register sets, alternating: trip t + 1 is in flight while trip t is summed
        uint32_t Xa[U][F::UNIT_NW], Pa[RPW][U][F::UNIT_DW], Xb[U][F::UNIT_NW], Pb[RPW][U][F::UNIT_DW];
        int64_t g0 = unit0 + sl;
        if (g0 < nunits) load_trip(g0, Xa, Pa);
        while (g0 < nunits) {
            if (g0 + STEP < nunits) load_trip(g0 + STEP, Xb, Pb);
            fma_trip(g0, Xa, Pa);
            g0 += STEP;
            if (g0 >= nunits) break;
            if (g0 + STEP < nunits) load_trip(g0 + STEP, Xa, Pa);
            fma_trip(g0, Xb, Pb);
            g0 += STEP;
        }
    } else {
        for (int64_t g0 = unit0 + sl; g0 < nunits; g0 += STEP) {
            uint32_t X[U][F::UNIT_NW], P[RPW][U][F::UNIT_DW];
            load_trip(g0, X, P);
            fma_trip(g0, X, P);
        }
    }
    // columns after the last whole unit: one element per lane
    {
        const int64_t c = nunits * F::UNIT + sl;
        if (sl < F::UNIT && c < a.n) {
            const N xv = static_cast<const N*>(a.x)[c];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const uint8_t* p = reinterpret_cast<const uint8_t*>(rowp[r]) + c * F::k;
                acc[r] = fma_n(as_native<F>(load_elem_unpacked<F>(p)), xv, acc[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = group_sum<N, LPR>(acc[r]);
    if constexpr (KS > 1) {
        // wave partials of each row, combined in wave order by the first wave
        __shared__ N part[kGemvWaves][64 / LPR][RPW];
        if (gl == 0) {
#pragma unroll
            for (int r = 0; r < RPW; ++r) part[wave][grp][r] = acc[r];
        }
        __syncthreads();
        if (ws == 0 && gl == 0) {
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                N s = part[wave][grp][r];
#pragma unroll
                for (int w = 1; w < KS; ++w) s = s + part[wave + w][grp][r];
                acc[r] = s;
            }
        }
        __syncthreads();   // the block may run another tile (persistent kernel) and reuse part
    }
    if (ws == 0 && gl == 0) {
        if (a.yk == 0) {
            N* y = static_cast<N*>(a.y);
#pragma unroll
            for (int r = 0; r < RPW; ++r)
                if (r0 + r < a.m) y[r0 + r] = acc[r];
        } else {
            // packed output: one rounding of the base-type result, byte stores
            uint8_t* y = static_cast<uint8_t*>(a.y);
#pragma unroll
            for (int r = 0; r < RPW; ++r)
                if (r0 + r < a.m)
                    store_bytes_rt(y + (r0 + r) * a.yk,
                                   pack_runtime((uint64_t)as_bits<F>(acc[r]), F::base, a.yk, a.ymode), a.yk);
        }
    }
}

// The tile configurations, in index order (the index is the public config
// id): (lanes per row group, rows per lane group, units per lane per trip,
// waves per row group, non-temporal A loads, LDS byte staging, pipelined).
#define FLYTE_GEMV_TILES(X)                   \
    X(0, 64, 1, 2, 1, false, false, false)    \
    X(1, 64, 1, 4, 1, false, false, false)    \
    X(2, 64, 2, 2, 1, false, false, false)    \
    X(3, 64, 2, 4, 1, false, false, false)    \
    X(4, 64, 4, 1, 1, false, false, false)    \
    X(5, 64, 4, 2, 1, false, false, false)    \
    X(6, 64, 8, 1, 1, false, false, false)    \
    X(7, 32, 2, 2, 1, false, false, false)    \
    X(8, 16, 1, 2, 1, false, false, false)    \
    X(9, 16, 2, 2, 1, false, false, false)    \
    X(10, 16, 4, 1, 1, false, false, false)   \
    X(11, 8, 2, 1, 1, false, false, false)    \
    X(12, 8, 4, 1, 1, false, false, false)    \
    X(13, 64, 2, 2, 2, false, false, false)   \
    X(14, 64, 4, 1, 2, false, false, false)   \
    X(15, 64, 4, 2, 2, false, false, false)   \
    X(16, 64, 2, 2, 4, false, false, false)   \
    X(17, 64, 4, 1, 4, false, false, false)   \
    X(18, 64, 8, 1, 4, false, false, false)   \
    X(19, 64, 4, 2, 1, true, false, false)    \
    X(20, 64, 2, 4, 1, true, false, false)    \
    X(21, 64, 4, 1, 2, true, false, false)    \
    X(22, 64, 4, 1, 4, true, false, false)    \
    X(23, 64, 1, 1, 1, true, true, false)     \
    X(24, 64, 2, 1, 1, true, true, false)     \
    X(25, 64, 4, 1, 1, true, true, false)     \
    X(26, 64, 2, 1, 2, true, true, false)     \
    X(27, 64, 4, 1, 2, true, true, false)     \
    X(28, 64, 2, 1, 4, true, true, false)     \
    X(29, 64, 4, 1, 4, true, true, false)     \
    X(30, 64, 8, 1, 4, true, true, false)     \
    X(31, 32, 2, 2, 1, true, false, false)    \
    X(32, 16, 2, 2, 1, true, false, false)    \
    X(33, 8, 2, 1, 1, true, false, false)     \
    X(34, 64, 1, 2, 4, true, false, false)    \
    X(35, 64, 1, 4, 4, true, false, false)    \
    X(36, 64, 2, 2, 4, true, false, false)    \
    X(37, 64, 1, 1, 4, true, true, false)     \
    X(38, 64, 8, 2, 4, true, false, false)    \
    X(39, 64, 4, 2, 2, true, false, false)    \
    X(40, 64, 8, 2, 4, true, false, true)     \
    X(41, 64, 2, 2, 4, true, false, true)     \
    X(42, 64, 4, 2, 2, true, false, true)     \
    X(43, 64, 4, 2, 1, true, false, true)

constexpr int kGemvNumTiles = 44;

struct TileInfo {
    int lpr, rpw, u, ks, nt, staged, rows_per_block;
};

inline TileInfo gemv_tile_info(int id)
{
    switch (id) {
#define FLYTE_TILE_CASE(ID, LPR, RPW, U, KS, NT, ST, PP) \
    case ID: return TileInfo{LPR, RPW, U, KS, NT, ST, GemvTile<LPR, RPW, U, KS, NT, ST, PP>::rows_per_block};
        FLYTE_GEMV_TILES(FLYTE_TILE_CASE)
#undef FLYTE_TILE_CASE
    }
    return TileInfo{0, 0, 0, 0, 0, 0, 0};
}

// Default tile when the autotuner cache has no entry for a shape (measured on
// MI355X with 8192 x 8192 matrices for the long rows; shorter rows use fewer
// lanes per row).
inline int gemv_default_tile(int64_t m, int64_t n, int k)
{
    const int64_t units = n * k / 16;   // ~16-byte units per row
    if (units >= 512 && n >= 1024 && m >= 1024) {
        if (k == 5 || k == 7) return 29;   // LDS-staged, 4 rows per wave, 4 waves per row group
        if (k == 4 || k == 6) return 22;
        return 19;                          // k = 2, 3, 8
    }
    if (units >= 512) return m >= 4096 ? 2 : 0;
    if (units >= 128) return 7;
    if (units >= 32) return 9;
    return 11;
}

}  // namespace flyte
