// GEMV y = A x over a packed row-major A (the paper's BLAS level-2 kernel,
// Section 6.2; its 2x unrolled variant is one point of the tile space here).
//
// A workgroup is 4 waves.  Each wave splits into 64/LPR lane groups; a group
// of LPR lanes owns RPW consecutive rows and walks them together: lane l of
// the group reads units l, l+LPR, ... of every row (U units per loop trip, so
// U*RPW independent loads are in flight per lane), unpacks them with
// compile-time v_perm_b32 and accumulates with fma in the base type.  x is read
// directly (it stays in L1/L2: one x unit serves RPW rows).  The LPR partial
// sums of a row are combined with a fixed xor butterfly, so every result is a
// fixed sequence of base-type operations for a given tile configuration.
#pragma once

#include "codec.hpp"

namespace flyte {

constexpr int kGemvBlock = 256;
constexpr int kGemvWaves = kGemvBlock / 64;

struct GemvArgs {
    const uint8_t* A;      // packed matrix
    int64_t row_bytes;     // lda * k
    const void* x;         // native
    void* y;               // native
    int32_t m, n;
};

template <int LPR, int RPW, int U>
struct GemvTile {
    static constexpr int lpr = LPR, rpw = RPW, u = U;
    static constexpr int rows_per_wave = (64 / LPR) * RPW;
    static constexpr int rows_per_block = kGemvWaves * rows_per_wave;
};

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
    constexpr int LPR = TILE::lpr, RPW = TILE::rpw, U = TILE::u;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int grp = lane / LPR, gl = lane % LPR;
    const int64_t r0 = tile_row0 + (int64_t)wave * TILE::rows_per_wave + (int64_t)grp * RPW;
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

    for (int64_t g0 = gl; g0 < nunits; g0 += (int64_t)LPR * U) {
        uint32_t X[U][F::UNIT_NW];
        uint32_t P[RPW][U][F::UNIT_DW];
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + (int64_t)u * LPR;
            if (g < nunits) {
                load_dwords(xw + g * F::UNIT_NW, X[u]);
#pragma unroll
                for (int r = 0; r < RPW; ++r) load_dwords(rowp[r] + g * F::UNIT_DW, P[r][u]);
            }
        });
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + (int64_t)u * LPR;
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
    }
    // columns after the last whole unit: one element per lane
    {
        const int64_t c = nunits * F::UNIT + gl;
        if (gl < F::UNIT && c < a.n) {
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
    if (gl == 0) {
        N* y = static_cast<N*>(a.y);
#pragma unroll
        for (int r = 0; r < RPW; ++r)
            if (r0 + r < a.m) y[r0 + r] = acc[r];
    }
}

// The tile configurations, in index order (the index is the public config id).
#define FLYTE_GEMV_TILES(X) \
    X(0, 64, 1, 2)          \
    X(1, 64, 1, 4)          \
    X(2, 64, 2, 2)          \
    X(3, 64, 2, 4)          \
    X(4, 64, 4, 1)          \
    X(5, 64, 4, 2)          \
    X(6, 64, 8, 1)          \
    X(7, 32, 2, 2)          \
    X(8, 16, 1, 2)          \
    X(9, 16, 2, 2)          \
    X(10, 16, 4, 1)         \
    X(11, 8, 2, 1)          \
    X(12, 8, 4, 1)

constexpr int kGemvNumTiles = 13;

struct TileInfo {
    int lpr, rpw, u, rows_per_block;
};

inline TileInfo gemv_tile_info(int id)
{
    switch (id) {
#define FLYTE_TILE_CASE(ID, LPR, RPW, U) \
    case ID: return TileInfo{LPR, RPW, U, GemvTile<LPR, RPW, U>::rows_per_block};
        FLYTE_GEMV_TILES(FLYTE_TILE_CASE)
#undef FLYTE_TILE_CASE
    }
    return TileInfo{0, 0, 0, 0};
}

// Default tile when the autotuner cache has no entry for a shape.
inline int gemv_default_tile(int64_t m, int64_t n, int k)
{
    const int64_t units = n * k / 16;   // ~16-byte units per row
    if (units >= 512) return m >= 4096 ? 2 : 0;
    if (units >= 128) return 7;
    if (units >= 32) return 9;
    return 11;
}

}  // namespace flyte
