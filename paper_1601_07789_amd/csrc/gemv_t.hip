// Transposed GEMV y = A^T x over a packed row-major A (m x n): y_j = sum_i
// A_ij x_i, the other access order of the paper's BLAS level-2 kernel.
//
// A workgroup of four waves owns a strip of 64 consecutive column units (one
// unit per lane) and a slab of consecutive rows.  The slab's rows are dealt to
// the waves in chunks of U rows (chunk c to wave c mod 4); a lane walks its
// unit down its chunks, so every wave-wide load reads one contiguous span of
// a row, and accumulates UNIT column sums with fma in the base type.  The
// four wave sums are added in wave order through LDS.  With more than one
// slab, the slab sums go to a per-stream workspace and a second kernel adds
// them (slabs q = j mod 4 by thread group j, then the four groups in order),
// so the result is a fixed sequence of operations for given sizes; the last
// step writes y native or packed (one rounding, byte stores).  A is streamed
// once, so units that one load instruction covers (at most 4 dwords) are read
// non-temporally.  5- and 7-dword units (two load instructions per unit, which
// would share cache lines) are read as lane-contiguous row spans and passed
// through LDS instead, in strips of 64 whole units.
#include "codec.hpp"
#include "common.hpp"
#include "gemv_impl.hpp"

namespace flyte {

constexpr int kGtBlock = 256;
constexpr int kGtWaves = kGtBlock / 64;
constexpr int kGtTarget = 1024;     // workgroups to aim for (strips x slabs), see gt_target

// Rows per chunk (loads in flight per lane) and workgroups to aim for, per
// format, as measured on 8192 x 8192: 8 rows and 1024 workgroups, except 12
// rows for binary64 k = 4 (+2-3%), 16 for k = 5 (+2-3%) and 768 workgroups for
// k = 8 (+3%); each of these lost elsewhere (16 rows: -10% at k = 3; 768
// workgroups: -10% at k = 3, -1% at k = 6).
template <class F>
constexpr int gt_rows()
{
    return F::base == 64 && F::k == 4 ? 12 : (F::base == 64 && F::k == 5 ? 16 : 8);
}

template <class F>
constexpr int64_t gt_target()
{
    return F::base == 64 && F::k == 8 ? 768 : kGtTarget;
}

template <class F>
__device__ __forceinline__ void gemv_t_store(typename F::native_t v, int64_t c, typename F::native_t* partial,
                                             void* y, int yk, int ymode)
{
    using N = typename F::native_t;
    if (partial) partial[c] = v;
    else if (yk == 0) static_cast<N*>(y)[c] = v;
    else store_bytes_rt(static_cast<uint8_t*>(y) + c * yk, pack_runtime((uint64_t)as_bits<F>(v), F::base, yk, ymode), yk);
}

template <class F, int U>
__global__ void __launch_bounds__(kGtBlock)
k_gemv_t(const uint8_t* __restrict__ A, int64_t row_bytes, const void* __restrict__ xv, int m, int n, int rows_per_slab,
         typename F::native_t* __restrict__ partial, void* __restrict__ y, int yk, int ymode)
{
    using T = typename F::bits_t;
    using N = typename F::native_t;
    __shared__ N red[kGtWaves - 1][F::UNIT][64];
    const N* x = static_cast<const N*>(xv);
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int64_t nunits = n / F::UNIT;
    const int64_t g = (int64_t)blockIdx.x * 64 + lane;     // column unit of this lane
    const int r0 = blockIdx.y * rows_per_slab;
    const int r1 = min(m, r0 + rows_per_slab);
    const int tail = (int)(n - nunits * F::UNIT);          // columns after the last whole unit
    N acc[F::UNIT];
#pragma unroll
    for (int e = 0; e < F::UNIT; ++e) acc[e] = N(0);
    if (g < nunits) {
        const uint8_t* col = A + g * (F::UNIT_DW * 4);
        int r = r0 + w * U;
        if constexpr (F::UNIT_DW > 4) {
            // 5- and 7-dword units: a full strip's span of each row (64 units) is read
            // with two lane-contiguous non-temporal loads (the first KiB as dwordx4, the
            // rest as one more piece per lane), passed through the wave's LDS row buffer,
            // and each lane reads its own unit back (odd dword stride: no bank conflicts)
            if (((int64_t)blockIdx.x + 1) * 64 <= nunits) {
                constexpr int SPAN = 64 * F::UNIT_DW;   // dwords of one row of the strip
                constexpr int REST = F::UNIT_DW - 4;    // dwords per lane after the first KiB
                __shared__ __attribute__((aligned(16))) uint32_t stage[kGtWaves][SPAN];
                const uint8_t* strip = A + (int64_t)blockIdx.x * SPAN * 4;
                for (; r + U <= r1; r += kGtWaves * U) {
                    uint32_t L[U][4], Q[U][REST];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const uint32_t* rp = reinterpret_cast<const uint32_t*>(strip + (int64_t)(r + u) * row_bytes);
                        load_dwords_nt(rp + lane * 4, L[u]);
                        load_dwords_nt(rp + 256 + lane * REST, Q[u]);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        *reinterpret_cast<u32x4*>(&stage[w][lane * 4]) = u32x4{L[u][0], L[u][1], L[u][2], L[u][3]};
#pragma unroll
                        for (int j = 0; j < REST; ++j) stage[w][256 + lane * REST + j] = Q[u][j];
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        uint32_t P[F::UNIT_DW];
#pragma unroll
                        for (int j = 0; j < F::UNIT_DW; ++j) P[j] = stage[w][lane * F::UNIT_DW + j];
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        T ab[F::UNIT];
                        unpack_elems<F, F::UNIT>(P, ab);
                        const N xr = x[r + u];
#pragma unroll
                        for (int e = 0; e < F::UNIT; ++e) acc[e] = fma_n(as_native<F>(ab[e]), xr, acc[e]);
                    }
                }
            }
        }
        for (; r + U <= r1; r += kGtWaves * U) {
            uint32_t P[U][F::UNIT_DW];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if constexpr (F::UNIT_DW <= 4)
                    load_dwords_nt(reinterpret_cast<const uint32_t*>(col + (int64_t)(r + u) * row_bytes), P[u]);
                else
                    load_dwords(reinterpret_cast<const uint32_t*>(col + (int64_t)(r + u) * row_bytes), P[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                T ab[F::UNIT];
                unpack_elems<F, F::UNIT>(P[u], ab);
                const N xr = x[r + u];
#pragma unroll
                for (int e = 0; e < F::UNIT; ++e) acc[e] = fma_n(as_native<F>(ab[e]), xr, acc[e]);
            }
        }
        for (; r < r1; ++r) {     // the slab's last, partial chunk (one wave at most)
            uint32_t P[F::UNIT_DW];
            load_dwords(reinterpret_cast<const uint32_t*>(col + (int64_t)r * row_bytes), P);
            T ab[F::UNIT];
            unpack_elems<F, F::UNIT>(P, ab);
            const N xr = x[r];
#pragma unroll
            for (int e = 0; e < F::UNIT; ++e) acc[e] = fma_n(as_native<F>(ab[e]), xr, acc[e]);
        }
    } else if (g == nunits && tail > 0) {
        for (int r = r0 + w; r < r1; r += kGtWaves) {
            const uint8_t* row = A + (int64_t)r * row_bytes;
            const N xr = x[r];
            for (int e = 0; e < tail; ++e)
                acc[e] = fma_n(as_native<F>(load_elem_unpacked<F>(row + (nunits * F::UNIT + e) * F::k)), xr, acc[e]);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int e = 0; e < F::UNIT; ++e) red[w - 1][e][lane] = acc[e];
    }
    __syncthreads();
    if (w > 0) return;
    const int ncols = g < nunits ? F::UNIT : (g == nunits ? tail : 0);
    N* dst = partial ? partial + (int64_t)blockIdx.y * n : nullptr;
#pragma unroll
    for (int e = 0; e < F::UNIT; ++e) {
        if (e < ncols) {
            N v = acc[e];
#pragma unroll
            for (int q = 0; q < kGtWaves - 1; ++q) v = v + red[q][e][lane];
            gemv_t_store<F>(v, g * F::UNIT + e, dst, y, yk, ymode);
        }
    }
}

template <class F>
__global__ void __launch_bounds__(kGtBlock)
k_gemv_t_final(const typename F::native_t* __restrict__ partial, int nslabs, int n, void* __restrict__ y, int yk,
               int ymode)
{
    using N = typename F::native_t;
    __shared__ N red[kGtWaves - 1][64];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int64_t c = (int64_t)blockIdx.x * 64 + lane;
    N s = N(0);
    if (c < n) {
        int q = w;
        for (; q + 3 * kGtWaves < nslabs; q += 4 * kGtWaves) {     // four loads in flight, added in q order
            N v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = partial[(int64_t)(q + i * kGtWaves) * n + c];
#pragma unroll
            for (int i = 0; i < 4; ++i) s = s + v[i];
        }
        for (; q < nslabs; q += kGtWaves) s = s + partial[(int64_t)q * n + c];
    }
    if (w > 0) red[w - 1][lane] = s;
    __syncthreads();
    if (w > 0 || c >= n) return;
#pragma unroll
    for (int q = 0; q < kGtWaves - 1; ++q) s = s + red[q][lane];
    gemv_t_store<F>(s, c, nullptr, y, yk, ymode);
}

template <class F>
__global__ void k_zero_native(void* y, int64_t n, int yk)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t bytes = n * (yk ? yk : F::W);
    for (int64_t b = i; b < bytes; b += (int64_t)gridDim.x * blockDim.x) static_cast<uint8_t*>(y)[b] = 0;
}

fb_status gemv_t_launch(fb_format fa, fb_format fy, int64_t m, int64_t n, const void* A, int64_t lda, const void* x,
                        void* y, hipStream_t stream)
{
    if (n == 0) return FB_OK;
    // y (n elements) is written even when m = 0 (empty sums), and the shared
    // argument checks stop at m = 0, so y is checked here
    if (!y) return set_error(FB_ERR_ARG, "fb_gemv_ex: null y");
    if (!aligned4(y)) return set_error(FB_ERR_ALIGN, "fb_gemv_ex: y must be 4-byte aligned");
    const int yk = (fy.k * 8 == fy.base) ? 0 : fy.k;
    return dispatch_format(fa, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        using N = typename F::native_t;
        if (m == 0) {
            // empty sums: +0, all zero bytes in every format
            k_zero_native<F><<<256, 256, 0, stream>>>(y, n, yk);
            return check_launch("fb_gemv_ex");
        }
        const int64_t ncolunits = n / F::UNIT + (n % F::UNIT ? 1 : 0);   // + the tail unit
        const int64_t nstrips = (ncolunits + 63) / 64;
        constexpr int U = gt_rows<F>();
        constexpr int64_t kChunkRows = (int64_t)kGtWaves * U;     // one chunk per wave
        int64_t nslabs = (gt_target<F>() + nstrips - 1) / nstrips;
        const int64_t max_slabs = (m + 2 * kChunkRows - 1) / (2 * kChunkRows);   // >= 2 chunks per wave
        if (nslabs > max_slabs) nslabs = max_slabs;
        if (nslabs < 1) nslabs = 1;
        int64_t rows = (m + nslabs - 1) / nslabs;
        rows = (rows + kChunkRows - 1) / kChunkRows * kChunkRows;        // slabs hold whole chunks
        nslabs = (m + rows - 1) / rows;
        N* partial = nullptr;
        if (nslabs > 1) {
            void* ws = nullptr;
            fb_status st = stream_workspace(stream, (size_t)nslabs * (size_t)n * sizeof(N), &ws);
            if (st != FB_OK) return st;
            partial = static_cast<N*>(ws);
        }
        dim3 grid((unsigned)nstrips, (unsigned)nslabs);
        k_gemv_t<F, U><<<grid, kGtBlock, 0, stream>>>(static_cast<const uint8_t*>(A), lda * F::k, x, (int)m, (int)n,
                                                       (int)rows, partial, y, yk, fy.round);
        if (partial)
            k_gemv_t_final<F><<<(unsigned)((n + 63) / 64), kGtBlock, 0, stream>>>(partial, (int)nslabs, (int)n, y, yk,
                                                                                fy.round);
        return check_launch("fb_gemv_ex");
    });
}

}  // namespace flyte
