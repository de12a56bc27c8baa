// Transposed GEMV y = A^T x over a packed row-major A (m x n): y_j = sum_i
// A_ij x_i, the other access order of the paper's BLAS level-2 kernel.
//
// A workgroup of 256 threads owns a strip of 256 consecutive column units and
// a slab of consecutive rows; each thread walks its unit down the slab's rows
// (U rows per loop trip), so every wave-wide load reads one contiguous span of
// a row, and accumulates UNIT column sums with fma in the base type; x_i is
// the same for the whole workgroup.  With more than one slab, the slab sums go
// to a per-stream workspace and a second kernel adds them in slab order, so
// the result is a fixed sequence of operations; the last step writes y native
// or packed (one rounding, byte stores).
#include "codec.hpp"
#include "common.hpp"

namespace flyte {

constexpr int kGtBlock = 256;

template <class F, int U>
__global__ void __launch_bounds__(kGtBlock)
k_gemv_t(const uint8_t* __restrict__ A, int64_t row_bytes, const void* __restrict__ xv, int m, int n, int rows_per_slab,
         typename F::native_t* __restrict__ partial, void* __restrict__ y, int yk, int ymode)
{
    using T = typename F::bits_t;
    using N = typename F::native_t;
    const N* x = static_cast<const N*>(xv);
    const int64_t nunits = n / F::UNIT;
    const int64_t g = (int64_t)blockIdx.x * kGtBlock + threadIdx.x;     // column unit of this thread
    const int r0 = blockIdx.y * rows_per_slab;
    const int r1 = min(m, r0 + rows_per_slab);
    N acc[F::UNIT];
#pragma unroll
    for (int e = 0; e < F::UNIT; ++e) acc[e] = N(0);
    const int tail = (int)(n - nunits * F::UNIT);   // columns after the last whole unit
    if (g < nunits) {
        int r = r0;
        for (; r + U <= r1; r += U) {
            uint32_t P[U][F::UNIT_DW];
#pragma unroll
            for (int u = 0; u < U; ++u)
                load_dwords(reinterpret_cast<const uint32_t*>(A + (int64_t)(r + u) * row_bytes) + g * F::UNIT_DW, P[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                T ab[F::UNIT];
                unpack_elems<F, F::UNIT>(P[u], ab);
                const N xr = x[r + u];
#pragma unroll
                for (int e = 0; e < F::UNIT; ++e) acc[e] = fma_n(as_native<F>(ab[e]), xr, acc[e]);
            }
        }
        for (; r < r1; ++r) {
            uint32_t P[F::UNIT_DW];
            load_dwords(reinterpret_cast<const uint32_t*>(A + (int64_t)r * row_bytes) + g * F::UNIT_DW, P);
            T ab[F::UNIT];
            unpack_elems<F, F::UNIT>(P, ab);
            const N xr = x[r];
#pragma unroll
            for (int e = 0; e < F::UNIT; ++e) acc[e] = fma_n(as_native<F>(ab[e]), xr, acc[e]);
        }
    } else if (g == nunits && tail > 0) {
        for (int r = r0; r < r1; ++r) {
            const uint8_t* row = A + (int64_t)r * row_bytes;
            const N xr = x[r];
            for (int e = 0; e < tail; ++e)
                acc[e] = fma_n(as_native<F>(load_elem_unpacked<F>(row + (nunits * F::UNIT + e) * F::k)), xr, acc[e]);
        }
    } else {
        return;
    }
    const int ncols = g < nunits ? F::UNIT : tail;
#pragma unroll
    for (int e = 0; e < F::UNIT; ++e) {
        if (e >= ncols) break;
        const int64_t c = g * F::UNIT + e;
        if (partial) {
            partial[(int64_t)blockIdx.y * n + c] = acc[e];
        } else if (yk == 0) {
            static_cast<N*>(y)[c] = acc[e];
        } else {
            store_bytes_rt(static_cast<uint8_t*>(y) + c * yk, pack_runtime((uint64_t)as_bits<F>(acc[e]), F::base, yk, ymode),
                           yk);
        }
    }
}

template <class F>
__global__ void __launch_bounds__(kGtBlock)
k_gemv_t_final(const typename F::native_t* __restrict__ partial, int nslabs, int n, void* __restrict__ y, int yk,
               int ymode)
{
    using N = typename F::native_t;
    const int64_t c = (int64_t)blockIdx.x * kGtBlock + threadIdx.x;
    if (c >= n) return;
    N s = N(0);
    for (int q = 0; q < nslabs; ++q) s = s + partial[(int64_t)q * n + c];
    if (yk == 0) static_cast<N*>(y)[c] = s;
    else store_bytes_rt(static_cast<uint8_t*>(y) + c * yk, pack_runtime((uint64_t)as_bits<F>(s), F::base, yk, ymode), yk);
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
    const int yk = (fy.k * 8 == fy.base) ? 0 : fy.k;
    return dispatch_format(fa, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        using N = typename F::native_t;
        if (m == 0) {
            // empty sums: +0, all zero bytes in every format
            k_zero_native<F><<<256, 256, 0, stream>>>(y, n, yk);
            return check_launch("fb_gemv_ex");
        }
        const int64_t ncolunits = n / F::UNIT + 1;            // + the tail unit
        const int64_t nstrips = (ncolunits + kGtBlock - 1) / kGtBlock;
        int64_t nslabs = (2048 + nstrips - 1) / nstrips;       // aim for ~2048 workgroups
        const int64_t max_slabs = (m + 15) / 16;               // at least 16 rows per slab
        if (nslabs > max_slabs) nslabs = max_slabs;
        if (nslabs < 1) nslabs = 1;
        const int64_t rows = (m + nslabs - 1) / nslabs;
        nslabs = (m + rows - 1) / rows;
        N* partial = nullptr;
        if (nslabs > 1) {
            void* ws = nullptr;
            fb_status st = stream_workspace(stream, (size_t)nslabs * (size_t)n * sizeof(N), &ws);
            if (st != FB_OK) return st;
            partial = static_cast<N*>(ws);
        }
        dim3 grid((unsigned)nstrips, (unsigned)nslabs);
        k_gemv_t<F, 4><<<grid, kGtBlock, 0, stream>>>(static_cast<const uint8_t*>(A), lda * F::k, x, (int)m, (int)n,
                                                       (int)rows, partial, y, yk, fy.round);
        if (partial)
            k_gemv_t_final<F><<<(unsigned)((n + kGtBlock - 1) / kGtBlock), kGtBlock, 0, stream>>>(partial, (int)nslabs,
                                                                                              (int)n, y, yk, fy.round);
        return check_launch("fb_gemv_ex");
    });
}

}  // namespace flyte
