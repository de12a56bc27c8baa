// Streaming kernels over packed arrays: pack, unpack, axpy, scale, dot and
// the vector magnitude (norm).  Kernels that produce packed values take the
// rounding mode of the format as a template parameter.
//
// Every kernel walks the array in units of F::UNIT elements (whole dwords of
// packed data); unpack, which writes W/k times what it reads, uses a unit
// sized by its 16-byte output instead.  pack, unpack, axpy and scale give
// each workgroup a chunk of kBlock * U consecutive units (thread t holds units
// t, t + kBlock, ..., U of them), one chunk per workgroup, so each wave-wide
// memory instruction touches one contiguous span and the workgroups in flight
// sweep a compact stretch of memory (chunk_grid).  dot and the norm, which
// keep one partial sum per workgroup, walk the array grid-stride with at most
// 63 workgroups per CU, a count kept off powers of two (stream_grid).  The
// fewer than a unit of elements after the last whole unit are handled one by
// one with byte accesses by the first threads of block 0.
#include <mutex>
#include <unordered_map>

#include "codec.hpp"
#include "common.hpp"

namespace flyte {

// Streaming loads and stores: every byte is touched once, so a lane's unit
// that one instruction covers (at most 4 dwords: the wave's instruction spans
// one contiguous range) goes through the non-temporal path; units of more
// dwords take two instructions whose spans interleave by lane, and stay on the
// ordinary path (non-temporal there measured slower, as low as 0.75x).
template <int N>
__device__ __forceinline__ void load_stream(const uint32_t* __restrict__ p, uint32_t (&out)[N])
{
    if constexpr (N == 4) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else if constexpr (N == 3) {
        const u32x3 v = __builtin_nontemporal_load(reinterpret_cast<const u32x3*>(p));
        out[0] = v.x; out[1] = v.y; out[2] = v.z;
    } else if constexpr (N == 2) {
        const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
        out[0] = v.x; out[1] = v.y;
    } else if constexpr (N == 1) {
        out[0] = __builtin_nontemporal_load(p);
    } else {
        load_dwords(p, out);
    }
}

template <int N>
__device__ __forceinline__ void store_stream(uint32_t* __restrict__ p, const uint32_t (&in)[N])
{
    if constexpr (N == 4) {
        u32x4 v; v.x = in[0]; v.y = in[1]; v.z = in[2]; v.w = in[3];
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(p));
    } else if constexpr (N == 3) {
        u32x3 v; v.x = in[0]; v.y = in[1]; v.z = in[2];
        __builtin_nontemporal_store(v, reinterpret_cast<u32x3*>(p));
    } else if constexpr (N == 2) {
        u32x2 v; v.x = in[0]; v.y = in[1];
        __builtin_nontemporal_store(v, reinterpret_cast<u32x2*>(p));
    } else if constexpr (N == 1) {
        __builtin_nontemporal_store(in[0], p);
    } else {
        store_dwords(p, in);
    }
}


// Wave-cooperative reads of 64 consecutive lane units of D dwords, D = 5 or 7
// (units a lane alone would read with two instructions whose spans interleave
// by lane): the wave reads the 64 D dwords as lane-contiguous 16-byte chunks,
// non-temporal (span_load), then passes them through its LDS slice so each
// lane gets its own unit (span_unit).  All 64 lanes must be active and the
// whole span in range; base is 16-byte aligned when the array is (a wave's
// first unit is a multiple of 64).
template <int D>
struct SpanChunks {
    u32x4 c0, c1;
};

template <int D>
__device__ __forceinline__ SpanChunks<D> span_load(const uint32_t* __restrict__ base, int lane)
{
    constexpr int CH = 64 * D / 4;   // 16-byte chunks of the span: 80 or 112
    SpanChunks<D> c;
    c.c0 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base) + lane);
    if (64 + lane < CH) c.c1 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base) + 64 + lane);
    return c;
}

template <int D>
__device__ __forceinline__ void span_unit(uint32_t* slice, int lane, const SpanChunks<D>& c, uint32_t (&out)[D])
{
    constexpr int CH = 64 * D / 4;
    *reinterpret_cast<u32x4*>(slice + 4 * lane) = c.c0;
    if (64 + lane < CH) *reinterpret_cast<u32x4*>(slice + 4 * (64 + lane)) = c.c1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < D; ++j) out[j] = slice[D * lane + j];   // odd stride: no bank conflicts
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The reverse: each lane's unit into the LDS slice, then the 64 D dwords
// written as lane-contiguous 16-byte chunks (non-temporal).
template <int D>
__device__ __forceinline__ void span_store(uint32_t* __restrict__ base, uint32_t* slice, int lane, const uint32_t (&in)[D])
{
    constexpr int CH = 64 * D / 4;
#pragma unroll
    for (int j = 0; j < D; ++j) slice[D * lane + j] = in[j];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const u32x4 c0 = *reinterpret_cast<const u32x4*>(slice + 4 * lane);
    u32x4 c1;
    if (64 + lane < CH) c1 = *reinterpret_cast<const u32x4*>(slice + 4 * (64 + lane));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_nontemporal_store(c0, reinterpret_cast<u32x4*>(base) + lane);
    if (64 + lane < CH) __builtin_nontemporal_store(c1, reinterpret_cast<u32x4*>(base) + 64 + lane);
}

constexpr int kBlock = 256;
constexpr int kUnroll = 4;

// ---------------------------------------------------------------- pack
// A lane unit is NE elements (a whole number of dword groups): NE * W bytes
// read, NE * k written.
template <class F, int MODE, int U, int NE>
__global__ void __launch_bounds__(kBlock)
k_pack(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int64_t nunits, int64_t n)
{
    using T = typename F::bits_t;
    static_assert(NE % F::G == 0, "unit must be whole dword groups");
    constexpr int D = NE * F::k / 4;          // packed dwords per lane unit
    constexpr int NW = NE * F::W / 4;         // native dwords per lane unit
    constexpr bool STG = D == 5 || D == 7;   // two-instruction packed units: written as wave spans
    // 32-byte input units (4 binary64 values) would take two load instructions
    // whose spans interleave by lane; when all 64 units of a wave are in range
    // the wave reads its 2 KiB as two lane-contiguous non-temporal KiB and hands
    // each lane its unit through the wave's LDS slice
    constexpr bool ISTG = NW == 8;
    constexpr int SLICE = (ISTG ? 64 * NW : 4) > (STG ? 64 * D : 4) ? (ISTG ? 64 * NW : 4) : (STG ? 64 * D : 4);
    __shared__ __attribute__((aligned(16))) uint32_t slices[(STG || ISTG) ? kBlock / 64 : 1][SLICE];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    constexpr int64_t chunk = (int64_t)kBlock * U;   // units per workgroup chunk
    for (int64_t g0 = (int64_t)blockIdx.x * chunk + threadIdx.x; g0 < nunits; g0 += (int64_t)gridDim.x * chunk) {
        uint32_t w[U][NW];
        u32x4 wc[ISTG ? U : 1][2];
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            if constexpr (ISTG) {
                const int64_t gw = g - lane;   // the wave's first unit (lanes hold consecutive units)
                if (gw + 63 < nunits) {        // wave-uniform: every lane in range and active
                    const u32x4* base = reinterpret_cast<const u32x4*>(src + gw * NW);
                    wc[u][0] = __builtin_nontemporal_load(base + lane);
                    wc[u][1] = __builtin_nontemporal_load(base + 64 + lane);
                    return;
                }
            }
            if (g < nunits) load_stream(src + g * NW, w[u]);
        });
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            if constexpr (ISTG) {
                if (g - lane + 63 < nunits) {
                    uint32_t* sl = slices[wave];
                    *reinterpret_cast<u32x4*>(sl + 4 * lane) = wc[u][0];
                    *reinterpret_cast<u32x4*>(sl + 256 + 4 * lane) = wc[u][1];
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    const u32x4 a0 = *reinterpret_cast<const u32x4*>(sl + 8 * lane);
                    const u32x4 a1 = *reinterpret_cast<const u32x4*>(sl + 8 * lane + 4);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    w[u][0] = a0.x; w[u][1] = a0.y; w[u][2] = a0.z; w[u][3] = a0.w;
                    w[u][4] = a1.x; w[u][5] = a1.y; w[u][6] = a1.z; w[u][7] = a1.w;
                }
            }
            if (g < nunits) {
                T b[NE];
                words_to_bits<F, NE>(w[u], b);
#pragma unroll
                for (int e = 0; e < NE; ++e) b[e] = round_pack<F, MODE>(b[e]);
                uint32_t P[D];
                assemble_elems<F, NE>(b, P);
                if constexpr (STG) {
                    if (g - lane + 63 < nunits) {   // wave-uniform: every lane in range and active
                        span_store<D>(dst + (g - lane) * D, slices[wave], lane, P);
                        return;
                    }
                }
                store_stream(dst + g * D, P);
            }
        });
    }
    if (blockIdx.x == 0) {
        const int64_t i = nunits * NE + threadIdx.x;
        if (threadIdx.x < NE && i < n) {
            T u;
            if constexpr (F::W == 4) u = src[i];
            else u = (uint64_t(src[2 * i + 1]) << 32) | src[2 * i];
            store_elem_bytes<F>(reinterpret_cast<uint8_t*>(dst) + i * F::k, round_pack<F, MODE>(u));
        }
    }
}

// ---------------------------------------------------------------- unpack
template <class F, int U, int NE>
__global__ void __launch_bounds__(kBlock)
k_unpack(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int64_t nunits, int64_t n)
{
    using T = typename F::bits_t;
    constexpr int OW = NE * F::W / 4;    // output dwords per lane unit
    // A unit of 8 output dwords (four binary64 values, odd k) takes two store
    // instructions whose spans interleave by lane; when all 64 units of a wave
    // are in range they go through the wave's LDS slice and leave as two
    // lane-contiguous KiB (non-temporal) instead.
    constexpr bool STAGE = OW == 8;
    __shared__ __attribute__((aligned(16))) uint32_t stage[STAGE ? kBlock / 64 : 1][STAGE ? 64 * OW : 4];
    constexpr int D = NE * F::k / 4;          // input dwords per lane unit
    constexpr bool STG = D == 5 || D == 7;   // two-instruction input units: read as wave spans
    __shared__ __attribute__((aligned(16))) uint32_t slices[STG ? kBlock / 64 : 1][STG ? 64 * D : 4];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    constexpr int64_t chunk = (int64_t)kBlock * U;   // units per workgroup chunk
    if constexpr (!STAGE && !STG) {
        // one instruction per unit each way: each unit is loaded, unpacked and stored
        // before the next is loaded.  With all U loads first and the stores after them,
        // the loop (or any code after the stores) makes the compiler wait for every load
        // before the first store, measured 5-11% slower on 16-byte outputs.
        for (int64_t g0 = (int64_t)blockIdx.x * chunk + threadIdx.x; g0 < nunits; g0 += (int64_t)gridDim.x * chunk) {
            static_for<U>([&](auto iu) {
                const int64_t g = g0 + decltype(iu)::value * kBlock;
                if (g < nunits) {
                    uint32_t P[D], w[OW];
                    load_stream(src + g * D, P);
                    T b[NE];
                    unpack_elems<F, NE>(P, b);
                    bits_to_words<F, NE>(b, w);
                    store_stream(dst + g * OW, w);
                }
            });
        }
    } else for (int64_t g0 = (int64_t)blockIdx.x * chunk + threadIdx.x; g0 < nunits; g0 += (int64_t)gridDim.x * chunk) {
        uint32_t P[U][D];
        SpanChunks<D> SP[STG ? U : 1];
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            if constexpr (STG) {
                const int64_t gw = g - lane;   // the wave's first unit (lanes hold consecutive units)
                if (gw + 63 < nunits) {        // wave-uniform: every lane in range and active
                    SP[u] = span_load<D>(src + gw * D, lane);
                    return;
                }
            }
            if (g < nunits) load_stream(src + g * D, P[u]);
        });
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            if constexpr (STG) {
                if (g - lane + 63 < nunits) span_unit<D>(slices[wave], lane, SP[u], P[u]);
            }
            uint32_t w[OW];
            if (g < nunits) {
                T b[NE];
                unpack_elems<F, NE>(P[u], b);
                bits_to_words<F, NE>(b, w);
            }
            if constexpr (STAGE) {
                const int64_t gw = g - lane;   // the wave's first unit (lanes hold consecutive units)
                if (gw + 63 < nunits) {        // wave-uniform: every lane in range and active
                    *reinterpret_cast<u32x4*>(&stage[wave][lane * 8]) = u32x4{w[0], w[1], w[2], w[3]};
                    *reinterpret_cast<u32x4*>(&stage[wave][lane * 8 + 4]) = u32x4{w[4], w[5], w[6], w[7]};
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    uint32_t v0[4], v1[4];
                    const u32x4 a = *reinterpret_cast<const u32x4*>(&stage[wave][lane * 4]);
                    const u32x4 c = *reinterpret_cast<const u32x4*>(&stage[wave][256 + lane * 4]);
                    v0[0] = a.x; v0[1] = a.y; v0[2] = a.z; v0[3] = a.w;
                    v1[0] = c.x; v1[1] = c.y; v1[2] = c.z; v1[3] = c.w;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    store_stream(dst + gw * OW + lane * 4, v0);
                    store_stream(dst + gw * OW + 256 + lane * 4, v1);
                } else if (g < nunits) {
                    store_stream(dst + g * OW, w);
                }
            } else if (g < nunits) {
                store_stream(dst + g * OW, w);
            }
        });
    }
    if (blockIdx.x == 0) {
        const int64_t i = nunits * NE + threadIdx.x;
        if (threadIdx.x < NE && i < n) {
            const T u = load_elem_unpacked<F>(reinterpret_cast<const uint8_t*>(src) + i * F::k);
            if constexpr (F::W == 4) {
                dst[i] = u;
            } else {
                dst[2 * i] = uint32_t(u);
                dst[2 * i + 1] = uint32_t(u >> 32);
            }
        }
    }
}

// ---------------------------------------------------------------- axpy
template <class F, int MODE, int U>
__global__ void __launch_bounds__(kBlock)
k_axpy(typename F::native_t alpha, const uint32_t* __restrict__ x, uint32_t* __restrict__ y, int64_t nunits,
       int64_t n)
{
    using T = typename F::bits_t;
    constexpr int D = F::UNIT_DW;
    constexpr bool STG = D == 5 || D == 7;   // two-instruction units: read and written as wave spans
    __shared__ __attribute__((aligned(16))) uint32_t slices[STG ? kBlock / 64 : 1][2][STG ? 64 * D : 4];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    constexpr int64_t chunk = (int64_t)kBlock * U;   // units per workgroup chunk
    for (int64_t g0 = (int64_t)blockIdx.x * chunk + threadIdx.x; g0 < nunits; g0 += (int64_t)gridDim.x * chunk) {
        uint32_t PX[U][D], PY[U][D];
        SpanChunks<D> SX[STG ? U : 1], SY[STG ? U : 1];
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            if constexpr (STG) {
                const int64_t gw = g - lane;   // the wave's first unit (lanes hold consecutive units)
                if (gw + 63 < nunits) {        // wave-uniform: every lane in range and active
                    SX[u] = span_load<D>(x + gw * D, lane);
                    SY[u] = span_load<D>(y + gw * D, lane);
                    return;
                }
            }
            if (g < nunits) {
                load_stream(x + g * D, PX[u]);
                load_stream(y + g * D, PY[u]);
            }
        });
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            bool span = false;
            if constexpr (STG) {
                span = g - lane + 63 < nunits;
                if (span) {
                    span_unit<D>(slices[wave][0], lane, SX[u], PX[u]);
                    span_unit<D>(slices[wave][1], lane, SY[u], PY[u]);
                }
            }
            if (g < nunits) {
                T bx[F::UNIT], by[F::UNIT];
                unpack_elems<F, F::UNIT>(PX[u], bx);
                unpack_elems<F, F::UNIT>(PY[u], by);
#pragma unroll
                for (int e = 0; e < F::UNIT; ++e)
                    by[e] = round_pack<F, MODE>(as_bits<F>(fma_n(alpha, as_native<F>(bx[e]), as_native<F>(by[e]))));
                uint32_t P[D];
                assemble_elems<F, F::UNIT>(by, P);
                if constexpr (STG) {
                    if (span) {
                        span_store<D>(y + (g - lane) * D, slices[wave][0], lane, P);
                        return;
                    }
                }
                store_stream(y + g * D, P);
            }
        });
    }
    if (blockIdx.x == 0) {
        const int64_t i = nunits * F::UNIT + threadIdx.x;
        if (threadIdx.x < F::UNIT && i < n) {
            const uint8_t* xb = reinterpret_cast<const uint8_t*>(x) + i * F::k;
            uint8_t* yb = reinterpret_cast<uint8_t*>(y) + i * F::k;
            const auto r = fma_n(alpha, as_native<F>(load_elem_unpacked<F>(xb)),
                                 as_native<F>(load_elem_unpacked<F>(yb)));
            store_elem_bytes<F>(yb, round_pack<F, MODE>(as_bits<F>(r)));
        }
    }
}

// ---------------------------------------------------------------- scale (in place)
template <class F, int MODE, int U>
__global__ void __launch_bounds__(kBlock)
k_scale(typename F::native_t alpha, uint32_t* __restrict__ x, int64_t nunits, int64_t n)
{
    using T = typename F::bits_t;
    constexpr int D = F::UNIT_DW;
    constexpr bool STG = D == 5 || D == 7;   // two-instruction units: read and written as wave spans
    __shared__ __attribute__((aligned(16))) uint32_t slices[STG ? kBlock / 64 : 1][STG ? 64 * D : 4];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    constexpr int64_t chunk = (int64_t)kBlock * U;   // units per workgroup chunk
    for (int64_t g0 = (int64_t)blockIdx.x * chunk + threadIdx.x; g0 < nunits; g0 += (int64_t)gridDim.x * chunk) {
        uint32_t PX[U][D];
        SpanChunks<D> SX[STG ? U : 1];
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            if constexpr (STG) {
                const int64_t gw = g - lane;   // the wave's first unit (lanes hold consecutive units)
                if (gw + 63 < nunits) {        // wave-uniform: every lane in range and active
                    SX[u] = span_load<D>(x + gw * D, lane);
                    return;
                }
            }
            if (g < nunits) load_stream(x + g * D, PX[u]);
        });
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * kBlock;
            bool span = false;
            if constexpr (STG) {
                span = g - lane + 63 < nunits;
                if (span) span_unit<D>(slices[wave], lane, SX[u], PX[u]);
            }
            if (g < nunits) {
                T bx[F::UNIT];
                unpack_elems<F, F::UNIT>(PX[u], bx);
#pragma unroll
                for (int e = 0; e < F::UNIT; ++e) bx[e] = round_pack<F, MODE>(as_bits<F>(alpha * as_native<F>(bx[e])));
                uint32_t P[D];
                assemble_elems<F, F::UNIT>(bx, P);
                if constexpr (STG) {
                    if (span) {
                        span_store<D>(x + (g - lane) * D, slices[wave], lane, P);
                        return;
                    }
                }
                store_stream(x + g * D, P);
            }
        });
    }
    if (blockIdx.x == 0) {
        const int64_t i = nunits * F::UNIT + threadIdx.x;
        if (threadIdx.x < F::UNIT && i < n) {
            uint8_t* xb = reinterpret_cast<uint8_t*>(x) + i * F::k;
            store_elem_bytes<F>(xb, round_pack<F, MODE>(as_bits<F>(alpha * as_native<F>(load_elem_unpacked<F>(xb)))));
        }
    }
}

// ---------------------------------------------------------------- dot
template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
    // xor butterfly: every lane ends with the same, order-fixed total
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

template <class T>
__device__ __forceinline__ T block_sum(T v)
{
    __shared__ T part[kBlock / 64];
    v = wave_sum(v);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) s = s + part[w];
    return s;
}

// SQ: y is x (the sum of squares of fb_nrm2), read once.
template <class F, int U, bool SQ = false>
__global__ void __launch_bounds__(kBlock)
k_dot_partial(const uint32_t* __restrict__ x, const uint32_t* __restrict__ y, int64_t nunits, int64_t n,
              typename F::native_t* __restrict__ partials)
{
    using T = typename F::bits_t;
    using N = typename F::native_t;
    constexpr int D = F::UNIT_DW;
    constexpr bool STG = D == 5 || D == 7;   // two-instruction units: read as wave spans
    __shared__ __attribute__((aligned(16))) uint32_t slices[STG ? kBlock / 64 : 1][2][STG ? 64 * D : 4];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    N acc = N(0);
    for (int64_t g0 = tid; g0 < nunits; g0 += nthreads * U) {
        uint32_t PX[U][D], PY[U][D];
        SpanChunks<D> SX[STG ? U : 1], SY[STG ? U : 1];
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * nthreads;
            if constexpr (STG) {
                const int64_t gw = g - lane;   // the wave's first unit (lanes hold consecutive units)
                if (gw + 63 < nunits) {        // wave-uniform: every lane in range and active
                    SX[u] = span_load<D>(x + gw * D, lane);
                    if constexpr (!SQ) SY[u] = span_load<D>(y + gw * D, lane);
                    return;
                }
            }
            if (g < nunits) {
                load_stream(x + g * D, PX[u]);
                if constexpr (!SQ) load_stream(y + g * D, PY[u]);
            }
        });
        static_for<U>([&](auto iu) {
            constexpr int u = decltype(iu)::value;
            const int64_t g = g0 + u * nthreads;
            if constexpr (STG) {
                if (g - lane + 63 < nunits) {
                    span_unit<D>(slices[wave][0], lane, SX[u], PX[u]);
                    if constexpr (!SQ) span_unit<D>(slices[wave][1], lane, SY[u], PY[u]);
                }
            }
            if (g < nunits) {
                T bx[F::UNIT], by[F::UNIT];
                unpack_elems<F, F::UNIT>(PX[u], bx);
                if constexpr (SQ) unpack_elems<F, F::UNIT>(PX[u], by);
                else unpack_elems<F, F::UNIT>(PY[u], by);
#pragma unroll
                for (int e = 0; e < F::UNIT; ++e) acc = fma_n(as_native<F>(bx[e]), as_native<F>(by[e]), acc);
            }
        });
    }
    if (blockIdx.x == 0) {
        const int64_t i = nunits * F::UNIT + threadIdx.x;
        if (threadIdx.x < F::UNIT && i < n) {
            acc = fma_n(as_native<F>(load_elem_unpacked<F>(reinterpret_cast<const uint8_t*>(x) + i * F::k)),
                        as_native<F>(load_elem_unpacked<F>(reinterpret_cast<const uint8_t*>(y) + i * F::k)), acc);
        }
    }
    const N s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <class N, bool SQRT>
__global__ void __launch_bounds__(kBlock) k_dot_final(const N* __restrict__ partials, int nparts, N* __restrict__ out)
{
    N acc = N(0);
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc = acc + partials[i];
    const N s = block_sum(acc);
    if (threadIdx.x == 0) {
        if constexpr (SQRT) {
            // one correctly rounded square root in the base type
            if constexpr (sizeof(N) == 4) *out = __builtin_sqrtf(s);
            else *out = __builtin_sqrt(s);
        } else {
            *out = s;
        }
    }
}

template <class N>
__global__ void k_store_zero(N* out)
{
    *out = N(0);
}

// Sum of the partials in a fixed order, rounded once to a packed result.
template <class F>
__global__ void __launch_bounds__(kBlock)
k_dot_final_packed(const typename F::native_t* __restrict__ partials, int nparts, uint8_t* __restrict__ out, int rk,
                   int rmode)
{
    using N = typename F::native_t;
    N acc = N(0);
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc = acc + partials[i];
    const N s = block_sum(acc);
    if (threadIdx.x == 0) store_bytes_rt(out, pack_runtime((uint64_t)as_bits<F>(s), F::base, rk, rmode), rk);
}

// ---------------------------------------------------------------- host side
// At most 1984 = 31 x 64 partial sums (not a power of two, see stream_grid).
constexpr int kMaxDotBlocks = 1984;

// Workgroups of a grid-stride launch over nunits lane units.  A lane keeps
// `unroll` units in flight, one grid's worth of units apart; with 16-byte
// units and a power-of-two number of threads those addresses are a power of
// two apart and fall on the same DRAM banks (measured at k = 4 and 8: dot
// 15-17% and axpy 8-11% slower than with a grid of 63 workgroups per CU).  So
// the count is kept off powers of two: at most 63 workgroups per CU, and one
// fewer than any power of two below that.
static int stream_grid(int64_t nunits, int unroll)
{
    const int64_t per_block = (int64_t)kBlock * unroll;
    int64_t blocks = (nunits + per_block - 1) / per_block;
    const int64_t cap = (int64_t)device_cu_count() * 63;
    if (blocks > cap) blocks = cap;
    if (blocks > 2 && (blocks & (blocks - 1)) == 0) blocks -= 1;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

// Workgroups of a chunked launch (pack, unpack, axpy, scale): one chunk of
// kBlock * unroll units per workgroup, so the workgroups in flight at any time
// cover a compact stretch of the arrays (measured with a plain 2 GiB copy:
// 16 KiB per workgroup, 5.9-6.0 TB/s, against 5.3-5.5 for the grid-stride walk
// at any grid size and 5.3-5.7 for chunks of 32-128 KiB).  The kernels still
// loop, so a capped grid stays correct.
static int chunk_grid(int64_t nunits, int unroll)
{
    const int64_t per_block = (int64_t)kBlock * unroll;
    int64_t blocks = (nunits + per_block - 1) / per_block;
    if (blocks > (1 << 30)) blocks = 1 << 30;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

// Partial sums of fb_dot / fb_nrm2 live in the per-stream workspace.
static fb_status dot_workspace(hipStream_t stream, void** out)
{
    return stream_workspace(stream, kMaxDotBlocks * sizeof(double), out);
}

static fb_status check_vec(const char* what, fb_format f, const void* a, const void* b, size_t n)
{
    if (!format_ok(f)) return set_error(FB_ERR_FORMAT, "%s: invalid format {%d,%d}", what, f.base, f.k);
    if (n > (size_t)INT64_MAX / 16) return set_error(FB_ERR_ARG, "%s: n too large", what);
    if (n == 0) return FB_OK;
    if (!a || !b) return set_error(FB_ERR_ARG, "%s: null pointer", what);
    if (!aligned4(a) || !aligned4(b)) return set_error(FB_ERR_ALIGN, "%s: pointers must be 4-byte aligned", what);
    return FB_OK;
}

}  // namespace flyte

using namespace flyte;

extern "C" fb_status fb_pack(fb_format f, const void* src_native, void* dst_packed, size_t n, hipStream_t stream)
{
    fb_status st = check_vec("fb_pack", f, src_native, dst_packed, n);
    if (st != FB_OK || n == 0) return st;
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        // pack reads W/k times what it writes, so its lane unit is sized by the
        // input where whole dword groups allow it: 16 bytes (2 binary64 or 4
        // binary32 values, one lane-contiguous load per wave instruction),
        // else the format's own unit
        constexpr int NE = (F::base == 64 && F::G <= 2) ? 2 : (F::base == 32 && F::G <= 4) ? 4 : F::UNIT;
        const int64_t nunits = (int64_t)(n / NE);
        return dispatch_round(f, [&](auto rt) {
            k_pack<F, decltype(rt)::value, kUnroll, NE><<<chunk_grid(nunits, kUnroll), kBlock, 0, stream>>>(
                static_cast<const uint32_t*>(src_native), static_cast<uint32_t*>(dst_packed), nunits, (int64_t)n);
            return check_launch("fb_pack");
        });
    });
}

extern "C" fb_status fb_unpack(fb_format f, const void* src_packed, void* dst_native, size_t n, hipStream_t stream)
{
    fb_status st = check_vec("fb_unpack", f, src_packed, dst_native, n);
    if (st != FB_OK || n == 0) return st;
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        // unpack writes W/k times what it reads, so its lane unit is sized by the
        // output: 16 bytes (2 binary64 or 4 binary32 values, one store instruction)
        // for binary64 of even k and binary32, else 4 binary64 values (odd k: a
        // whole number of dwords in; 32 bytes out, stored through the wave's LDS
        // slice as two lane-contiguous KiB)
        constexpr int NE = (F::base == 64) ? ((F::k % 2 == 0) ? 2 : 4) : 4;
        static_assert(NE % F::G == 0, "unit must be whole dword groups");
        const int64_t nunits = (int64_t)(n / NE);
        k_unpack<F, kUnroll, NE><<<chunk_grid(nunits, kUnroll), kBlock, 0, stream>>>(
            static_cast<const uint32_t*>(src_packed), static_cast<uint32_t*>(dst_native), nunits, (int64_t)n);
        return check_launch("fb_unpack");
    });
}

extern "C" fb_status fb_axpy(fb_format f, size_t n, double alpha, const void* x, void* y, hipStream_t stream)
{
    fb_status st = check_vec("fb_axpy", f, x, y, n);
    if (st != FB_OK || n == 0) return st;
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        using N = typename F::native_t;
        const int64_t nunits = (int64_t)(n / F::UNIT);
        return dispatch_round(f, [&](auto rt) {
            k_axpy<F, decltype(rt)::value, kUnroll><<<chunk_grid(nunits, kUnroll), kBlock, 0, stream>>>(
                (N)alpha, static_cast<const uint32_t*>(x), static_cast<uint32_t*>(y), nunits, (int64_t)n);
            return check_launch("fb_axpy");
        });
    });
}

// The two launches of a dot product with its partial sums in `partials`
// (room for kMaxDotBlocks native values).  Arguments are validated.
static fb_status dot_launch(fb_format f, size_t n, const void* x, const void* y, void* result, void* partials,
                            hipStream_t stream)
{
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        using N = typename F::native_t;
        const int64_t nunits = (int64_t)(n / F::UNIT);
        int grid = stream_grid(nunits, kUnroll);
        if (grid > kMaxDotBlocks) grid = kMaxDotBlocks;
        k_dot_partial<F, kUnroll><<<grid, kBlock, 0, stream>>>(static_cast<const uint32_t*>(x),
                                                               static_cast<const uint32_t*>(y), nunits,
                                                               (int64_t)n, static_cast<N*>(partials));
        k_dot_final<N, false><<<1, kBlock, 0, stream>>>(static_cast<const N*>(partials), grid, static_cast<N*>(result));
        return check_launch("fb_dot");
    });
}

static fb_status dot_zero(fb_format f, void* result, hipStream_t stream)
{
    return dispatch_format(f, [&](auto tag) {
        using N = typename Fmt<decltype(tag.first)::value, decltype(tag.second)::value>::native_t;
        k_store_zero<N><<<1, 1, 0, stream>>>(static_cast<N*>(result));
        return check_launch("fb_dot");
    });
}

static fb_status dot_check(const char* what, fb_format f, size_t n, const void* x, const void* y, void* result)
{
    if (!result) return set_error(FB_ERR_ARG, "%s: null result", what);
    if (!aligned4(result)) return set_error(FB_ERR_ALIGN, "%s: result must be 4-byte aligned", what);
    return check_vec(what, f, x, y, n);
}

extern "C" fb_status fb_dot(fb_format f, size_t n, const void* x, const void* y, void* result, hipStream_t stream)
{
    fb_status st = dot_check("fb_dot", f, n, x, y, result);
    if (st != FB_OK) return st;
    if (n == 0) return dot_zero(f, result, stream);
    void* ws = nullptr;
    st = dot_workspace(stream, &ws);
    if (st != FB_OK) return st;
    return dot_launch(f, n, x, y, result, ws, stream);
}

// ---------------------------------------------------------------- allocation-free dot
// The partial sums of fb_dot_noalloc live in this array instead of the stream
// workspace: kMaxDotBlocks binary64 values (15.5 KiB), one copy per device,
// kept until the process ends and shared by every call on that device.  Host
// code never names it directly (on the host the name is only a stand-in): its
// device address is looked up once per device and kept.
constexpr size_t kScratchBytes = (size_t)kMaxDotBlocks * sizeof(double);
static __device__ __align__(256) double scratch[kMaxDotBlocks];

static fb_status scratch_address(void** out)
{
    static std::mutex mu;
    static std::unordered_map<int, void*> addr;   // device -> that device's copy of scratch
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(FB_ERR_RUNTIME, "fb_dot_noalloc: hipGetDevice failed");
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(FB_ERR_RUNTIME, "fb_dot_noalloc: hipGetSymbolAddress failed on device %d: %s", dev,
                             hipGetErrorString(e));
        it = addr.emplace(dev, p).first;
    }
    *out = it->second;
    return FB_OK;
}

extern "C" fb_status fb_dot_noalloc(fb_format f, size_t n, const void* x, const void* y, void* result,
                                    hipStream_t stream)
{
    fb_status st = dot_check("fb_dot_noalloc", f, n, x, y, result);
    if (st != FB_OK) return st;
    if (n == 0) return dot_zero(f, result, stream);
    // The partial count is capped at kMaxDotBlocks whatever n is, so every n
    // fits; the check guards the size of the array against a larger cap.
    const size_t need = (size_t)kMaxDotBlocks * (f.base / 8);
    if (need > kScratchBytes)
        return set_error(FB_ERR_UNSUPPORTED, "fb_dot_noalloc: %zu bytes of partial sums exceed the %zu-byte scratch",
                         need, kScratchBytes);
    void* p = nullptr;
    st = scratch_address(&p);
    if (st != FB_OK) return st;
    return dot_launch(f, n, x, y, result, p, stream);
}

extern "C" fb_status fb_dot_packed(fb_format f, fb_format fr, size_t n, const void* x, const void* y, void* result,
                                   hipStream_t stream)
{
    if (!result) return set_error(FB_ERR_ARG, "fb_dot_packed: null result");
    if (!format_ok(fr) || fr.base != f.base)
        return set_error(FB_ERR_FORMAT, "fb_dot_packed: result format must be a valid format of the same base");
    fb_status st = check_vec("fb_dot_packed", f, x, y, n);
    if (st != FB_OK) return st;
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        using N = typename F::native_t;
        void* ws = nullptr;
        fb_status s2 = dot_workspace(stream, &ws);
        if (s2 != FB_OK) return s2;
        const int64_t nunits = (int64_t)(n / F::UNIT);
        int grid = n ? stream_grid(nunits, kUnroll) : 0;
        if (grid > kMaxDotBlocks) grid = kMaxDotBlocks;
        if (grid > 0)
            k_dot_partial<F, kUnroll><<<grid, kBlock, 0, stream>>>(static_cast<const uint32_t*>(x),
                                                                   static_cast<const uint32_t*>(y), nunits,
                                                                   (int64_t)n, static_cast<N*>(ws));
        k_dot_final_packed<F><<<1, kBlock, 0, stream>>>(static_cast<const N*>(ws), grid, static_cast<uint8_t*>(result),
                                                        fr.k, fr.round);
        return check_launch("fb_dot_packed");
    });
}

extern "C" fb_status fb_nrm2(fb_format f, size_t n, const void* x, void* result, hipStream_t stream)
{
    if (!result) return set_error(FB_ERR_ARG, "fb_nrm2: null result");
    if (!aligned4(result)) return set_error(FB_ERR_ALIGN, "fb_nrm2: result must be 4-byte aligned");
    fb_status st = check_vec("fb_nrm2", f, x, x, n);
    if (st != FB_OK) return st;
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        using N = typename F::native_t;
        if (n == 0) {
            k_store_zero<N><<<1, 1, 0, stream>>>(static_cast<N*>(result));
            return check_launch("fb_nrm2");
        }
        void* ws = nullptr;
        fb_status s2 = dot_workspace(stream, &ws);
        if (s2 != FB_OK) return s2;
        const int64_t nunits = (int64_t)(n / F::UNIT);
        int grid = stream_grid(nunits, kUnroll);
        if (grid > kMaxDotBlocks) grid = kMaxDotBlocks;
        k_dot_partial<F, kUnroll, true><<<grid, kBlock, 0, stream>>>(static_cast<const uint32_t*>(x),
                                                                     static_cast<const uint32_t*>(x), nunits,
                                                                     (int64_t)n, static_cast<N*>(ws));
        k_dot_final<N, true><<<1, kBlock, 0, stream>>>(static_cast<const N*>(ws), grid, static_cast<N*>(result));
        return check_launch("fb_nrm2");
    });
}

extern "C" fb_status fb_scale(fb_format f, size_t n, double alpha, void* x, hipStream_t stream)
{
    fb_status st = check_vec("fb_scale", f, x, x, n);
    if (st != FB_OK || n == 0) return st;
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        using N = typename F::native_t;
        const int64_t nunits = (int64_t)(n / F::UNIT);
        return dispatch_round(f, [&](auto rt) {
            k_scale<F, decltype(rt)::value, kUnroll><<<chunk_grid(nunits, kUnroll), kBlock, 0, stream>>>(
                (N)alpha, static_cast<uint32_t*>(x), nunits, (int64_t)n);
            return check_launch("fb_scale");
        });
    });
}
