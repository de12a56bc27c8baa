// Device codec for k-byte ("flyte") floating point on gfx950.
//
// A flyte value derived from an IEEE-754 base type of W bits keeps the sign
// and exponent fields of that type and the top m = 8k - 1 - E mantissa bits
// (Table 1 of Anderson & Gregg, extended to binary64 with k = 2..4 by the
// same rule).  Element i of a packed array occupies bytes [i*k, i*k + k) and
// holds the top k bytes of the little-endian base pattern, in little-endian
// order (the bit-field layout of Section 3.2).
//
// Unpack (Sections 3.2 and 4.1): move the k bytes to the top of the base word
// and zero-fill the rest.  Pack (Sections 5.2 and 5.3): round to nearest even
// at the cut, with carry into the exponent; a NaN is truncated and, if that
// cleared its kept mantissa, given the quiet bit, so it stays NaN.
//
// Memory access: a lane owns a "unit" of UNIT consecutive elements whose
// UNIT*k bytes are a whole number of dwords (a multiple of the dword-aligned
// group of G = 4/gcd(4,k) elements, grown towards 16 bytes), and consecutive
// lanes own consecutive units, so one wave-wide load or store instruction
// covers one contiguous span and no two lanes ever write the same dword (the
// paper's non-overlapping vector stores, Section 4.3).  Inside a unit every
// byte move is a compile-time v_perm_b32: one per binary32 element, one or
// two per binary64 element.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace flyte {

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

template <int BASE, int K>
struct Fmt {
    static_assert((BASE == 32 && K >= 2 && K <= 4) || (BASE == 64 && K >= 2 && K <= 8),
                  "not a flyte format");
    static constexpr int base = BASE;
    static constexpr int k = K;
    static constexpr int W = BASE / 8;                 // native bytes
    static constexpr int E = BASE == 32 ? 8 : 11;      // exponent bits
    static constexpr int D = BASE - 8 * K;             // dropped bits
    static constexpr int M = 8 * K - 1 - E;            // kept mantissa bits
    static constexpr int G = 4 / cgcd(4, K);           // elements per dword-aligned group
    static constexpr int UNIT = G * ((16 / (G * K)) > 1 ? (16 / (G * K)) : 1);  // elements per lane unit
    static constexpr int UNIT_DW = UNIT * K / 4;       // packed dwords per unit
    static constexpr int UNIT_NW = UNIT * W / 4;       // native dwords per unit
    using native_t = std::conditional_t<BASE == 32, float, double>;
    using bits_t = std::conditional_t<BASE == 32, uint32_t, uint64_t>;
};

// ---------------------------------------------------------------- compile-time loops
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

template <int N, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------- byte gather
constexpr int min_valid4(int a, int b, int c, int d)
{
    int m = 1 << 30;
    if (a >= 0 && a < m) m = a;
    if (b >= 0 && b < m) m = b;
    if (c >= 0 && c < m) m = c;
    if (d >= 0 && d < m) m = d;
    return m == (1 << 30) ? -1 : m;
}

// v_perm_b32 selector byte: source byte s taken from the 8-byte window that
// starts at byte `lo` of the stream, or 0x0C (a zero byte) when s is outside.
constexpr uint32_t perm_sel(int s, int lo) { return (s >= lo && s < lo + 8) ? uint32_t(s - lo) : 0x0Cu; }

constexpr uint32_t perm_sel4(int s0, int s1, int s2, int s3, int lo)
{
    return perm_sel(s0, lo) | (perm_sel(s1, lo) << 8) | (perm_sel(s2, lo) << 16) | (perm_sel(s3, lo) << 24);
}

// Byte j of the result is byte Sj of the little-endian byte stream held in the
// dword array S (a negative Sj gives a zero byte).  The four source bytes must
// lie within 16 consecutive stream bytes; every index is a compile-time
// constant, so this is one or two v_perm_b32 (or a plain register move).
template <int S0, int S1, int S2, int S3, int NS>
__device__ __forceinline__ uint32_t gather4(const uint32_t (&S)[NS])
{
    constexpr int lo = min_valid4(S0, S1, S2, S3);
    if constexpr (lo < 0) {
        return 0u;
    } else {
        constexpr int w0 = lo / 4;
        constexpr int b0 = 4 * w0;
        if constexpr (S0 == b0 && S1 == b0 + 1 && S2 == b0 + 2 && S3 == b0 + 3) {
            return S[w0];
        } else {
            constexpr uint32_t selA = perm_sel4(S0, S1, S2, S3, b0);
            constexpr bool needB = S0 >= b0 + 8 || S1 >= b0 + 8 || S2 >= b0 + 8 || S3 >= b0 + 8;
            static_assert(S0 < b0 + 16 && S1 < b0 + 16 && S2 < b0 + 16 && S3 < b0 + 16,
                          "gather window too wide");
            const uint32_t hiA = (w0 + 1 < NS) ? S[(w0 + 1 < NS) ? w0 + 1 : w0] : 0u;
            uint32_t r = __builtin_amdgcn_perm(hiA, S[w0], selA);
            if constexpr (needB) {
                constexpr int w1 = w0 + 2;
                constexpr uint32_t selB = perm_sel4(S0, S1, S2, S3, b0 + 8);
                const uint32_t hiB = (w1 + 1 < NS) ? S[(w1 + 1 < NS) ? w1 + 1 : w1] : 0u;
                r |= __builtin_amdgcn_perm(hiB, S[w1], selB);
            }
            return r;
        }
    }
}

// ---------------------------------------------------------------- unpack
// Source byte of byte t (0 = least significant) of the native pattern of
// element e: the top k bytes come from the stored element, the rest are zero.
template <class F>
constexpr int unpack_src(int e, int t)
{
    return t < F::W - F::k ? -1 : e * F::k + t - (F::W - F::k);
}

// P: the NE*k/4 packed dwords of NE consecutive elements (NE a multiple of
// G); out: their NE native bit patterns.
template <class F, int NE>
__device__ __forceinline__ void unpack_elems(const uint32_t (&P)[NE * F::k / 4],
                                             typename F::bits_t (&out)[NE])
{
    static_assert(NE % F::G == 0, "unit must be whole dword groups");
    static_for<NE>([&](auto ic) {
        constexpr int e = decltype(ic)::value;
        if constexpr (F::base == 32) {
            out[e] = gather4<unpack_src<F>(e, 0), unpack_src<F>(e, 1), unpack_src<F>(e, 2),
                             unpack_src<F>(e, 3)>(P);
        } else {
            const uint32_t lo = gather4<unpack_src<F>(e, 0), unpack_src<F>(e, 1), unpack_src<F>(e, 2),
                                        unpack_src<F>(e, 3)>(P);
            const uint32_t hi = gather4<unpack_src<F>(e, 4), unpack_src<F>(e, 5), unpack_src<F>(e, 6),
                                        unpack_src<F>(e, 7)>(P);
            out[e] = (uint64_t(hi) << 32) | lo;
        }
    });
}

// ---------------------------------------------------------------- pack
// Round to nearest even at the cut.  For a non-NaN pattern u,
// (u + 2^(D-1) - 1 + lsb) >> D rounds up exactly when the dropped part
// exceeds half an ulp, or equals it with an odd kept part; the carry runs
// into the exponent by itself and cannot reach the sign (the largest non-NaN
// input is -Inf, whose dropped bits are zero).  NaN: truncate, and set the
// quiet bit if the kept mantissa became zero.
template <class F>
__device__ __forceinline__ typename F::bits_t rne_pack(typename F::bits_t u)
{
    using T = typename F::bits_t;
    if constexpr (F::D == 0) {
        return u;
    } else {
        constexpr T one = 1;
        constexpr T abs_mask = (one << (F::base - 1)) - 1;
        constexpr T inf_bits = ((one << F::E) - 1) << (F::base - 1 - F::E);
        constexpr T half_m1 = (one << (F::D - 1)) - 1;
        constexpr T kept_mant = (one << F::M) - 1;
        constexpr T quiet = one << (F::M - 1);
        const T q = u >> F::D;
        const T r = (u + half_m1 + (q & one)) >> F::D;
        const T qn = ((q & kept_mant) == 0) ? (q | quiet) : q;
        return ((u & abs_mask) > inf_bits) ? qn : r;
    }
}

// Pack in a rounding mode: 0 nearest even (above), 1 toward zero (drop the
// low bytes; Section 5.1), 2 to odd (drop them and set the lowest kept bit if
// any dropped bit was set; Section 7).  NaNs take the same rule in every mode.
template <class F, int MODE>
__device__ __forceinline__ typename F::bits_t round_pack(typename F::bits_t u)
{
    using T = typename F::bits_t;
    if constexpr (MODE == 0 || F::D == 0) {
        return rne_pack<F>(u);
    } else {
        constexpr T one = 1;
        constexpr T abs_mask = (one << (F::base - 1)) - 1;
        constexpr T inf_bits = ((one << F::E) - 1) << (F::base - 1 - F::E);
        constexpr T kept_mant = (one << F::M) - 1;
        constexpr T quiet = one << (F::M - 1);
        constexpr T dropped = (one << F::D) - 1;
        const T q = u >> F::D;
        const T qn = ((q & kept_mant) == 0) ? (q | quiet) : q;
        T r = q;
        if constexpr (MODE == 2) r = q | (T)((u & dropped) != 0);
        return ((u & abs_mask) > inf_bits) ? qn : r;
    }
}

// Pack with the format given at run time (base width W = 32 or 64, k bytes,
// rounding mode): the same rules as round_pack, with runtime shift amounts.
// Used where one value is packed per result (GEMV/dot outputs), so the cost
// of variable shifts does not matter.
__device__ __forceinline__ uint64_t pack_runtime(uint64_t u, int W, int k, int mode)
{
    const int E = W == 32 ? 8 : 11;
    const int D = W - 8 * k;
    if (D == 0) return u;
    const int M = 8 * k - 1 - E;
    const uint64_t one = 1;
    const uint64_t abs_mask = (W == 64) ? ~(one << 63) : ((one << 31) - 1);
    const uint64_t inf_bits = ((one << E) - 1) << (W - 1 - E);
    const uint64_t q = u >> D;
    if ((u & abs_mask) > inf_bits) return ((q & ((one << M) - 1)) == 0) ? (q | (one << (M - 1))) : q;
    if (mode == 0) return (u + ((one << (D - 1)) - 1) + (q & one)) >> D;
    if (mode == 2) return q | (uint64_t)((u & ((one << D) - 1)) != 0);
    return q;
}

__device__ __forceinline__ void store_bytes_rt(uint8_t* p, uint64_t q, int k)
{
    for (int j = 0; j < k; ++j) p[j] = uint8_t(q >> (8 * j));
}

// Stream byte that holds byte bi of packed element e, when the packed values
// sit one per native word (low k bytes of a 4- or 8-byte word).
template <class F>
constexpr int pack_src(int p)
{
    return (p / F::k) * F::W + (p % F::k);
}

// q: NE packed values (low k bytes of each word); out: NE*k/4 dwords.
template <class F, int NE>
__device__ __forceinline__ void assemble_elems(const typename F::bits_t (&q)[NE],
                                               uint32_t (&out)[NE * F::k / 4])
{
    static_assert(NE % F::G == 0, "unit must be whole dword groups");
    constexpr int NS = NE * F::W / 4;
    uint32_t S[NS];
    static_for<NE>([&](auto ic) {
        constexpr int e = decltype(ic)::value;
        if constexpr (F::base == 32) {
            S[e] = q[e];
        } else {
            S[2 * e] = uint32_t(q[e]);
            S[2 * e + 1] = uint32_t(q[e] >> 32);
        }
    });
    static_for<NE * F::k / 4>([&](auto iw) {
        constexpr int w = decltype(iw)::value;
        out[w] = gather4<pack_src<F>(4 * w), pack_src<F>(4 * w + 1), pack_src<F>(4 * w + 2),
                         pack_src<F>(4 * w + 3)>(S);
    });
}

// ---------------------------------------------------------------- value helpers
template <class F>
__device__ __forceinline__ typename F::native_t as_native(typename F::bits_t u)
{
    if constexpr (F::base == 32) return __uint_as_float(u);
    else return __longlong_as_double((long long)u);
}

template <class F>
__device__ __forceinline__ typename F::bits_t as_bits(typename F::native_t v)
{
    if constexpr (F::base == 32) return __float_as_uint(v);
    else return (uint64_t)__double_as_longlong(v);
}

// Explicit fused multiply-add in the base type (FP_CONTRACT on, Section 4.4).
__device__ __forceinline__ float fma_n(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_n(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- scalar element access (tails)
// Unpacked bit pattern of the element whose k bytes start at p (byte loads).
template <class F>
__device__ __forceinline__ typename F::bits_t load_elem_unpacked(const uint8_t* p)
{
    typename F::bits_t q = 0;
#pragma unroll
    for (int j = 0; j < F::k; ++j) q |= typename F::bits_t(p[j]) << (8 * j);
    return q << F::D;
}

// Stores the k bytes of packed value q at p (byte stores).
template <class F>
__device__ __forceinline__ void store_elem_bytes(uint8_t* p, typename F::bits_t q)
{
#pragma unroll
    for (int j = 0; j < F::k; ++j) p[j] = uint8_t(q >> (8 * j));
}

// ---------------------------------------------------------------- vector memory
// Multi-dword accesses that need only 4-byte alignment (gfx9 memory
// instructions accept any dword-aligned address for dwordx2/x3/x4).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3), aligned(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4), aligned(4)));

template <int N>
__device__ __forceinline__ void load_dwords(const uint32_t* __restrict__ p, uint32_t (&out)[N])
{
    static_for<(N + 3) / 4>([&](auto iv) {
        constexpr int o = 4 * decltype(iv)::value;
        constexpr int r = N - o < 4 ? N - o : 4;
        if constexpr (r == 4) {
            const u32x4 v = *reinterpret_cast<const u32x4*>(p + o);
            out[o] = v.x; out[o + 1] = v.y; out[o + 2] = v.z; out[o + 3] = v.w;
        } else if constexpr (r == 3) {
            const u32x3 v = *reinterpret_cast<const u32x3*>(p + o);
            out[o] = v.x; out[o + 1] = v.y; out[o + 2] = v.z;
        } else if constexpr (r == 2) {
            const u32x2 v = *reinterpret_cast<const u32x2*>(p + o);
            out[o] = v.x; out[o + 1] = v.y;
        } else {
            out[o] = p[o];
        }
    });
}

template <int N>
__device__ __forceinline__ void store_dwords(uint32_t* __restrict__ p, const uint32_t (&in)[N])
{
    static_for<(N + 3) / 4>([&](auto iv) {
        constexpr int o = 4 * decltype(iv)::value;
        constexpr int r = N - o < 4 ? N - o : 4;
        if constexpr (r == 4) {
            u32x4 v; v.x = in[o]; v.y = in[o + 1]; v.z = in[o + 2]; v.w = in[o + 3];
            *reinterpret_cast<u32x4*>(p + o) = v;
        } else if constexpr (r == 3) {
            u32x3 v; v.x = in[o]; v.y = in[o + 1]; v.z = in[o + 2];
            *reinterpret_cast<u32x3*>(p + o) = v;
        } else if constexpr (r == 2) {
            u32x2 v; v.x = in[o]; v.y = in[o + 1];
            *reinterpret_cast<u32x2*>(p + o) = v;
        } else {
            p[o] = in[o];
        }
    });
}

// Native words -> bit patterns and back.
template <class F, int NE>
__device__ __forceinline__ void words_to_bits(const uint32_t (&w)[NE * F::W / 4], typename F::bits_t (&u)[NE])
{
    static_for<NE>([&](auto ie) {
        constexpr int e = decltype(ie)::value;
        if constexpr (F::base == 32) u[e] = w[e];
        else u[e] = (uint64_t(w[2 * e + 1]) << 32) | w[2 * e];
    });
}

template <class F, int NE>
__device__ __forceinline__ void bits_to_words(const typename F::bits_t (&u)[NE], uint32_t (&w)[NE * F::W / 4])
{
    static_for<NE>([&](auto ie) {
        constexpr int e = decltype(ie)::value;
        if constexpr (F::base == 32) {
            w[e] = u[e];
        } else {
            w[2 * e] = uint32_t(u[e]);
            w[2 * e + 1] = uint32_t(u[e] >> 32);
        }
    });
}

}  // namespace flyte
