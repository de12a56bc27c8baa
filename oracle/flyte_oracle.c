/*
 * flyte oracle -- TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.
 *
 * A plain, slow, obviously-correct CPU model of the multibyte ("flyte")
 * floating-point storage scheme of Anderson & Gregg, "Vectorization of
 * Multibyte Floating Point Data Formats" (PACT 2016).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load this code; the
 * HIP library never includes, links or calls it, and it includes nothing from
 * the library.
 *
 * Notation (Section 3.1 and Table 1 of the paper): a flyte value derived from
 * an IEEE-754 base type of W bits (binary32 or binary64) keeps the sign and
 * the full exponent field of that base type and cuts the mantissa at a byte
 * boundary, so it occupies k whole bytes.
 *   W = base width, E = exponent bits (8 or 11), d = W - 8k dropped bits,
 *   m = 8k - 1 - E kept mantissa bits.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - Byte order: the stored bytes of an element are the top k bytes of the
 *     little-endian base pattern, kept in little-endian order (the bit-field
 *     class of Section 3.2 on x86).  Element i occupies bytes [i*k, i*k+k).
 *   - Rounding on pack is round-to-nearest-even decided by the guard, round,
 *     sticky and pre-guard bits (Section 5.2); the increment may carry into
 *     the exponent (next binade, or infinity from the largest finite value).
 *   - NaN on pack: the kept bits are truncated; if that leaves the kept
 *     mantissa zero, its top (quiet) bit is set so the value stays NaN; the
 *     sign is kept (Section 5.3, NaN values; Section 5.1 for truncation of
 *     quiet NaNs).
 *   - binary64 with k = 2, 3, 4 follows the same rule, m = 8k - 12.
 *   - Rounding modes other than nearest-even (Section 5.1 round toward zero;
 *     Section 7 round to odd after Boldo and Melquiond) decide only the
 *     finite/infinite inputs; NaNs follow the same NaN rule in every mode.
 *
 * Build: plain C11, compiled with -O2 -ffp-contract=off so that every fused
 * multiply-add below is the explicit fma()/fmaf() call and nothing else.
 *
 * MUTATION hooks: building with -DFBO_MUTATION=<n> plants one deliberate
 * mistake, so the test suite can show that its pins catch it:
 *   1 = ties round away from zero (P bit ignored)
 *   2 = NaN fix dropped (plain round-to-nearest applied to NaNs)
 *   3 = the add-half-ULP heuristic of Section 5.2 (no tie rule, no NaN fix)
 *   4 = unpack shifts by one byte too few (wrong alignment of stored bytes)
 *   5 = sign bit lost on pack
 *   6 = round to odd that never sets the lowest bit (plain truncation)
 *   7 = the exact accumulator ignores the sign of products
 *   8 = the transposed GEMV multiplies column c by x in reversed row order
 *   9 = axpy computes alpha*y + x
 *  10 = the naive dot rounds each product before adding (no contraction)
 *  11 = axpy ignores its rounding mode (always nearest even)
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>

#ifndef FBO_MUTATION
#define FBO_MUTATION 0
#endif

/* ------------------------------------------------------------------ */
/* Format description (Table 1, extended to binary64 k = 2..4).         */
/* ------------------------------------------------------------------ */

/* Returns 1 when {base, k} names a flyte format: binary32 with k = 2..4 or
 * binary64 with k = 2..8. */
int fbo_format_valid(int base, int k)
{
    if (base == 32) return k >= 2 && k <= 4;
    if (base == 64) return k >= 2 && k <= 8;
    return 0;
}

static int exp_bits(int base) { return base == 32 ? 8 : 11; }

/* Kept mantissa bits m = 8k - 1 - E. */
int fbo_mant_bits(int base, int k) { return 8 * k - 1 - exp_bits(base); }

static uint64_t low_mask(int bits)
{
    return bits >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << bits) - 1);
}

/* ------------------------------------------------------------------ */
/* C1: unpack one element (Section 3.2 and Section 4.1).                */
/* The stored k-byte integer is moved up to the base width and the      */
/* dropped low bytes are filled with zeros.  No special cases.          */
/* ------------------------------------------------------------------ */
uint64_t fbo_unpack_bits(int base, int k, uint64_t q)
{
    int d = base - 8 * k;
#if FBO_MUTATION == 4
    d -= 8;
    if (d < 0) d = 0;
#endif
    return (q << d) & low_mask(base);
}

/* ------------------------------------------------------------------ */
/* C2: pack one element (Sections 5.2 and 5.3).                         */
/* ------------------------------------------------------------------ */
uint64_t fbo_pack_bits(int base, int k, uint64_t u)
{
    const int W = base;
    const int E = exp_bits(base);
    const int d = W - 8 * k;              /* dropped bits */
    const int m = 8 * k - 1 - E;          /* kept mantissa bits */
    u &= low_mask(W);
    if (d == 0) return u;                 /* the base type itself */

    const uint64_t expo = (u >> (W - 1 - E)) & low_mask(E);
    const uint64_t frac = u & low_mask(W - 1 - E);
    const int is_nan = (expo == low_mask(E)) && frac != 0;

    /* Truncation keeps the top k bytes: sign, exponent, top m mantissa bits. */
    uint64_t q = u >> d;

#if FBO_MUTATION == 3
    /* The paper's add-half-ULP heuristic (negative control). */
    (void)is_nan; (void)m;
    return ((u + ((uint64_t)1 << (d - 1))) & low_mask(W)) >> d;
#endif

    if (is_nan
#if FBO_MUTATION == 2
        && 0
#endif
       ) {
        /* NaN stays NaN: truncation may have cleared every kept mantissa bit
         * (a signalling NaN whose payload sat in the dropped bytes); then the
         * top kept mantissa bit, the quiet bit, is set.  The sign is kept and
         * no rounding increment is applied. */
        if ((q & low_mask(m)) == 0) q |= (uint64_t)1 << (m - 1);
        return q;
    }

    /* Round to nearest, ties to even, from the bits around the cut:
     *   P = pre-guard bit (lowest kept bit),
     *   G = guard bit (first dropped bit),
     *   R = round bit (second dropped bit),
     *   S = sticky bit (OR of every lower dropped bit). */
    const int P = (int)(q & 1);
    const int G = (int)((u >> (d - 1)) & 1);
    const int R = (int)((u >> (d - 2)) & 1);
    const int S = (u & low_mask(d - 2)) != 0;
#if FBO_MUTATION == 1
    const int up = G;                     /* ties away from zero */
    (void)P; (void)R; (void)S;
#else
    const int up = G && (R || S || P);
#endif
    /* The increment may carry out of the mantissa into the exponent: that is
     * the correct result (next binade; infinity above the largest finite
     * value).  It never reaches the sign: a finite input has an exponent
     * below all-ones, and an infinity has no dropped bits set. */
    if (up) q += 1;
#if FBO_MUTATION == 5
    q &= low_mask(8 * k - 1);
#endif
    return q;
}

/* ------------------------------------------------------------------ */
/* Pack with a rounding mode: 0 nearest even (above), 1 toward zero      */
/* (Section 5.1: drop the low bytes), 2 to odd (Section 7: drop the low  */
/* bytes and, if any dropped bit was set, force the lowest kept bit to   */
/* 1).  NaNs are handled as in the nearest-even pack.                    */
/* ------------------------------------------------------------------ */
enum { FBO_RNE = 0, FBO_RTZ = 1, FBO_RTO = 2 };

uint64_t fbo_pack_bits_mode(int base, int k, uint64_t u, int mode)
{
    if (mode == FBO_RNE) return fbo_pack_bits(base, k, u);
    const int W = base;
    const int E = exp_bits(base);
    const int d = W - 8 * k;
    const int m = 8 * k - 1 - E;
    u &= low_mask(W);
    if (d == 0) return u;
    const uint64_t expo = (u >> (W - 1 - E)) & low_mask(E);
    const uint64_t frac = u & low_mask(W - 1 - E);
    uint64_t q = u >> d;
    if (expo == low_mask(E) && frac != 0) {          /* NaN */
        if ((q & low_mask(m)) == 0) q |= (uint64_t)1 << (m - 1);
        return q;
    }
    if (mode == FBO_RTO) {
        const int inexact = (u & low_mask(d)) != 0;
#if FBO_MUTATION == 6
        (void)inexact;
#else
        if (inexact) q |= 1;                          /* the odd neighbour */
#endif
    }
    return q;                                         /* toward zero: truncation */
}

/* ------------------------------------------------------------------ */
/* Arrays of packed elements (Section 4.1: consecutive, no padding).    */
/* ------------------------------------------------------------------ */
static uint64_t load_elem(const uint8_t *p, int k, size_t i)
{
    uint64_t q = 0;
    for (int j = 0; j < k; ++j) q |= (uint64_t)p[i * (size_t)k + j] << (8 * j);
    return q;
}

static void store_elem(uint8_t *p, int k, size_t i, uint64_t q)
{
    for (int j = 0; j < k; ++j) p[i * (size_t)k + j] = (uint8_t)(q >> (8 * j));
}

static uint64_t load_native_bits(const void *p, int base, size_t i)
{
    if (base == 32) { uint32_t v; memcpy(&v, (const uint8_t *)p + 4 * i, 4); return v; }
    uint64_t v; memcpy(&v, (const uint8_t *)p + 8 * i, 8); return v;
}

static void store_native_bits(void *p, int base, size_t i, uint64_t v)
{
    if (base == 32) { uint32_t w = (uint32_t)v; memcpy((uint8_t *)p + 4 * i, &w, 4); return; }
    memcpy((uint8_t *)p + 8 * i, &v, 8);
}

/* dst_native[i] = C1(src_packed[i]) for i < n. */
void fbo_unpack(int base, int k, const uint8_t *src, void *dst, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        store_native_bits(dst, base, i, fbo_unpack_bits(base, k, load_elem(src, k, i)));
}

/* dst_packed[i] = C2(src_native[i]) for i < n. */
void fbo_pack(int base, int k, const void *src, uint8_t *dst, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        store_elem(dst, k, i, fbo_pack_bits(base, k, load_native_bits(src, base, i)));
}

void fbo_pack_mode(int base, int k, int mode, const void *src, uint8_t *dst, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        store_elem(dst, k, i, fbo_pack_bits_mode(base, k, load_native_bits(src, base, i), mode));
}

static double elem_value(int base, int k, const uint8_t *p, size_t i)
{
    uint64_t u = fbo_unpack_bits(base, k, load_elem(p, k, i));
    if (base == 32) { uint32_t w = (uint32_t)u; float f; memcpy(&f, &w, 4); return (double)f; }
    double v; memcpy(&v, &u, 8); return v;
}

static uint64_t bits_of_double(double v) { uint64_t u; memcpy(&u, &v, 8); return u; }
static uint32_t bits_of_float(float v) { uint32_t u; memcpy(&u, &v, 4); return u; }

/* ------------------------------------------------------------------ */
/* C3 axpy: y[i] <- pack(fma(alpha, unpack(x[i]), unpack(y[i]))).       */
/* Arithmetic is in the base type (Section 3.1: convert to the next     */
/* largest native type, compute there, convert back); the multiply-add  */
/* is contracted (FP_CONTRACT on, Section 4.4 and Section 6).  alpha is */
/* first rounded to the base type.                                      */
/* ------------------------------------------------------------------ */
void fbo_axpy_mode(int base, int k, int mode, size_t n, double alpha, const uint8_t *x, uint8_t *y)
{
    for (size_t i = 0; i < n; ++i) {
        uint64_t r;
#if FBO_MUTATION == 9
        const uint8_t *xa = y, *ya = x;
#else
        const uint8_t *xa = x, *ya = y;
#endif
        if (base == 32) {
            float a = (float)alpha;
            float xi = (float)elem_value(base, k, xa, i);
            float yi = (float)elem_value(base, k, ya, i);
            r = bits_of_float(fmaf(a, xi, yi));
        } else {
            double xi = elem_value(base, k, xa, i);
            double yi = elem_value(base, k, ya, i);
            r = bits_of_double(fma(alpha, xi, yi));
        }
#if FBO_MUTATION == 11
        store_elem(y, k, i, fbo_pack_bits(base, k, r));
#else
        store_elem(y, k, i, fbo_pack_bits_mode(base, k, r, mode));
#endif
    }
}

/* axpy with the default cut, round to nearest even. */
void fbo_axpy(int base, int k, size_t n, double alpha, const uint8_t *x, uint8_t *y)
{
    fbo_axpy_mode(base, k, FBO_RNE, n, alpha, x, y);
}

/* The paper's in-place BLAS-1 "scale" program: x[i] <- pack(alpha * x[i]),
 * one multiplication in the base type (alpha first rounded to it). */
void fbo_scale(int base, int k, int mode, size_t n, double alpha, uint8_t *x)
{
    for (size_t i = 0; i < n; ++i) {
        uint64_t r;
        if (base == 32) r = bits_of_float((float)alpha * (float)elem_value(base, k, x, i));
        else r = bits_of_double(alpha * elem_value(base, k, x, i));
        store_elem(x, k, i, fbo_pack_bits_mode(base, k, r, mode));
    }
}

/* ------------------------------------------------------------------ */
/* Dot products.                                                        */
/* naive: sequential fma in the base type, the AT_LEAST accumulator of  */
/*        Section 4.4 held in the base type.                            */
/* exact: the real value of sum x_i*y_i, rounded once to nearest-even   */
/*        in the base type, computed with a long fixed-point            */
/*        accumulator (Kulisch's exact scalar product).                 */
/* ------------------------------------------------------------------ */
double fbo_dot_naive(int base, int k, size_t n, const uint8_t *x, const uint8_t *y)
{
    if (base == 32) {
        float s = 0.0f;
        for (size_t i = 0; i < n; ++i)
            s = fmaf((float)elem_value(base, k, x, i), (float)elem_value(base, k, y, i), s);
        return (double)s;
    }
    double s = 0.0;
#if FBO_MUTATION == 10
    for (size_t i = 0; i < n; ++i) {
        volatile double p = elem_value(base, k, x, i) * elem_value(base, k, y, i);
        s = s + p;
    }
#else
    for (size_t i = 0; i < n; ++i) s = fma(elem_value(base, k, x, i), elem_value(base, k, y, i), s);
#endif
    return s;
}

/* Long accumulator.  Bit 0 has weight 2^-2148, the smallest product of two
 * binary64 values (2^-1074 squared).  The largest product is below 2^2048,
 * so 2^40 such terms stay below 2^2088; ACC_LIMBS*64 = 4480 bits cover that
 * range with room for a two's-complement sign. */
#define ACC_LIMBS 70
#define ACC_BIAS 2148

typedef struct {
    uint64_t limb[ACC_LIMBS];
    int nan;        /* an invalid product or Inf - Inf was seen */
    int pos_inf;    /* +Inf product seen */
    int neg_inf;    /* -Inf product seen */
} longacc;

static void acc_init(longacc *a) { memset(a, 0, sizeof *a); }

/* Adds (neg ? -1 : 1) * mag * 2^(shift - ACC_BIAS), mag < 2^106. */
static void acc_add(longacc *a, int neg, unsigned __int128 mag, int shift)
{
    uint64_t part[ACC_LIMBS];
    memset(part, 0, sizeof part);
    int L = shift / 64, b = shift % 64;
    uint64_t lo = (uint64_t)mag, hi = (uint64_t)(mag >> 64);
    /* mag << b spread over three limbs */
    part[L] = lo << b;
    uint64_t c1 = b ? (lo >> (64 - b)) | (hi << b) : hi;
    uint64_t c2 = b ? (hi >> (64 - b)) : 0;
    if (L + 1 < ACC_LIMBS) part[L + 1] = c1;
    if (L + 2 < ACC_LIMBS) part[L + 2] = c2;
    if (neg) {
        /* two's complement negate of part */
        int carry = 1;
        for (int i = 0; i < ACC_LIMBS; ++i) {
            uint64_t v = ~part[i];
            uint64_t s = v + (uint64_t)carry;
            carry = (carry && s == 0) ? 1 : 0;
            part[i] = s;
        }
    }
    unsigned __int128 carry = 0;
    for (int i = 0; i < ACC_LIMBS; ++i) {
        unsigned __int128 s = (unsigned __int128)a->limb[i] + part[i] + carry;
        a->limb[i] = (uint64_t)s;
        carry = s >> 64;
    }
}

/* Splits a finite double into integer mantissa and exponent: v = M * 2^e. */
static void split_double(double v, int *neg, uint64_t *M, int *e)
{
    uint64_t u = bits_of_double(v);
    *neg = (int)(u >> 63);
    uint64_t be = (u >> 52) & 0x7FF, fr = u & low_mask(52);
    if (be == 0) { *M = fr; *e = -1074; }
    else { *M = fr | ((uint64_t)1 << 52); *e = (int)be - 1075; }
}

static void acc_add_product(longacc *a, double x, double y)
{
    if (isnan(x) || isnan(y)) { a->nan = 1; return; }
    if (isinf(x) || isinf(y)) {
        if (x == 0.0 || y == 0.0) { a->nan = 1; return; }
        int neg = signbit(x) != signbit(y);
        if (neg) a->neg_inf = 1; else a->pos_inf = 1;
        return;
    }
    int nx, ny, ex, ey;
    uint64_t mx, my;
    split_double(x, &nx, &mx, &ex);
    split_double(y, &ny, &my, &ey);
    if (mx == 0 || my == 0) return;
#if FBO_MUTATION == 7
    (void)nx;
    (void)ny;
    acc_add(a, 0, (unsigned __int128)mx * my, ex + ey + ACC_BIAS);
#else
    acc_add(a, nx != ny, (unsigned __int128)mx * my, ex + ey + ACC_BIAS);
#endif
}

static int acc_bit(const uint64_t *v, int i) { return (int)((v[i / 64] >> (i % 64)) & 1); }

/* Rounds the accumulated exact value to nearest-even with precision p bits
 * and minimum normal exponent emin (binary64: 53, -1022; binary32: 24,
 * -126); returns it as a double (exactly representable in the target). */
static double acc_round(const longacc *a, int p, int emin, int emax)
{
    if (a->nan || (a->pos_inf && a->neg_inf)) return NAN;
    if (a->pos_inf) return INFINITY;
    if (a->neg_inf) return -INFINITY;
    uint64_t mag[ACC_LIMBS];
    memcpy(mag, a->limb, sizeof mag);
    int neg = (int)(mag[ACC_LIMBS - 1] >> 63);
    if (neg) {
        int carry = 1;
        for (int i = 0; i < ACC_LIMBS; ++i) {
            uint64_t v = ~mag[i];
            uint64_t s = v + (uint64_t)carry;
            carry = (carry && s == 0) ? 1 : 0;
            mag[i] = s;
        }
    }
    int h = -1;
    for (int i = ACC_LIMBS * 64 - 1; i >= 0; --i)
        if (acc_bit(mag, i)) { h = i; break; }
    if (h < 0) return 0.0;                /* exact zero; +0 by convention */
    int E = h - ACC_BIAS;                 /* 2^E <= |value| < 2^(E+1) */
    int qexp = (E > emin ? E : emin) - (p - 1);   /* weight of the last kept bit */
    int t = qexp + ACC_BIAS;              /* its bit index; always > 0 here */
    uint64_t kept = 0;
    for (int i = h; i >= t; --i) kept = (kept << 1) | (uint64_t)acc_bit(mag, i);
    int G = acc_bit(mag, t - 1);
    int S = 0;
    for (int i = t - 2; i >= 0 && !S; --i) S = acc_bit(mag, i);
    if (G && (S || (kept & 1))) kept += 1;
    if (kept == ((uint64_t)1 << p)) { kept >>= 1; qexp += 1; }
    double r;
    if (qexp + p - 1 > emax) r = INFINITY;
    else r = ldexp((double)kept, qexp);
    return neg ? -r : r;
}

double fbo_dot_exact(int base, int k, size_t n, const uint8_t *x, const uint8_t *y)
{
    longacc a;
    acc_init(&a);
    for (size_t i = 0; i < n; ++i) acc_add_product(&a, elem_value(base, k, x, i), elem_value(base, k, y, i));
    if (base == 32) return (double)(float)acc_round(&a, 24, -126, 127);
    return acc_round(&a, 53, -1022, 1023);
}

/* "magnitude": the Euclidean norm sqrt(sum x_i^2) of a packed vector.
 * naive: sequential fma of squares in the base type, then sqrt in it;
 * exact: the sum of squares exactly (long accumulator), rounded once to the
 * base type, then its correctly rounded square root. */
double fbo_nrm2_naive(int base, int k, size_t n, const uint8_t *x)
{
    if (base == 32) {
        float s = 0.0f;
        for (size_t i = 0; i < n; ++i) {
            float v = (float)elem_value(base, k, x, i);
            s = fmaf(v, v, s);
        }
        return (double)sqrtf(s);
    }
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double v = elem_value(base, k, x, i);
        s = fma(v, v, s);
    }
    return sqrt(s);
}

double fbo_nrm2_exact(int base, int k, size_t n, const uint8_t *x)
{
    double s2 = fbo_dot_exact(base, k, n, x, x);
    if (base == 32) return (double)sqrtf((float)s2);
    return sqrt(s2);
}

/* ------------------------------------------------------------------ */
/* GEMV y = A x.  A is m x n, row-major, leading dimension lda (in      */
/* elements), stored as k-byte elements; x and y are native of the base.*/
/* ------------------------------------------------------------------ */
static double native_at(const void *p, int base, size_t i)
{
    if (base == 32) { float f; memcpy(&f, (const uint8_t *)p + 4 * i, 4); return (double)f; }
    double v; memcpy(&v, (const uint8_t *)p + 8 * i, 8); return v;
}

static void native_set(void *p, int base, size_t i, double v)
{
    if (base == 32) { float f = (float)v; memcpy((uint8_t *)p + 4 * i, &f, 4); return; }
    memcpy((uint8_t *)p + 8 * i, &v, 8);
}

void fbo_gemv_naive(int base, int k, int64_t m, int64_t n, const uint8_t *A, int64_t lda,
                    const void *x, void *y)
{
    for (int64_t r = 0; r < m; ++r) {
        const uint8_t *row = A + (size_t)r * (size_t)lda * (size_t)k;
        if (base == 32) {
            float s = 0.0f;
            for (int64_t c = 0; c < n; ++c)
                s = fmaf((float)elem_value(base, k, row, (size_t)c), (float)native_at(x, base, (size_t)c), s);
            native_set(y, base, (size_t)r, (double)s);
        } else {
            double s = 0.0;
            for (int64_t c = 0; c < n; ++c)
                s = fma(elem_value(base, k, row, (size_t)c), native_at(x, base, (size_t)c), s);
            native_set(y, base, (size_t)r, s);
        }
    }
}

/* Per row: the correctly rounded exact dot.  Also returns, if absrow is not
 * NULL, sum_c |A_rc * x_c| rounded to double (used by error bounds). */
void fbo_gemv_exact(int base, int k, int64_t m, int64_t n, const uint8_t *A, int64_t lda,
                    const void *x, double *y_exact, double *absrow)
{
    for (int64_t r = 0; r < m; ++r) {
        const uint8_t *row = A + (size_t)r * (size_t)lda * (size_t)k;
        longacc a, b;
        acc_init(&a);
        acc_init(&b);
        for (int64_t c = 0; c < n; ++c) {
            double av = elem_value(base, k, row, (size_t)c), xv = native_at(x, base, (size_t)c);
            acc_add_product(&a, av, xv);
            if (absrow) acc_add_product(&b, fabs(av), fabs(xv));
        }
        double v = acc_round(&a, 53, -1022, 1023);
        if (base == 32) v = (double)(float)acc_round(&a, 24, -126, 127);
        y_exact[r] = v;
        if (absrow) absrow[r] = acc_round(&b, 53, -1022, 1023);
    }
}

/* Transposed GEMV y = A^T x: A is m x n row-major (lda), x has m native
 * values, y has n.  naive: for each column, a sequential fma over the rows in
 * increasing order; exact: per column the long-accumulator sum rounded once
 * (returned as double), and sum_i |A_ij x_i|. */
void fbo_gemv_t_naive(int base, int k, int64_t m, int64_t n, const uint8_t *A, int64_t lda,
                      const void *x, void *y)
{
    for (int64_t c = 0; c < n; ++c) {
        if (base == 32) {
            float s = 0.0f;
            for (int64_t r = 0; r < m; ++r)
                s = fmaf((float)elem_value(base, k, A + (size_t)r * (size_t)lda * (size_t)k, (size_t)c),
                         (float)native_at(x, base, (size_t)r), s);
            native_set(y, base, (size_t)c, (double)s);
        } else {
            double s = 0.0;
            for (int64_t r = 0; r < m; ++r)
                s = fma(elem_value(base, k, A + (size_t)r * (size_t)lda * (size_t)k, (size_t)c),
                        native_at(x, base, (size_t)r), s);
            native_set(y, base, (size_t)c, s);
        }
    }
}

void fbo_gemv_t_exact(int base, int k, int64_t m, int64_t n, const uint8_t *A, int64_t lda,
                      const void *x, double *y_exact, double *abscol)
{
    for (int64_t c = 0; c < n; ++c) {
        longacc a, b;
        acc_init(&a);
        acc_init(&b);
        for (int64_t r = 0; r < m; ++r) {
            double av = elem_value(base, k, A + (size_t)r * (size_t)lda * (size_t)k, (size_t)c);
#if FBO_MUTATION == 8
            double xv = native_at(x, base, (size_t)(m - 1 - r));
#else
            double xv = native_at(x, base, (size_t)r);
#endif
            acc_add_product(&a, av, xv);
            if (abscol) acc_add_product(&b, fabs(av), fabs(xv));
        }
        y_exact[c] = base == 32 ? (double)(float)acc_round(&a, 24, -126, 127) : acc_round(&a, 53, -1022, 1023);
        if (abscol) abscol[c] = acc_round(&b, 53, -1022, 1023);
    }
}

/* ------------------------------------------------------------------ */
/* GEMM C = A B.  A is M x K (lda), B is K x N (ldb), row-major, packed */
/* in formats fa, fb.  For each requested entry (i, j) the exact dot of  */
/* row i of A and column j of B is rounded once to binary64; also the   */
/* matching entry of |A||B|.  Entries are given as two index arrays.    */
/* ------------------------------------------------------------------ */
void fbo_gemm_entries(int abase, int ak, int bbase, int bk, int64_t K,
                      const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
                      int64_t count, const int64_t *ii, const int64_t *jj,
                      double *c_exact, double *c_abs)
{
    for (int64_t t = 0; t < count; ++t) {
        const uint8_t *arow = A + (size_t)ii[t] * (size_t)lda * (size_t)ak;
        longacc a, b;
        acc_init(&a);
        acc_init(&b);
        for (int64_t p = 0; p < K; ++p) {
            double av = elem_value(abase, ak, arow, (size_t)p);
            double bv = elem_value(bbase, bk, B + (size_t)p * (size_t)ldb * (size_t)bk, (size_t)jj[t]);
            acc_add_product(&a, av, bv);
            acc_add_product(&b, fabs(av), fabs(bv));
        }
        c_exact[t] = acc_round(&a, 53, -1022, 1023);
        if (c_abs) c_abs[t] = acc_round(&b, 53, -1022, 1023);
    }
}

/* Plain triple-loop GEMM in binary64 with sequential fma over the inner
 * index (timing baseline and a second opinion); C is binary64 M x N. */
void fbo_gemm_naive(int abase, int ak, int bbase, int bk, int64_t M, int64_t N, int64_t K,
                    const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
                    double *C, int64_t ldc)
{
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0;
            for (int64_t p = 0; p < K; ++p)
                s = fma(elem_value(abase, ak, A + (size_t)i * (size_t)lda * (size_t)ak, (size_t)p),
                        elem_value(bbase, bk, B + (size_t)p * (size_t)ldb * (size_t)bk, (size_t)j), s);
            C[(size_t)i * (size_t)ldc + (size_t)j] = s;
        }
}

/* The mutation number this object was built with (0 = the real oracle). */
int fbo_mutation(void) { return FBO_MUTATION; }
