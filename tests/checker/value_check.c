/*
 * Independent value-domain check of the oracle's pack (round to nearest even,
 * Section 5.2 of Anderson & Gregg) for binary32-derived formats.
 *
 * This file shares no code with the oracle: it computes the expected result
 * from the VALUE of each input, by the classic magic-constant rounding in
 * binary64 arithmetic, and compares it with the oracle's bit-level pack loaded
 * through dlopen().  For a finite non-NaN binary32 x with binade exponent
 * e = floor(log2 |x|), the target grid spacing is 2^s with
 * s = max(e, -126) - m (m kept mantissa bits).  With C = 1.5 * 2^(52+s),
 * the binary64 sum x + C lies in [2^(52+s), 2^(53+s)), where binary64 spacing
 * is exactly 2^s and C is a multiple of 2^(s+1), so the hardware's
 * round-to-nearest-even addition rounds x to the nearest multiple of 2^s with
 * ties to an even multiple; subtracting C again is exact.  A result at or
 * above 2^128 is an overflow to infinity; a zero result takes the sign of x.
 *
 * For NaN inputs the checker asserts only what the paper requires of every
 * rounding mode (Section 5.3, NaN values): the result is a NaN of the same
 * sign.  Infinities must map to infinities of the same sign.
 *
 * Round toward zero and round to odd (the other modes of the pack, Sections
 * 5.1 and 7) are checked the same way: y = trunc(x / 2^s) * 2^s in binary64
 * (exact), and for round to odd, if y != x and y / 2^s is even, y moves one
 * step of 2^s away from zero.
 *
 * Usage:
 *   value_check <oracle.so> <k> <start> <count> <threads> [mode]
 *     mode 0 nearest even (default), 1 toward zero, 2 to odd;
 *     checks binary32 patterns start .. start+count-1 (count 0 means all 2^32)
 *     and that pack(unpack(q)) == q for every k-byte pattern q in that range;
 *   value_check <oracle.so> rt <base> <k> <threads>
 *     checks pack(unpack(q)) == q for every k-byte pattern q (k <= 4) of the
 *     format {base, k}: unpack is injective and pack inverts it exactly;
 *   value_check <oracle.so> bm <k> <kwide> <threads>
 *     checks, for every binary32 input, that rounding to odd into kwide bytes
 *     and then to nearest even into k bytes equals rounding to nearest even
 *     into k bytes directly (Boldo and Melquiond: the intermediate has at
 *     least two more bits).
 * Prints the number of mismatches and the first few.
 */
#include <dlfcn.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t (*pack_fn)(int, int, uint64_t);
typedef uint64_t (*pack_mode_fn)(int, int, uint64_t, int);

static pack_fn g_pack, g_unpack;
static pack_mode_fn g_pack_mode;
static int g_k, g_base, g_mode, g_kwide;

typedef struct {
    uint64_t lo, hi;          /* pattern range [lo, hi) */
    uint64_t bad;
    uint64_t first_bad[4];
    uint64_t got[4], want[4];
} job;

static float f_of(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t u_of(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* Expected packed pattern, toward zero (mode 1) or to odd (mode 2). */
static uint32_t expected_directed(uint32_t u, int k, int mode)
{
    const int m = 8 * k - 9;
    const int dropped = 32 - 8 * k;
    double xd = (double)f_of(u);
    double y = xd;
    if (!isinf(xd) && xd != 0.0) {
        int e;
        (void)frexp(xd, &e);
        e -= 1;
        int s = (e > -126 ? e : -126) - m;
        double steps = trunc(ldexp(xd, -s));        /* exact: |x| / 2^s < 2^54 */
        y = ldexp(steps, s);
        if (mode == 2 && y != xd && fmod(fabs(steps), 2.0) == 0.0) y = ldexp(steps + copysign(1.0, xd), s);
        if (y == 0.0) y = copysign(0.0, xd);
    }
    return u_of((float)y) >> dropped;
}

/* Expected packed pattern for a non-NaN binary32 input, from its value. */
static uint32_t expected(uint32_t u, int k)
{
    const int m = 8 * k - 9;            /* kept mantissa bits, 8 exponent bits */
    const int dropped = 32 - 8 * k;
    float x = f_of(u);
    double xd = (double)x;
    double y;
    if (isinf(xd)) {
        y = xd;
    } else if (xd == 0.0) {
        y = xd;
    } else {
        int e;
        (void)frexp(xd, &e);
        e -= 1;                         /* 2^e <= |x| < 2^(e+1) */
        int s = (e > -126 ? e : -126) - m;
        double C = ldexp(1.5, 52 + s);
        volatile double t = xd + C;     /* one rounding, to a multiple of 2^s */
        y = t - C;                      /* exact */
        if (fabs(y) >= ldexp(1.0, 128)) y = copysign(INFINITY, xd);
        if (y == 0.0) y = copysign(0.0, xd);
    }
    float yf = (float)y;                /* exact: y is on the target grid */
    return u_of(yf) >> dropped;
}

static void *worker(void *arg)
{
    job *J = (job *)arg;
    const int k = g_k;
    const int dropped = 32 - 8 * k;
    for (uint64_t p = J->lo; p < J->hi; ++p) {
        uint32_t u = (uint32_t)p;
        uint32_t got = g_mode ? (uint32_t)g_pack_mode(32, k, u, g_mode) : (uint32_t)g_pack(32, k, u);
        int ok;
        uint32_t want;
        int is_nan = (u & 0x7FFFFFFFu) > 0x7F800000u;
        if (is_nan) {
            uint32_t back = got << dropped;
            ok = ((back & 0x7FFFFFFFu) > 0x7F800000u) && ((back >> 31) == (u >> 31));
            want = 0xFFFFFFFFu;
        } else {
            want = g_mode ? expected_directed(u, k, g_mode) : expected(u, k);
            ok = got == want;
        }
        if (!ok) {
            if (J->bad < 4) { J->first_bad[J->bad] = u; J->got[J->bad] = got; J->want[J->bad] = want; }
            J->bad++;
        }
        /* round trip on the k-byte patterns: pack(unpack(q)) == q */
        if (p < ((uint64_t)1 << (8 * k)) && p >= J->lo) {
            uint32_t q = u;
            uint32_t back = (uint32_t)g_pack(32, k, g_unpack(32, k, q));
            if (back != q) {
                if (J->bad < 4) { J->first_bad[J->bad] = q | 0x100000000ull; J->got[J->bad] = back; J->want[J->bad] = q; }
                J->bad++;
            }
        }
    }
    return NULL;
}

static void *bm_worker(void *arg)
{
    job *J = (job *)arg;
    for (uint64_t p = J->lo; p < J->hi; ++p) {
        uint32_t u = (uint32_t)p;
        if ((u & 0x7FFFFFFFu) > 0x7F800000u) continue;   /* NaNs: no rounding takes place */
        uint64_t wide = g_unpack(32, g_kwide, g_pack_mode(32, g_kwide, u, 2));
        uint64_t two_step = g_pack(32, g_k, wide);
        uint64_t direct = g_pack(32, g_k, u);
        if (two_step != direct) {
            if (J->bad < 4) { J->first_bad[J->bad] = u; J->got[J->bad] = two_step; J->want[J->bad] = direct; }
            J->bad++;
        }
    }
    return NULL;
}

static void *rt_worker(void *arg)
{
    job *J = (job *)arg;
    for (uint64_t q = J->lo; q < J->hi; ++q) {
        uint64_t back = g_pack(g_base, g_k, g_unpack(g_base, g_k, q));
        if (back != q) {
            if (J->bad < 4) { J->first_bad[J->bad] = q; J->got[J->bad] = back; J->want[J->bad] = q; }
            J->bad++;
        }
    }
    return NULL;
}

int main(int argc, char **argv)
{
    if (argc < 6) {
        fprintf(stderr, "usage: %s oracle.so k start count threads\n", argv[0]);
        return 2;
    }
    void *h = dlopen(argv[1], RTLD_NOW | RTLD_LOCAL);
    if (!h) { fprintf(stderr, "dlopen: %s\n", dlerror()); return 2; }
    g_pack = (pack_fn)dlsym(h, "fbo_pack_bits");
    g_unpack = (pack_fn)dlsym(h, "fbo_unpack_bits");
    g_pack_mode = (pack_mode_fn)dlsym(h, "fbo_pack_bits_mode");
    if (!g_pack || !g_unpack || !g_pack_mode) { fprintf(stderr, "missing symbols\n"); return 2; }
    int roundtrip = strcmp(argv[2], "rt") == 0;
    int bm = strcmp(argv[2], "bm") == 0;
    uint64_t start, count;
    int nt;
    if (bm) {
        g_k = atoi(argv[3]);
        g_kwide = atoi(argv[4]);
        nt = atoi(argv[5]);
        start = 0;
        count = (uint64_t)1 << 32;
    } else if (roundtrip) {
        g_base = atoi(argv[3]);
        g_k = atoi(argv[4]);
        nt = atoi(argv[5]);
        if (g_k < 1 || g_k > 4) { fprintf(stderr, "rt mode needs k <= 4\n"); return 2; }
        start = 0;
        count = (uint64_t)1 << (8 * g_k);
    } else {
        g_base = 32;
        g_k = atoi(argv[2]);
        start = strtoull(argv[3], NULL, 0);
        count = strtoull(argv[4], NULL, 0);
        nt = atoi(argv[5]);
        g_mode = argc > 6 ? atoi(argv[6]) : 0;
        if (count == 0) count = (uint64_t)1 << 32;
    }
    if (nt < 1) nt = 1;
    if (nt > 64) nt = 64;
    job jobs[64];
    pthread_t th[64];
    memset(jobs, 0, sizeof jobs);
    uint64_t per = (count + (uint64_t)nt - 1) / (uint64_t)nt;
    for (int t = 0; t < nt; ++t) {
        jobs[t].lo = start + per * (uint64_t)t;
        jobs[t].hi = jobs[t].lo + per;
        if (jobs[t].hi > start + count) jobs[t].hi = start + count;
        if (jobs[t].lo > jobs[t].hi) jobs[t].lo = jobs[t].hi;
        pthread_create(&th[t], NULL, bm ? bm_worker : (roundtrip ? rt_worker : worker), &jobs[t]);
    }
    uint64_t bad = 0;
    int shown = 0;
    for (int t = 0; t < nt; ++t) {
        pthread_join(th[t], NULL);
        bad += jobs[t].bad;
        for (uint64_t i = 0; i < jobs[t].bad && i < 4 && shown < 8; ++i, ++shown)
            printf("mismatch input=%#llx got=%#llx want=%#llx\n",
                   (unsigned long long)jobs[t].first_bad[i], (unsigned long long)jobs[t].got[i],
                   (unsigned long long)jobs[t].want[i]);
    }
    printf("checked=%llu mismatches=%llu\n", (unsigned long long)count, (unsigned long long)bad);
    return bad ? 1 : 0;
}
