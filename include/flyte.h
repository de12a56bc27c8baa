/*
 * flyte.h -- C ABI of libflyte, multibyte ("flyte") floating point on AMD
 * Instinct MI355X (gfx950).
 *
 * Storage format (Anderson & Gregg, "Vectorization of Multibyte Floating
 * Point Data Formats", PACT 2016, Section 3.1 and Table 1): a value derived
 * from an IEEE-754 base type (binary32 or binary64) keeps the sign and the
 * full exponent field of that type and the top m = 8k - 1 - E bits of its
 * mantissa, so it is stored in k bytes: binary32 with k = 2, 3, 4 (4 is
 * binary32 itself; 2 is bit-for-bit bfloat16) and binary64 with k = 2..8
 * (5, 6, 7 are the paper's 40-, 48- and 56-bit formats; 8 is binary64).
 *
 * Packed arrays (Section 4.1): element i occupies bytes [i*k, i*k + k) with no
 * padding; those bytes are the top k bytes of the little-endian base bit
 * pattern, in little-endian order.  Matrices are row-major; a leading
 * dimension (lda, ldb, ldc) counts elements, and row r starts at byte
 * r*ld*k.
 *
 * Conversion: unpack shifts the k bytes to the top of the base word and fills
 * the dropped bytes with zeros (Section 3.2).  pack rounds to nearest, ties to
 * even, at the cut (Section 5.2), with the increment carrying into the
 * exponent: values round up into the next binade, the largest finite values
 * can round to infinity, subnormals underflow gradually (Section 5.3); the
 * format's round field can select round toward zero or round to odd instead.
 * In every mode a NaN is truncated and, if that leaves its kept mantissa
 * zero, gets the quiet bit (the top kept mantissa bit), so NaN stays NaN with
 * its sign.  Denormals are never flushed.
 *
 * Arithmetic (Section 3.1, and the AT_LEAST accumulator and FP_CONTRACT of
 * Section 4.4): every operation computes in the base type -- binary32 formats
 * in FP32, binary64 formats in FP64 -- with fused multiply-adds; accumulators
 * are held in the base type.  The GEMMs are the exception, see fb_gemm.
 *
 * Conventions for every call:
 *  - "native" means float for base 32 and double for base 64.
 *  - All data pointers are DEVICE pointers owned by the caller.  Every
 *    pointer must be 4-byte aligned, and every packed matrix row must start on
 *    a 4-byte boundary ((ld*k) % 4 == 0); otherwise FB_ERR_ALIGN.  Kernels
 *    read and write whole dwords (up to 4 per instruction) at 4-byte aligned
 *    addresses, so no stronger alignment is needed.
 *  - All calls are asynchronous on `stream` (0 = the null stream).  Argument
 *    errors are detected on the host, return immediately and launch nothing.
 *    A launch failure returns FB_ERR_RUNTIME.  Details of the last error on
 *    the calling thread are in fb_last_error().
 *  - n = 0 (or m = 0) is valid and launches nothing (fb_dot writes 0).
 *  - Nothing aborts, throws or prints.  Hot calls allocate no device memory,
 *    except a per-(device, stream) workspace for partial sums (fb_dot,
 *    fb_dot_packed, fb_nrm2: 16 KiB; transposed fb_gemv_ex: slabs * n native
 *    values; fb_gemm on {64,2..4}: scales and band flags, about 73 bytes per
 *    row of A and column of B),
 *    allocated on first use on that stream and kept.  A call that needs more
 *    allocates a larger buffer and keeps the old one allocated as well (until
 *    the process ends), so queued work and graphs captured earlier never
 *    write freed memory; sizes at least double, so the retired buffers hold
 *    less than the current one.  Calls can be captured into a HIP graph; one
 *    that needs a larger workspace than its stream has returns FB_ERR_RUNTIME
 *    during capture, so make one call of that size on the stream beforehand.
 *  - Input and output ranges must not overlap unless a call says so.
 */
#ifndef FLYTE_H
#define FLYTE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Format descriptor {base, k, round}: base 32 with k in 2..4, or base 64 with
 * k in 2..8.  round selects how values are cut to k bytes wherever a call
 * packs results (fb_pack, fb_axpy, fb_scale, a packed fb_gemm C); it is
 * ignored by calls that only read packed data.  reserved must be 0. */
typedef enum fb_round {
    FB_ROUND_NEAREST_EVEN = 0,   /* Section 5.2 (the default) */
    FB_ROUND_TOWARD_ZERO = 1,    /* Section 5.1: drop the low bytes */
    FB_ROUND_TO_ODD = 2          /* Section 7 (Boldo-Melquiond): drop the low bytes, set the
                                    lowest kept bit if any dropped bit was set */
} fb_round;

typedef struct fb_format {
    uint8_t base;
    uint8_t k;
    uint8_t round;      /* fb_round */
    uint8_t reserved;
} fb_format;

typedef enum fb_status {
    FB_OK = 0,
    FB_ERR_FORMAT = 1,       /* {base, k} is not a flyte format */
    FB_ERR_ARG = 2,          /* null pointer, negative size, bad leading dimension */
    FB_ERR_ALIGN = 3,        /* pointer or row start not 4-byte aligned */
    FB_ERR_UNSUPPORTED = 4,  /* valid formats, but no kernel for this combination */
    FB_ERR_RUNTIME = 5       /* HIP runtime error (launch, allocation, graph) */
} fb_status;

/* ------------------------------------------------------------------ codec */

/* Pack n native values into n k-byte elements (Sections 5.2 and 5.3).
 * src_native: n floats/doubles; dst_packed: n*k bytes.  Bit-exact. */
fb_status fb_pack(fb_format f, const void *src_native, void *dst_packed, size_t n,
                  hipStream_t stream);

/* Unpack n k-byte elements into n native values (Sections 3.2 and 4.1).
 * src_packed: n*k bytes; dst_native: n floats/doubles.  Bit-exact. */
fb_status fb_unpack(fb_format f, const void *src_packed, void *dst_native, size_t n,
                    hipStream_t stream);

/* ------------------------------------------------------------------ BLAS 1 */

/* result = sum_i unpack(x_i) * unpack(y_i), x and y packed (n*k bytes each):
 * a BLAS level-1 program of Sections 6.1 and 6.3.1 over k-byte data (Section 3.1).
 * Products and sums in the base type with fma; the reduction order is fixed
 * (per-thread sequential, then fixed trees), so repeated calls on the same
 * device give identical bits.  result: one native value in device memory. */
fb_status fb_dot(fb_format f, size_t n, const void *x, const void *y, void *result,
                 hipStream_t stream);

/* fb_dot for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): same arguments,
 * kernels, order and result bits as fb_dot, but the partial sums go to a
 * static device array of 1984 binary64 values (15.5 KiB) instead of the
 * stream workspace, so the call allocates nothing, ever.  Every n is
 * accepted (the partial count is capped at 1984 whatever n is).  The array
 * exists once per device and is shared by all calls on that device: calls
 * that overlap in time on one device (on different streams, or from
 * different threads) race on it and give wrong results; calls ordered on one
 * stream are fine.  Nothing in it needs to start at zero. */
fb_status fb_dot_noalloc(fb_format f, size_t n, const void *x, const void *y, void *result,
                         hipStream_t stream);

/* fb_dot with the result stored in format fr (same base as f): the base-type
 * sum rounded once in fr's rounding mode, fr.k bytes in device memory. */
fb_status fb_dot_packed(fb_format f, fb_format fr, size_t n, const void *x, const void *y,
                        void *result, hipStream_t stream);

/* y_i <- pack(fma(alpha, unpack(x_i), unpack(y_i))), in place on y: a BLAS
 * level-1 program of Sections 6.1 and 6.3.1, one fused multiply-add in the base type and one
 * cut (Sections 3.1, 5.2).  alpha is first rounded to the native type.
 * Bit-exact per element.
 * x and y are packed (n*k bytes); x must not overlap y. */
fb_status fb_axpy(fb_format f, size_t n, double alpha, const void *x, void *y,
                  hipStream_t stream);

/* x_i <- pack(alpha * unpack(x_i)), in place (the paper's BLAS-1 "scale"
 * program, Section 6): one multiplication in the base type, alpha first
 * rounded to it, then the cut in the format's rounding mode.  Bit-exact. */
fb_status fb_scale(fb_format f, size_t n, double alpha, void *x, hipStream_t stream);

/* result = sqrt(sum_i unpack(x_i)^2) (the vector "magnitude"): squares summed
 * with fma in the base type in a fixed order, then one square root in it.
 * No rescaling: squares that overflow the base type give Inf.  result: one
 * native value in device memory. */
fb_status fb_nrm2(fb_format f, size_t n, const void *x, void *result, hipStream_t stream);

/* ------------------------------------------------------------------ BLAS 2 */

/* y = A x, the BLAS level-2 GEMV of Sections 6.2 and 6.3.2 over a packed A
 * (codec fused into the loads, Sections 3.2 and 4.1).  A: m x n packed,
 * row-major, leading dimension lda >= n (elements).
 * x: n native values; y: m native values.  Each y_r is a sequence of fmas in
 * the base type in an order fixed by the tile configuration (chosen by the
 * autotuner cache, else a default for the shape). */
fb_status fb_gemv(fb_format f, int64_t m, int64_t n, const void *A, int64_t lda,
                  const void *x, void *y, hipStream_t stream);

/* y = op(A) x with y stored in format fy (same base as fa; fy with k bytes =
 * the base width means a native y; otherwise each y element is the base-type
 * result rounded once to fy in fy's rounding mode).  trans = 0: y (m
 * elements) = A x, x has n values, same kernels and order as fb_gemv.
 * trans = 1: y (n elements) = A^T x, x has m values: each y_j is a fixed
 * sequence of fmas over slabs of rows plus a fixed-order sum of the slab
 * results (kept in the per-stream workspace, which grows to slabs * n native
 * values and then stays allocated).  y is written even when m = 0 (zeros), so
 * it must be valid whenever n > 0. */
fb_status fb_gemv_ex(fb_format fa, fb_format fy, int32_t trans, int64_t m, int64_t n, const void *A,
                     int64_t lda, const void *x, void *y, hipStream_t stream);

/* Same as fb_gemv with the tile configuration forced: config is an index in
 * [0, fb_gemv_num_configs()).  Used by the autotuner and for reproducibility. */
fb_status fb_gemv_config(fb_format f, int64_t m, int64_t n, const void *A, int64_t lda,
                         const void *x, void *y, int32_t config, hipStream_t stream);

/* Number of GEMV tile configurations, and a description of one: returns the
 * lanes that share a row group (0 if config is out of range) and writes the
 * rows per wave, the waves that sweep the same rows together, and the units
 * each lane loads per loop trip. */
int32_t fb_gemv_num_configs(void);
int32_t fb_gemv_config_info(int32_t config, int32_t *rows_per_wave, int32_t *waves_per_block,
                            int32_t *chunks_per_lane);

/* ------------------------------------------------------------------ autotuner */

/* Times every GEMV tile configuration on the caller's buffers (A, x, y as for
 * fb_gemv; y is overwritten) with `reps` timed launches each on `stream`,
 * records the fastest for the (format, shape bucket) in the in-process cache,
 * and returns its index in *best (may be NULL).  Synchronises the stream. */
fb_status fb_tune_gemv(fb_format f, int64_t m, int64_t n, const void *A, int64_t lda,
                       const void *x, void *y, int32_t reps, int32_t *best, hipStream_t stream);

/* The cached choice for (format, m, n), or -1 if none. */
int32_t fb_tune_lookup(fb_format f, int64_t m, int64_t n);

/* Records a choice measured by the caller (for example with rotating buffers
 * so that the 256 MB last-level cache holds none of A) for the shape bucket of
 * (m, n).  us is the measured time per launch, kept for the saved cache. */
fb_status fb_tune_record(fb_format f, int64_t m, int64_t n, int32_t config, double us);

/* Saves / loads the tile cache as JSON (path NULL: $FLYTE_TUNE_CACHE).
 * Loading merges into the in-process cache. */
fb_status fb_tune_save(const char *path);
fb_status fb_tune_load(const char *path);
void fb_tune_clear(void);

/* ------------------------------------------------------------------ batched GEMV */

/* One independent GEMV y = A x of a batch (same semantics as fb_gemv; the
 * batched schedule itself is not in the paper). */
typedef struct fb_gemv_desc {
    fb_format f;
    int32_t m;
    int32_t n;
    int32_t reserved1;
    int64_t lda;
    const void *A;
    const void *x;
    void *y;
} fb_gemv_desc;   /* 48 bytes */

typedef struct fb_plan fb_plan;

/* Validates `count` descriptors (host array), picks a tile configuration per
 * descriptor from the autotuner cache, orders the work, and uploads a device
 * work table.  The plan owns that table and its work counter; the descriptor
 * array may be freed afterwards.  Buffers named by the descriptors must stay
 * valid while the plan is launched.  Distinct descriptors must not share y. */
fb_status fb_gemv_batched_plan(const fb_gemv_desc *descs, int32_t count, fb_plan **out);

/* Autotunes the plan: descriptors are grouped by (format, log2 m, log2 n);
 * for each group, up to 64 of its own GEMVs are run alone in the persistent
 * kernel with every tile compiled into it (their y are overwritten), the
 * fastest tile is stored in the tile cache and assigned to the whole group,
 * and the device tables are rebuilt.  Synchronises `stream`. */
fb_status fb_gemv_batched_tune(fb_plan *plan, int32_t reps, hipStream_t stream);

/* Runs every GEMV of the plan in ONE persistent kernel: workgroups take
 * (descriptor, row tile) work items from a device counter until none remain.
 * The first launch builds and instantiates a HIP graph of two kernel nodes
 * (counter reset, persistent kernel); later launches replay it, on any
 * stream.  Launches of one plan must not overlap.  Each y equals
 * fb_gemv_config on the same descriptor with the plan's configuration
 * (fb_plan_config), bit for bit. */
fb_status fb_gemv_batched_launch(fb_plan *plan, hipStream_t stream);

/* Reference schedules: one fb_gemv_config launch per descriptor, in order,
 * either issued from the host (loop) or as a prebuilt HIP graph with one
 * kernel node per descriptor, chained in order (loop_graph, built on its first
 * call).  Same results as fb_gemv_batched_launch. */
fb_status fb_gemv_batched_loop(fb_plan *plan, hipStream_t stream);
fb_status fb_gemv_batched_loop_graph(fb_plan *plan, hipStream_t stream);

/* Algorithmic bytes of the plan (sum of m*n*k + native bytes of x and y). */
int64_t fb_plan_bytes(const fb_plan *plan);
/* Tile configuration chosen for descriptor i (or -1). */
int32_t fb_plan_config(const fb_plan *plan, int32_t i);

/* Frees the plan's device memory and graphs; waits for all work on the plan's device
 * first (hipDeviceSynchronize), so a launch still in flight is not cut short. */
void fb_plan_destroy(fb_plan *plan);

/* ------------------------------------------------------------------ BLAS 3 */

/* C = A B with A M x K (lda), B K x N (ldb), C M x N (ldc), row-major: the
 * matrix-matrix benchmark of Section 6 with the codec fused into the operand
 * loaders and, for a packed C, into the epilogue (Sections 3.2, 4.3, 5.2).
 * Any M, N, K >= 0 (edge tiles and the K tail are bounded; no byte past a
 * row's last element is read and no C element outside the M x N block is
 * written).  Supported combinations (others: FB_ERR_UNSUPPORTED):
 *  - fa = fb = {32,2}, fc = {32,4}: the stored 2-byte patterns are bfloat16
 *    operands of BF16 matrix-core instructions, FP32 accumulation, FP32 C.
 *  - fa = fb = {32,3}, fc = {32,4}: each operand element is split, while it is
 *    loaded, into hi = its top two bytes (a bfloat16; a NaN gets the quiet
 *    bit, so it stays NaN) and lo = x - hi rounded to bfloat16 (exact for
 *    biased exponent >= 9; 0 for Inf/NaN); C = hi*hi + hi*lo + lo*hi in FP32
 *    accumulators (lo*lo dropped, |lo| < 2^-7 |x|): three BF16 products.  An
 *    infinite element (hi = Inf, lo = 0) can meet a partner whose lo is 0 in a
 *    hi*lo term, Inf * 0, so entries whose exact value is +-Inf may come out
 *    NaN; NaN stays NaN.  No workspace.
 *  - fa = fb = {64,2}, {64,3} or {64,4} (5, 13, 21 significant bits), fc any
 *    binary64 format: every row of A and column of B is scaled by an exact
 *    power of two (its largest element to [1, 2)), each scaled element cut
 *    into 1, 2 or 3 bfloat16 pieces (8 + 8 + 5 bits, exact), the products of
 *    pieces (exact in FP32) summed on BF16 matrix cores in FP32, scaled back
 *    exactly in FP64 and rounded to fc in the epilogue.  By default the
 *    products of pieces i, j with i + j <= k - 2 are formed ({64,3}: 3 of 4,
 *    dropping at most 2^-14 |a||b| per term; {64,4}: 6 of 9, dropping below
 *    2^-20 |a||b|).  A row or column with an element more than 2^40 below its
 *    largest, a binary64 subnormal, Inf or NaN cannot be scaled exactly: every
 *    128 x 128 tile of C in its 128-row band of A (128-column band of B) is
 *    then computed as below, on FP64 matrix cores.  A pass before the GEMM
 *    finds the scales and bands; they live in the per-stream workspace
 *    (about 73 bytes per row of A plus column of B).
 *  - fa = fb = any binary64 format {64,2..8} (k >= 5, or with FB_GEMM_FP64),
 *    fc any binary64 format: operands unpacked to FP64, FP64 matrix-core
 *    products and accumulation (products exact for k <= 4), C rounded to fc
 *    in the epilogue in fc's rounding mode (one rounding of the FP64 result).
 * K = 0 gives C = +0.  Rows of A, B and C start 4-byte aligned (ld * k a
 * multiple of 4), else FB_ERR_ALIGN. */
fb_status fb_gemm(fb_format fa, fb_format fb, fb_format fc, int64_t M, int64_t N, int64_t K,
                  const void *A, int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc,
                  hipStream_t stream);

/* fb_gemm with options.  FB_GEMM_ALL_PRODUCTS (split operands: {32,3}, and
 * {64,3}, {64,4} on the bfloat16 pieces): every product of pieces is formed
 * (4 for {32,3} and {64,3}, 9 for {64,4}), so only the FP32 accumulation
 * rounds.  FB_GEMM_FP64 (binary64 operands): the FP64 matrix-core path for
 * k <= 4 as well.  Other flag bits: FB_ERR_ARG; a flag that does not apply
 * to the formats: FB_ERR_UNSUPPORTED. */
typedef enum fb_gemm_flags {
    FB_GEMM_DEFAULT = 0,
    FB_GEMM_ALL_PRODUCTS = 1,
    FB_GEMM_FOUR_PRODUCTS = 1,   /* the {32,3} name of FB_GEMM_ALL_PRODUCTS */
    FB_GEMM_FP64 = 2
} fb_gemm_flags;

fb_status fb_gemm_ex(fb_format fa, fb_format fb, fb_format fc, int64_t M, int64_t N, int64_t K,
                     const void *A, int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc,
                     uint32_t flags, hipStream_t stream);

/* ------------------------------------------------------------------ errors */

const char *fb_status_str(fb_status status);
/* Detail of the last failing call on this thread ("" if none). */
const char *fb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FLYTE_H */
