// GEMM on {32,2} operands with BF16 matrix cores (gfx950): the stored 2-byte
// patterns are bfloat16 operands as they are (the 16-bit flyte of Table 1 is
// bit-for-bit bfloat16).  C = A B, A M x K and B K x N row-major packed, C
// FP32 row-major, any M, N, K (the split products of {32,3} run on the
// bfloat16-piece GEMM).
//
// Tiling: a workgroup computes a BM x BN tile of C with WGM x WGN waves, each
// wave a (BM/WGM) x (BN/WGN) tile of v_mfma_f32_16x16x32_bf16 results.  Large
// wave tiles keep LDS operand traffic low.  8 waves per workgroup, two per
// SIMD, in 256 x 256 x 64 tiles as 4 x 2 waves of 64 x 128 (136 KiB of LDS);
// shapes that are not multiples of 256 use 128 x 128 x 64.  K is walked in BK
// steps through double-buffered LDS (one barrier per step; the next step's
// global loads are issued before the current step's MFMAs; the last step is
// peeled).  A is stored m-major (k contiguous, rows padded by 16 bytes, so
// the 16-byte operand reads of 16 lanes hit distinct banks) and read with
// ds_read_b128.  B is stored as it is in memory, k-major (n contiguous), from
// 16-byte global loads, and each operand fragment is read with two
// transposing LDS reads (ds_read_b64_tr_b16: the 16 lanes of a group address
// a 4 x 16 block, 4 k-rows of 16 columns, and lane i receives column i's 4
// k-values).  A 32-lane read phase covers k-rows r..r+3 and r+8..r+11; B
// rows are unpadded and 16-byte chunk c of k-row R sits at c ^ 2 g(R), with
// g(R) = (R & 3) | ((R >> 1) & 4), so those 8 rows' 32-byte pieces fall in 8
// distinct 32-byte bank groups.  Workgroups are renumbered so that consecutive tiles
// of C run on the same XCD (sharing its L2), grouped 8 tile-rows at a time.
//
// Shapes that are not tile multiples run the EDGE instances, whose K loop has
// the same loads as the full-tile instance: a thread's rows of A past M read
// row M - 1 and its 8-column chunks of B past N read the last chunk (those
// results are not stored; the clamps are fixed per thread).  A last, partial
// K step is peeled after the loop and loads elements (positions past K read
// as zero, so nothing past a row's end is read).  When N is not a multiple of
// 8 (EDGE = 2), the chunk of B that N cuts is read element by element in every
// step.  Only the entries inside M x N are stored.
#include "codec.hpp"
#include "common.hpp"

namespace flyte {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef short i16x4_t __attribute__((ext_vector_type(4)));
typedef short i16x8_t __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) i16x4_t lds_i16x4_t;

// Tile index of this workgroup: XCD-aware renumbering, then 8-row groups.
__device__ __forceinline__ void gemm_tile_coords(int ntm, int ntn, int& tm, int& tn)
{
    const int nb = ntm * ntn;
    int pid = blockIdx.x;
    if (nb % 8 == 0) pid = (pid % 8) * (nb / 8) + pid / 8;
    constexpr int GROUP = 8;
    const int per_group = GROUP * ntn;
    const int group = pid / per_group;
    const int first_m = group * GROUP;
    const int gsize = (ntm - first_m) < GROUP ? (ntm - first_m) : GROUP;
    tm = first_m + (pid % per_group) % gsize;
    tn = (pid % per_group) / gsize;
}

// Tile configuration: BM x BN x BK workgroup tile, WGM x WGN waves (wave tile
// (BM/WGM) x (BN/WGN) as 16 x 16 MFMA tiles).
template <int BM, int BN, int BK, int WGM, int WGN>
struct B32Tile {
    static constexpr int THREADS = 64 * WGM * WGN;
    static constexpr int TM = BM / WGM, TN = BN / WGN;
    static constexpr int FM = TM / 16, FN = TN / 16;
    static constexpr int ROW = BK + 8;                  // bf16 per padded LDS row of A
    static constexpr int BROW = BN;                     // bf16 per LDS row of B (k-major, swizzled)
    static constexpr int A_TILE = BM * ROW, B_TILE = BK * BROW;
    static constexpr int STAGE = A_TILE + B_TILE;
    // A: chunks of 8 consecutive bf16 of a row (16 bytes); B: the same along n
    static constexpr int CPR = BK / 8, A_N = BM * CPR / THREADS;
    static constexpr int BCPR = BN / 8, B_N = BK * BCPR / THREADS;
    static_assert(BK % 32 == 0 && TM % 16 == 0 && TN % 16 == 0, "tile shape");
    static_assert(A_N * THREADS == BM * CPR && A_N >= 1, "A staging must divide evenly");
    static_assert(B_N * THREADS == BK * BCPR && B_N >= 1, "B staging must divide evenly");
    static_assert(BN >= 128, "the B swizzle permutes 8 blocks of 16 columns");
};

__device__ __forceinline__ int clamp8(int v) { return v < 0 ? 0 : (v > 8 ? 8 : v); }

// 8 bfloat16 from p, element e read only when e < nvalid (else zero; nvalid may be <= 0).
__device__ __forceinline__ u32x4_t load8_edge(const uint8_t* p, int nvalid)
{
    uint32_t w[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t lo = (2 * d < nvalid) ? *reinterpret_cast<const uint16_t*>(p + 4 * d) : 0u;
        const uint32_t hi = (2 * d + 1 < nvalid) ? *reinterpret_cast<const uint16_t*>(p + 4 * d + 2) : 0u;
        w[d] = lo | (hi << 16);
    }
    return u32x4_t{w[0], w[1], w[2], w[3]};
}

template <int BM, int BN, int BK, int WGM, int WGN, int EDGE>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm_b32(const uint8_t* __restrict__ A, int64_t lda, const uint8_t* __restrict__ B, int64_t ldb,
           float* __restrict__ C, int64_t ldc, int M, int N, int K)
{
    // A and B are the packed {32,2} matrices (bfloat16 patterns).
    using T = B32Tile<BM, BN, BK, WGM, WGN>;
    constexpr int THREADS = T::THREADS, ROW = T::ROW, BROW = T::BROW;
    constexpr int FM = T::FM, FN = T::FN;
    // [stage][A, B]
    __shared__ __attribute__((aligned(16))) uint16_t lds[2][T::STAGE];

    const int ntm = (M + BM - 1) / BM, ntn = (N + BN - 1) / BN;
    int tm, tn;
    gemm_tile_coords(ntm, ntn, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x, lane = t % 64, wid = t / 64;
    const int wm = wid / WGN, wn = wid % WGN;

    u32x4_t ra[T::A_N], rb[T::B_N];

    auto a_tile = [&](int s) { return lds[s]; };
    auto b_tile = [&](int s) { return lds[s] + T::A_TILE; };

    // a thread's rows of A and 8-column chunks of B, clamped into the matrix (EDGE)
    auto a_row = [&](int i) {
        const int row = m0 + (t + THREADS * i) / T::CPR;
        return (int64_t)(EDGE && row >= M ? M - 1 : row);
    };
    auto b_col = [&](int i) {
        const int col = n0 + ((t + THREADS * i) % T::BCPR) * 8;
        return (int64_t)(EDGE == 1 && col >= N ? N - 8 : col);
    };
    // elements of B's chunk i inside the matrix (EDGE = 2: N cuts a chunk), 0..8
    auto b_valid = [&](int i) { return clamp8(N - (n0 + ((t + THREADS * i) % T::BCPR) * 8)); };

    // a full K step at k0
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int i = 0; i < T::A_N; ++i) {
            const int kc = (t + THREADS * i) % T::CPR;
            ra[i] = *reinterpret_cast<const u32x4_t*>(A + (a_row(i) * lda + k0 + kc * 8) * 2);
        }
#pragma unroll
        for (int i = 0; i < T::B_N; ++i) {
            const int row = (t + THREADS * i) / T::BCPR;
            const uint8_t* p = B + ((int64_t)(k0 + row) * ldb + b_col(i)) * 2;
            if (EDGE == 2 && b_valid(i) < 8) rb[i] = load8_edge(p, b_valid(i));
            else rb[i] = *reinterpret_cast<const u32x4_t*>(p);
        }
    };
    // the last, partial K step at k0: positions past K read as zero
    auto load_tail = [&](int k0) {
#pragma unroll
        for (int i = 0; i < T::A_N; ++i) {
            const int kk = k0 + ((t + THREADS * i) % T::CPR) * 8;
            ra[i] = load8_edge(A + (a_row(i) * lda + kk) * 2, K - kk);
        }
#pragma unroll
        for (int i = 0; i < T::B_N; ++i) {
            const int kr = k0 + (t + THREADS * i) / T::BCPR;
            const uint8_t* p = B + ((int64_t)(kr < K ? kr : K - 1) * ldb + b_col(i)) * 2;
            if (kr >= K) rb[i] = u32x4_t{0u, 0u, 0u, 0u};
            else if (EDGE == 2) rb[i] = load8_edge(p, b_valid(i));
            else rb[i] = *reinterpret_cast<const u32x4_t*>(p);
        }
    };

    auto store_tiles = [&](int s) {
#pragma unroll
        for (int i = 0; i < T::A_N; ++i) {
            const int c = t + THREADS * i, row = c / T::CPR, kc = c % T::CPR;
            *reinterpret_cast<u32x4_t*>(a_tile(s) + row * ROW + kc * 8) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < T::B_N; ++i) {
            const int c = t + THREADS * i, row = c / T::BCPR, nc = c % T::BCPR;
            const int g = (row & 3) | ((row >> 1) & 4);
            *reinterpret_cast<u32x4_t*>(b_tile(s) + row * BROW + (nc ^ (2 * g)) * 8) = rb[i];
        }
    };

    f32x4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int s) {
        const uint16_t* Ah = a_tile(s);
        const uint16_t* Bh = b_tile(s);
        const int r16 = lane % 16, kq = 8 * (lane / 16);
        // One read-ahead pipeline over the K sub-steps of the stage: each B
        // fragment is read one column block ahead of the MFMAs that use it
        // (the last block reads the next sub-step's first B fragment), and
        // the next sub-step's A fragments are read halfway through the
        // current one, so the wave waits for at most one LDS read before an
        // MFMA group.  The group barriers keep the compiler to this order.
        // The wave raises its issue priority for the block, so the other
        // wave on the SIMD does its staging while this one feeds the
        // matrix core.
        constexpr int KSN = BK / 32, JA = FN / 2;
        auto read_a = [&](int ks, int i) {
            return *reinterpret_cast<const bf16x8_t*>(Ah + (wm * T::TM + i * 16 + r16) * ROW + ks * 32 + kq);
        };
        // transposing read: lane s of a 16-lane group addresses k-row 8 (lane / 16) + s / 4 (+ 4 for
        // the upper half) and columns 4 (s % 4) .. + 3 of the fragment's 16 columns, whose block of
        // 16 columns sits at block index ^ g(row) (g of those rows is the same for every ks and half)
        const uint16_t* Bl = Bh + (8 * (lane / 16) + r16 / 4) * BROW + 4 * (r16 % 4);
        const int bg = (r16 / 4) | (((lane / 16) & 1) << 2);
        auto read_b = [&](int ks, int j) {
            const uint16_t* p = Bl + ks * 32 * BROW + ((wn * FN + j) ^ bg) * 16;
            const i16x4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4_t*)(p));
            const i16x4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4_t*)(p + 4 * BROW));
            return __builtin_bit_cast(bf16x8_t, i16x8_t(__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7)));
        };
        bf16x8_t a[2][FM], b[FN];
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int i = 0; i < FM; ++i) a[0][i] = read_a(0, i);
        b[0] = read_b(0, 0);
#pragma unroll
        for (int ks = 0; ks < KSN; ++ks) {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if (j + 1 < FN) b[j + 1] = read_b(ks, j + 1);
                else if (ks + 1 < KSN) b[0] = read_b(ks + 1, 0);
                if (j == JA && ks + 1 < KSN) {
#pragma unroll
                    for (int i = 0; i < FM; ++i) a[(ks + 1) & 1][i] = read_a(ks + 1, i);
                }
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks & 1][i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        __builtin_amdgcn_sched_group_barrier(0x100, FM + 2, 0);   // LDS reads
#pragma unroll
        for (int ks = 0; ks < KSN; ++ks) {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if (ks < KSN - 1 || j < FN - 1) {
                    if (j == JA && ks + 1 < KSN) __builtin_amdgcn_sched_group_barrier(0x100, 2 + FM, 0);
                    else __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, FM, 0);   // MFMAs
            }
        }
        __builtin_amdgcn_s_setprio(0);
    };

    // the last K step is peeled so the loop body has no branches; a partial
    // last step (EDGE instances) is loaded after the loop
    const int KF = K / BK, KT = EDGE ? (K + BK - 1) / BK : KF;
    if (!EDGE || KF > 0) load_tiles(0);
    else load_tail(0);
    store_tiles(0);
    __syncthreads();
    for (int kt = 0; kt < KF - 1; ++kt) {
        const int s = kt & 1;
        load_tiles((kt + 1) * BK);
        // keep the next step's global loads ahead of this step's MFMAs, so
        // their latency is covered by the whole step
        __builtin_amdgcn_sched_barrier(0);
        compute(s);
        store_tiles(s ^ 1);
        __syncthreads();
    }
    if (EDGE && KT > KF && KF > 0) {
        const int s = (KF - 1) & 1;
        load_tail(KF * BK);
        compute(s);
        store_tiles(s ^ 1);
        __syncthreads();
    }
    compute((KT - 1) & 1);

    // ---- epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * T::TM + i * 16 + 4 * (lane / 16) + r;
                const int col = n0 + wn * T::TN + j * 16 + lane % 16;
                if (!EDGE || (row < M && col < N)) C[(int64_t)row * ldc + col] = acc[i][j][r];
            }
}

template <int BM, int BN, int BK, int WGM, int WGN, int EDGE>
static void launch_b32(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                       int64_t ldc, hipStream_t stream)
{
    const unsigned blocks = (unsigned)(((M + BM - 1) / BM) * ((N + BN - 1) / BN));
    k_gemm_b32<BM, BN, BK, WGM, WGN, EDGE><<<blocks, 64 * WGM * WGN, 0, stream>>>(
        static_cast<const uint8_t*>(A), lda, static_cast<const uint8_t*>(B), ldb, static_cast<float*>(C), ldc, (int)M,
        (int)N, (int)K);
}

template <int BM, int BN, int WGM, int WGN>
static void launch_b32_shape(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb,
                             void* C, int64_t ldc, hipStream_t stream)
{
    if (M % BM == 0 && N % BN == 0 && K % 64 == 0)
        launch_b32<BM, BN, 64, WGM, WGN, 0>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    else if (N % 8 == 0)
        launch_b32<BM, BN, 64, WGM, WGN, 1>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    else
        launch_b32<BM, BN, 64, WGM, WGN, 2>(M, N, K, A, lda, B, ldb, C, ldc, stream);
}

// {32,2} operands, any M, N >= 1 and K >= 1 (checked by the caller): 256 x 256
// tiles when the full-tile instance applies or when those tiles still give
// every compute unit one, else 128 x 128.
fb_status gemm_bf16_launch(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb,
                           void* C, int64_t ldc, hipStream_t stream)
{
    const bool full256 = M % 256 == 0 && N % 256 == 0 && K % 64 == 0;
    if (full256 || ((M + 255) / 256) * ((N + 255) / 256) >= device_cu_count())
        launch_b32_shape<256, 256, 4, 2>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    else
        launch_b32_shape<128, 128, 2, 2>(M, N, K, A, lda, B, ldb, C, ldc, stream);
    return check_launch("fb_gemm");
}

}  // namespace flyte
