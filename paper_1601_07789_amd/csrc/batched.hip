// Batched GEMV: thousands of independent y_d = A_d x_d with mixed formats and
// uneven shapes in one persistent kernel.
//
// The plan (host) validates the descriptors, picks a tile configuration for
// each from the autotuner cache (restricted to the tiles compiled into the
// persistent kernel), splits every GEMV into row tiles of one workgroup each,
// orders those work items by decreasing cost (longest first, so the tail of
// the schedule is made of small items), and uploads the descriptor and work
// tables.  The persistent kernel runs as many workgroups as fit on the device
// at once; each workgroup repeatedly takes the next work item from a device
// counter and runs the same per-block GEMV body as fb_gemv, so every y is
// bit-identical to fb_gemv_config with the same tile.  Every workgroup leaves
// the loop once the counter passes the last item.
//
// Launch: a HIP graph of two kernel nodes (counter reset, persistent kernel),
// built and instantiated on the first launch and replayed afterwards.  The
// counter is cleared by a kernel, not a memset node.
#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "gemv_impl.hpp"

namespace flyte {

fb_status gemv_validate(const char* what, fb_format f, int64_t m, int64_t n, const void* A, int64_t lda,
                        const void* x, const void* y);
int tune_lookup(fb_format f, int64_t m, int64_t n);
void tune_store(fb_format f, int64_t m, int64_t n, int tile, double us);
const void* gemv_kernel_fn(fb_format f, int tile, int64_t m, unsigned* blocks);
int tune_bucket(int64_t v);

// Tiles compiled into the persistent kernel (public GEMV config ids); the
// order is the slot order of run_format below.  The set keeps the kernel at
// three workgroups per CU without spilling (the kernel's register budget is
// the largest of its paths).  A set of two-row tiles only fits four
// workgroups per CU but measured slower: the four-row tiles' reuse of x is
// worth more than the extra occupancy.
constexpr int kBatchedNumTiles = 8;
static const int kBatchedTile[kBatchedNumTiles] = {11, 12, 9, 10, 33, 32, 21, 7};

static int batched_slot(int tile)
{
    for (int i = 0; i < kBatchedNumTiles; ++i)
        if (kBatchedTile[i] == tile) return i;
    return -1;
}

static int format_index(fb_format f)
{
    return f.base == 32 ? f.k - 2 : 3 + (f.k - 2);   // 0..9
}

struct DescDev {
    GemvArgs a;
    int32_t code;     // format_index * kBatchedNumTiles + slot
    int32_t pad;
};

struct WorkItem {
    int32_t desc;
    int32_t row0;
};

__global__ void k_reset_counter(uint32_t* counter) { *counter = 0u; }

// One out-of-line function per (format, tile): each path gets its own register
// allocation instead of the union of all paths inlined into one body.
template <class F, class TILE>
__device__ __noinline__ void run_tile(GemvArgs a, int64_t row0)
{
    gemv_block<F, TILE>(a, row0);
}

template <int B, int K>
__device__ __forceinline__ void run_format(const DescDev& d, int slot, int64_t row0)
{
    using F = Fmt<B, K>;
    switch (slot) {
        case 0: run_tile<F, GemvTile<8, 2, 1>>(d.a, row0); break;              // config 11
        case 1: run_tile<F, GemvTile<8, 4, 1>>(d.a, row0); break;              // config 12
        case 2: run_tile<F, GemvTile<16, 2, 2>>(d.a, row0); break;             // config 9
        case 3: run_tile<F, GemvTile<16, 4, 1>>(d.a, row0); break;             // config 10
        case 4: run_tile<F, GemvTile<8, 2, 1, 1, true>>(d.a, row0); break;     // config 33
        case 5: run_tile<F, GemvTile<16, 2, 2, 1, true>>(d.a, row0); break;    // config 32
        case 6: run_tile<F, GemvTile<64, 4, 1, 2, true>>(d.a, row0); break;    // config 21
        default: run_tile<F, GemvTile<32, 2, 2>>(d.a, row0); break;            // config 7
    }
}

__global__ void __launch_bounds__(kGemvBlock, 3)
k_gemv_batched(const DescDev* __restrict__ descs, const WorkItem* __restrict__ items, int32_t nitems,
               uint32_t* __restrict__ counter)
{
    // The next item is claimed before the current one is processed, so the
    // atomic's round trip overlaps the work; a workgroup claims one item past
    // the end before it leaves (the counter is reset before every launch).
    __shared__ int32_t s_item;
    if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(counter, 1u);
    __syncthreads();
    int32_t it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    while (it < nitems) {
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
        const WorkItem w = items[it];
        const DescDev d = descs[w.desc];
        const int code = __builtin_amdgcn_readfirstlane(d.code);
        const int fi = code / kBatchedNumTiles, slot = code % kBatchedNumTiles;
        switch (fi) {
            case 0: run_format<32, 2>(d, slot, w.row0); break;
            case 1: run_format<32, 3>(d, slot, w.row0); break;
            case 2: run_format<32, 4>(d, slot, w.row0); break;
            case 3: run_format<64, 2>(d, slot, w.row0); break;
            case 4: run_format<64, 3>(d, slot, w.row0); break;
            case 5: run_format<64, 4>(d, slot, w.row0); break;
            case 6: run_format<64, 5>(d, slot, w.row0); break;
            case 7: run_format<64, 6>(d, slot, w.row0); break;
            case 8: run_format<64, 7>(d, slot, w.row0); break;
            default: run_format<64, 8>(d, slot, w.row0); break;
        }
        if (threadIdx.x == 0) s_item = (int32_t)next;
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
    }
}

}  // namespace flyte

using namespace flyte;

struct fb_plan {
    std::vector<fb_gemv_desc> descs;
    std::vector<int> tiles;          // public config id per descriptor
    int64_t bytes = 0;
    int32_t nitems = 0;
    int device = 0;
    DescDev* d_descs = nullptr;
    WorkItem* d_items = nullptr;
    uint32_t* d_counter = nullptr;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t loop_graph = nullptr;
    hipGraphExec_t loop_exec = nullptr;
    std::mutex mu;
};

static void plan_free_device(fb_plan* p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->loop_exec) (void)hipGraphExecDestroy(p->loop_exec);
    if (p->loop_graph) (void)hipGraphDestroy(p->loop_graph);
    if (p->d_descs) (void)hipFree(p->d_descs);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_counter) (void)hipFree(p->d_counter);
    p->exec = nullptr;
    p->graph = nullptr;
    p->loop_exec = nullptr;
    p->loop_graph = nullptr;
    p->d_descs = nullptr;
    p->d_items = nullptr;
    p->d_counter = nullptr;
}

// Untuned choice inside the persistent kernel: few lanes per row (many rows
// per work item) measured fastest for rows of up to a few thousand elements.
static int pick_batched_tile(const fb_gemv_desc& d)
{
    const int t = tune_lookup(d.f, d.m, d.n);
    if (t >= 0 && batched_slot(t) >= 0) return t;
    return 11;
}

// Device tables of a set of descriptors with their tiles: descriptor table,
// work items (longest first) and the persistent grid size.
struct Tables {
    DescDev* d_descs = nullptr;
    WorkItem* d_items = nullptr;
    int32_t nitems = 0;
    int grid = 0;
};

static void free_tables(Tables& t)
{
    if (t.d_descs) (void)hipFree(t.d_descs);
    if (t.d_items) (void)hipFree(t.d_items);
    t = Tables{};
}

static fb_status build_tables(const std::vector<fb_gemv_desc>& descs, const std::vector<int>& tiles, Tables& out)
{
    const int count = (int)descs.size();
    std::vector<DescDev> dd(count);
    struct Run {
        int desc;
        int rows_per_block;
        int64_t cost;   // bytes of one work item
        int nt;
    };
    std::vector<Run> runs;
    runs.reserve(count);
    int64_t total_items = 0;
    for (int i = 0; i < count; ++i) {
        const fb_gemv_desc& d = descs[i];
        const int tile = tiles[i];
        const TileInfo ti = gemv_tile_info(tile);
        dd[i].a = GemvArgs{static_cast<const uint8_t*>(d.A), d.lda * d.f.k, d.x, d.y, d.m, d.n, 0, 0};
        dd[i].code = format_index(d.f) * kBatchedNumTiles + batched_slot(tile);
        dd[i].pad = 0;
        if (d.m == 0) continue;
        const int nt = (d.m + ti.rows_per_block - 1) / ti.rows_per_block;
        runs.push_back(Run{i, ti.rows_per_block, (int64_t)ti.rows_per_block * d.n * d.f.k + 1, nt});
        total_items += nt;
    }
    if (total_items > INT32_MAX - 1024) return set_error(FB_ERR_ARG, "fb_gemv_batched_plan: too many work items");
    std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.cost > b.cost; });
    std::vector<WorkItem> items;
    items.reserve((size_t)total_items);
    for (const Run& r : runs)
        for (int t = 0; t < r.nt; ++t) items.push_back(WorkItem{r.desc, t * r.rows_per_block});
    out.nitems = (int32_t)items.size();
    if (hipMalloc(&out.d_descs, sizeof(DescDev) * std::max(1, count)) != hipSuccess ||
        hipMalloc(&out.d_items, sizeof(WorkItem) * std::max<size_t>(1, items.size())) != hipSuccess) {
        free_tables(out);
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_plan: device allocation failed");
    }
    if ((count && hipMemcpy(out.d_descs, dd.data(), sizeof(DescDev) * count, hipMemcpyHostToDevice) != hipSuccess) ||
        (!items.empty() &&
         hipMemcpy(out.d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess)) {
        free_tables(out);
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_plan: upload failed");
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_gemv_batched),
                                                     kGemvBlock, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    out.grid = std::max(1, std::min<int>(per_cu * device_cu_count(), std::max<int32_t>(1, out.nitems)));
    return FB_OK;
}

// Builds (or rebuilds) the plan's device tables from p->descs and p->tiles.
static fb_status plan_upload(fb_plan* p)
{
    plan_free_device(p);
    Tables t;
    fb_status st = build_tables(p->descs, p->tiles, t);
    if (st != FB_OK) return st;
    if (hipMalloc(&p->d_counter, 256) != hipSuccess) {
        free_tables(t);
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_plan: device allocation failed");
    }
    p->d_descs = t.d_descs;
    p->d_items = t.d_items;
    p->nitems = t.nitems;
    p->grid = t.grid;
    return FB_OK;
}

extern "C" fb_status fb_gemv_batched_plan(const fb_gemv_desc* descs, int32_t count, fb_plan** out)
{
    if (!out) return set_error(FB_ERR_ARG, "fb_gemv_batched_plan: null output");
    *out = nullptr;
    if (count < 0 || (count > 0 && !descs)) return set_error(FB_ERR_ARG, "fb_gemv_batched_plan: bad descriptor array");
    for (int i = 0; i < count; ++i) {
        const fb_gemv_desc& d = descs[i];
        fb_status st = gemv_validate("fb_gemv_batched_plan", d.f, d.m, d.n, d.A, d.lda, d.x, d.y);
        if (st != FB_OK) return set_error(st, "fb_gemv_batched_plan: descriptor %d: %s", i, fb_last_error());
    }
    fb_plan* p = new (std::nothrow) fb_plan();
    if (!p) return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_plan: out of host memory");
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_plan: no device");
    }
    p->descs.assign(descs, descs + count);
    p->tiles.resize(count);
    for (int i = 0; i < count; ++i) {
        const fb_gemv_desc& d = descs[i];
        p->tiles[i] = pick_batched_tile(d);
        const int W = d.f.base / 8;
        p->bytes += (int64_t)d.m * d.n * d.f.k + (int64_t)(d.m + d.n) * W;
    }
    fb_status st = plan_upload(p);
    if (st != FB_OK) {
        delete p;
        return st;
    }
    *out = p;
    return FB_OK;
}

static fb_status build_graph(fb_plan* p)
{
    hipGraph_t g = nullptr;
    if (hipGraphCreate(&g, 0) != hipSuccess) return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_launch: graph create");
    hipGraphNode_t n_reset = nullptr, n_run = nullptr;
    void* reset_args[] = {&p->d_counter};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(k_reset_counter);
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(1);
    kp.sharedMemBytes = 0;
    kp.kernelParams = reset_args;
    kp.extra = nullptr;
    fb_status st = FB_OK;
    if (hipGraphAddKernelNode(&n_reset, g, nullptr, 0, &kp) != hipSuccess) st = FB_ERR_RUNTIME;
    void* run_args[] = {&p->d_descs, &p->d_items, &p->nitems, &p->d_counter};
    hipKernelNodeParams kr{};
    kr.func = reinterpret_cast<void*>(k_gemv_batched);
    kr.gridDim = dim3((unsigned)p->grid);
    kr.blockDim = dim3(kGemvBlock);
    kr.sharedMemBytes = 0;
    kr.kernelParams = run_args;
    kr.extra = nullptr;
    if (st == FB_OK && hipGraphAddKernelNode(&n_run, g, &n_reset, 1, &kr) != hipSuccess) st = FB_ERR_RUNTIME;
    hipGraphExec_t e = nullptr;
    if (st == FB_OK && hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) st = FB_ERR_RUNTIME;
    if (st != FB_OK) {
        (void)hipGraphDestroy(g);
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_launch: graph construction failed");
    }
    p->graph = g;
    p->exec = e;
    return FB_OK;
}

extern "C" fb_status fb_gemv_batched_tune(fb_plan* plan, int32_t reps, hipStream_t stream)
{
    if (!plan) return set_error(FB_ERR_ARG, "fb_gemv_batched_tune: null plan");
    std::lock_guard<std::mutex> lk(plan->mu);
    if (reps < 1) reps = 1;
    // group descriptors by (format, m bucket, n bucket)
    struct Key {
        int fi, mb, nb;
        bool operator<(const Key& o) const
        {
            return fi != o.fi ? fi < o.fi : (mb != o.mb ? mb < o.mb : nb < o.nb);
        }
    };
    std::vector<std::pair<Key, int>> order;
    for (int i = 0; i < (int)plan->descs.size(); ++i) {
        const fb_gemv_desc& d = plan->descs[i];
        if (d.m == 0 || d.n == 0) continue;
        order.push_back({Key{format_index(d.f), tune_bucket(d.m), tune_bucket(d.n)}, i});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<Key, int>& a, const std::pair<Key, int>& b) { return a.first < b.first; });
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_tune: hipEventCreate failed");
    uint32_t* counter = nullptr;
    if (hipMalloc(&counter, 256) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_tune: allocation failed");
    }
    fb_status result = FB_OK;
    for (size_t g0 = 0; g0 < order.size() && result == FB_OK;) {
        size_t g1 = g0;
        while (g1 < order.size() && !(order[g0].first < order[g1].first) && !(order[g1].first < order[g0].first)) ++g1;
        // the group's GEMVs (up to 64) run alone in the persistent kernel with each candidate tile
        std::vector<fb_gemv_desc> sub;
        for (size_t j = g0; j < g1 && sub.size() < 64; ++j) sub.push_back(plan->descs[order[j].second]);
        int best = -1;
        double best_us = 1e300;
        for (int s = 0; s < kBatchedNumTiles && result == FB_OK; ++s) {
            std::vector<int> tiles(sub.size(), kBatchedTile[s]);
            Tables t;
            result = build_tables(sub, tiles, t);
            if (result != FB_OK) break;
            auto run = [&]() {
                k_reset_counter<<<1, 1, 0, stream>>>(counter);
                k_gemv_batched<<<t.grid, kGemvBlock, 0, stream>>>(t.d_descs, t.d_items, t.nitems, counter);
            };
            run();
            float ms = 0.f;
            bool ok = hipEventRecord(e0, stream) == hipSuccess;
            for (int r = 0; r < reps && ok; ++r) run();
            ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1, stream) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            free_tables(t);
            if (!ok) {
                result = set_error(FB_ERR_RUNTIME, "fb_gemv_batched_tune: timing failed");
                break;
            }
            const double us = 1000.0 * ms / reps;
            if (us < best_us) {
                best_us = us;
                best = kBatchedTile[s];
            }
        }
        if (result == FB_OK && best >= 0) {
            const fb_gemv_desc& rep = plan->descs[order[g0].second];
            tune_store(rep.f, rep.m, rep.n, best, best_us);
            for (size_t j = g0; j < g1; ++j) plan->tiles[order[j].second] = best;
        }
        g0 = g1;
    }
    (void)hipStreamSynchronize(stream);
    (void)hipFree(counter);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != FB_OK) return result;
    return plan_upload(plan);
}

extern "C" fb_status fb_gemv_batched_launch(fb_plan* plan, hipStream_t stream)
{
    if (!plan) return set_error(FB_ERR_ARG, "fb_gemv_batched_launch: null plan");
    std::lock_guard<std::mutex> lk(plan->mu);
    if (plan->nitems == 0) return FB_OK;
    if (!plan->exec) {
        fb_status st = build_graph(plan);
        if (st != FB_OK) return st;
    }
    if (hipGraphLaunch(plan->exec, stream) != hipSuccess)
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_launch: hipGraphLaunch failed");
    return FB_OK;
}

extern "C" fb_status fb_gemv_batched_loop(fb_plan* plan, hipStream_t stream)
{
    if (!plan) return set_error(FB_ERR_ARG, "fb_gemv_batched_loop: null plan");
    for (size_t i = 0; i < plan->descs.size(); ++i) {
        const fb_gemv_desc& d = plan->descs[i];
        if (d.m == 0) continue;
        fb_status st = gemv_launch_tile(d.f, d.m, d.n, d.A, d.lda, d.x, d.y, plan->tiles[i], stream);
        if (st != FB_OK) return st;
    }
    return FB_OK;
}

extern "C" fb_status fb_gemv_batched_loop_graph(fb_plan* plan, hipStream_t stream)
{
    if (!plan) return set_error(FB_ERR_ARG, "fb_gemv_batched_loop_graph: null plan");
    std::lock_guard<std::mutex> lk(plan->mu);
    if (!plan->loop_exec) {
        hipGraph_t g = nullptr;
        if (hipGraphCreate(&g, 0) != hipSuccess) return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_loop_graph: create");
        hipGraphNode_t prev = nullptr;
        bool ok = true;
        for (size_t i = 0; i < plan->descs.size() && ok; ++i) {
            const fb_gemv_desc& d = plan->descs[i];
            if (d.m == 0) continue;
            GemvArgs a{static_cast<const uint8_t*>(d.A), d.lda * d.f.k, d.x, d.y, d.m, d.n, 0, 0};
            unsigned blocks = 0;
            const void* fn = gemv_kernel_fn(d.f, plan->tiles[i], d.m, &blocks);
            void* args[] = {&a};
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(fn);
            kp.gridDim = dim3(blocks);
            kp.blockDim = dim3(kGemvBlock);
            kp.sharedMemBytes = 0;
            kp.kernelParams = args;
            kp.extra = nullptr;
            hipGraphNode_t node = nullptr;
            ok = fn && hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp) == hipSuccess;
            prev = node;
        }
        hipGraphExec_t e = nullptr;
        if (!ok || hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_loop_graph: graph construction failed");
        }
        plan->loop_graph = g;
        plan->loop_exec = e;
    }
    if (hipGraphLaunch(plan->loop_exec, stream) != hipSuccess)
        return set_error(FB_ERR_RUNTIME, "fb_gemv_batched_loop_graph: hipGraphLaunch failed");
    return FB_OK;
}

extern "C" int64_t fb_plan_bytes(const fb_plan* plan) { return plan ? plan->bytes : 0; }

extern "C" int32_t fb_plan_config(const fb_plan* plan, int32_t i)
{
    if (!plan || i < 0 || i >= (int32_t)plan->tiles.size()) return -1;
    return plan->tiles[i];
}

extern "C" void fb_plan_destroy(fb_plan* plan)
{
    if (!plan) return;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    if (have_cur && cur != plan->device) (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    plan_free_device(plan);
    if (have_cur && cur != plan->device) (void)hipSetDevice(cur);
    delete plan;
}
