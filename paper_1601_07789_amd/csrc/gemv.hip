// fb_gemv, its forced-configuration variant, and the tile autotuner.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "gemv_impl.hpp"

namespace flyte {

template <class F, class TILE>
__global__ void __launch_bounds__(kGemvBlock) k_gemv(GemvArgs a)
{
    gemv_block<F, TILE>(a, (int64_t)blockIdx.x * TILE::rows_per_block);
}

template <class F>
static fb_status launch_gemv(const GemvArgs& a, int tile, hipStream_t stream)
{
    switch (tile) {
#define FLYTE_TILE_LAUNCH(ID, LPR, RPW, U, KS, NT, ST, PP)                                   \
    case ID: {                                                                               \
        using TL = GemvTile<LPR, RPW, U, KS, NT, ST, PP>;                                    \
        const int64_t blocks = (a.m + TL::rows_per_block - 1) / TL::rows_per_block;          \
        k_gemv<F, TL><<<(unsigned)blocks, kGemvBlock, 0, stream>>>(a);                       \
        return check_launch("fb_gemv");                                                      \
    }
        FLYTE_GEMV_TILES(FLYTE_TILE_LAUNCH)
#undef FLYTE_TILE_LAUNCH
    }
    return set_error(FB_ERR_ARG, "fb_gemv: bad tile configuration %d", tile);
}

// Kernel entry point and grid size of one GEMV launch with a given tile (used
// to build graphs of GEMV launches).
const void* gemv_kernel_fn(fb_format f, int tile, int64_t m, unsigned* blocks)
{
    return dispatch_format(f, [&](auto tag) -> const void* {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        switch (tile) {
#define FLYTE_TILE_FN(ID, LPR, RPW, U, KS, NT, ST, PP)                                     \
    case ID: {                                                                             \
        using TL = GemvTile<LPR, RPW, U, KS, NT, ST, PP>;                                  \
        *blocks = (unsigned)((m + TL::rows_per_block - 1) / TL::rows_per_block);           \
        return reinterpret_cast<const void*>(k_gemv<F, TL>);                               \
    }
            FLYTE_GEMV_TILES(FLYTE_TILE_FN)
#undef FLYTE_TILE_FN
        }
        return nullptr;
    });
}

fb_status gemv_validate(const char* what, fb_format f, int64_t m, int64_t n, const void* A, int64_t lda,
                        const void* x, const void* y)
{
    if (!format_ok(f)) return set_error(FB_ERR_FORMAT, "%s: invalid format {%d,%d}", what, f.base, f.k);
    if (m < 0 || n < 0 || m > INT32_MAX || n > INT32_MAX)
        return set_error(FB_ERR_ARG, "%s: bad sizes m=%lld n=%lld", what, (long long)m, (long long)n);
    if (lda < n || lda < 0) return set_error(FB_ERR_ARG, "%s: lda=%lld < n=%lld", what, (long long)lda, (long long)n);
    if (m == 0) return FB_OK;
    if (!A || !x || !y) return set_error(FB_ERR_ARG, "%s: null pointer", what);
    if (!aligned4(A) || !aligned4(x) || !aligned4(y) || ((lda * f.k) % 4) != 0)
        return set_error(FB_ERR_ALIGN, "%s: pointers and rows (lda*k) must be 4-byte aligned", what);
    return FB_OK;
}

fb_status gemv_launch_tile(fb_format f, int64_t m, int64_t n, const void* A, int64_t lda, const void* x, void* y,
                           int tile, hipStream_t stream, int yk, int ymode)
{
    GemvArgs a{static_cast<const uint8_t*>(A), lda * f.k, x, y, (int32_t)m, (int32_t)n, yk, ymode};
    return dispatch_format(f, [&](auto tag) {
        using F = Fmt<decltype(tag.first)::value, decltype(tag.second)::value>;
        return launch_gemv<F>(a, tile, stream);
    });
}

// ---------------------------------------------------------------- tile cache
struct TuneKey {
    int base, k, mb, nb;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(base, k, mb, nb) < std::tie(o.base, o.k, o.mb, o.nb);
    }
};

int tune_bucket(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

static std::mutex g_tune_mu;
static std::map<TuneKey, std::pair<int, double>> g_tune;   // tile, microseconds

int tune_lookup(fb_format f, int64_t m, int64_t n)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{f.base, f.k, tune_bucket(m), tune_bucket(n)});
    return it == g_tune.end() ? -1 : it->second.first;
}

void tune_store(fb_format f, int64_t m, int64_t n, int tile, double us)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey{f.base, f.k, tune_bucket(m), tune_bucket(n)}] = {tile, us};
}

int gemv_pick_tile(fb_format f, int64_t m, int64_t n)
{
    const int t = tune_lookup(f, m, n);
    return t >= 0 ? t : gemv_default_tile(m, n, f.k);
}

}  // namespace flyte

using namespace flyte;

extern "C" int32_t fb_gemv_num_configs(void) { return kGemvNumTiles; }

extern "C" int32_t fb_gemv_config_info(int32_t config, int32_t* rows_per_wave, int32_t* waves_per_block,
                                       int32_t* chunks_per_lane)
{
    if (config < 0 || config >= kGemvNumTiles) return 0;
    const TileInfo t = gemv_tile_info(config);
    if (rows_per_wave) *rows_per_wave = (64 / t.lpr) * t.rpw;
    if (waves_per_block) *waves_per_block = t.ks;
    if (chunks_per_lane) *chunks_per_lane = t.u;
    return t.lpr;
}

extern "C" fb_status fb_gemv_config(fb_format f, int64_t m, int64_t n, const void* A, int64_t lda, const void* x,
                                    void* y, int32_t config, hipStream_t stream)
{
    fb_status st = gemv_validate("fb_gemv", f, m, n, A, lda, x, y);
    if (st != FB_OK || m == 0) return st;
    if (config < 0 || config >= kGemvNumTiles) return set_error(FB_ERR_ARG, "fb_gemv: config %d out of range", config);
    return gemv_launch_tile(f, m, n, A, lda, x, y, config, stream);
}

extern "C" fb_status fb_gemv(fb_format f, int64_t m, int64_t n, const void* A, int64_t lda, const void* x, void* y,
                             hipStream_t stream)
{
    fb_status st = gemv_validate("fb_gemv", f, m, n, A, lda, x, y);
    if (st != FB_OK || m == 0) return st;
    return gemv_launch_tile(f, m, n, A, lda, x, y, gemv_pick_tile(f, m, n), stream);
}

extern "C" fb_status fb_gemv_ex(fb_format fa, fb_format fy, int32_t trans, int64_t m, int64_t n, const void* A,
                                int64_t lda, const void* x, void* y, hipStream_t stream)
{
    fb_status st = gemv_validate("fb_gemv_ex", fa, m, n, A, lda, x, y);
    if (st != FB_OK) return st;
    if (!format_ok(fy) || fy.base != fa.base)
        return set_error(FB_ERR_FORMAT, "fb_gemv_ex: y format must be a valid format of the same base");
    if (trans != 0 && trans != 1) return set_error(FB_ERR_ARG, "fb_gemv_ex: trans must be 0 or 1");
    if (trans == 1) return gemv_t_launch(fa, fy, m, n, A, lda, x, y, stream);
    if (m == 0) return FB_OK;
    const int yk = (fy.k * 8 == fy.base) ? 0 : fy.k;
    return gemv_launch_tile(fa, m, n, A, lda, x, y, gemv_pick_tile(fa, m, n), stream, yk, fy.round);
}

extern "C" int32_t fb_tune_lookup(fb_format f, int64_t m, int64_t n)
{
    if (!format_ok(f)) return -1;
    return tune_lookup(f, m, n);
}

extern "C" fb_status fb_tune_gemv(fb_format f, int64_t m, int64_t n, const void* A, int64_t lda, const void* x,
                                  void* y, int32_t reps, int32_t* best, hipStream_t stream)
{
    fb_status st = gemv_validate("fb_tune_gemv", f, m, n, A, lda, x, y);
    if (st != FB_OK) return st;
    if (m == 0 || n == 0) return set_error(FB_ERR_ARG, "fb_tune_gemv: empty shape");
    if (reps < 1) reps = 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(FB_ERR_RUNTIME, "fb_tune_gemv: hipEventCreate failed");
    int best_tile = -1;
    double best_us = 1e300;
    fb_status result = FB_OK;
    for (int t = 0; t < kGemvNumTiles && result == FB_OK; ++t) {
        for (int w = 0; w < 2 && result == FB_OK; ++w) result = gemv_launch_tile(f, m, n, A, lda, x, y, t, stream);
        if (result != FB_OK) break;
        if (hipEventRecord(e0, stream) != hipSuccess) {
            result = set_error(FB_ERR_RUNTIME, "fb_tune_gemv: hipEventRecord failed");
            break;
        }
        for (int r = 0; r < reps && result == FB_OK; ++r) result = gemv_launch_tile(f, m, n, A, lda, x, y, t, stream);
        float ms = 0.f;
        if (result != FB_OK || hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            if (result == FB_OK) result = set_error(FB_ERR_RUNTIME, "fb_tune_gemv: timing failed");
            break;
        }
        const double us = 1000.0 * ms / reps;
        if (us < best_us) {
            best_us = us;
            best_tile = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != FB_OK) return result;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[TuneKey{f.base, f.k, tune_bucket(m), tune_bucket(n)}] = {best_tile, best_us};
    }
    if (best) *best = best_tile;
    return FB_OK;
}

extern "C" fb_status fb_tune_record(fb_format f, int64_t m, int64_t n, int32_t config, double us)
{
    if (!format_ok(f)) return set_error(FB_ERR_FORMAT, "fb_tune_record: invalid format {%d,%d}", f.base, f.k);
    if (m <= 0 || n <= 0) return set_error(FB_ERR_ARG, "fb_tune_record: empty shape");
    if (config < 0 || config >= kGemvNumTiles) return set_error(FB_ERR_ARG, "fb_tune_record: bad config %d", config);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey{f.base, f.k, tune_bucket(m), tune_bucket(n)}] = {config, us};
    return FB_OK;
}

static const char* cache_path(const char* path)
{
    if (path && *path) return path;
    const char* env = getenv("FLYTE_TUNE_CACHE");
    return (env && *env) ? env : nullptr;
}

extern "C" fb_status fb_tune_save(const char* path)
{
    const char* p = cache_path(path);
    if (!p) return set_error(FB_ERR_ARG, "fb_tune_save: no path and FLYTE_TUNE_CACHE unset");
    FILE* fh = fopen(p, "w");
    if (!fh) return set_error(FB_ERR_ARG, "fb_tune_save: cannot open %s", p);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    fprintf(fh, "{\"version\": 1, \"kind\": \"flyte-gemv-tiles\", \"entries\": [\n");
    size_t i = 0;
    for (const auto& kv : g_tune) {
        fprintf(fh, "  {\"base\": %d, \"k\": %d, \"m_bucket\": %d, \"n_bucket\": %d, \"tile\": %d, \"us\": %.3f}%s\n",
                kv.first.base, kv.first.k, kv.first.mb, kv.first.nb, kv.second.first, kv.second.second,
                ++i < g_tune.size() ? "," : "");
    }
    fprintf(fh, "]}\n");
    fclose(fh);
    return FB_OK;
}

extern "C" fb_status fb_tune_load(const char* path)
{
    const char* p = cache_path(path);
    if (!p) return set_error(FB_ERR_ARG, "fb_tune_load: no path and FLYTE_TUNE_CACHE unset");
    FILE* fh = fopen(p, "r");
    if (!fh) return set_error(FB_ERR_ARG, "fb_tune_load: cannot open %s", p);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, fh)) > 0) text.append(buf, got);
    fclose(fh);
    // one entry object per '{' after the entries key
    size_t pos = text.find("\"entries\"");
    if (pos == std::string::npos) return set_error(FB_ERR_ARG, "fb_tune_load: %s has no entries", p);
    std::vector<std::pair<TuneKey, std::pair<int, double>>> parsed;
    while ((pos = text.find('{', pos + 1)) != std::string::npos) {
        int base, k, mb, nb, tile;
        double us;
        if (sscanf(text.c_str() + pos,
                   "{\"base\": %d, \"k\": %d, \"m_bucket\": %d, \"n_bucket\": %d, \"tile\": %d, \"us\": %lf}", &base,
                   &k, &mb, &nb, &tile, &us) != 6)
            return set_error(FB_ERR_ARG, "fb_tune_load: malformed entry in %s", p);
        if (!format_ok(fb_format{(uint8_t)base, (uint8_t)k}) || tile < 0 || tile >= kGemvNumTiles)
            return set_error(FB_ERR_ARG, "fb_tune_load: invalid entry in %s", p);
        parsed.push_back({TuneKey{base, k, mb, nb}, {tile, us}});
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& e : parsed) g_tune[e.first] = e.second;
    return FB_OK;
}

extern "C" void fb_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}
