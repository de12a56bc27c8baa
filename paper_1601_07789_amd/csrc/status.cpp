// Status strings, per-thread error detail, and small device queries.
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace flyte {

static thread_local char g_last_error[512] = "";

fb_status set_error(fb_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return st;
}

void clear_error() { g_last_error[0] = '\0'; }

int device_cu_count()
{
    static std::mutex mu;
    static std::unordered_map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    cache[dev] = cus;
    return cus;
}

fb_status stream_workspace(hipStream_t stream, size_t bytes, void** out)
{
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, std::pair<void*, size_t>> cache;
    // Buffers handed out before a stream's workspace grew.  They are never
    // freed: a graph captured from an earlier call still names its buffer, and
    // replaying it must not write freed memory.  Each growth at least doubles
    // the size, so these hold less than the current buffer.
    static std::vector<void*> retired;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(FB_ERR_RUNTIME, "workspace: hipGetDevice failed");
    std::lock_guard<std::mutex> lk(mu);
    auto& slot = cache[std::make_pair(dev, stream)];
    if (slot.second < bytes) {
        // allocating is not allowed while the stream is being captured into a graph
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
            return set_error(FB_ERR_RUNTIME,
                             "workspace: %zu bytes needed while the stream is being captured; make one call of "
                             "the same size on this stream outside capture first",
                             bytes);
        size_t want = bytes < 2 * slot.second ? 2 * slot.second : bytes;
        if (want < 16384) want = 16384;
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) return set_error(FB_ERR_RUNTIME, "workspace: allocation failed");
        if (slot.first) retired.push_back(slot.first);
        slot = {p, want};
    }
    *out = slot.first;
    return FB_OK;
}

}  // namespace flyte

extern "C" const char* fb_status_str(fb_status status)
{
    switch (status) {
        case FB_OK: return "FB_OK";
        case FB_ERR_FORMAT: return "FB_ERR_FORMAT";
        case FB_ERR_ARG: return "FB_ERR_ARG";
        case FB_ERR_ALIGN: return "FB_ERR_ALIGN";
        case FB_ERR_UNSUPPORTED: return "FB_ERR_UNSUPPORTED";
        case FB_ERR_RUNTIME: return "FB_ERR_RUNTIME";
    }
    return "FB_ERR_UNKNOWN";
}

extern "C" const char* fb_last_error(void) { return flyte::g_last_error; }
