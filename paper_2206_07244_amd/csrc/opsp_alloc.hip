// Device-memory cache of the library (OpSparse Section 5.3-5.4: the paper
// keeps metadata in one self-managed allocation and hides cudaMalloc behind
// running kernels because allocation is far slower than memory access).
//
// On this stack a stream-ordered pool allocation or release costs tens to
// hundreds of microseconds of host time per call, which is more than a whole
// small SpGEMM.  The library therefore keeps released blocks in per-device
// free lists keyed by (stream, size class) and hands them out again without
// any HIP call.  A block released on stream s is reused only by work ordered
// after the release on the same stream, so no synchronisation is needed.
// Blocks come from hipMallocAsync on the requesting stream; when that fails,
// the cache of the device is returned to HIP (after a device synchronise)
// and the allocation is retried.  opsp_cache_release() empties the cache.
#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "opsp.h"
#include "opsp_internal.h"

namespace opsp {
namespace {

struct Block {
    void *ptr;
    size_t bytes;   // size class actually allocated
};

struct DeviceCache {
    // (stream, size class) -> free blocks
    std::map<std::pair<hipStream_t, size_t>, std::vector<void *>> free_lists;
    std::unordered_map<void *, Block> live;    // handed-out blocks
    size_t cached_bytes = 0;
    size_t live_bytes = 0;
};

std::mutex g_cache_mu;
std::unordered_map<int, DeviceCache> g_cache;

// Testing: allocations still to succeed before one fails (-1 = never).
std::atomic<int64_t> g_fail_after{-1};

bool injected_failure() {
    int64_t n = g_fail_after.load();
    while (n >= 0) {
        if (g_fail_after.compare_exchange_weak(n, n - 1)) return n == 0;
    }
    return false;
}

// Size classes: multiples of 256 B below 64 KB, then 8 classes per power of
// two (at most 12.5 % rounding).
size_t size_class(size_t bytes) {
    if (bytes <= 65536) return (bytes + 255) & ~size_t(255);
    size_t p = 1;
    while ((p << 1) <= bytes) p <<= 1;
    const size_t step = p >> 3;
    return (bytes + step - 1) / step * step;
}

// Frees every cached block of device `dev` (current) and, with `trim`,
// shrinks the device's default pool to what is still allocated from it: the
// library raises the pool's release threshold, so freed blocks would stay
// reserved by the pool and out of reach of other allocators in the process.
void release_device(int dev, DeviceCache &dc, bool trim) {
    for (auto &kv : dc.free_lists)
        for (void *p : kv.second) (void)hipFree(p);
    dc.free_lists.clear();
    dc.cached_bytes = 0;
    hipMemPool_t pool;
    if (trim && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        (void)hipDeviceSynchronize();
        (void)hipMemPoolTrimTo(pool, 0);
    }
}

}  // namespace

hipError_t cache_alloc(void **out, size_t bytes, hipStream_t s) {
    *out = nullptr;
    if (bytes == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (injected_failure()) return hipErrorOutOfMemory;
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        DeviceCache &dc = g_cache[dev];
        auto it = dc.free_lists.find({s, cls});
        if (it != dc.free_lists.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            dc.cached_bytes -= cls;
            dc.live_bytes += cls;
            dc.live[p] = Block{p, cls};
            *out = p;
            return hipSuccess;
        }
    }
    e = hipMallocAsync(out, cls, s);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            release_device(dev, g_cache[dev], false);
        }
        e = hipMallocAsync(out, cls, s);
    }
    if (e != hipSuccess) {
        // the status goes back to the caller; leave no error behind for the
        // next HIP call of the process to report as its own
        (void)hipGetLastError();
        *out = nullptr;
        return e;
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[dev].live[*out] = Block{*out, cls};
    g_cache[dev].live_bytes += cls;
    return hipSuccess;
}

// Returns the block to the cache of the current device.  Pointers the cache
// did not hand out are released with hipFreeAsync.
hipError_t cache_free(void *p, hipStream_t s) {
    if (!p) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        DeviceCache &dc = g_cache[dev];
        auto it = dc.live.find(p);
        if (it != dc.live.end()) {
            const size_t cls = it->second.bytes;
            dc.live.erase(it);
            dc.live_bytes -= cls;
            dc.free_lists[{s, cls}].push_back(p);
            dc.cached_bytes += cls;
            return hipSuccess;
        }
    }
    return hipFreeAsync(p, s);
}

hipError_t cache_release_all() {
    hipError_t e = hipDeviceSynchronize();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    release_device(dev, g_cache[dev], true);
    return e;
}

size_t cache_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return g_cache[dev].cached_bytes;
}

size_t live_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return g_cache[dev].live_bytes;
}

}  // namespace opsp

extern "C" {

opsp_status opsp_cache_release(void) {
    return opsp::cache_release_all() == hipSuccess ? OPSP_OK : OPSP_ERR_HIP;
}

int64_t opsp_cache_bytes(void) { return (int64_t)opsp::cache_bytes(); }

int64_t opsp_cache_live_bytes(void) { return (int64_t)opsp::live_bytes(); }

void opsp_debug_fail_alloc(int64_t n) { opsp::g_fail_after.store(n < 0 ? -1 : n); }

}  // extern "C"
