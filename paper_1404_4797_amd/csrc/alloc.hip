// Device memory for every temporary of the library: a stream-ordered block
// cache in front of the device's memory pool.
//
// Freeing large blocks with hipFreeAsync was measured to hold the calling
// host thread for milliseconds per call while the device ran out of queued
// work.  Freed blocks are therefore kept per (device, stream, size class) and
// handed out again to later allocations of the same class on the same
// stream.  No event is needed for that reuse: the stream runs every earlier
// user of a block before any later one.  Size classes round a request up to
// an eighth of its leading power of two (at most 12.5 % slack).  At most a
// quarter of the device's memory stays cached; blocks beyond that go back to
// the pool.  An allocation that fails empties the cache (after a device
// synchronisation) and is tried once more.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "sclap.h"

namespace sclap {

namespace {

struct CacheKey {
    int dev;
    hipStream_t s;
    size_t cls;
    bool operator<(const CacheKey& o) const { return std::tie(dev, s, cls) < std::tie(o.dev, o.s, o.cls); }
};

struct Cache {
    std::mutex mu;
    std::map<CacheKey, std::vector<void*>> blocks;
    size_t cached[256] = {};
    size_t cap[256] = {};
    bool pool_ready[256] = {};
};

Cache& cache() {
    static Cache* c = new Cache;  // outlives static destructors of callers
    return *c;
}

size_t size_class(size_t bytes) {
    if (bytes <= 4096) return 4096;
    int lead = 63 - __builtin_clzll(static_cast<unsigned long long>(bytes));
    const size_t step = static_cast<size_t>(1) << (lead - 3);
    return (bytes + step - 1) / step * step;
}

int current_device() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256) fail(SCLAP_ERR_HIP, "device ordinal out of range");
    return dev;
}

// Called with the cache lock held.
void ready_device(Cache& c, int dev) {
    if (c.pool_ready[dev]) return;
    hipMemPool_t pool;
    HIPCHK(hipDeviceGetDefaultMemPool(&pool, dev));
    uint64_t keep = ~0ULL;  // the pool itself keeps freed memory too
    HIPCHK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    size_t fr = 0, total = 0;
    HIPCHK(hipMemGetInfo(&fr, &total));
    c.cap[dev] = total / 4;
    c.pool_ready[dev] = true;
}

// Frees every cached block of dev (all streams) or of one stream; lock held.
void drop_blocks(Cache& c, int dev, bool one_stream, hipStream_t s) {
    for (auto it = c.blocks.begin(); it != c.blocks.end();) {
        if (it->first.dev == dev && (!one_stream || it->first.s == s)) {
            for (void* p : it->second) {
                (void)hipFreeAsync(p, it->first.s);
                c.cached[dev] -= it->first.cls;
            }
            it = c.blocks.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s) {
    Cache& c = cache();
    const int dev = current_device();
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        ready_device(c, dev);
        auto it = c.blocks.find(CacheKey{dev, s, cls});
        if (it != c.blocks.end() && !it->second.empty()) {
            void* p = it->second.back();
            it->second.pop_back();
            c.cached[dev] -= cls;
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMallocAsync(&p, cls, s);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(c.mu);
            drop_blocks(c, dev, false, nullptr);
        }
        (void)hipDeviceSynchronize();
        e = hipMallocAsync(&p, cls, s);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? SCLAP_ERR_NO_MEMORY : SCLAP_ERR_HIP,
             "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    return p;
}

void dev_free(void* p, size_t bytes, hipStream_t s) {
    if (!p) return;
    Cache& c = cache();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) {
        (void)hipFreeAsync(p, s);
        return;
    }
    const size_t cls = size_class(bytes);
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.pool_ready[dev] || c.cached[dev] + cls > c.cap[dev]) {
        (void)hipFreeAsync(p, s);
        return;
    }
    c.blocks[CacheKey{dev, s, cls}].push_back(p);
    c.cached[dev] += cls;
}

void release_cached(hipStream_t s, bool all_streams) {
    Cache& c = cache();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) return;
    std::lock_guard<std::mutex> lk(c.mu);
    drop_blocks(c, dev, !all_streams, s);
}

}  // namespace sclap
