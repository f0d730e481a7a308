// Stream-keyed cache of device scratch blocks.
//
// Returning a block to the stream-ordered pool (hipFreeAsync) costs about a
// quarter of a millisecond of host time on this runtime, which would make a
// CP-ALS sweep (tens of temporaries) host-bound.  Blocks released here are
// kept per (device, stream, size class) and handed out again to later
// requests on the same stream: stream order guarantees that the earlier work
// using the block has finished before later work touches it.  Blocks are
// never shared across streams.  The cache is bounded; beyond the bound a
// released block goes back to the pool.
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

namespace cpd {
namespace {

constexpr size_t kCacheMax = 24ull << 30;  // bytes kept cached per process

std::atomic<int64_t> g_alloc_limit{-1};  // bytes; -1: no limit

struct Cache {
    std::mutex mu;
    std::multimap<std::tuple<int, uintptr_t, size_t>, void *> blocks;  // (device, stream, class) -> block
    size_t bytes = 0;
};

Cache &cache() {
    static Cache *c = new Cache();  // never destroyed: blocks live until the process ends
    return *c;
}

// size classes: 4 KiB, then 2^k * {1, 1.25, 1.5, 1.75} (at most 25% slack)
size_t size_class(size_t b) {
    if (b <= 4096) return 4096;
    int k = 63 - __builtin_clzll(b);
    const size_t base = (size_t)1 << k;
    for (int q = 0; q <= 4; ++q) {
        const size_t c = base + (base >> 2) * q;
        if (c >= b) return c;
    }
    return base << 1;
}

}  // namespace

cpd_status device_alloc(void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    const int64_t lim = g_alloc_limit.load();
    if (lim >= 0 && bytes > (size_t)lim)
        CPD_FAIL(CPD_ENOMEM, "device allocation of %zu bytes refused (limit %lld bytes)", bytes, (long long)lim);
    if (hipMallocAsync(p, bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        CPD_FAIL(CPD_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    return CPD_OK;
}

cpd_status scratch_get(size_t bytes, hipStream_t s, void **p) {
    *p = nullptr;
    // the limit applies to cached blocks too (a request is refused or not
    // whatever the cache holds)
    const int64_t lim = g_alloc_limit.load();
    if (lim >= 0 && bytes > (size_t)lim)
        CPD_FAIL(CPD_ENOMEM, "device allocation of %zu bytes refused (limit %lld bytes)", bytes, (long long)lim);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        CPD_FAIL(CPD_EHIP, "no current device");
    }
    const size_t cls = size_class(bytes);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.blocks.find(std::make_tuple(dev, (uintptr_t)s, cls));
        if (it != c.blocks.end()) {
            *p = it->second;
            c.blocks.erase(it);
            c.bytes -= cls;
            return CPD_OK;
        }
    }
    return device_alloc(p, cls, s);
}

void scratch_put(void *p, size_t bytes, hipStream_t s) {
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFreeAsync(p, s);
        return;
    }
    const size_t cls = size_class(bytes);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        if (c.bytes + cls <= kCacheMax) {
            c.blocks.emplace(std::make_tuple(dev, (uintptr_t)s, cls), p);
            c.bytes += cls;
            return;
        }
    }
    (void)hipFreeAsync(p, s);
}

}  // namespace cpd

extern "C" cpd_status cpd_set_alloc_limit(int64_t bytes) {
    cpd::g_alloc_limit.store(bytes < 0 ? -1 : bytes);
    return CPD_OK;
}
