// Device and pinned-host memory caches.
//
// Every build, partition and count allocates and frees scratch arrays whose
// sizes repeat from call to call.  The stream-ordered HIP allocator was
// measured at tens of microseconds per allocation and up to milliseconds per
// free of a large block on this stack, with the GPU idle meanwhile, so the
// library keeps its own caches:
//
//  - sizes are rounded up to one of four classes per power of two (at most
//    25% slack, 512 B minimum), and a freed block waits in its class's free
//    list for the next request of that class;
//  - a free records an event on the stream it is freed on; the next user
//    waits for that event on its own stream (hipStreamWaitEvent) unless the
//    event has already completed, so reuse is ordered after every earlier use
//    whatever stream takes the block;
//  - pinned host blocks (for small copies between host tables and the
//    device, which would otherwise be pageable and synchronous, and for the
//    host block store of a streamed graph) work the same way, except that
//    the host waits for the event before reuse;
//  - when the free lists exceed a limit (a quarter of device memory; for
//    pinned memory an eighth of physical memory, within 4 - 64 GiB) the
//    largest blocks go back to HIP; a failed allocation returns every
//    cached block and tries once more.
//
// While a caller's allocator hook is installed, new device allocations go
// through it instead; blocks the cache handed out still come back to it.
#include <unistd.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace pgabb {

namespace {

std::mutex g_hook_mu;
pgabb_alloc_fn g_alloc = nullptr;
pgabb_free_fn g_free = nullptr;
void *g_alloc_ctx = nullptr;

size_t size_class(size_t b) {
    if (b <= 512) return 512;
    const int e = 63 - __builtin_clzll(static_cast<unsigned long long>(b - 1));  // 2^e < b <= 2^(e+1)
    const size_t step = (size_t(1) << e) / 4;
    return (b + step - 1) / step * step;
}

struct FreeBlock {
    void *p;
    hipEvent_t ev;
};

struct Cache {
    std::mutex mu;
    std::multimap<size_t, FreeBlock> free;  // class -> blocks
    std::unordered_map<void *, size_t> live;  // pointer -> class
    std::vector<hipEvent_t> events;           // spare events
    size_t cached = 0;
    size_t limit = 0;
    bool host = false;

    hipEvent_t take_event() {
        if (!events.empty()) {
            hipEvent_t e = events.back();
            events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        PGABB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return e;
    }

    void hip_free(void *p) {
        if (host) (void)hipHostFree(p);
        else (void)hipFree(p);
    }

    // Return free blocks to HIP, largest first, until `keep` bytes remain.
    // Called with mu held.
    void trim(size_t keep) {
        while (cached > keep && !free.empty()) {
            auto it = std::prev(free.end());
            (void)hipEventSynchronize(it->second.ev);
            hip_free(it->second.p);
            events.push_back(it->second.ev);
            cached -= it->first;
            free.erase(it);
        }
    }
};

std::mutex g_caches_mu;
std::vector<std::unique_ptr<Cache>> g_dev_caches;
Cache g_host_cache;

Cache &device_cache() {
    int dev = 0;
    PGABB_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_caches_mu);
    if (g_dev_caches.size() <= static_cast<size_t>(dev)) g_dev_caches.resize(dev + 1);
    if (!g_dev_caches[dev]) {
        auto c = std::make_unique<Cache>();
        size_t fr = 0, total = 0;
        PGABB_HIP(hipMemGetInfo(&fr, &total));
        c->limit = total / 4;
        g_dev_caches[dev] = std::move(c);
    }
    return *g_dev_caches[dev];
}

Cache &host_cache() {
    static std::once_flag once;
    std::call_once(once, [] {
        g_host_cache.host = true;
        // room for a streamed graph's block store between calls: an eighth
        // of physical memory, at least 4 GiB and at most 64 GiB
        const long pages = sysconf(_SC_PHYS_PAGES), psz = sysconf(_SC_PAGE_SIZE);
        const size_t phys = pages > 0 && psz > 0 ? static_cast<size_t>(pages) * static_cast<size_t>(psz) : 0;
        g_host_cache.limit = std::clamp(phys / 8, size_t(4) << 30, size_t(64) << 30);
    });
    return g_host_cache;
}

// Take a cached block of class `cls`, or nullptr.  For device blocks the
// stream `s` is made to wait for the block's last free; for host blocks the
// host waits.
void *take(Cache &c, size_t cls, hipStream_t s) {
    FreeBlock fb{nullptr, nullptr};
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto range = c.free.equal_range(cls);
        if (range.first == range.second) return nullptr;
        auto pick = range.first;
        for (auto it = range.first; it != range.second; ++it)
            if (hipEventQuery(it->second.ev) == hipSuccess) {
                pick = it;
                break;
            }
        fb = pick->second;
        c.free.erase(pick);
        c.cached -= cls;
        c.live[fb.p] = cls;
    }
    if (hipEventQuery(fb.ev) != hipSuccess) {
        if (c.host) PGABB_HIP(hipEventSynchronize(fb.ev));
        else PGABB_HIP(hipStreamWaitEvent(s, fb.ev, 0));
    }
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(c.mu);
    c.events.push_back(fb.ev);
    return fb.p;
}

void *fresh(Cache &c, size_t cls) {
    void *p = nullptr;
    for (int attempt = 0; attempt < 2; ++attempt) {
        hipError_t e = c.host ? hipHostMalloc(&p, cls, hipHostMallocDefault) : hipMalloc(&p, cls);
        if (e == hipSuccess && p) {
            std::lock_guard<std::mutex> lk(c.mu);
            c.live[p] = cls;
            return p;
        }
        (void)hipGetLastError();
        p = nullptr;
        if (attempt == 0) {
            std::lock_guard<std::mutex> lk(c.mu);
            if (c.cached == 0) break;
            c.trim(0);
        }
    }
    fail(PGABB_ENOMEM, "%s(%zu bytes) failed", c.host ? "hipHostMalloc" : "hipMalloc", cls);
    return nullptr;
}

// Returns false if `p` did not come from this cache.
bool give_back(Cache &c, void *p, hipStream_t s) {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return false;
    const size_t cls = it->second;
    c.live.erase(it);
    hipEvent_t ev = c.take_event();
    if (hipEventRecord(ev, s) != hipSuccess) {
        // the stream is unusable: wait for the whole device instead
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();
        (void)hipEventRecord(ev, nullptr);
        (void)hipGetLastError();
    }
    c.free.insert({cls, FreeBlock{p, ev}});
    c.cached += cls;
    if (c.cached > c.limit) c.trim(c.limit / 2);
    return true;
}

}  // namespace

void set_allocator_hook(pgabb_alloc_fn fa, pgabb_free_fn ff, void *ctx) {
    std::lock_guard<std::mutex> lk(g_hook_mu);
    g_alloc = fa;
    g_free = ff;
    g_alloc_ctx = ctx;
}

void *dalloc(size_t bytes, hipStream_t s) {
    if (!bytes) return nullptr;
    pgabb_alloc_fn fa;
    void *ctx;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        fa = g_alloc;
        ctx = g_alloc_ctx;
    }
    if (fa) {
        void *p = fa(bytes, s, ctx);
        if (!p) fail(PGABB_ENOMEM, "allocator hook failed for %zu bytes", bytes);
        return p;
    }
    Cache &c = device_cache();
    const size_t cls = size_class(bytes);
    if (void *p = take(c, cls, s)) return p;
    return fresh(c, cls);
}

void dfree(void *p, hipStream_t s) noexcept {
    if (!p) return;
    try {
        // blocks from a cache go back to it even if a hook was installed since
        if (give_back(device_cache(), p, s)) return;
        std::vector<Cache *> others;
        {
            std::lock_guard<std::mutex> lk(g_caches_mu);
            for (auto &c : g_dev_caches)
                if (c) others.push_back(c.get());
        }
        for (Cache *c : others)
            if (give_back(*c, p, s)) return;  // freed while another device is current
        pgabb_free_fn ff;
        void *ctx;
        {
            std::lock_guard<std::mutex> lk(g_hook_mu);
            ff = g_free;
            ctx = g_alloc_ctx;
        }
        if (ff) ff(p, s, ctx);
    } catch (...) {
        // reached from destructors: nothing useful to report
    }
}

void *halloc(size_t bytes) {
    if (!bytes) return nullptr;
    Cache &c = host_cache();
    const size_t cls = size_class(bytes);
    if (void *p = take(c, cls, nullptr)) return p;
    return fresh(c, cls);
}

void hfree(void *p, hipStream_t s) noexcept {
    if (!p) return;
    try {
        (void)give_back(host_cache(), p, s);
    } catch (...) {
    }
}

void release_cached_memory() {
    std::vector<Cache *> all;
    {
        std::lock_guard<std::mutex> lk(g_caches_mu);
        for (auto &c : g_dev_caches)
            if (c) all.push_back(c.get());
    }
    all.push_back(&host_cache());
    for (Cache *c : all) {
        std::lock_guard<std::mutex> lk(c->mu);
        c->trim(0);
    }
}

size_t cached_bytes(bool host) {
    if (host) {
        Cache &c = host_cache();
        std::lock_guard<std::mutex> lk(c.mu);
        return c.cached;
    }
    Cache &c = device_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    return c.cached;
}

}  // namespace pgabb
