// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pgabb.h"

namespace pgabb {

// ------------------------------------------------------------------ errors

struct Error {
    pgabb_status status;
    std::string message;
};

[[noreturn]] void fail(pgabb_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define PGABB_HIP(call)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            ::pgabb::fail(e_ == hipErrorOutOfMemory ? PGABB_ENOMEM : PGABB_EDEVICE,           \
                          "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define PGABB_REQUIRE(cond, st, ...)        \
    do {                                    \
        if (!(cond)) ::pgabb::fail(st, __VA_ARGS__); \
    } while (0)

// --------------------------------------------------------- device memory

// Device allocation goes through the caller's hook when one is installed,
// else through the library's caching allocator (memory.cpp): blocks are
// reused by size class, and reuse on any stream is ordered after the
// block's last free by an event.
void *dalloc(size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s) noexcept;
// Pinned host blocks from a cache of the same kind; hfree(p, s) returns the
// block once the work enqueued on s so far has finished with it.
void *halloc(size_t bytes);
void hfree(void *p, hipStream_t s) noexcept;
void set_allocator_hook(pgabb_alloc_fn fa, pgabb_free_fn ff, void *ctx);
void release_cached_memory();
size_t cached_bytes(bool host);

// Owning device array.  Freed on the stream it was allocated on.
template <class T>
class DArray {
  public:
    DArray() = default;
    DArray(size_t n, hipStream_t s) { reset(n, s); }
    ~DArray() { release(); }
    DArray(const DArray &) = delete;
    DArray &operator=(const DArray &) = delete;
    DArray(DArray &&o) noexcept { swap(o); }
    DArray &operator=(DArray &&o) noexcept {
        if (this != &o) {
            release();
            swap(o);
        }
        return *this;
    }
    void reset(size_t n, hipStream_t s) {
        release();
        stream_ = s;
        n_ = n;
        ptr_ = n ? static_cast<T *>(dalloc(n * sizeof(T), s)) : nullptr;
    }
    void release() {
        if (ptr_) dfree(ptr_, stream_);
        ptr_ = nullptr;
        n_ = 0;
    }
    void swap(DArray &o) noexcept {
        std::swap(ptr_, o.ptr_);
        std::swap(n_, o.n_);
        std::swap(stream_, o.stream_);
    }
    T *get() const { return ptr_; }
    size_t size() const { return n_; }
    size_t bytes() const { return n_ * sizeof(T); }

  private:
    T *ptr_ = nullptr;
    size_t n_ = 0;
    hipStream_t stream_ = nullptr;
};

// Pinned host array.  reset(n) allocates with hipHostMalloc; reset(n, s,
// true) takes the block from the pinned cache (halloc) instead, and release
// returns it there, ordered after the work then queued on s: for large
// stores that are rebuilt call after call, whose hipHostMalloc and
// hipHostFree would otherwise repeat.
template <class T>
class PinnedArray {
  public:
    PinnedArray() = default;
    ~PinnedArray() { release(); }
    PinnedArray(const PinnedArray &) = delete;
    PinnedArray &operator=(const PinnedArray &) = delete;
    void reset(size_t n, hipStream_t s = nullptr, bool cached = false) {
        release();
        if (n) {
            if (cached) {
                ptr_ = static_cast<T *>(halloc(n * sizeof(T)));
            } else {
                void *p = nullptr;
                hipError_t e = hipHostMalloc(&p, n * sizeof(T), hipHostMallocDefault);
                if (e != hipSuccess)
                    fail(PGABB_ENOMEM, "hipHostMalloc(%zu bytes): %s", n * sizeof(T), hipGetErrorString(e));
                ptr_ = static_cast<T *>(p);
            }
        }
        n_ = n;
        stream_ = s;
        cached_ = cached;
    }
    void release() {
        if (ptr_) {
            if (cached_) hfree(ptr_, stream_);
            else (void)hipHostFree(ptr_);
        }
        ptr_ = nullptr;
        n_ = 0;
        cached_ = false;
    }
    T *get() const { return ptr_; }
    size_t size() const { return n_; }
    T &operator[](size_t i) { return ptr_[i]; }

  private:
    T *ptr_ = nullptr;
    size_t n_ = 0;
    hipStream_t stream_ = nullptr;
    bool cached_ = false;
};

// Pinned host staging array from the host cache, for copies between host
// tables and the device.  Released on the stream given at construction.
template <class T>
class Staged {
  public:
    Staged(size_t n, hipStream_t s) : n_(n), stream_(s) {
        ptr_ = n ? static_cast<T *>(halloc(n * sizeof(T))) : nullptr;
    }
    ~Staged() {
        if (ptr_) hfree(ptr_, stream_);
    }
    Staged(const Staged &) = delete;
    Staged &operator=(const Staged &) = delete;
    T *get() const { return ptr_; }
    size_t size() const { return n_; }
    size_t bytes() const { return n_ * sizeof(T); }
    T &operator[](size_t i) { return ptr_[i]; }
    const T &operator[](size_t i) const { return ptr_[i]; }

  private:
    T *ptr_ = nullptr;
    size_t n_ = 0;
    hipStream_t stream_ = nullptr;
};

// Event pair timing a region of one stream.
class StreamTimer {
  public:
    StreamTimer();
    ~StreamTimer();
    void start(hipStream_t s);
    void stop(hipStream_t s);
    double ms();  // waits for the stop event

  private:
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// ------------------------------------------------------------- primitives

// Exclusive prefix sum of n values; out may alias in.  Returns nothing; the
// total is out[n-1] + in[n-1] and is written to *total_dev when not null.
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total_dev,
                        hipStream_t s);
void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev,
                        hipStream_t s);

// Stable LSD radix sort on bits [0, nbits) of the keys.  `keys`/`vals` hold
// the input; `keys_alt`/`vals_alt` are scratch of the same size.  Returns
// true when the sorted data ended in the *_alt buffers.  vals may be null.
bool radix_sort_u64(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                    int64_t n, int nbits, hipStream_t s);
bool radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                    int64_t n, int nbits, hipStream_t s);

// Persisted autotuner results (tune_cache.cpp).
bool tune_lookup(const std::string &key, std::vector<int> &val);
void tune_store(const std::string &key, const std::vector<int> &val);
void tune_forget_all();
void tune_reload();

// Number of bits needed to hold v (0 for v = 0).
inline int bit_width_u64(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 2147483647LL) g = 2147483647LL;
    return static_cast<unsigned>(g);
}

}  // namespace pgabb
