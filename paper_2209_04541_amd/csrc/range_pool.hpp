// First-fit allocator of byte ranges of a device pool (the block caches of
// the streamed counts).
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace pgabb {

// First-fit allocator over [0, cap) with coalescing of free ranges.
class RangePool {
  public:
    explicit RangePool(uint64_t cap) { free_[0] = cap; }
    // Returns offset or UINT64_MAX.
    uint64_t alloc(uint64_t bytes) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const uint64_t off = it->first;
                const uint64_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return off;
            }
        }
        return UINT64_MAX;
    }
    void release(uint64_t off, uint64_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

}  // namespace pgabb
