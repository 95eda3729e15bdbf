// First-fit sub-allocator over one device allocation, used by the serving loop
// to hold every admitted request's device buffers within the HBM budget. Plain
// host C++ (no HIP): offsets only, the caller owns the memory at `base`.
//
// Sizes are rounded up to 256-byte granules, so every offset is 256-byte
// aligned when `base` is. The free list maps offset -> bytes, disjoint and
// coalesced (no two free blocks touch). Not thread-safe: the server calls it
// under its own lock.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace gw {

struct Arena {
    static constexpr size_t kGranule = 256;
    uint8_t *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes, coalesced

    static size_t granules(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }

    void init(void *p, size_t bytes) {
        base = (uint8_t *)p;
        size = bytes / kGranule * kGranule;
        free_.clear();
        if (size) free_[0] = size;
    }
    // The lowest-offset free block that fits; false (and *off untouched) if none.
    bool alloc(size_t bytes, size_t *off) {
        bytes = granules(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, o2 = it->first + bytes;
                free_.erase(it);
                if (rest) free_[o2] = rest;
                return true;
            }
        return false;
    }
    // Return a block that alloc gave out, with the size it was asked for.
    void release(size_t off, size_t bytes) {
        bytes = granules(bytes ? bytes : 1);
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
    size_t free_bytes() const {
        size_t s = 0;
        for (const auto &f : free_) s += f.second;
        return s;
    }
};

}  // namespace gw
