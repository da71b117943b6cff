// First-fit allocator of the serving loop's device arena (host-side
// bookkeeping only: offsets into [0, size), no memory is touched).  Kept in
// a header of its own so that the host-side checks (tests/host_check.cpp)
// exercise the very allocator the server uses.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace swe {

constexpr size_t kArenaAlign = 256;

inline size_t arena_align_up(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
public:
    void reset(size_t size)
    {
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = arena_align_up(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = arena_align_up(std::max<size_t>(bytes, 1));
        used_ -= bytes;
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
    // visits the free blocks (offset, bytes) in address order
    template <class F>
    void each_free(F f) const
    {
        for (const auto &kv : free_) f(kv.first, kv.second);
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

}  // namespace swe
