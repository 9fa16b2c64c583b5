// pool.h -- first-fit sub-allocator over one device allocation (the job
// service's HBM budget).  Host-only bookkeeping: offsets into the pool,
// 256-byte aligned, adjacent free ranges coalesced.  Not thread-safe; the
// service calls it under its lock.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace stk {

class PoolAllocator {
   public:
    static constexpr uint64_t kAlign = 256;

    explicit PoolAllocator(uint64_t size = 0) { reset(size); }

    void reset(uint64_t size) {
        size_ = size / kAlign * kAlign;
        free_.clear();
        used_ = 0;
        high_ = 0;
        if (size_) free_[0] = size_;
    }

    static uint64_t round_up(uint64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

    // Returns true and the offset of a block of at least `bytes` bytes, or
    // false when no free range is large enough.
    bool alloc(uint64_t bytes, uint64_t *off) {
        const uint64_t b = round_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= b) {
                *off = it->first;
                const uint64_t rest = it->second - b;
                const uint64_t start = it->first + b;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += b;
                if (used_ > high_) high_ = used_;
                return true;
            }
        }
        return false;
    }

    void release(uint64_t off, uint64_t bytes) {
        const uint64_t b = round_up(bytes ? bytes : 1);
        used_ -= b;
        auto it = free_.emplace(off, b).first;
        // merge with the following range
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        // merge with the preceding range
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t high_water() const { return high_; }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (const auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t free_ranges() const { return free_.size(); }

   private:
    uint64_t size_ = 0, used_ = 0, high_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
};

}  // namespace stk
