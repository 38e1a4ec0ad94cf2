// arena.h -- byte ranges inside one preallocated device region, for the
// request server: each resident sample's slab is carved out of the region
// when the sample is admitted and given back when it retires, so serving
// never allocates or frees device memory while kernels run.
//
// Best fit over a free list kept sorted by offset; a released range merges
// with free neighbours.  Plain C++ (no HIP), so it is tested on the host.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace rsa {

class Arena {
public:
    static constexpr uint64_t kAlign = 4096;   // every range starts and ends on this

    explicit Arena(uint64_t bytes = 0) { reset(bytes); }

    void reset(uint64_t bytes)
    {
        free_.clear();
        size_ = bytes / kAlign * kAlign;
        used_ = peak_ = 0;
        if (size_) free_[0] = size_;
    }

    static uint64_t round(uint64_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

    // Smallest free range that holds `bytes`; false (nothing changes) if none.
    bool alloc(uint64_t bytes, uint64_t &off)
    {
        const uint64_t need = round(bytes ? bytes : 1);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= need && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return false;
        off = best->first;
        const uint64_t left = best->second - need;
        free_.erase(best);
        if (left) free_[off + need] = left;
        used_ += need;
        if (used_ > peak_) peak_ = used_;
        return true;
    }

    // Give back a range that alloc returned for the same `bytes`.
    void release(uint64_t off, uint64_t bytes)
    {
        uint64_t len = round(bytes ? bytes : 1);
        used_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return;
            }
        }
        free_[off] = len;
    }

    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (const auto &f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    size_t free_ranges() const { return free_.size(); }

private:
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
};

}  // namespace rsa
