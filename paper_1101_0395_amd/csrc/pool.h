// First-fit allocator of byte ranges of a fixed pool: the host bookkeeping
// behind the serving engine's admission of jobs by device-memory footprint.
// Offsets only; nothing here touches the device.
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>

namespace cq {

class ExtentPool {
public:
    explicit ExtentPool(size_t bytes = 0, size_t align = 256) : align_(align ? align : 1)
    {
        total_ = bytes / align_ * align_;
        if (total_ > 0) free_[0] = total_;
    }

    size_t total() const { return total_; }
    size_t used() const { return used_; }
    size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

    // Lowest-offset free range of at least `bytes` (rounded up to the
    // alignment); false if none is large enough.
    bool alloc(size_t bytes, size_t* off)
    {
        const size_t need = round(bytes);
        if (need == 0) return false;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const size_t rest = it->second - need;
            const size_t at = it->first + need;
            free_.erase(it);
            if (rest > 0) free_[at] = rest;
            used_ += need;
            return true;
        }
        return false;
    }

    // Returns a range from alloc(bytes) (same size argument); merges it with
    // free neighbours so free ranges never touch.
    void release(size_t off, size_t bytes)
    {
        size_t size = round(bytes);
        used_ -= size;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += size;
                return;
            }
        }
        free_[off] = size;
    }

    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }

    size_t free_ranges() const { return free_.size(); }

private:
    size_t align_;
    size_t total_ = 0;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> size; disjoint, never adjacent
};

}  // namespace cq
