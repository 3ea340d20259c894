// First-fit allocator over one device-memory budget (host-side bookkeeping
// only: offsets into a reservation made elsewhere), used by the serving loop.
// A free range remembers the fences (per-stream sequence numbers) of the work
// that used it last, merged conservatively when ranges coalesce, so memory
// freed on one stream is reused on another only after that work. Plain C++,
// no device calls: it also builds in the host-only sanitizer check.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace ssmap {

constexpr int kMaxLanes = 4;

struct Fence {
    uint64_t seq[kMaxLanes] = {};
};
inline void merge_fence(Fence &a, const Fence &b) {
    for (int i = 0; i < kMaxLanes; ++i) a.seq[i] = std::max(a.seq[i], b.seq[i]);
}

// First-fit allocator over [0, cap). A free range carries the fences of the
// work that used it last (merged conservatively when ranges coalesce).
class Slab {
  public:
    void init(size_t cap) {
        free_.clear();
        free_[0] = Range{cap, Fence{}};
        used_ = peak_ = 0;
    }
    bool alloc(size_t n, size_t &off, Fence &f) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second.size < n) continue;
            off = it->first;
            f = it->second.fence;
            const size_t rest = it->second.size - n;
            free_.erase(it);
            if (rest) free_[off + n] = Range{rest, f};
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n, const Fence &f) {
        used_ -= n;
        Range r{n, f};
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            r.size += next->second.size;
            merge_fence(r.fence, next->second.fence);
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second.size == off) {
                prev->second.size += r.size;
                merge_fence(prev->second.fence, r.fence);
                return;
            }
        }
        free_[off] = r;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    // free ranges as (offset, size), in offset order (for checks)
    template <typename Fn> void each_free(Fn &&fn) const {
        for (const auto &kv : free_) fn(kv.first, kv.second.size);
    }

  private:
    struct Range {
        size_t size;
        Fence fence;
    };
    std::map<size_t, Range> free_;
    size_t used_ = 0, peak_ = 0;
};


}  // namespace ssmap
