// Host-side core of the serving runtime: byte arenas and FIFO admission.
// No HIP dependency, so the admission logic is tested on the host alone.
//
// A timeslice is admitted to the device when (1) a stream slot is free and
// (2) the device arena can hold its footprint (inputs, outputs, workspace).
// Admission is first-come first-served: a slice that does not fit blocks the
// ones behind it, so a large slice cannot starve.  Freed memory is coalesced.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>

namespace trig {
namespace serve {

// First-fit allocator over [0, capacity) with free-block coalescing.  Offsets
// and sizes are multiples of `align` (a power of two).
class Arena {
public:
    explicit Arena(size_t capacity = 0, size_t align = 256) { reset(capacity, align); }

    void reset(size_t capacity, size_t align = 256) {
        align_ = align;
        capacity_ = capacity & ~(align - 1);
        free_.clear();
        used_.clear();
        if (capacity_) free_[0] = capacity_;
        in_use_ = 0;
    }

    static constexpr size_t kFail = ~size_t(0);

    size_t round(size_t n) const { return (n + align_ - 1) & ~(align_ - 1); }

    // Offset of a new block of n bytes, or kFail.
    size_t alloc(size_t n) {
        n = round(n == 0 ? 1 : n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                used_[off] = n;
                in_use_ += n;
                return off;
            }
        }
        return kFail;
    }

    // Would alloc(n) succeed now?
    bool fits(size_t n) const {
        n = round(n == 0 ? 1 : n);
        for (const auto& f : free_)
            if (f.second >= n) return true;
        return false;
    }

    // Returns false for an offset that is not a live block.
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return true;
            }
        }
        free_[off] = len;
        return true;
    }

    size_t capacity() const { return capacity_; }
    size_t in_use() const { return in_use_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    size_t live_blocks() const { return used_.size(); }

private:
    size_t align_ = 256, capacity_ = 0, in_use_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> used_;  // offset -> length
};

// Device bytes a slice needs: CSR offsets, hit coordinates, per-event
// outputs (count, flag, accepted id), one counter and the selection
// workspace, each rounded to `align`.
inline size_t slice_footprint(int64_t n_events, int64_t n_hits, size_t workspace, size_t align = 256) {
    auto r = [&](size_t b) { return (b + align - 1) & ~(align - 1); };
    return r(4 * (size_t)(3 * n_events + 1)) + 2 * r(4 * (size_t)n_hits) + r(4 * (size_t)n_events) +
           r((size_t)n_events) + r(4 * (size_t)(n_events > 0 ? n_events : 1)) + r(4) + r(4) + r(workspace);
}

// FIFO admission: pending tickets wait until a slot is free and their
// footprint fits the arena.
struct Pending {
    uint64_t ticket;
    size_t bytes;
};

class Admission {
public:
    Admission(size_t arena_bytes, int slots) : arena_(arena_bytes), free_slots_(slots) {}

    // A slice whose footprint exceeds the whole arena can never be admitted.
    bool admissible(size_t bytes) const { return arena_.round(bytes) <= arena_.capacity(); }

    void enqueue(uint64_t ticket, size_t bytes) { queue_.push_back({ticket, bytes}); }

    // Admits the queue head if possible: returns true with its ticket, slot
    // use and arena offset.
    bool admit_next(uint64_t& ticket, size_t& offset) {
        if (queue_.empty() || free_slots_ <= 0) return false;
        const Pending& p = queue_.front();
        const size_t off = arena_.alloc(p.bytes);
        if (off == Arena::kFail) return false;
        ticket = p.ticket;
        offset = off;
        queue_.pop_front();
        --free_slots_;
        return true;
    }

    // Removes a queued (not admitted) ticket; false if not queued.
    bool cancel(uint64_t ticket) {
        for (auto it = queue_.begin(); it != queue_.end(); ++it)
            if (it->ticket == ticket) {
                queue_.erase(it);
                return true;
            }
        return false;
    }

    void complete(size_t offset) {
        arena_.release(offset);
        ++free_slots_;
    }

    size_t queued() const { return queue_.size(); }
    int free_slots() const { return free_slots_; }
    const Arena& arena() const { return arena_; }

private:
    Arena arena_;
    int free_slots_;
    std::deque<Pending> queue_;
};

}  // namespace serve
}  // namespace trig
