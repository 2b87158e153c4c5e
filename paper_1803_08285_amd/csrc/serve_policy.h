// Host-side policy of the query server, free of any device code so that it is
// tested on the CPU (with the address and undefined-behaviour sanitizers) as
// well as used by server.hip:
//   * Arena: first-fit allocator over one device allocation made at server
//     creation (256-byte granules, coalescing free ranges), so serving never
//     calls the device allocator;
//   * pick_admission: which pending query to start next.
//
// Admission is cost-aware.  A query's cost is its number of map terms
// (segments x bins x pixels).  Heavy queries (cost >= the heavy threshold) fill
// the whole GPU on their own, so at most max_heavy (default one) run at a time
// and they start in arrival order; light queries run beside it in the other slots, in arrival
// order among themselves, and pass a heavy query that is waiting for the heavy
// slot.  A heavy query therefore waits only for the heavy queries before it
// (never behind a queue of light ones) and shares the GPU only with light
// work, and a light query never waits for a heavy one to finish.  Neither kind
// can starve the other: a waiting heavy query starts as soon as the running one
// ends, and light queries need only a free slot and memory.  A query that waits
// for memory holds back every query behind it (arrival order), so memory
// pressure cannot starve it either.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>
#include <vector>

namespace sgwb {
namespace serve {

class Arena {
  public:
    void init(char *base, size_t size)
    {
        base_ = base;
        size_ = size;
        free_.clear();
        sizes_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    static size_t granule(size_t n)
    {
        n = (n + 255) / 256 * 256;
        return n ? n : 256;
    }
    char *alloc(size_t n)
    {
        n = granule(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                sizes_[off] = n;
                used_ += n;
                return base_ + off;
            }
        }
        return nullptr;
    }
    // Returns false for a pointer that is not a live block (ignored).
    bool release(char *p)
    {
        if (!p || p < base_) return false;
        const size_t off = (size_t)(p - base_);
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return false;
        size_t start = off, len = s->second;
        used_ -= len;
        sizes_.erase(s);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
        return true;
    }
    // Would a request of n bytes fit now (first fit)?
    bool fits(size_t n) const
    {
        n = granule(n);
        for (const auto &kv : free_)
            if (kv.second >= n) return true;
        return false;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t live_blocks() const { return sizes_.size(); }
    // Free ranges (offset -> length), for checks.
    const std::map<size_t, size_t> &free_ranges() const { return free_; }
    const std::map<size_t, size_t> &live() const { return sizes_; }

  private:
    char *base_ = nullptr;
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> sizes_;  // offset -> length of live blocks
};

// Default heavy threshold: 3e10 map-term equivalents (a query's estimated GPU
// time at 4.2e13 terms/s), about 0.7 ms of the whole GPU; queries above it
// occupy every compute unit for long enough that letting them overlap only
// stretches both, while those below it finish quickly enough to run beside a
// heavy one.
constexpr double kHeavyTermsDefault = 3e10;

struct PendingView {
    double cost;  // map terms
    size_t need;  // arena bytes the query needs to start (incl. new seeds)
};

struct RunningView {
    int free_slots;
    int heavy_running;  // heavy queries running now
};

enum : int { kAdmitNone = -1 };

// Index (into pending, arrival order) of the query to start now, or kAdmitNone.
// fits(i) says whether pending[i]'s footprint fits in the arena now; at most
// max_heavy heavy queries run at a time.
template <class Fits>
int pick_admission(const std::vector<PendingView> &pending, const RunningView &run, double heavy_terms, Fits fits,
                   int max_heavy = 1)
{
    if (run.free_slots <= 0) return kAdmitNone;
    bool heavy_seen = false;
    for (size_t i = 0; i < pending.size(); ++i) {
        const bool heavy = pending[i].cost >= heavy_terms;
        if (heavy && (heavy_seen || run.heavy_running >= max_heavy)) {
            heavy_seen = true;  // waits for the heavy slot; light queries may pass it
            continue;
        }
        heavy_seen = heavy_seen || heavy;
        if (fits(i)) return (int)i;
        // waits for memory: nothing behind it passes, so it cannot starve
        return kAdmitNone;
    }
    return kAdmitNone;
}

}  // namespace serve
}  // namespace sgwb
