// Host-side scheduling of the continuous-batching server: admission of
// queued requests against a device-memory budget, the per-tick iteration
// counts of the resident jobs, and deferred release of finished jobs'
// memory.  No HIP calls here, so the logic is testable on any host.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

namespace fe {

// First-fit allocator over byte offsets [0, capacity), 256-byte granules.
class Arena {
  public:
    explicit Arena(size_t capacity = 0) { reset(capacity); }

    void reset(size_t capacity)
    {
        cap_ = capacity & ~(size_t)255;
        free_.clear();
        if (cap_) free_[0] = cap_;
        used_ = 0;
    }

    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }

    bool alloc(size_t bytes, size_t *off)
    {
        const size_t need = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const size_t rest = it->second - need, at = it->first + need;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += need;
            return true;
        }
        return false;
    }

    void release(size_t off, size_t bytes)
    {
        const size_t need = round(bytes);
        used_ -= need;
        auto it = free_.emplace(off, need).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {  // merge right
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {  // merge left
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t largest_free() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct SchedJob {
    uint64_t id = 0;     // server-assigned, increasing in submission order
    size_t bytes = 0;    // device memory the job holds while resident
    long px = 0;         // pixels of the image (work per iteration)
    int total = 0;       // iterations requested
    int done = 0;        // iterations enqueued so far
    size_t off = 0;      // arena offset once admitted
    double t_submit = 0, t_admit = 0;
};

// One scheduling tick: which queued jobs become resident, how many
// iterations every resident job receives, and which jobs finish with it.
struct TickPlan {
    std::vector<uint64_t> admitted;   // need their initial state
    std::vector<uint64_t> active;     // every resident job, in admission order
    std::vector<int> done_before;     // iterations applied before this tick
    std::vector<int> count;           // iterations added this tick
    std::vector<uint64_t> finishing;  // reach their total with this tick
};

// Admission is in arrival order (no overtaking).  Each tick offers every
// resident job up to iters_per_tick iterations, oldest first; with a work
// budget (tick_work > 0 pixel-iterations) the offer stops once the tick
// holds that much work, so that a tick's duration stays bounded however
// many jobs are resident and the oldest jobs finish first (the oldest
// always advances, so every job finishes).  Without a budget every resident
// job advances every tick (processor sharing).
class Scheduler {
  public:
    Scheduler(size_t budget, int iters_per_tick, int max_active, long long tick_work = 0)
        : arena_(budget), per_tick_(std::max(1, iters_per_tick)),
          max_active_(max_active > 0 ? max_active : 1 << 30),
          tick_work_(tick_work > 0 ? tick_work : 0)
    {
    }

    // A job larger than the whole budget could never run.
    bool fits_ever(size_t bytes) const { return Arena::round(bytes) <= arena_.capacity(); }

    uint64_t submit(size_t bytes, int total, double now, long px = 0)
    {
        SchedJob j;
        j.id = next_id_++;
        j.bytes = bytes;
        j.px = px;
        j.total = std::max(0, total);
        j.t_submit = now;
        pending_.push_back(j);
        return j.id;
    }

    // Admit in arrival order while memory and the active cap allow (the
    // queue head blocks later arrivals: no overtaking), then give the
    // resident jobs, oldest first, min(per_tick, remaining) iterations each
    // until the tick's work budget (if any) is spent; the rest get none
    // this tick.
    TickPlan plan(double now)
    {
        TickPlan t;
        while (!pending_.empty() && (int)active_.size() < max_active_) {
            SchedJob &h = pending_.front();
            size_t off = 0;
            if (!arena_.alloc(h.bytes, &off)) break;
            h.off = off;
            h.t_admit = now;
            active_.push_back(h);
            t.admitted.push_back(h.id);
            pending_.pop_front();
        }
        std::vector<SchedJob> keep;
        long long work = 0;
        for (SchedJob &j : active_) {
            const bool spent = tick_work_ > 0 && work >= tick_work_;
            const int c = spent ? 0 : std::min(per_tick_, j.total - j.done);
            work += (long long)c * j.px;
            t.active.push_back(j.id);
            t.done_before.push_back(j.done);
            t.count.push_back(c);
            j.done += c;
            if (j.done >= j.total) {
                t.finishing.push_back(j.id);
                retiring_.push_back(j);
            } else {
                keep.push_back(j);
            }
        }
        active_.swap(keep);
        return t;
    }

    // The tick that finished these jobs has completed on the device: their
    // memory may be reused.
    void retire(const std::vector<uint64_t> &ids)
    {
        for (uint64_t id : ids) {
            auto it = std::find_if(retiring_.begin(), retiring_.end(),
                                   [&](const SchedJob &j) { return j.id == id; });
            if (it == retiring_.end()) continue;
            arena_.release(it->off, it->bytes);
            retiring_.erase(it);
        }
    }

    const SchedJob *find(uint64_t id) const
    {
        for (auto *v : {&active_, &retiring_})
            for (const SchedJob &j : *v)
                if (j.id == id) return &j;
        for (const SchedJob &j : pending_)
            if (j.id == id) return &j;
        return nullptr;
    }

    size_t pending() const { return pending_.size(); }
    size_t active() const { return active_.size(); }
    size_t retiring() const { return retiring_.size(); }
    const Arena &arena() const { return arena_; }

  private:
    Arena arena_;
    int per_tick_, max_active_;
    long long tick_work_;
    uint64_t next_id_ = 1;
    std::deque<SchedJob> pending_;
    std::vector<SchedJob> active_, retiring_;
};

}  // namespace fe
