// Scheduling policy of the burn server, host-only and free of HIP: the device arena,
// first-come-first-served admission, cutting requests into slices, the choice of what
// each launch carries (shortest remaining work first, one kernel class per launch) and
// the accounting of completed launches.  The device side (copies, launches, events)
// comes in through a `Dev` class, so the CPU tests drive the same code with a fake
// device.
//
// Dev supplies:
//   using Handle = ...;                              one launch in flight
//   double now();                                    seconds, monotonic
//   bool upload(SchedRequest *r);                    start the input copy into r's block
//   int64_t slice(const void *cls, int max_nr);      zones per slice for a kernel class
//   bool launch(int stream, const std::vector<Part> &parts, Handle *h);
//   int query(const Handle &h);                      0 done, 1 running, -1 failed
//   void retire(const Handle &h);                    the launch's resources are free again
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace zbh {

constexpr size_t ARENA_ALIGN = 256;
inline size_t arena_round(size_t b) { return (b + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1); }

// First-fit allocator over one device block; offsets only, no device access.
class Arena {
public:
    void init(size_t bytes)
    {
        free_.clear();
        free_[0] = bytes;
        size_ = bytes;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = arena_round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = arena_round(bytes);
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
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t free_blocks() const { return free_.size(); }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

enum ReqState { PENDING, ADMITTED, DONE };

// What the policy knows of a request; the server's request type extends it.
struct SchedRequest {
    uint64_t ticket = 0;
    int64_t zones = 0;
    size_t bytes = 0, off = 0;   // device block in the arena
    const void *cls = nullptr;   // kernel class: only requests of one class share a launch
    int nr = 0;                  // reactions of the network (a slice's size depends on it)
    double cost = 1.0;           // relative device work per zone
    int64_t next = 0;            // first zone not yet in a launch
    int64_t finished = 0;        // zones whose launch has completed
    ReqState st = PENDING;
    double t_submit = 0, t_admit = 0, t_first = 0, t_done = 0;
};

// Zones [first, first + n) of a request, carried by one launch.
struct Part {
    SchedRequest *r;
    int64_t first, n;
};

// The parts of the next launch, taken from `active` (admitted requests); empty when no
// zone is left to launch.  The request with the least estimated work left decides the
// kernel class, and the launch takes slices of the requests of that class in that
// order, at most `maxseg` of them and 2 slices of zones in all: new small requests pass
// large ones at launch granularity, while a large request still gets every launch slot
// nobody else needs.  Advances each request's `next`.
template <class SliceFn>
std::vector<Part> plan_launch(const std::vector<SchedRequest *> &active, int maxseg, double now, SliceFn &&slice)
{
    std::vector<Part> parts;
    std::vector<SchedRequest *> cand;
    for (SchedRequest *r : active)
        if (r->next < r->zones) cand.push_back(r);
    if (cand.empty()) return parts;
    auto left = [](const SchedRequest *r) { return (double)(r->zones - r->next) * r->cost; };
    std::stable_sort(cand.begin(), cand.end(),
                     [&](const SchedRequest *a, const SchedRequest *b) { return left(a) < left(b); });
    const void *cls = cand[0]->cls;
    int max_nr = 0;
    for (SchedRequest *r : cand)
        if (r->cls == cls) max_nr = std::max(max_nr, r->nr);
    const int64_t sl = std::max<int64_t>(slice(cls, max_nr), 1);
    const int64_t cap = 2 * sl;
    int64_t total = 0;
    for (SchedRequest *r : cand) {
        if ((int)parts.size() >= maxseg || total >= cap) break;
        if (r->cls != cls) continue;
        const int64_t n = std::min({r->zones - r->next, sl, cap - total});
        parts.push_back({r, r->next, n});
        r->next += n;
        total += n;
        if (r->t_first == 0) r->t_first = now;
    }
    return parts;
}

template <class Dev>
class Scheduler {
public:
    struct Inflight {
        typename Dev::Handle h;
        int stream;
        std::vector<Part> parts;
    };
    enum Outcome { IDLE, PROGRESS, FAILED };

    void init(size_t arena_bytes, int nstreams, int depth, int maxseg)
    {
        arena.init(arena_bytes);
        nstreams_ = nstreams;
        depth_ = depth;
        maxseg_ = maxseg;
        per_stream_.assign(nstreams, 0);
    }

    // Queue a request (state PENDING, its bytes and class set).
    void enqueue(SchedRequest *r) { pending.push_back(r); }

    // One pass: completions, then admission, then launches on every stream up to `depth`
    // in flight.  Called with `lk` held; the input copies run with it released.
    // Requests that finished are appended to `done`.  On FAILED, `error` says why and the
    // scheduler's state is left for the caller to tear down.
    Outcome step(Dev &dev, std::unique_lock<std::mutex> &lk, std::vector<SchedRequest *> &done)
    {
        bool any = false;
        // 1. completions
        for (size_t i = 0; i < inflight.size();) {
            Inflight &L = inflight[i];
            const int q = dev.query(L.h);
            if (q == 1) {
                ++i;
                continue;
            }
            if (q != 0) {
                error = "burn launch failed";
                return FAILED;
            }
            const double t = dev.now();
            for (const Part &p : L.parts) {
                SchedRequest *r = p.r;
                r->finished += p.n;
                if (r->finished == r->zones) {
                    r->st = DONE;
                    r->t_done = t;
                    n_done++;
                    zones_done += r->zones;
                    active.erase(std::find(active.begin(), active.end(), r));
                    done.push_back(r);
                }
            }
            per_stream_[L.stream]--;
            dev.retire(L.h);
            inflight.erase(inflight.begin() + i);
            any = true;
        }
        // 2. admission, first come first served: the head waits until its block fits
        while (!pending.empty()) {
            SchedRequest *r = pending.front();
            size_t off = 0;
            if (!arena.alloc(r->bytes, &off)) break;
            pending.pop_front();
            r->off = off;
            peak_used = std::max(peak_used, arena.used());
            // the copy from pageable host memory may block: run it without the lock; the
            // request is in no list meanwhile, so nothing else sees it
            lk.unlock();
            const bool ok = dev.upload(r);
            lk.lock();
            if (!ok) {
                error = "upload of a request failed";
                return FAILED;
            }
            r->st = ADMITTED;
            r->t_admit = dev.now();
            active.push_back(r);
            any = true;
        }
        // 3. launches
        for (int s = 0; s < nstreams_; ++s) {
            while (per_stream_[s] < depth_) {
                Inflight L;
                L.parts = plan_launch(active, maxseg_, dev.now(),
                                      [&](const void *cls, int nr) { return dev.slice(cls, nr); });
                if (L.parts.empty()) return any ? PROGRESS : IDLE;
                L.stream = s;
                if (!dev.launch(s, L.parts, &L.h)) {
                    error = "burn launch could not be issued";
                    return FAILED;
                }
                per_stream_[s]++;
                n_launches++;
                inflight.push_back(std::move(L));
                any = true;
            }
        }
        return any ? PROGRESS : IDLE;
    }

    // Frees a fetched request's device block.
    void release(const SchedRequest *r) { arena.release(r->off, r->bytes); }
    int in_flight(int stream) const { return per_stream_[stream]; }

    Arena arena;
    std::deque<SchedRequest *> pending;
    std::vector<SchedRequest *> active;   // admitted, not all zones launched or finished
    std::vector<Inflight> inflight;
    std::string error;
    uint64_t n_launches = 0, n_done = 0;
    int64_t zones_done = 0;
    size_t peak_used = 0;

private:
    int nstreams_ = 0, depth_ = 0, maxseg_ = 1;
    std::vector<int> per_stream_;
};

}  // namespace zbh
