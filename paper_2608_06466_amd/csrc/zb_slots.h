// Rotating per-call device scratch of a context (zone-queue counters, FP64 fallback lists):
// which slot a call gets, and when it must first wait for the slot's previous user.
// Host-only, no HIP: the runtime supplies the wait (an event synchronisation), and the CPU
// tests build this header on its own.
#pragma once

#include <vector>

namespace zbh {

// A ring of `eager` slots for ordinary (eager) calls, then a pool of `capture` slots for
// calls captured into a graph.  An eager slot handed out again is first waited for: the
// work of its last user has ended before the new call may clear and reuse it.  A captured
// call keeps its slot for as long as its graph may be replayed, which the library cannot
// see, so capture slots are never handed out twice; once they are all taken, a captured
// call is refused.
class SlotRing {
public:
    void init(int eager, int capture)
    {
        eager_ = eager;
        capture_ = capture;
        next_ = next_cap_ = 0;
        pending_.assign(eager, 0);
    }
    int eager() const { return eager_; }
    int capture() const { return capture_; }

    // The next eager slot, after wait(slot) if its previous user may still be running.
    template <class Wait>
    int acquire(Wait &&wait)
    {
        const int s = next_;
        next_ = (next_ + 1) % eager_;
        if (pending_[s]) {
            wait(s);
            pending_[s] = 0;
        }
        return s;
    }
    // The caller recorded an event after the last work that uses eager slot s.
    void mark(int s) { pending_[s] = 1; }
    bool pending(int s) const { return pending_[s] != 0; }
    // A capture slot (index eager + k, never handed out again), or -1 when none is left.
    int acquire_capture()
    {
        if (next_cap_ >= capture_) return -1;
        return eager_ + next_cap_++;
    }
    int captures_left() const { return capture_ - next_cap_; }

private:
    int eager_ = 0, capture_ = 0, next_ = 0, next_cap_ = 0;
    std::vector<unsigned char> pending_;
};

}  // namespace zbh
