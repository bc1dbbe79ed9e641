// CPU test of the context's slot rotation (zb_slots.h): a slot is never handed out while
// the work of its previous user may still run, captured calls never share a slot, and the
// capture pool runs out with a refusal instead of a reuse.  Built with ASan and UBSan.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "zb_slots.h"

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                             \
        }                                                             \
    } while (0)

int main()
{
    const int E = 8, C = 3;
    zbh::SlotRing r;
    r.init(E, C);
    std::vector<int> in_flight(E, 0);   // work queued after the slot's last marked use
    int waits = 0;
    auto wait = [&](int s) { in_flight[s] = 0; ++waits; };
    // the first E calls take fresh slots without waiting
    for (int i = 0; i < E; ++i) {
        const int s = r.acquire(wait);
        CHECK(s == i && waits == 0 && !in_flight[s]);
        in_flight[s] = 1;
        r.mark(s);
    }
    // the next one reuses slot 0 and must wait for it
    int s = r.acquire(wait);
    CHECK(s == 0 && waits == 1 && !in_flight[0]);
    in_flight[0] = 1;
    r.mark(0);
    // captured calls: distinct slots past the ring, never reused, then refused
    std::set<int> cap;
    for (int i = 0; i < C; ++i) {
        const int c = r.acquire_capture();
        CHECK(c >= E && c < E + C && !cap.count(c));
        cap.insert(c);
    }
    CHECK(r.acquire_capture() == -1 && r.captures_left() == 0);
    // random traffic: calls of 1..4 launches, work that finishes on its own at random
    std::mt19937 rng(5);
    for (int call = 0; call < 100000; ++call) {
        const int launches = 1 + (int)(rng() % 4);
        std::vector<int> got;
        for (int k = 0; k < launches; ++k) {
            const int t = r.acquire(wait);
            CHECK(t >= 0 && t < E);
            CHECK(!in_flight[t]);                   // never handed out while in use
            for (int u : got) CHECK(u != t);        // a call's slots are distinct (launches <= E)
            got.push_back(t);
        }
        for (int t : got) {
            in_flight[t] = 1;
            r.mark(t);
        }
        for (int t = 0; t < E; ++t)                 // some work ends by itself; the ring
            if (rng() % 3 == 0) in_flight[t] = 0;   // still waits (an event query is cheap)
        CHECK(r.acquire_capture() == -1);
    }
    std::printf("slots ok: %d waits\n", waits);
    return 0;
}
