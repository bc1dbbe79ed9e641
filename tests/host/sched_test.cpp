// CPU test of the burn server's scheduling policy (zb_sched.h) on a fake device: the
// arena against a brute-force model, first-come-first-served admission within the byte
// budget, the slicing and class rules of every launch, shortest-remaining-work order,
// zone coverage, completion accounting and failure reporting; then the same policy
// driven by a scheduler thread, a fake GPU thread and client threads, as the server runs
// it.  Built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <map>
#include <set>
#include <thread>

#include "zb_sched.h"

using namespace zbh;

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            exit(1);                                                         \
        }                                                                    \
    } while (0)

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 1) {}
    uint64_t next()
    {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return s;
    }
    int64_t range(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }
};

// ---- the arena against a model that marks every 256-byte unit ----
static void test_arena()
{
    for (uint64_t seed = 1; seed <= 20; ++seed) {
        Rng g(seed);
        const size_t units = 512;
        Arena a;
        a.init(units * ARENA_ALIGN);
        std::vector<char> used(units, 0);
        std::map<size_t, size_t> live;   // offset -> bytes asked
        for (int it = 0; it < 4000; ++it) {
            if (g.next() % 2 || live.empty()) {
                const size_t bytes = (size_t)g.range(1, 40 * ARENA_ALIGN);
                const size_t nu = arena_round(bytes) / ARENA_ALIGN;
                // first fit in the model: the lowest run of nu free units
                long want = -1;
                for (size_t u = 0, run = 0; u < units; ++u) {
                    run = used[u] ? 0 : run + 1;
                    if (run == nu) {
                        want = (long)(u + 1 - nu);
                        break;
                    }
                }
                size_t off = 0;
                const bool ok = a.alloc(bytes, &off);
                CHECK(ok == (want >= 0));
                if (ok) {
                    CHECK(off == (size_t)want * ARENA_ALIGN);
                    for (size_t u = 0; u < nu; ++u) used[off / ARENA_ALIGN + u] = 1;
                    live[off] = bytes;
                }
            } else {
                auto it2 = live.begin();
                std::advance(it2, g.range(0, (int64_t)live.size() - 1));
                a.release(it2->first, it2->second);
                const size_t nu = arena_round(it2->second) / ARENA_ALIGN;
                for (size_t u = 0; u < nu; ++u) used[it2->first / ARENA_ALIGN + u] = 0;
                live.erase(it2);
            }
            size_t nused = 0;
            for (char c : used) nused += c;
            CHECK(a.used() == nused * ARENA_ALIGN);
            // adjacent free runs are always merged: free blocks == free runs of the model
            size_t runs = 0;
            for (size_t u = 0; u < units; ++u) runs += !used[u] && (u == 0 || used[u - 1]);
            CHECK(a.free_blocks() == runs);
        }
        for (auto &kv : live) a.release(kv.first, kv.second);
        CHECK(a.used() == 0 && a.free_blocks() == 1);
    }
    printf("arena ok\n");
}

// ---- the launch plan alone ----
static void test_plan()
{
    static const int A = 0, B = 0;   // two kernel classes, told apart by address
    const void *ca = &A, *cb = &B;
    std::vector<SchedRequest> rs(5);
    // remaining work: zones * cost
    const int64_t zones[5] = {1000, 10, 300, 50, 5000};
    const double cost[5] = {1.0, 4.0, 1.0, 1.0, 0.001};
    const void *cls[5] = {ca, ca, cb, ca, ca};
    std::vector<SchedRequest *> act;
    for (int i = 0; i < 5; ++i) {
        rs[i].ticket = i + 1;
        rs[i].zones = zones[i];
        rs[i].cost = cost[i];
        rs[i].cls = cls[i];
        rs[i].nr = 10 * (i + 1);
        act.push_back(&rs[i]);
    }
    int seen_nr = -1;
    auto slice = [&](const void *c, int nr) {
        CHECK(c == ca);
        seen_nr = nr;
        return (int64_t)64;
    };
    // least work left: request 4 (5 units), then 1 (40), 3 (50), 0 (1000); 2 is class B
    std::vector<Part> p = plan_launch(act, 8, 1.0, slice);
    CHECK(seen_nr == 50);   // the largest reaction count among class A requests
    CHECK(p.size() == 4);
    CHECK(p[0].r == &rs[4] && p[0].first == 0 && p[0].n == 64);   // one slice at most
    CHECK(p[1].r == &rs[1] && p[1].first == 0 && p[1].n == 10);
    CHECK(p[2].r == &rs[3] && p[2].first == 0 && p[2].n == 50);
    // 64 + 10 + 50 = 124 zones: request 0 gets the 4 left below 2 slices
    CHECK(p[3].r == &rs[0] && p[3].first == 0 && p[3].n == 4);
    CHECK(rs[0].next == 4 && rs[4].next == 64 && rs[2].next == 0);
    // the next launch continues where this one stopped
    p = plan_launch(act, 8, 2.0, slice);
    CHECK(p[0].r == &rs[1] || p[0].r == &rs[4]);
    for (const Part &q : p) CHECK(q.r->cls == ca && q.first + q.n == q.r->next);
    // maxseg caps the number of parts
    for (auto &r : rs) r.next = 0;
    p = plan_launch(act, 2, 1.0, slice);
    CHECK(p.size() == 2);
    printf("plan ok\n");
}

// ---- a fake device, stepped by hand ----
struct FakeDev {
    struct Handle {
        int id = -1;
    };
    struct Launch {
        int stream;
        std::vector<Part> parts;
        bool finished = false, retired = false;
    };
    Scheduler<FakeDev> *sch = nullptr;
    std::vector<Launch> launches;
    std::set<int> running;
    std::set<uint64_t> uploaded;
    std::map<uint64_t, int64_t> covered;   // ticket -> zones handed to launches
    double t = 0;
    int64_t slice_zones = 37;
    int maxseg = 4;
    bool fail_upload = false, fail_query = false;

    double now() { return t += 1.0; }
    bool upload(SchedRequest *r)
    {
        CHECK(r->st == PENDING);
        CHECK(r->off + arena_round(r->bytes) <= sch->arena.size());
        CHECK(uploaded.insert(r->ticket).second);
        return !fail_upload;
    }
    int64_t slice(const void *, int) { return slice_zones; }
    bool launch(int stream, const std::vector<Part> &parts, Handle *h)
    {
        CHECK(!parts.empty() && (int)parts.size() <= maxseg);
        CHECK(sch->in_flight(stream) < 2);
        int64_t total = 0;
        // the request that leads had the least work left among all admitted requests
        // with zones still to launch (its `next` before this launch)
        std::map<const SchedRequest *, int64_t> taken;
        for (const Part &p : parts) taken[p.r] += p.n;
        auto left_before = [&](const SchedRequest *r) {
            return (double)(r->zones - r->next + (taken.count(r) ? taken[r] : 0)) * r->cost;
        };
        for (const SchedRequest *r : sch->active)
            if (r->next - (taken.count(r) ? taken[r] : 0) < r->zones)
                CHECK(left_before(parts[0].r) <= left_before(r));
        for (const Part &p : parts) {
            CHECK(p.r->cls == parts[0].r->cls);
            CHECK(p.r->st == ADMITTED);
            CHECK(uploaded.count(p.r->ticket));
            CHECK(p.n > 0 && p.n <= slice_zones);
            CHECK(p.first == covered[p.r->ticket]);   // zones in order, each once
            covered[p.r->ticket] += p.n;
            CHECK(covered[p.r->ticket] <= p.r->zones);
            total += p.n;
        }
        CHECK(total <= 2 * slice_zones);
        h->id = (int)launches.size();
        launches.push_back({stream, parts});
        running.insert(h->id);
        return true;
    }
    int query(const Handle &h)
    {
        if (fail_query) return -1;
        return launches[h.id].finished ? 0 : 1;
    }
    void retire(const Handle &h)
    {
        CHECK(launches[h.id].finished && !launches[h.id].retired);
        launches[h.id].retired = true;
    }
};

static void test_simulation(uint64_t seed)
{
    Rng g(seed);
    static const int C[3] = {0, 0, 0};
    const size_t budget = 64 * 1024;
    const int nstreams = 3, depth = 2;
    FakeDev dev;
    Scheduler<FakeDev> sch;
    dev.sch = &sch;
    dev.maxseg = (int)g.range(1, 6);
    dev.slice_zones = g.range(8, 80);
    sch.init(budget, nstreams, depth, dev.maxseg);
    std::mutex mu;
    std::unique_lock<std::mutex> lk(mu);
    std::vector<SchedRequest *> all, done, admitted_order;
    std::set<SchedRequest *> fetched, done_set;
    const int nreq = (int)g.range(20, 60);
    int submitted = 0;
    int64_t total_zones = 0;
    for (int round = 0; round < 100000 && (int)fetched.size() < nreq; ++round) {
        // clients: submit now and then, fetch what is done
        if (submitted < nreq && g.next() % 3 == 0) {
            SchedRequest *r = new SchedRequest();
            r->ticket = ++submitted;
            r->zones = g.range(1, 200);
            r->bytes = (size_t)g.range(1, budget / 3);
            r->cls = &C[g.range(0, 2)];
            r->nr = (int)g.range(1, 30);
            r->cost = (double)g.range(1, 5);
            r->t_submit = dev.now();
            total_zones += r->zones;
            sch.enqueue(r);
            all.push_back(r);
        }
        for (SchedRequest *r : done_set)
            if (!fetched.count(r) && g.next() % 2) {
                sch.release(r);
                fetched.insert(r);
            }
        // the device finishes some of the running launches, in any order
        for (auto it = dev.running.begin(); it != dev.running.end();)
            if (g.next() % 4 == 0) {
                dev.launches[*it].finished = true;
                it = dev.running.erase(it);
            } else {
                ++it;
            }
        const size_t nact = sch.active.size();
        done.clear();
        const auto o = sch.step(dev, lk, done);
        CHECK(o != Scheduler<FakeDev>::FAILED);
        for (SchedRequest *r : sch.active)
            if (std::find(admitted_order.begin(), admitted_order.end(), r) == admitted_order.end())
                admitted_order.push_back(r);
        for (SchedRequest *r : done) {
            CHECK(done_set.insert(r).second);   // reported once
            CHECK(r->st == DONE && r->finished == r->zones && dev.covered[r->ticket] == r->zones);
            if (std::find(admitted_order.begin(), admitted_order.end(), r) == admitted_order.end())
                admitted_order.push_back(r);
        }
        (void)nact;
        // a request is done exactly when every launch that carried it has completed
        for (SchedRequest *r : all) {
            if (r->st == PENDING) continue;
            int64_t fin = 0;
            for (auto &L : dev.launches)
                if (L.retired)
                    for (const Part &p : L.parts)
                        if (p.r == r) fin += p.n;
            CHECK(fin == r->finished);
            CHECK((r->st == DONE) == (fin == r->zones));
        }
        // admitted blocks are disjoint and inside the budget
        std::vector<std::pair<size_t, size_t>> blocks;
        for (SchedRequest *r : all)
            if (r->st != PENDING && !fetched.count(r)) blocks.push_back({r->off, arena_round(r->bytes)});
        std::sort(blocks.begin(), blocks.end());
        size_t sum = 0;
        for (size_t i = 0; i < blocks.size(); ++i) {
            CHECK(blocks[i].first + blocks[i].second <= budget);
            if (i) CHECK(blocks[i - 1].first + blocks[i - 1].second <= blocks[i].first);
            sum += blocks[i].second;
        }
        CHECK(sum == sch.arena.used());
        CHECK(sch.peak_used <= budget);
        // the head of the queue waits only because its block does not fit
        if (!sch.pending.empty()) {
            size_t off;
            Arena probe = sch.arena;
            CHECK(!probe.alloc(sch.pending.front()->bytes, &off));
        }
        for (int s = 0; s < nstreams; ++s) CHECK(sch.in_flight(s) <= depth);
    }
    CHECK((int)fetched.size() == nreq);
    CHECK(sch.n_done == (uint64_t)nreq && sch.zones_done == total_zones);
    CHECK(sch.n_launches == dev.launches.size());
    CHECK(sch.arena.used() == 0 && sch.arena.free_blocks() == 1);
    CHECK(sch.inflight.empty() && sch.active.empty() && sch.pending.empty());
    // first come, first served
    for (size_t i = 0; i < admitted_order.size(); ++i) CHECK(admitted_order[i]->ticket == i + 1);
    for (auto &L : dev.launches) CHECK(L.retired);
    for (SchedRequest *r : all) {
        CHECK(r->t_submit <= r->t_admit && r->t_admit <= r->t_first && r->t_first <= r->t_done);
        delete r;
    }
}

static void test_failures()
{
    static const int C = 0;
    for (int which = 0; which < 2; ++which) {
        FakeDev dev;
        Scheduler<FakeDev> sch;
        dev.sch = &sch;
        sch.init(1 << 20, 2, 2, 4);
        std::mutex mu;
        std::unique_lock<std::mutex> lk(mu);
        SchedRequest r;
        r.ticket = 1;
        r.zones = 10;
        r.bytes = 1000;
        r.cls = &C;
        sch.enqueue(&r);
        std::vector<SchedRequest *> done;
        if (which == 0) {
            dev.fail_upload = true;
            CHECK(sch.step(dev, lk, done) == Scheduler<FakeDev>::FAILED);
            CHECK(sch.error.find("upload") != std::string::npos);
        } else {
            CHECK(sch.step(dev, lk, done) == Scheduler<FakeDev>::PROGRESS);
            CHECK(dev.launches.size() == 1);
            dev.fail_query = true;
            CHECK(sch.step(dev, lk, done) == Scheduler<FakeDev>::FAILED);
            CHECK(sch.error.find("launch failed") != std::string::npos);
            CHECK(done.empty());
        }
    }
    printf("failures ok\n");
}

// ---- threads: a scheduler loop, a fake GPU, clients that submit, wait and fetch ----
struct ThreadDev {
    struct Handle {
        int id = -1;
    };
    std::mutex gm;   // the fake GPU's own state
    std::vector<int> state;   // per launch: 0 queued, 1 done
    std::vector<int64_t> zones;
    std::atomic<int64_t> executed{0};
    double now()
    {
        using namespace std::chrono;
        return duration<double>(steady_clock::now().time_since_epoch()).count();
    }
    bool upload(SchedRequest *)
    {
        std::this_thread::sleep_for(std::chrono::microseconds(20));   // a copy, lock released
        return true;
    }
    int64_t slice(const void *, int) { return 50; }
    bool launch(int, const std::vector<Part> &parts, Handle *h)
    {
        std::lock_guard<std::mutex> g(gm);
        int64_t n = 0;
        for (const Part &p : parts) n += p.n;
        h->id = (int)state.size();
        state.push_back(0);
        zones.push_back(n);
        return true;
    }
    int query(const Handle &h)
    {
        std::lock_guard<std::mutex> g(gm);
        return state[h.id] ? 0 : 1;
    }
    void retire(const Handle &) {}
    // the GPU: finish the oldest queued launch
    bool run_one()
    {
        std::lock_guard<std::mutex> g(gm);
        for (size_t i = 0; i < state.size(); ++i)
            if (!state[i]) {
                state[i] = 1;
                executed += zones[i];
                return true;
            }
        return false;
    }
};

static void test_threads()
{
    static const int C[2] = {0, 0};
    ThreadDev dev;
    Scheduler<ThreadDev> sch;
    sch.init(256 * 1024, 4, 2, 8);
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::thread worker([&] {
        std::unique_lock<std::mutex> lk(mu);
        std::vector<SchedRequest *> done;
        while (!stop) {
            done.clear();
            const auto o = sch.step(dev, lk, done);
            CHECK(o != Scheduler<ThreadDev>::FAILED);
            if (!done.empty()) cv_done.notify_all();
            if (o == Scheduler<ThreadDev>::IDLE) cv_work.wait_for(lk, std::chrono::microseconds(200));
        }
    });
    std::atomic<bool> gpu_stop{false};
    std::thread gpu([&] {
        while (!gpu_stop) {
            if (!dev.run_one()) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    });
    const int nclients = 4, per_client = 40;
    std::atomic<int64_t> submitted_zones{0};
    std::vector<std::thread> clients;
    for (int c = 0; c < nclients; ++c)
        clients.emplace_back([&, c] {
            Rng g(100 + c);
            for (int i = 0; i < per_client; ++i) {
                SchedRequest *r = new SchedRequest();
                r->zones = g.range(1, 300);
                r->bytes = (size_t)g.range(1000, 60000);
                r->cls = &C[g.range(0, 1)];
                r->nr = 5;
                submitted_zones += r->zones;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    r->ticket = (uint64_t)(c * per_client + i + 1);
                    sch.enqueue(r);
                }
                cv_work.notify_all();
                std::unique_lock<std::mutex> lk(mu);
                CHECK(cv_done.wait_for(lk, std::chrono::seconds(30), [&] { return r->st == DONE; }));
                CHECK(r->finished == r->zones);
                sch.release(r);
                lk.unlock();
                cv_work.notify_all();   // memory freed: admission may proceed
                delete r;
            }
        });
    for (auto &t : clients) t.join();
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
        CHECK(sch.n_done == (uint64_t)(nclients * per_client));
        CHECK(sch.zones_done == submitted_zones.load());
        CHECK(sch.arena.used() == 0 && sch.arena.free_blocks() == 1);
        CHECK(sch.active.empty() && sch.pending.empty());
    }
    cv_work.notify_all();
    worker.join();
    gpu_stop = true;
    gpu.join();
    CHECK(dev.executed.load() == submitted_zones.load());
    printf("threads ok\n");
}

int main()
{
    test_arena();
    test_plan();
    for (uint64_t s = 1; s <= 200; ++s) test_simulation(s);
    printf("simulation ok\n");
    test_failures();
    test_threads();
    printf("sched ok\n");
    return 0;
}
