// Burn server: continuous batching of burn requests on one GPU.
//
// A request (network, zones, dt, tolerances, host input) is copied at submit,
// queued, and admitted first-come-first-served as soon as its device state fits
// in the server's HBM budget (one arena, allocated once, so no allocation on
// the request path).  Admitted requests are cut into slices of zones; a
// scheduler thread keeps a few persistent launches in flight on several
// streams, each launch holding up to MAXSEG slices of requests that use the
// same kernel class (any network or tolerance of that class), taken
// shortest-remaining-work first.  Requests that
// arrive while others run join the next launch, and their kernels overlap the
// ones in flight (a launch's tail is filled by the next).  Results stay in
// device memory until fetched.  A zone's result depends only on its own input
// and the kernel class, so it is the same whether the request ran alone or in
// a mix.

#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "zb_host_internal.h"
#include "zb_sched.h"

using namespace zb;
using namespace zbh;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request : SchedRequest {
    const zb_network *net = nullptr;
    const KernelInfo *k = nullptr;
    int row = 0;
    double dt = 0, rtol = 0, atol = 0;
    std::vector<double> in_state, in_scale;
    double *state = nullptr, *scale = nullptr;
    int32_t *status = nullptr;
    zb_zone_stats *stats = nullptr;
    hipEvent_t uploaded = nullptr;
};

// The scheduler's device side: copies on the copy stream, launches on the server's
// streams, one event and one block of zone-queue counters per launch in flight.
struct HipDev {
    struct Handle {
        hipEvent_t done = nullptr;
        int qblock = 0;
    };
    zb_server *S = nullptr;
    zb_err err = ZB_EDEVICE;   // why the last failed call failed
    std::string msg;

    double now() { return now_s(); }
    bool upload(SchedRequest *sr);
    int64_t slice(const void *cls, int max_nr);
    bool launch(int stream, const std::vector<Part> &parts, Handle *h);
    int query(const Handle &h);
    void retire(const Handle &h);
};

}  // namespace

struct zb_server {
    zb_context *ctx = nullptr;
    zb_opts opts{};
    int nstreams = 4, depth = 2;
    int64_t slice_req = 0;   // 0: from the kernel's capacity
    size_t max_pending = 1024;

    char *arena_base = nullptr;
    std::vector<hipStream_t> streams;
    hipStream_t copy = nullptr;
    unsigned long long *queues = nullptr;   // nstreams * depth blocks of MAXSEG
    unsigned long long *nfail = nullptr;
    std::vector<int> free_qblocks;
    std::vector<hipEvent_t> free_events;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    zb_err broken = ZB_OK;
    std::string broken_msg;

    uint64_t next_ticket = 1;
    std::map<uint64_t, Request *> all;   // every request not yet fetched
    Scheduler<HipDev> sched;             // arena, queue, launches in flight, totals
    HipDev dev;
};

static int64_t slice_zones(zb_server *S, const KernelInfo *k, int nr)
{
    if (S->slice_req > 0) return S->slice_req;
    int per_cu = blocks_per_cu(k, nr);
    int64_t cap = (int64_t)std::max(per_cu, 1) * S->ctx->cus * (64 / k->lanes);
    // One GPU of resident zones per slice, so a launch (two slices) gives each slot about
    // two zones.  At most four kernels run at once (one per hardware queue) and a launch
    // holds its stream until its slowest zone ends, which for the 48-variable network is
    // several times the mean zone time; with half a GPU per slice the launches' tails
    // left the GPU part idle (500 Poisson requests: 75k zone-burns/s, latency p99 74 s).
    return std::max<int64_t>(cap, 64);
}

bool HipDev::upload(SchedRequest *sr)
{
    Request *r = static_cast<Request *>(sr);
    char *base = S->arena_base + r->off;
    const int64_t z = r->zones;
    size_t o = 0;
    r->state = (double *)(base + o);
    o += arena_round(sizeof(double) * r->row * z);
    r->status = (int32_t *)(base + o);
    o += arena_round(sizeof(int32_t) * z);
    r->stats = (zb_zone_stats *)(base + o);
    o += arena_round(sizeof(zb_zone_stats) * z);
    r->scale = r->in_scale.empty() ? nullptr : (double *)(base + o);
    hipError_t e1 = hipMemcpyAsync(r->state, r->in_state.data(), sizeof(double) * r->row * z,
                                   hipMemcpyHostToDevice, S->copy);
    hipError_t e2 = r->scale ? hipMemcpyAsync(r->scale, r->in_scale.data(), r->in_scale.size() * sizeof(double),
                                              hipMemcpyHostToDevice, S->copy)
                             : hipSuccess;
    hipError_t e3 = hipEventRecord(r->uploaded, S->copy);
    return e1 == hipSuccess && e2 == hipSuccess && e3 == hipSuccess;
}

int64_t HipDev::slice(const void *cls, int max_nr)
{
    return slice_zones(S, static_cast<const KernelInfo *>(cls), max_nr);
}

bool HipDev::launch(int s, const std::vector<Part> &parts, Handle *h)
{
    const KernelInfo *k = static_cast<const KernelInfo *>(parts[0].r->cls);
    std::vector<zb_segment> segs;
    hipStream_t st = S->streams[s];
    for (const Part &p : parts) {
        const Request *r = static_cast<const Request *>(p.r);
        zb_segment g;
        g.net = r->net;
        g.state = r->state + (size_t)p.first * r->row;
        g.zones = p.n;
        g.dt = r->dt;
        g.rtol = r->rtol;
        g.atol = r->atol;
        g.rate_scale = r->scale ? r->scale + (size_t)p.first * r->net->dn.nr : nullptr;
        g.zone_status = r->status + p.first;
        g.stats = r->stats + p.first;
        g.source = nullptr;
        segs.push_back(g);
        if (hipStreamWaitEvent(st, r->uploaded, 0) != hipSuccess) {
            err = ZB_EDEVICE;
            msg = "stream wait failed";
            return false;
        }
    }
    // one block and one event per launch in flight: nstreams * depth of each exist
    h->qblock = S->free_qblocks.back();
    S->free_qblocks.pop_back();
    h->done = S->free_events.back();
    S->free_events.pop_back();
    Workspace ws{S->queues + (size_t)h->qblock * MAXSEG, 1, S->nfail};
    zb_opts o = S->opts;
    zb_err e = burn_impl(S->ctx, segs.data(), (int)segs.size(), &o, st, k->lanes, nullptr, &ws);
    if (e == ZB_OK && hipEventRecord(h->done, st) != hipSuccess) e = ZB_EDEVICE;
    if (e != ZB_OK) {
        err = e;
        msg = "burn launch could not be issued";
        return false;
    }
    return true;
}

int HipDev::query(const Handle &h)
{
    const hipError_t q = hipEventQuery(h.done);
    if (q == hipErrorNotReady) return 1;
    if (q == hipSuccess) return 0;
    err = ZB_EDEVICE;
    msg = std::string("burn launch failed: ") + hipGetErrorString(q);
    return -1;
}

void HipDev::retire(const Handle &h)
{
    S->free_qblocks.push_back(h.qblock);
    S->free_events.push_back(h.done);
}

static void fail_all(zb_server *S, zb_err e, const std::string &msg)
{
    S->broken = e;
    S->broken_msg = msg;
    for (auto &kv : S->all) {
        if (kv.second->st != DONE) {
            kv.second->st = DONE;
            kv.second->t_done = now_s();
        }
    }
    S->sched.pending.clear();
    S->sched.active.clear();
    S->cv_done.notify_all();
}

static void server_loop(zb_server *S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    std::vector<SchedRequest *> done;
    while (!S->stop) {
        bool any = false;
        if (S->broken == ZB_OK) {
            done.clear();
            S->dev.msg.clear();
            const auto o = S->sched.step(S->dev, lk, done);
            if (!done.empty()) S->cv_done.notify_all();
            if (o == Scheduler<HipDev>::FAILED)
                fail_all(S, S->dev.msg.empty() ? ZB_EDEVICE : S->dev.err,
                         S->dev.msg.empty() ? S->sched.error : S->dev.msg);
            any = o != Scheduler<HipDev>::IDLE;
        }
        if (S->stop) break;
        if (!any) {
            // poll launches in flight often; sleep longer when idle
            if (S->sched.inflight.empty())
                S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            else
                S->cv_work.wait_for(lk, std::chrono::microseconds(100));
        }
    }
}

static zb_err server_free(zb_server *S)
{
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    DeviceGuard g(S->ctx->device);
    for (auto s : S->streams) (void)hipStreamSynchronize(s);
    if (S->copy) (void)hipStreamSynchronize(S->copy);
    for (auto &kv : S->all) {
        if (kv.second->uploaded) (void)hipEventDestroy(kv.second->uploaded);
        delete kv.second;
    }
    for (auto &L : S->sched.inflight) (void)hipEventDestroy(L.h.done);
    for (auto e : S->free_events) (void)hipEventDestroy(e);
    for (auto s : S->streams) (void)hipStreamDestroy(s);
    if (S->copy) (void)hipStreamDestroy(S->copy);
    if (S->arena_base) (void)hipFree(S->arena_base);
    if (S->queues) (void)hipFree(S->queues);
    delete S;
    return ZB_OK;
}

extern "C" zb_err zb_server_create(zb_context *ctx, const zb_server_opts *so, zb_server **out)
{
    if (!ctx || !so || !out) return fail(ZB_EINVAL, "NULL argument");
    *out = nullptr;
    if (so->hbm_budget_bytes < (1u << 20)) return fail(ZB_EINVAL, "hbm_budget_bytes must be at least 1 MiB");
    if (so->streams < 0 || so->streams > 8) return fail(ZB_EINVAL, "streams must be 0..8");
    if (so->launches_per_stream < 0 || so->launches_per_stream > 4)
        return fail(ZB_EINVAL, "launches_per_stream must be 0..4");
    if (so->slice_zones < 0 || so->max_pending < 0) return fail(ZB_EINVAL, "negative size");
    const zb_opts &bo = so->burn;
    if (bo.precision != ZB_FP64 && bo.precision != ZB_MIXED) return fail(ZB_EINVAL, "precision %d", bo.precision);
    if (bo.mapping != ZB_MAP_AUTO && (bo.mapping < 1 || bo.mapping > 64 || (bo.mapping & (bo.mapping - 1))))
        return fail(ZB_EINVAL, "mapping must be 0 or a power of two 1..64");
    if (bo.retry && !(isfinite(bo.retry_rtol) && bo.retry_rtol > 0.0 && isfinite(bo.retry_atol) &&
                      bo.retry_atol > 0.0))
        return fail(ZB_EINVAL, "retry needs finite retry_rtol > 0 and retry_atol > 0");
    if (bo.jac_policy != ZB_JAC_EVERY_STEP && bo.jac_policy != ZB_JAC_REUSE)
        return fail(ZB_EINVAL, "jac_policy %d", bo.jac_policy);
    if (bo.integrator != ZB_BDF && bo.integrator != ZB_RKC && bo.integrator != ZB_BDF_VARIABLE)
        return fail(ZB_EINVAL, "integrator %d", bo.integrator);
    if (bo.integrator == ZB_RKC && bo.precision == ZB_MIXED)
        return fail(ZB_EINVAL, "the RKC integrator has no LU: use ZB_FP64");
    if (bo.retry && bo.retry_jac != ZB_RETRY_JAC_ANALYTIC && bo.retry_jac != ZB_RETRY_JAC_FD)
        return fail(ZB_EINVAL, "retry_jac %d", bo.retry_jac);
    if (bo.retry && bo.integrator == ZB_RKC && bo.retry_jac == ZB_RETRY_JAC_FD)
        return fail(ZB_EINVAL, "the finite-difference retry Jacobian is a BDF option");
    {
        const zb_err e = check_lu(&bo, bo.precision);
        if (e != ZB_OK) return e;
    }
    if (bo.fp64_fallback != 0 && bo.fp64_fallback != 1)
        return fail(ZB_EINVAL, "fp64_fallback %d", bo.fp64_fallback);
    if (bo.fp64_fallback && bo.precision == ZB_MIXED)
        return fail(ZB_EUNSUPPORTED, "the server has no FP64 fallback");
    DeviceGuard g(ctx->device);
    zb_server *S = new (std::nothrow) zb_server();
    if (!S) return fail(ZB_ENOMEM, "host allocation failed");
    S->ctx = ctx;
    S->opts = bo;
    S->nstreams = so->streams ? so->streams : 4;
    S->depth = so->launches_per_stream ? so->launches_per_stream : 2;
    S->slice_req = so->slice_zones;
    S->max_pending = so->max_pending ? (size_t)so->max_pending : 1024;
    const int nblocks = S->nstreams * S->depth;
    if (hipMalloc((void **)&S->arena_base, so->hbm_budget_bytes) != hipSuccess) {
        delete S;
        return fail(ZB_ENOMEM, "could not allocate the HBM budget of %zu bytes", (size_t)so->hbm_budget_bytes);
    }
    S->dev.S = S;
    if (hipMalloc((void **)&S->queues, sizeof(unsigned long long) * (MAXSEG * (size_t)nblocks + 1)) != hipSuccess) {
        (void)hipFree(S->arena_base);
        delete S;
        return fail(ZB_ENOMEM, "queue allocation failed");
    }
    S->nfail = S->queues + (size_t)MAXSEG * nblocks;
    S->streams.resize(S->nstreams, nullptr);
    S->sched.init(so->hbm_budget_bytes, S->nstreams, S->depth, MAXSEG);
    bool ok = launch_reset(S->nfail, 1, nullptr) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    for (int i = 0; ok && i < S->nstreams; ++i) ok = hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&S->copy, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < nblocks; ++i) {
        hipEvent_t e = nullptr;
        ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (ok) S->free_events.push_back(e);
        S->free_qblocks.push_back(i);
    }
    if (!ok) {
        server_free(S);
        return fail(ZB_EDEVICE, "stream or event creation failed");
    }
    S->worker = std::thread(server_loop, S);
    *out = S;
    return ZB_OK;
}

extern "C" zb_err zb_server_submit(zb_server *S, const zb_network *net, const double *host_state,
                                   int64_t zones, double dt, double rtol, double atol,
                                   const double *host_rate_scale, uint64_t *ticket)
{
    if (!S || !net || !ticket) return fail(ZB_EINVAL, "NULL argument");
    if (net->ctx != S->ctx) return fail(ZB_EINVAL, "network belongs to another context");
    if (zones <= 0 || !host_state) return fail(ZB_EINVAL, "a request needs zones > 0 and a state");
    if (!(isfinite(dt) && dt > 0.0) || !(isfinite(rtol) && rtol > 0.0) || !(isfinite(atol) && atol > 0.0))
        return fail(ZB_EINVAL, "dt, rtol and atol must be finite and > 0");
    const int row = net->dn.ns + 1;
    const int lanes = lanes_for(S->ctx, net, S->opts.precision, &S->opts);
    const zb_opts ro = resolved_opts(S->ctx, net, S->opts.precision, &S->opts);
    const KernelInfo *k = kernel_for(net->dn.nv, lanes, S->opts.precision == ZB_MIXED,
                                     method_of(&ro));
    if (!k) return fail(ZB_EUNSUPPORTED, "no kernel for nv=%d with %d lanes", net->dn.nv, lanes);
    auto al = arena_round;
    size_t bytes = al(sizeof(double) * row * (size_t)zones) + al(sizeof(int32_t) * (size_t)zones) +
                   al(sizeof(zb_zone_stats) * (size_t)zones) +
                   (host_rate_scale ? al(sizeof(double) * net->dn.nr * (size_t)zones) : 0);
    if (bytes > S->sched.arena.size())
        return fail(ZB_EINVAL, "request needs %zu device bytes, more than the whole budget", bytes);
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(ZB_ENOMEM, "host allocation failed");
    r->net = net;
    r->k = k;
    r->cls = k;
    r->nr = net->dn.nr;
    r->row = row;
    r->zones = zones;
    r->dt = dt;
    r->rtol = rtol;
    r->atol = atol;
    r->bytes = bytes;
    // relative work per zone for the launch order: per step the LU and solves grow
    // with the square of the padded size, the rates and Jacobian with the reactions
    r->cost = (double)k->nvp * k->nvp * (double)(net->dn.nr + net->dn.nv);
    r->t_submit = now_s();
    try {
        r->in_state.assign(host_state, host_state + (size_t)row * zones);
        if (host_rate_scale) r->in_scale.assign(host_rate_scale, host_rate_scale + (size_t)net->dn.nr * zones);
    } catch (...) {
        delete r;
        return fail(ZB_ENOMEM, "host copy of the request failed");
    }
    {
        DeviceGuard g(S->ctx->device);
        if (hipEventCreateWithFlags(&r->uploaded, hipEventDisableTiming) != hipSuccess) {
            delete r;
            return fail(ZB_EDEVICE, "event creation failed");
        }
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->broken != ZB_OK) {
            (void)hipEventDestroy(r->uploaded);
            delete r;
            return fail(S->broken, "server stopped: %s", S->broken_msg.c_str());
        }
        if (S->sched.pending.size() >= S->max_pending) {
            (void)hipEventDestroy(r->uploaded);
            delete r;
            return fail(ZB_EBUSY, "pending queue full (%zu requests)", S->max_pending);
        }
        r->ticket = S->next_ticket++;
        S->sched.enqueue(r);
        S->all[r->ticket] = r;
        *ticket = r->ticket;
    }
    S->cv_work.notify_all();
    return ZB_OK;
}

extern "C" zb_err zb_server_wait(zb_server *S, uint64_t ticket, double timeout_s, int32_t *done)
{
    if (!S || !done) return fail(ZB_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(ZB_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (timeout_s > 0.0)
        S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->st == DONE; });
    *done = r->st == DONE;
    if (S->broken != ZB_OK) return fail(S->broken, "server stopped: %s", S->broken_msg.c_str());
    return ZB_OK;
}

extern "C" zb_err zb_server_fetch(zb_server *S, uint64_t ticket, double *host_state_out,
                                  int32_t *zone_status_out, zb_zone_stats *stats_out,
                                  zb_request_info *info)
{
    if (!S) return fail(ZB_EINVAL, "NULL server");
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return fail(ZB_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        if (S->broken != ZB_OK) return fail(S->broken, "server stopped: %s", S->broken_msg.c_str());
        if (r->st != DONE) return fail(ZB_EBUSY, "request %llu is not finished", (unsigned long long)ticket);
        S->all.erase(it);
    }
    DeviceGuard g(S->ctx->device);
    const int64_t z = r->zones;
    zb_err e = ZB_OK;
    std::vector<int32_t> st;
    int32_t *st_dst = zone_status_out;
    if (info && !st_dst) {
        st.resize(z);
        st_dst = st.data();
    }
    if (host_state_out &&
        hipMemcpyAsync(host_state_out, r->state, sizeof(double) * r->row * z, hipMemcpyDeviceToHost, S->copy) != hipSuccess)
        e = ZB_EDEVICE;
    if (e == ZB_OK && st_dst &&
        hipMemcpyAsync(st_dst, r->status, sizeof(int32_t) * z, hipMemcpyDeviceToHost, S->copy) != hipSuccess)
        e = ZB_EDEVICE;
    if (e == ZB_OK && stats_out &&
        hipMemcpyAsync(stats_out, r->stats, sizeof(zb_zone_stats) * z, hipMemcpyDeviceToHost, S->copy) != hipSuccess)
        e = ZB_EDEVICE;
    if (e == ZB_OK && hipStreamSynchronize(S->copy) != hipSuccess) e = ZB_EDEVICE;
    if (info) {
        info->zones = z;
        int64_t ok = 0;
        if (e == ZB_OK)
            for (int64_t i = 0; i < z; ++i)
                ok += st_dst[i] == ZB_ZONE_OK || st_dst[i] == ZB_ZONE_OK_RETRY || st_dst[i] == ZB_ZONE_OK_FP64;
        info->zones_ok = ok;
        info->queue_s = r->t_admit - r->t_submit;
        info->latency_s = r->t_done - r->t_submit;
        info->first_launch_s = r->t_first - r->t_submit;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->sched.release(r);
    }
    S->cv_work.notify_all();   // memory freed: admission may proceed
    (void)hipEventDestroy(r->uploaded);
    delete r;
    return e == ZB_OK ? ZB_OK : fail(e, "copy of the results failed");
}

extern "C" zb_err zb_server_stats(zb_server *S, zb_server_totals *out)
{
    if (!S || !out) return fail(ZB_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out->requests_done = (int64_t)S->sched.n_done;
    out->zones_done = S->sched.zones_done;
    out->launches = (int64_t)S->sched.n_launches;
    out->pending = (int64_t)S->sched.pending.size();
    out->active = (int64_t)S->sched.active.size();
    out->bytes_in_use = (int64_t)S->sched.arena.used();
    out->peak_bytes_in_use = (int64_t)S->sched.peak_used;
    return ZB_OK;
}

extern "C" zb_err zb_server_destroy(zb_server *S)
{
    if (!S) return ZB_OK;
    return server_free(S);
}
