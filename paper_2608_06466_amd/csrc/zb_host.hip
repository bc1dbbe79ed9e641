// Host runtime of libzoneburn: contexts, device copies of networks, kernel
// selection, launch configuration and the C ABI declared in include/zoneburn.h.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "zb_host_internal.h"

using namespace zb;
using namespace zbh;

static thread_local std::string g_last_error;

zb_err zbh::fail(zb_err e, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return e;
}

// ------------------------------------------------------------------ context

// Scratch of zb_burn_batch_noalloc: the zone-queue counters of its launches.  Each GPU the
// library runs on holds its own copy until the process ends; every such call on a GPU
// shares that copy (calls that overlap on one GPU race).  In host code the name is not a
// device address: the address is taken once per device with hipGetSymbolAddress (at
// context creation) and only that address is used.
static __device__ __align__(256) unsigned long long scratch[STATIC_LAUNCHES * MAXSEG];

static std::mutex g_scratch_mu;
static unsigned long long *g_scratch_ptr[64];

// This device's address of `scratch` (the device is current).
static zb_err static_scratch_address(int device, unsigned long long **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= 64) return fail(ZB_EUNSUPPORTED, "device %d: no scratch slot", device);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ZB_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[device] = (unsigned long long *)ptr;
    }
    *out = g_scratch_ptr[device];
    return ZB_OK;
}

extern "C" zb_err zb_context_create(int device, zb_context **out)
{
    if (!out) return fail(ZB_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(ZB_EINVAL, "device %d out of range (%d devices)", device, n);
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(ZB_EUNSUPPORTED, "device %d is %s; the kernels are built for gfx950", device,
                    prop.gcnArchName);
    zb_context *c = new (std::nothrow) zb_context();
    if (!c) return fail(ZB_ENOMEM, "host allocation failed");
    c->device = device;
    c->cus = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    const size_t nq = 1 + (size_t)(QUEUE_SLOTS + QUEUE_CAPTURE_SLOTS) * MAXSEG;
    if (hipMalloc((void **)&c->ws, sizeof(unsigned long long) * nq) != hipSuccess) {
        delete c;
        return fail(ZB_ENOMEM, "workspace allocation failed");
    }
    if (hipMalloc((void **)&c->fb, sizeof(unsigned long long) * (FB_SLOTS + FB_CAPTURE_SLOTS) *
                                       (size_t)FB_STRIDE) != hipSuccess) {
        (void)hipFree(c->ws);
        delete c;
        return fail(ZB_ENOMEM, "workspace allocation failed");
    }
    if (static_scratch_address(device, &c->static_scratch) != ZB_OK) {
        (void)hipFree(c->ws);
        (void)hipFree(c->fb);
        delete c;
        return ZB_EDEVICE;
    }
    c->qring.init(QUEUE_SLOTS, QUEUE_CAPTURE_SLOTS);
    c->fbring.init(FB_SLOTS, FB_CAPTURE_SLOTS);
    c->qev.assign(QUEUE_SLOTS, nullptr);
    c->fbev.assign(FB_SLOTS, nullptr);
    if (launch_reset(c->ws, nq, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->ws);
        (void)hipFree(c->fb);
        delete c;
        return fail(ZB_EDEVICE, "workspace initialisation failed");
    }
    *out = c;
    return ZB_OK;
}

extern "C" zb_err zb_context_destroy(zb_context *ctx)
{
    if (!ctx) return ZB_OK;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ws);
        (void)hipFree(ctx->fb);
        for (auto s : ctx->side) (void)hipStreamDestroy(s);
        for (auto e : ctx->join) (void)hipEventDestroy(e);
        if (ctx->fork) (void)hipEventDestroy(ctx->fork);
        for (auto e : ctx->qev)
            if (e) (void)hipEventDestroy(e);
        for (auto e : ctx->fbev)
            if (e) (void)hipEventDestroy(e);
    }
    delete ctx;
    return ZB_OK;
}

// ------------------------------------------------------------------ network

extern "C" zb_err zb_network_create(zb_context *ctx, const zb_network_desc *d, zb_network **out)
{
    if (!ctx || !d || !out) return fail(ZB_EINVAL, "NULL argument");
    *out = nullptr;
    const int ns = d->n_species, nr = d->n_reactions, th = d->thermal ? 1 : 0;
    const int nv = ns + th;
    if (ns < 1 || nv > NVMAX) return fail(ZB_EINVAL, "n_species %d: need 1 <= n_species + thermal <= %d", ns, NVMAX);
    if (nr < 0 || nr > RMAX) return fail(ZB_EINVAL, "n_reactions %d out of range 0..%d", nr, RMAX);
    if (nr > 0 && (!d->reactant || !d->product || !d->lnA || !d->n_exp || !d->E || (th && !d->q)))
        return fail(ZB_EINVAL, "NULL reaction array");
    std::vector<int4> rct(std::max(nr, 1));
    std::vector<double4> par(std::max(nr, 1));
    for (int r = 0; r < nr; ++r) {
        int a = d->reactant[2 * r], b = d->reactant[2 * r + 1];
        int c = d->product[2 * r], e = d->product[2 * r + 1];
        if (a < 0 || a >= ns || b < -1 || b >= ns || c < 0 || c >= ns || e < -1 || e >= ns)
            return fail(ZB_EINVAL, "reaction %d: species index out of range", r);
        double q = th ? d->q[r] : 0.0;
        if (!isfinite(d->lnA[r]) || !isfinite(d->n_exp[r]) || !isfinite(d->E[r]) || !isfinite(q))
            return fail(ZB_EINVAL, "reaction %d: non-finite parameter", r);
        rct[r] = make_int4(a, b, c, e);
        par[r] = make_double4(d->lnA[r], d->n_exp[r], d->E[r], q);
    }
    // per-species involvement lists (net stoichiometry != 0)
    std::vector<std::vector<int2>> inv(ns);
    for (int r = 0; r < nr; ++r) {
        const int4 x = rct[r];
        for (int i = 0; i < ns; ++i) {
            int nu = (x.z == i) + (x.w == i) - (x.x == i) - (x.y == i);
            if (nu != 0) inv[i].push_back(make_int2(r | (int)((unsigned)nu << 16), x.x | ((x.y + 1) << 8)));
        }
    }
    int inv_len = 2;
    for (int i = 0; i < ns; ++i) inv_len = std::max<int>(inv_len, (int)inv[i].size());
    inv_len += inv_len & 1;   // even: the kernels take two entries per iteration
    std::vector<int2> invf((size_t)ns * inv_len, make_int2(0, 0));   // nu = 0 pads a row
    for (int i = 0; i < ns; ++i) std::copy(inv[i].begin(), inv[i].end(), invf.begin() + (size_t)i * inv_len);
    size_t o_rct = 0, o_par = o_rct + sizeof(int4) * rct.size();
    size_t o_inv = o_par + sizeof(double4) * par.size();
    size_t bytes = o_inv + sizeof(int2) * invf.size();
    zb_network *n = new (std::nothrow) zb_network();
    if (!n) return fail(ZB_ENOMEM, "host allocation failed");
    DeviceGuard g(ctx->device);
    char *dm = nullptr;
    if (hipMalloc((void **)&dm, bytes) != hipSuccess) {
        delete n;
        return fail(ZB_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    std::vector<char> host(bytes);
    memcpy(host.data() + o_rct, rct.data(), sizeof(int4) * rct.size());
    memcpy(host.data() + o_par, par.data(), sizeof(double4) * par.size());
    memcpy(host.data() + o_inv, invf.data(), sizeof(int2) * invf.size());
    if (hipMemcpy(dm, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dm);
        delete n;
        return fail(ZB_EDEVICE, "copy of the network to the device failed");
    }
    n->ctx = ctx;
    n->dmem = dm;
    n->dn.ns = ns;
    n->dn.nv = nv;
    n->dn.thermal = th;
    n->dn.nr = nr;
    n->dn.inv_len = inv_len;
    n->dn.rct = (const int4 *)(dm + o_rct);
    n->dn.par = (const double4 *)(dm + o_par);
    n->dn.inv = (const int2 *)(dm + o_inv);
    *out = n;
    return ZB_OK;
}

extern "C" zb_err zb_network_destroy(zb_network *n)
{
    if (!n) return ZB_OK;
    {
        DeviceGuard g(n->ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(n->dmem);
    }
    delete n;
    return ZB_OK;
}

extern "C" zb_err zb_network_info(const zb_network *n, int32_t *n_var, int32_t *n_reactions)
{
    if (!n) return fail(ZB_EINVAL, "NULL network");
    if (n_var) *n_var = n->dn.nv;
    if (n_reactions) *n_reactions = n->dn.nr;
    return ZB_OK;
}

// ------------------------------------------------------------- kernel choice

// LDS of a launch; rates as in lds_layout (true is the larger, for choices made before the
// segments are known).
static size_t launch_lds(const KernelInfo *k, int max_nr, bool rates = true)
{
    const int G = 64 / k->lanes;
    const int rpl = (k->nvp + k->lanes - 1) / k->lanes;
    const LdsLayout lay = lds_layout(k->nvp, k->lanes, rpl, max_nr, method_vc(k->jac),
                                     jac_f32(k->nvp, k->mixed != 0), rates,
                                     hist_regs(k->nvp, k->lanes, k->mixed != 0, k->jac));
    return (size_t)G * lay.total * sizeof(double);
}

// Lanes per zone when the caller does not choose.  Up to 4 variables, 4 lanes (one row each)
// beat one lane with every row: Robertson 2^19 zones in 64 against 79 ms, 4096 zones in 4.4
// against 9.3 ms (MI355X, mixed precision).
static int default_lanes(int nv)
{
    if (nv <= 4) return 4;
    if (nv <= 8) return 8;
    if (nv <= 16) return 16;
    if (nv <= 32) return 32;
    return 64;
}

// Smallest kernel with nvp >= nv for the given lanes and precision.
// The kernel of a method; the blocked-LU methods exist for the 48-row whole-wave kernels
// only, and other mappings take the same method with the vector-unit LU.
const KernelInfo *zbh::kernel_for(int nv, int lanes, int mixed, int method)
{
    const KernelInfo *k = find_kernel(nv, lanes, mixed, method);
    if (!k && method_blocked_lu(method))
        k = find_kernel(nv, lanes, mixed, method_vc(method) ? METHOD_BDF_VC : METHOD_BDF);
    return k;
}

const KernelInfo *zbh::find_kernel(int nv, int lanes, int mixed, int jac)
{
    const KernelInfo *tab;
    int n = kernel_table(&tab);
    const KernelInfo *best = nullptr;
    for (int i = 0; i < n; ++i) {
        if (tab[i].lanes != lanes || tab[i].mixed != mixed || tab[i].jac != jac || tab[i].nvp < nv)
            continue;
        if (!best || tab[i].nvp < best->nvp) best = &tab[i];
    }
    return best;
}

// ZB_LU_AUTO: the tuned LU where the options allow the matrix-core one (FP32 LU, Jacobian
// every step, a BDF integrator, the tuned lanes), else the vector LU.
int zbh::lu_for(zb_context *ctx, const zb_network *net, int prec, const zb_opts *o)
{
    if (!o) return ZB_LU_VALU;
    if (o->lu != ZB_LU_AUTO) return o->lu;
    if (prec != ZB_MIXED || o->integrator == ZB_RKC || o->jac_policy != ZB_JAC_EVERY_STEP)
        return ZB_LU_VALU;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &t : ctx->tuned)
        if (t.nv == net->dn.nv && t.nr == net->dn.nr && t.prec == prec)
            return (t.auto_lu == ZB_LU_MFMA &&
                    (o->mapping == ZB_MAP_AUTO || o->mapping == t.auto_lanes))
                       ? ZB_LU_MFMA
                       : ZB_LU_VALU;
    return ZB_LU_VALU;
}

zb_opts zbh::resolved_opts(zb_context *ctx, const zb_network *net, int prec, const zb_opts *o)
{
    zb_opts r{};
    if (o) r = *o;
    r.precision = prec;
    r.lu = lu_for(ctx, net, prec, o);
    return r;
}

int zbh::lanes_for(zb_context *ctx, const zb_network *net, int prec, const zb_opts *o)
{
    if (o && o->mapping != ZB_MAP_AUTO) return o->mapping;
    const bool auto_mfma = o && o->lu == ZB_LU_AUTO && lu_for(ctx, net, prec, o) == ZB_LU_MFMA;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &t : ctx->tuned)
        if (t.nv == net->dn.nv && t.nr == net->dn.nr && t.prec == prec)
            return auto_mfma ? t.auto_lanes : t.lanes;
    // The per-zone LDS area holds the reaction columns (5 doubles a reaction) once per zone of
    // the wave, so a small network with many reactions needs wider groups: widen until two
    // waves fit a CU.
    const int steps[] = {1, 4, 8, 16, 32, 64};
    const int L0 = default_lanes(net->dn.nv);
    for (int L : steps) {
        if (L < L0) continue;
        const KernelInfo *k = find_kernel(net->dn.nv, L, prec == ZB_MIXED, 0);
        if (k && launch_lds(k, net->dn.nr) <= 80 * 1024) return L;
    }
    return 64;
}

extern "C" zb_err zb_get_mapping(zb_context *ctx, const zb_network *net, int32_t precision, int32_t *lanes)
{
    if (!ctx || !net || !lanes) return fail(ZB_EINVAL, "NULL argument");
    *lanes = lanes_for(ctx, net, precision, nullptr);
    return ZB_OK;
}

// ------------------------------------------------------------------- launch

static bool valid_ptr(const void *p, int device)
{
    if (!p) return true;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) return a.device == device;
    return false;
}

zb_err zbh::check_lu(const zb_opts *o, int prec)
{
    if (!o || o->lu == ZB_LU_VALU || o->lu == ZB_LU_AUTO) return ZB_OK;
    if (o->lu != ZB_LU_MFMA) return fail(ZB_EINVAL, "lu %d", o->lu);
    if (prec != ZB_MIXED) return fail(ZB_EINVAL, "the matrix-core LU is FP32: use ZB_MIXED");
    if (o->integrator == ZB_RKC) return fail(ZB_EINVAL, "the RKC integrator has no LU");
    if (o->jac_policy != ZB_JAC_EVERY_STEP)
        return fail(ZB_EINVAL, "the matrix-core LU takes the Jacobian every step (its LDS staging "
                               "area holds the Jacobian otherwise)");
    return ZB_OK;
}

zb_err zbh::check_segment(zb_context *ctx, const zb_segment &s)
{
    if (!s.net) return fail(ZB_EINVAL, "NULL network");
    if (s.net->ctx != ctx) return fail(ZB_EINVAL, "network belongs to another context");
    if (s.zones < 0) return fail(ZB_EINVAL, "zones < 0");
    if (!(isfinite(s.dt) && s.dt > 0.0)) return fail(ZB_EINVAL, "dt must be finite and > 0");
    if (!(isfinite(s.rtol) && s.rtol > 0.0)) return fail(ZB_EINVAL, "rtol must be finite and > 0");
    if (!(isfinite(s.atol) && s.atol > 0.0)) return fail(ZB_EINVAL, "atol must be finite and > 0");
    if (s.zones > 0 && !s.state) return fail(ZB_EINVAL, "NULL state with zones > 0");
    if (s.zones > 0) {
        if (!valid_ptr(s.state, ctx->device)) return fail(ZB_EINVAL, "state is not device memory of device %d", ctx->device);
        if (!valid_ptr(s.rate_scale, ctx->device)) return fail(ZB_EINVAL, "rate_scale is not device memory");
        if (!valid_ptr(s.source, ctx->device)) return fail(ZB_EINVAL, "source is not device memory");
        if (!valid_ptr(s.zone_status, ctx->device)) return fail(ZB_EINVAL, "zone_status is not device memory");
        if (!valid_ptr(s.stats, ctx->device)) return fail(ZB_EINVAL, "stats is not device memory");
    }
    return ZB_OK;
}


int zbh::blocks_per_cu(const KernelInfo *k, int max_nr)
{
    const size_t lds = launch_lds(k, max_nr);
    if (lds > 160 * 1024) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k->fn, 64, lds) != hipSuccess) return 0;
    return per_cu;
}

// One persistent launch over segments that all use the same kernel.  queue:
// MAXSEG device counters the launch clears first; nfail: failed-zone counter.
namespace {
struct RunOpts {
    int max_steps, retry, retry_max_steps, jac_policy, retry_jac;
    double retry_rtol, retry_atol;
    int fallback;
};
}  // namespace

static RunOpts run_opts(const zb_opts *o)
{
    RunOpts r{100000, 0, 100000, 0, 0, 0.0, 0.0, 0};
    if (o && o->max_steps > 0) r.max_steps = o->max_steps;
    if (o) r.jac_policy = o->jac_policy;
    if (o) r.fallback = o->fp64_fallback;
    if (o && o->retry) {
        r.retry = 1;
        r.retry_rtol = o->retry_rtol;
        r.retry_atol = o->retry_atol;
        r.retry_max_steps = o->retry_max_steps > 0 ? o->retry_max_steps : r.max_steps;
        r.retry_jac = o->retry_jac;
    }
    return r;
}

// With the FP64 fallback (a mixed-precision kernel and fb lists): the mixed run lists the
// zones it fails, and the FP64 kernel of the same class then burns those from their inputs.
static zb_err launch_segments(zb_context *ctx, const KernelInfo *k, const zb_segment *segs, int n,
                              const RunOpts &ro, hipStream_t stream, unsigned long long *queue,
                              unsigned long long *nfail, float *ms_out, unsigned long long *fb)
{
    BurnArgs A;
    memset(&A, 0, sizeof A);
    int64_t total = 0;
    int max_nr = 0;
    bool rates = false;
    for (int i = 0; i < n; ++i) {
        Segment &S = A.seg[i];
        S.net = segs[i].net->dn;
        S.state = segs[i].state;
        S.scale = segs[i].rate_scale;
        S.source = segs[i].source;
        S.status = segs[i].zone_status;
        S.stats = (int32_t *)segs[i].stats;
        S.zones = segs[i].zones;
        S.dt = segs[i].dt;
        S.rtol = segs[i].rtol;
        S.atol = segs[i].atol;
        total += segs[i].zones;
        max_nr = std::max(max_nr, S.net.nr);
        rates = rates || S.scale != nullptr || !S.net.thermal;
    }
    if (total == 0) return ZB_OK;
    A.nseg = n;
    A.max_nr = max_nr;
    A.max_steps = ro.max_steps;
    A.retry = ro.retry;
    A.retry_max_steps = ro.retry_max_steps;
    A.retry_rtol = ro.retry_rtol;
    A.retry_atol = ro.retry_atol;
    A.retry_jac = ro.retry_jac;
    A.rates_lds = rates ? 1 : 0;
    const bool fb_on = ro.fallback && k->mixed && fb;
    A.fb = fb;
    A.fb_mode = fb_on ? 1 : 0;
    A.queue = queue;
    A.nfail = nfail;

    const int G = 64 / k->lanes;
    const size_t lds = launch_lds(k, max_nr, rates);
    if (lds > 160 * 1024) return fail(ZB_EUNSUPPORTED, "LDS need %zu bytes exceeds 160 KiB", lds);
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k->fn, 64, lds));
    if (per_cu < 1) return fail(ZB_EUNSUPPORTED, "kernel does not fit on a CU (LDS %zu)", lds);
    int64_t groups = (total + G - 1) / G;
    int64_t blocks = std::min<int64_t>((int64_t)per_cu * ctx->cus, groups);
    HIP_TRY(launch_reset(A.queue, MAXSEG, stream));
    if (fb_on) HIP_TRY(launch_reset(fb, MAXSEG, stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms_out) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, stream));
    }
    void *args[] = {&A};
    HIP_TRY(hipLaunchKernel(k->fn, dim3((unsigned)blocks), dim3(64), args, lds, stream));
    if (fb_on) {
        // the FP64 kernel of the class (the blocked-LU methods have none: their vector-LU form)
        const KernelInfo *kf = kernel_for(k->nvp, k->lanes, 0, k->jac);
        if (!kf) return fail(ZB_EUNSUPPORTED, "no FP64 kernel for the fallback (nvp %d)", k->nvp);
        const size_t ldsf = launch_lds(kf, max_nr, rates);
        int per_cu_f = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_f, kf->fn, 64, ldsf));
        if (per_cu_f < 1 || ldsf > 160 * 1024)
            return fail(ZB_EUNSUPPORTED, "fallback kernel does not fit on a CU (LDS %zu)", ldsf);
        const int Gf = 64 / kf->lanes;
        const int64_t listed = std::min<int64_t>(total, (int64_t)n * FB_CAP);
        const int64_t blocks_f = std::min<int64_t>((int64_t)per_cu_f * ctx->cus, (listed + Gf - 1) / Gf);
        BurnArgs B = A;
        B.fb_mode = 2;
        void *bargs[] = {&B};
        HIP_TRY(launch_reset(A.queue, MAXSEG, stream));
        HIP_TRY(hipLaunchKernel(kf->fn, dim3((unsigned)blocks_f), dim3(64), bargs, ldsf, stream));
    }
    if (ms_out) {
        HIP_TRY(hipEventRecord(e1, stream));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(ms_out, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return ZB_OK;
}

namespace {
// Segments that share a kernel: one persistent launch.
struct Group {
    const KernelInfo *k;
    std::vector<zb_segment> segs;
    double cost;   // relative device time, for ordering
};
}  // namespace

static zb_err plan_groups(zb_context *ctx, const zb_segment *segs, int n, const zb_opts *opts,
                          int force_lanes, std::vector<Group> &out)
{
    if (n < 0 || (n > 0 && !segs)) return fail(ZB_EINVAL, "bad segment list");
    const int prec = opts ? opts->precision : ZB_FP64;
    if (prec != ZB_FP64 && prec != ZB_MIXED) return fail(ZB_EINVAL, "precision %d", prec);
    if (opts && opts->mapping != ZB_MAP_AUTO &&
        (opts->mapping < 1 || opts->mapping > 64 || (opts->mapping & (opts->mapping - 1))))
        return fail(ZB_EINVAL, "mapping must be 0 or a power of two 1..64");
    if (opts && opts->retry &&
        !(isfinite(opts->retry_rtol) && opts->retry_rtol > 0.0 && isfinite(opts->retry_atol) &&
          opts->retry_atol > 0.0))
        return fail(ZB_EINVAL, "retry needs finite retry_rtol > 0 and retry_atol > 0");
    if (opts && opts->jac_policy != ZB_JAC_EVERY_STEP && opts->jac_policy != ZB_JAC_REUSE)
        return fail(ZB_EINVAL, "jac_policy %d", opts->jac_policy);
    if (opts && opts->integrator != ZB_BDF && opts->integrator != ZB_RKC &&
        opts->integrator != ZB_BDF_VARIABLE)
        return fail(ZB_EINVAL, "integrator %d", opts->integrator);
    const bool rkc = opts && opts->integrator == ZB_RKC;
    if (rkc && prec == ZB_MIXED) return fail(ZB_EINVAL, "the RKC integrator has no LU: use ZB_FP64");
    if (opts && opts->retry && opts->retry_jac != ZB_RETRY_JAC_ANALYTIC &&
        opts->retry_jac != ZB_RETRY_JAC_FD)
        return fail(ZB_EINVAL, "retry_jac %d", opts->retry_jac);
    if (opts && opts->retry && rkc && opts->retry_jac == ZB_RETRY_JAC_FD)
        return fail(ZB_EINVAL, "the finite-difference retry Jacobian is a BDF option");
    {
        const zb_err e = check_lu(opts, prec);
        if (e != ZB_OK) return e;
    }
    if (opts && opts->fp64_fallback != 0 && opts->fp64_fallback != 1)
        return fail(ZB_EINVAL, "fp64_fallback %d", opts->fp64_fallback);
    for (int i = 0; i < n; ++i) {
        zb_err e = check_segment(ctx, segs[i]);
        if (e != ZB_OK) return e;
    }
    out.clear();
    for (int i = 0; i < n; ++i) {
        if (segs[i].zones == 0) continue;
        const zb_opts so = resolved_opts(ctx, segs[i].net, prec, opts);
        const int jac = method_of(&so);
        int lanes = force_lanes ? force_lanes : lanes_for(ctx, segs[i].net, prec, opts);
        const KernelInfo *k = kernel_for(segs[i].net->dn.nv, lanes, prec == ZB_MIXED, jac);
        if (!k)
            return fail(ZB_EUNSUPPORTED, "no kernel for nv=%d with %d lanes per zone (%s)",
                        segs[i].net->dn.nv, lanes, prec == ZB_MIXED ? "mixed" : "fp64");
        Group *g = nullptr;
        for (auto &x : out)
            if (x.k == k && x.segs.size() < (size_t)MAXSEG) g = &x;
        if (!g) {
            out.push_back(Group{k, {}, 0.0});
            g = &out.back();
        }
        g->segs.push_back(segs[i]);
        // per-step work grows roughly with the square of the padded size
        g->cost += (double)segs[i].zones * (double)k->nvp * (double)k->nvp;
    }
    std::stable_sort(out.begin(), out.end(), [](const Group &a, const Group &b) { return a.cost > b.cost; });
    return ZB_OK;
}

int zbh::count_launches(zb_context *ctx, const zb_segment *segs, int n, const zb_opts *opts, int *launches)
{
    std::vector<Group> groups;
    zb_err e = plan_groups(ctx, segs, n, opts, 0, groups);
    if (e != ZB_OK) return e;
    *launches = (int)groups.size();
    return ZB_OK;
}

static zb_err side_streams(zb_context *ctx, int need)
{
    while ((int)ctx->side.size() < need) {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ctx->side.push_back(s);
        ctx->join.push_back(ev);
    }
    if (!ctx->fork) HIP_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    return ZB_OK;
}

// Launches the planned groups with the given queue counters and fallback lists.
static zb_err launch_groups(zb_context *ctx, std::vector<Group> &groups, const RunOpts &ro,
                            hipStream_t s0, std::vector<unsigned long long *> &queue,
                            unsigned long long *nfail, float *ms_out,
                            std::vector<unsigned long long *> &fb, bool serial = false)
{
    const int ng = (int)groups.size();
    if (ng == 1)
        return launch_segments(ctx, groups[0].k, groups[0].segs.data(), (int)groups[0].segs.size(),
                               ro, s0, queue[0], nfail, ms_out, fb[0]);
    if (serial) {
        for (int i = 0; i < ng; ++i) {
            zb_err e = launch_segments(ctx, groups[i].k, groups[i].segs.data(),
                                       (int)groups[i].segs.size(), ro, s0, queue[i], nfail, nullptr,
                                       fb[i]);
            if (e != ZB_OK) return e;
        }
        return ZB_OK;
    }
    // Several kernel classes: the costliest runs on the caller's stream and the
    // others on side streams forked from it and joined back, so the classes share
    // the GPU (a class's tail is filled by the others) instead of running in turn.
    std::lock_guard<std::mutex> lk(ctx->fork_mu);
    const int nside = std::min(ng - 1, MAX_SIDE_STREAMS);
    zb_err e = side_streams(ctx, nside);
    if (e != ZB_OK) return e;
    HIP_TRY(hipEventRecord(ctx->fork, s0));
    for (int j = 0; j < nside; ++j) HIP_TRY(hipStreamWaitEvent(ctx->side[j], ctx->fork, 0));
    for (int i = 0; i < ng; ++i) {
        hipStream_t s = i == 0 ? s0 : ctx->side[(i - 1) % nside];
        e = launch_segments(ctx, groups[i].k, groups[i].segs.data(), (int)groups[i].segs.size(),
                            ro, s, queue[i], nfail, nullptr, fb[i]);
        if (e != ZB_OK) return e;
    }
    for (int j = 0; j < nside; ++j) {
        HIP_TRY(hipEventRecord(ctx->join[j], ctx->side[j]));
        HIP_TRY(hipStreamWaitEvent(s0, ctx->join[j], 0));
    }
    return ZB_OK;
}

// Records, on s0 (which every launch of the call has joined), the event of each eager slot
// the call used, so that the slot's next user waits for it.
static zb_err mark_slots(zb_context *ctx, hipStream_t s0, SlotRing &ring,
                         std::vector<hipEvent_t> &ev, const std::vector<int> &slots)
{
    for (int q : slots) {
        if (!ev[q]) HIP_TRY(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev[q], s0));
        ring.mark(q);
    }
    return ZB_OK;
}

zb_err zbh::burn_impl(zb_context *ctx, const zb_segment *segs, int n, const zb_opts *opts,
                      void *stream, int force_lanes, float *ms_out, const Workspace *ws)
{
    if (!ctx) return fail(ZB_EINVAL, "NULL context");
    std::vector<Group> groups;
    zb_err e = plan_groups(ctx, segs, n, opts, force_lanes, groups);
    if (e != ZB_OK) return e;
    if (groups.empty()) return ZB_OK;
    const RunOpts ro = run_opts(opts);
    const int ng = (int)groups.size();
    if (ws && ng > ws->launches)
        return fail(ZB_EINVAL, "workspace holds queues for %d launches, %d needed", ws->launches, ng);
    DeviceGuard g(ctx->device);
    std::vector<unsigned long long *> queue(ng), fb(ng, nullptr);
    unsigned long long *nfail = ws ? ws->nfail : ctx->ws;
    const bool want_fb = ro.fallback && opts->precision == ZB_MIXED;
    hipStream_t s0 = (hipStream_t)stream;
    if (ws) {
        for (int i = 0; i < ng; ++i) queue[i] = ws->queue + (size_t)i * MAXSEG;
        if (want_fb && !ws->fb) return fail(ZB_EUNSUPPORTED, "this caller has no FP64 fallback lists");
        if (want_fb)
            for (int i = 0; i < ng; ++i) fb[i] = ws->fb + (size_t)i * FB_STRIDE;
        return launch_groups(ctx, groups, ro, s0, queue, nfail, ms_out, fb, ws->serial);
    }
    // The context's rotating slots.  A slot still in use by an earlier call is waited for
    // before this call clears it; a call being captured into a graph gets slots that no
    // other call will ever take.
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s0, &cst));
    const bool capturing = cst != hipStreamCaptureStatusNone;
    std::lock_guard<std::mutex> lk(ctx->slot_mu);
    std::vector<int> qs, fs;
    auto wait_q = [&](int s) { (void)hipEventSynchronize(ctx->qev[s]); };
    auto wait_f = [&](int s) { (void)hipEventSynchronize(ctx->fbev[s]); };
    for (int i = 0; i < ng; ++i) {
        const int q = capturing ? ctx->qring.acquire_capture() : ctx->qring.acquire(wait_q);
        if (q < 0)
            return fail(ZB_EBUSY, "all %d queue slots for captured calls are taken", QUEUE_CAPTURE_SLOTS);
        queue[i] = ctx->ws + 1 + (size_t)q * MAXSEG;
        if (!capturing) qs.push_back(q);
        if (want_fb) {
            const int f = capturing ? ctx->fbring.acquire_capture() : ctx->fbring.acquire(wait_f);
            if (f < 0)
                return fail(ZB_EBUSY, "all %d fallback lists for captured calls are taken",
                            FB_CAPTURE_SLOTS);
            fb[i] = ctx->fb + (size_t)f * FB_STRIDE;
            if (!capturing) fs.push_back(f);
        }
    }
    e = launch_groups(ctx, groups, ro, s0, queue, nfail, ms_out, fb);
    // mark the slots even after a failed launch: some of its kernels may be queued
    zb_err em = mark_slots(ctx, s0, ctx->qring, ctx->qev, qs);
    if (em == ZB_OK) em = mark_slots(ctx, s0, ctx->fbring, ctx->fbev, fs);
    return e != ZB_OK ? e : em;
}

extern "C" zb_err zb_burn(zb_context *ctx, const zb_network *net, double *state, int64_t zones,
                          double dt, double rtol, double atol, const double *rate_scale,
                          const zb_opts *opts, int32_t *zone_status, zb_zone_stats *stats, void *stream)
{
    zb_segment s;
    s.net = net;
    s.state = state;
    s.zones = zones;
    s.dt = dt;
    s.rtol = rtol;
    s.atol = atol;
    s.rate_scale = rate_scale;
    s.zone_status = zone_status;
    s.stats = stats;
    s.source = nullptr;
    return burn_impl(ctx, &s, 1, opts, stream);
}

extern "C" zb_err zb_burn_batch(zb_context *ctx, const zb_segment *segs, int32_t n_seg,
                                const zb_opts *opts, void *stream)
{
    return burn_impl(ctx, segs, n_seg, opts, stream);
}

extern "C" zb_err zb_burn_batch_noalloc(zb_context *ctx, const zb_segment *segs, int32_t n_seg,
                                        const zb_opts *opts, void *stream)
{
    if (!ctx) return fail(ZB_EINVAL, "NULL context");
    if (!ctx->static_scratch) return fail(ZB_EDEVICE, "no static scratch on this context's device");
    if (opts && opts->fp64_fallback && opts->precision == ZB_MIXED)
        return fail(ZB_EUNSUPPORTED, "fp64_fallback needs lists the static scratch does not hold");
    int launches = 0;
    zb_err e = (zb_err)count_launches(ctx, segs, n_seg, opts, &launches);   // validates everything
    if (e != ZB_OK) return e;
    if (launches > STATIC_LAUNCHES)
        return fail(ZB_EINVAL, "the call needs %d launches (kernel classes, at most %d segments "
                               "each); the static scratch holds the counters of %d",
                    launches, MAXSEG, STATIC_LAUNCHES);
    Workspace ws{ctx->static_scratch, STATIC_LAUNCHES, ctx->ws, nullptr};
    ws.serial = true;
    return burn_impl(ctx, segs, n_seg, opts, stream, 0, nullptr, &ws);
}

extern "C" zb_err zb_sync(zb_context *ctx, void *stream, int64_t *n_failed)
{
    if (!ctx) return fail(ZB_EINVAL, "NULL context");
    DeviceGuard g(ctx->device);
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    unsigned long long nf = 0;
    HIP_TRY(hipMemcpy(&nf, ctx->ws, sizeof nf, hipMemcpyDeviceToHost));
    if (nf) {
        HIP_TRY(launch_reset(ctx->ws, 1, nullptr));
        HIP_TRY(hipDeviceSynchronize());
    }
    if (n_failed) *n_failed = (int64_t)nf;
    return nf ? ZB_EZONES : ZB_OK;
}

// -------------------------------------------------------------------- graphs

struct zb_graph {
    zb_context *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long *queues = nullptr;   // launches x MAXSEG, private to this graph
    unsigned long long *fb = nullptr;       // launches x FB_STRIDE with the FP64 fallback
};

extern "C" zb_err zb_graph_create(zb_context *ctx, const zb_segment *segs, int32_t n_seg,
                                  const zb_opts *opts, zb_graph **out)
{
    if (!ctx || !out) return fail(ZB_EINVAL, "NULL argument");
    *out = nullptr;
    int launches = 0;
    zb_err e = (zb_err)count_launches(ctx, segs, n_seg, opts, &launches);   // validates everything
    if (e != ZB_OK) return e;
    DeviceGuard g(ctx->device);
    zb_graph *G = new (std::nothrow) zb_graph();
    if (!G) return fail(ZB_ENOMEM, "host allocation failed");
    G->ctx = ctx;
    const size_t qbytes = sizeof(unsigned long long) * MAXSEG * (size_t)std::max(launches, 1);
    if (hipMalloc((void **)&G->queues, qbytes) != hipSuccess) {
        delete G;
        return fail(ZB_ENOMEM, "graph queue allocation failed");
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(G->queues);
        delete G;
        return fail(ZB_EDEVICE, "stream creation failed");
    }
    if (opts && opts->fp64_fallback && opts->precision == ZB_MIXED &&
        hipMalloc((void **)&G->fb, sizeof(unsigned long long) * FB_STRIDE * (size_t)std::max(launches, 1)) !=
            hipSuccess) {
        (void)hipStreamDestroy(s);
        (void)hipFree(G->queues);
        delete G;
        return fail(ZB_ENOMEM, "graph fallback-list allocation failed");
    }
    Workspace ws{G->queues, std::max(launches, 1), ctx->ws, G->fb};
    e = ZB_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        e = fail(ZB_EDEVICE, "hipStreamBeginCapture failed");
    } else {
        zb_err eb = burn_impl(ctx, segs, n_seg, opts, s, 0, nullptr, &ws);
        hipError_t ec = hipStreamEndCapture(s, &G->graph);
        if (eb != ZB_OK) e = eb;
        else if (ec != hipSuccess) e = fail(ZB_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
        else if (hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0) != hipSuccess)
            e = fail(ZB_EDEVICE, "hipGraphInstantiate failed");
    }
    (void)hipStreamDestroy(s);
    if (e != ZB_OK) {
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
        if (G->graph) (void)hipGraphDestroy(G->graph);
        (void)hipFree(G->queues);
        delete G;
        return e;
    }
    *out = G;
    return ZB_OK;
}

extern "C" zb_err zb_graph_launch(zb_graph *G, void *stream)
{
    if (!G) return fail(ZB_EINVAL, "NULL graph");
    DeviceGuard g(G->ctx->device);
    HIP_TRY(hipGraphLaunch(G->exec, (hipStream_t)stream));
    return ZB_OK;
}

extern "C" zb_err zb_graph_destroy(zb_graph *G)
{
    if (!G) return ZB_OK;
    {
        DeviceGuard g(G->ctx->device);
        (void)hipDeviceSynchronize();
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
        if (G->graph) (void)hipGraphDestroy(G->graph);
        (void)hipFree(G->queues);
        (void)hipFree(G->fb);
    }
    delete G;
    return ZB_OK;
}

// ----------------------------------------------------------------- autotune

namespace {
struct TuneRun {
    zb_tune_candidate c;
    int li;   // log2 of the lanes
};
}  // namespace

// Times the candidates on a copy of the sample: every lanes-per-zone mapping with the vector
// LU, then (with_mfma) the matrix-core LU where a kernel of it exists for the network.  Each
// is compared with the first candidate that ran; best_valu / best_all index the fastest
// qualifying vector-LU candidate and the fastest qualifying one (-1: none).
static zb_err tune_impl(zb_context *ctx, const zb_network *net, const double *sample_state,
                        int64_t zones, double dt, double rtol, double atol, int32_t precision,
                        bool with_mfma, std::vector<TuneRun> &runs, int &best_valu, int &best_all)
{
    if (!ctx || !net || !sample_state || zones <= 0) return fail(ZB_EINVAL, "bad argument");
    if (precision != ZB_FP64 && precision != ZB_MIXED) return fail(ZB_EINVAL, "precision %d", precision);
    {
        const zb_segment probe = {net, (double *)sample_state, zones, dt, rtol, atol, nullptr, nullptr, nullptr};
        const zb_err e = check_segment(ctx, probe);
        if (e != ZB_OK) return e;
    }
    DeviceGuard g(ctx->device);
    const int row = net->dn.ns + 1;
    const size_t bytes = sizeof(double) * row * (size_t)zones;
    // the candidates: (lanes, LU)
    std::vector<std::pair<int, int>> cand;
    for (int lanes = 1; lanes <= 64; lanes *= 2) cand.push_back({lanes, ZB_LU_VALU});
    if (with_mfma && precision == ZB_MIXED && net->dn.nv > 32) {
        const KernelInfo *kb = find_kernel(net->dn.nv, 64, 1, METHOD_BDF_BLU);
        if (kb) cand.push_back({64, ZB_LU_MFMA});
    }
    // Each candidate's kernel, and how many copies of the sample it is timed on: the sample,
    // ordered longest zone first, fills the GPU's resident zones at least 8 times over
    // (copies of a zone side by side; at most 16 copies).  A sample that fills them only a
    // few times is timed mostly in its ramp-down, with few waves left to hide latencies: on
    // 8192 zones of the 48-variable network (4 times the resident 2048) the matrix-core LU
    // ran 5 % slower than the vector LU, from 16384 zones on 2.5 % faster, as on the whole
    // 262144-zone segment (1.7 %).
    struct Cand {
        int lanes, lu, reps;
        const KernelInfo *k;
    };
    std::vector<Cand> cs;
    int rmax = 1;
    for (auto [lanes, lu] : cand) {
        const KernelInfo *kk = lu == ZB_LU_MFMA ? find_kernel(net->dn.nv, lanes, 1, METHOD_BDF_BLU)
                                                : find_kernel(net->dn.nv, lanes, precision == ZB_MIXED, 0);
        int reps = 0;
        if (kk && launch_lds(kk, net->dn.nr) <= 160 * 1024) {
            const int64_t resident = (int64_t)blocks_per_cu(kk, net->dn.nr) * ctx->cus * (64 / lanes);
            reps = (int)std::min<int64_t>(16, std::max<int64_t>(1, (8 * resident + zones - 1) / zones));
            if (resident <= 0) kk = nullptr;
        } else {
            kk = nullptr;
        }
        cs.push_back({lanes, lu, kk ? reps : 0, kk});
        if (kk) rmax = std::max(rmax, reps);
    }
    const size_t rep_zones = (size_t)zones * rmax;
    double *work = nullptr, *ordered = nullptr;
    int32_t *st = nullptr;
    zb_zone_stats *zs = nullptr;
    HIP_TRY(hipMalloc((void **)&work, bytes * rmax));
    if (hipMalloc((void **)&ordered, bytes * rmax) != hipSuccess ||
        hipMalloc((void **)&st, sizeof(int32_t) * rep_zones) != hipSuccess ||
        hipMalloc((void **)&zs, sizeof(zb_zone_stats) * zones) != hipSuccess) {
        (void)hipFree(work);
        (void)hipFree(ordered);
        (void)hipFree(st);
        return fail(ZB_ENOMEM, "autotune scratch");
    }
    auto release = [&]() {
        (void)hipFree(work);
        (void)hipFree(ordered);
        (void)hipFree(st);
        (void)hipFree(zs);
    };
    std::vector<double> ref(row * (size_t)zones), cur(row * rep_zones), lpt(row * (size_t)zones);
    std::vector<int32_t> ref_st(zones), cur_st(rep_zones);
    // Zones are handed out in queue order, so the time of a sample in its given order is
    // mostly that of whichever long zones happen to start last: on 8192 zones of the
    // 48-variable network it scatters by about 2 % between runs, more than the candidates
    // differ.  The sample is therefore burned once first, for its step counts, and the
    // candidates are timed on it longest first: the time then follows the throughput.
    {
        zb_opts o{};
        o.precision = precision;
        zb_segment s = {net, work, zones, dt, rtol, atol, nullptr, st, zs};
        std::vector<zb_zone_stats> hs(zones);
        std::vector<int64_t> order(zones);
        zb_err e = ZB_OK;
        if (hipMemcpy(work, sample_state, bytes, hipMemcpyDeviceToDevice) != hipSuccess) e = ZB_EDEVICE;
        if (e == ZB_OK) e = burn_impl(ctx, &s, 1, &o, nullptr, 0, nullptr);
        if (e == ZB_OK && (hipDeviceSynchronize() != hipSuccess ||
                           hipMemcpy(hs.data(), zs, sizeof(zb_zone_stats) * zones, hipMemcpyDeviceToHost) != hipSuccess ||
                           hipMemcpy(ref.data(), sample_state, bytes, hipMemcpyDeviceToHost) != hipSuccess))
            e = ZB_EDEVICE;
        if (e != ZB_OK) {
            release();
            return e;
        }
        for (int64_t z = 0; z < zones; ++z) order[z] = z;
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t a, int64_t b) { return hs[a].nst > hs[b].nst; });
        for (int64_t z = 0; z < zones; ++z)
            memcpy(&lpt[z * row], &ref[order[z] * row], sizeof(double) * row);
    }
    bool have_ref = false;
    zb_err res = ZB_OK;
    best_valu = best_all = -1;
    runs.clear();
    for (const Cand &C : cs) {
        const int lanes = C.lanes, lu = C.lu;
        TuneRun R{{lanes, lu, -1.f, 0}, __builtin_ctz((unsigned)lanes)};
        if (!C.k) {   // this candidate cannot launch
            runs.push_back(R);
            continue;
        }
        const int r = C.reps;
        const int64_t nz = zones * (int64_t)r;
        const size_t nb = bytes * r;
        for (int64_t z = 0; z < zones; ++z)
            for (int c = 0; c < r; ++c)
                memcpy(&cur[(z * r + c) * row], &lpt[z * row], sizeof(double) * row);
        if (hipMemcpy(ordered, cur.data(), nb, hipMemcpyHostToDevice) != hipSuccess) {
            res = fail(ZB_EDEVICE, "autotune sample upload");
            break;
        }
        zb_opts o{};
        o.precision = precision;
        o.lu = lu;
        float ms = 0.f;
        // the first launch, over one copy, also loads the code object; the second is timed
        for (int rep = 0; rep < 2; ++rep) {
            zb_segment s = {net, work, rep ? nz : zones, dt, rtol, atol, nullptr, st, nullptr};
            if (hipMemcpy(work, ordered, rep ? nb : bytes, hipMemcpyDeviceToDevice) != hipSuccess) { res = ZB_EDEVICE; break; }
            zb_err e = burn_impl(ctx, &s, 1, &o, nullptr, lanes, &ms);
            if (e != ZB_OK) { res = e; break; }
        }
        if (res != ZB_OK) break;
        if (hipMemcpy(cur.data(), work, nb, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(cur_st.data(), st, sizeof(int32_t) * nz, hipMemcpyDeviceToHost) != hipSuccess) {
            res = ZB_EDEVICE;
            break;
        }
        // Every candidate runs the same integrator; the mappings differ only in the order of
        // the group reductions and the LUs in the rounding of the factorisation, so results
        // agree to rounding except on the rare ill-conditioned zone.  A candidate qualifies
        // when every zone (the first copy of each) ends with the status of the first
        // candidate that ran and at least 99% of the zones agree with it to a gated relative
        // 1e-6.
        bool ok = true;
        if (!have_ref) {
            for (int64_t z = 0; z < zones; ++z) {
                memcpy(&ref[z * row], &cur[z * r * row], sizeof(double) * row);
                ref_st[z] = cur_st[z * r];
            }
            have_ref = true;
        } else {
            int64_t agree = 0;
            for (int64_t z = 0; z < zones && ok; ++z) {
                if (cur_st[z * r] != ref_st[z]) ok = false;
                bool zok = true;
                for (int i = 0; i < row; ++i) {
                    double a = ref[z * row + i], b = cur[z * r * row + i];
                    double den = fmax(fabs(a), atol / rtol);
                    if (!(fabs(a - b) <= 1e-6 * den)) zok = false;
                }
                agree += zok;
            }
            if (ok && agree * 100 < zones * 99) ok = false;
        }
        ms /= (float)r;   // per copy of the sample
        R.c.ms = ms;
        R.c.qualified = ok ? 1 : 0;
        runs.push_back(R);
        const int idx = (int)runs.size() - 1;
        if (ok && (best_all < 0 || ms < runs[best_all].c.ms)) best_all = idx;
        if (ok && lu == ZB_LU_VALU && (best_valu < 0 || ms < runs[best_valu].c.ms)) best_valu = idx;
    }
    release();
    if (res != ZB_OK) return res;
    if (best_all < 0 || best_valu < 0) return fail(ZB_EUNSUPPORTED, "no mapping ran");
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        const zb_context::Tuned t{net->dn.nv, net->dn.nr, precision, runs[best_valu].c.lanes,
                                  runs[best_all].c.lanes, runs[best_all].c.lu};
        bool found = false;
        for (auto &x : ctx->tuned)
            if (x.nv == t.nv && x.nr == t.nr && x.prec == t.prec) {
                x = t;
                found = true;
            }
        if (!found) ctx->tuned.push_back(t);
    }
    return ZB_OK;
}

extern "C" zb_err zb_autotune(zb_context *ctx, const zb_network *net, const double *sample_state,
                              int64_t zones, double dt, double rtol, double atol, int32_t precision,
                              int32_t *best_lanes, float *times_ms)
{
    std::vector<TuneRun> runs;
    int bv = -1, ba = -1;
    const zb_err e = tune_impl(ctx, net, sample_state, zones, dt, rtol, atol, precision, false,
                               runs, bv, ba);
    if (times_ms) {
        for (int i = 0; i < 7; ++i) times_ms[i] = -1.f;
        for (auto &r : runs) times_ms[r.li] = r.c.ms;
    }
    if (e != ZB_OK) return e;
    if (best_lanes) *best_lanes = runs[bv].c.lanes;
    return ZB_OK;
}

extern "C" zb_err zb_autotune_candidates(zb_context *ctx, const zb_network *net,
                                         const double *sample_state, int64_t zones, double dt,
                                         double rtol, double atol, int32_t precision,
                                         zb_tune_candidate *out, int32_t max_out, int32_t *n_out,
                                         int32_t *best)
{
    if (max_out < 0 || (max_out > 0 && !out)) return fail(ZB_EINVAL, "bad candidate buffer");
    std::vector<TuneRun> runs;
    int bv = -1, ba = -1;
    const zb_err e = tune_impl(ctx, net, sample_state, zones, dt, rtol, atol, precision, true,
                               runs, bv, ba);
    for (int i = 0; i < (int)runs.size() && i < max_out; ++i) out[i] = runs[i].c;
    if (n_out) *n_out = (int32_t)runs.size();
    if (e != ZB_OK) return e;
    if (best) *best = ba;
    return ZB_OK;
}

// ------------------------------------------------------------ tuning cache

extern "C" zb_err zb_tune_save(zb_context *ctx, const char *path)
{
    if (!ctx || !path) return fail(ZB_EINVAL, "NULL argument");
    int rt = 0;
    HIP_TRY(hipRuntimeGetVersion(&rt));
    std::vector<TuneEntry> es;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        es = ctx->tuned;
    }
    const std::string text = tune_json(ctx->arch, rt, es);
    // written next to the target and renamed over it, so a reader never sees half a file
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return fail(ZB_EINVAL, "cannot write %s", tmp.c_str());
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) != 0 || !ok) {
        remove(tmp.c_str());
        return fail(ZB_EINVAL, "cannot write %s", tmp.c_str());
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return fail(ZB_EINVAL, "cannot replace %s", path);
    }
    return ZB_OK;
}

extern "C" zb_err zb_tune_load(zb_context *ctx, const char *path, int32_t *loaded)
{
    if (!ctx || !path) return fail(ZB_EINVAL, "NULL argument");
    if (loaded) *loaded = 0;
    FILE *f = fopen(path, "rb");
    if (!f) return fail(ZB_EINVAL, "cannot read %s", path);
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, n);
        if (text.size() > (1u << 20)) {
            fclose(f);
            return fail(ZB_EINVAL, "%s is larger than 1 MiB", path);
        }
    }
    const bool rd_err = ferror(f) != 0;
    fclose(f);
    if (rd_err) return fail(ZB_EINVAL, "cannot read %s", path);
    std::string arch, err;
    int rt_file = 0;
    std::vector<TuneEntry> es;
    if (!tune_parse(text, NVMAX, RMAX, arch, rt_file, es, err)) return fail(ZB_EINVAL, "%s: %s", path, err.c_str());
    int rt = 0;
    HIP_TRY(hipRuntimeGetVersion(&rt));
    // timings from another GPU or HIP runtime say nothing about this one
    if (arch != ctx->arch || rt_file != rt) return ZB_OK;
    int applied = 0;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const TuneEntry &e : es) {
        // an entry naming a kernel this library does not hold, or one whose LDS does not fit
        // a CU, is skipped
        const KernelInfo *kv = find_kernel(e.nv, e.lanes, e.prec == ZB_MIXED, METHOD_BDF);
        const KernelInfo *ka = e.auto_lu == ZB_LU_MFMA
                                   ? (e.prec == ZB_MIXED && e.nv > 32 ? find_kernel(e.nv, e.auto_lanes, 1, METHOD_BDF_BLU) : nullptr)
                                   : find_kernel(e.nv, e.auto_lanes, e.prec == ZB_MIXED, METHOD_BDF);
        if (!kv || !ka || launch_lds(kv, e.nr) > 160 * 1024 || launch_lds(ka, e.nr) > 160 * 1024) continue;
        bool found = false;
        for (auto &x : ctx->tuned)
            if (x.nv == e.nv && x.nr == e.nr && x.prec == e.prec) {
                x = e;
                found = true;
            }
        if (!found) ctx->tuned.push_back(e);
        ++applied;
    }
    if (loaded) *loaded = applied;
    return ZB_OK;
}

// -------------------------------------------------------------------- errors

extern "C" const char *zb_strerror(zb_err e)
{
    switch (e) {
    case ZB_OK: return "ZB_OK";
    case ZB_EINVAL: return "ZB_EINVAL";
    case ZB_ENOMEM: return "ZB_ENOMEM";
    case ZB_EDEVICE: return "ZB_EDEVICE";
    case ZB_EZONES: return "ZB_EZONES";
    case ZB_EBUSY: return "ZB_EBUSY";
    case ZB_ENOTFOUND: return "ZB_ENOTFOUND";
    case ZB_EUNSUPPORTED: return "ZB_EUNSUPPORTED";
    }
    return "unknown";
}

extern "C" const char *zb_last_error(void) { return g_last_error.c_str(); }
