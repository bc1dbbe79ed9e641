// Host-side internals shared by the runtime files of libzoneburn (not part of the ABI).
#pragma once

#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>
#include <vector>

#include "zb_internal.h"
#include "zb_slots.h"
#include "zb_tunecache.h"
#include "zoneburn.h"

namespace zbh {

zb_err fail(zb_err e, const char *fmt, ...);

#define HIP_TRY(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::zbh::fail(ZB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Zone-queue counter slots of a context (MAXSEG counters each): a ring for eager calls, and
// slots that a call captured into a graph keeps for good (SlotRing).
constexpr int QUEUE_SLOTS = 1024;
constexpr int QUEUE_CAPTURE_SLOTS = 64;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

constexpr int MAX_SIDE_STREAMS = 3;

// Device counters a call works with: per launch, MAXSEG zone-queue counters
// (cleared by the launch itself), and one failed-zone counter.
struct Workspace {
    unsigned long long *queue;   // launches x MAXSEG
    int launches;
    unsigned long long *nfail;
    unsigned long long *fb;      // launches x FB_STRIDE FP64 fallback lists (nullptr: none)
    bool serial = false;         // every launch on the caller's stream, one after another
};

// Kernel classes (launches) one call of the allocation-free entry point may make: the
// zone-queue counters of that many launches sit in the library's static device array.
constexpr int STATIC_LAUNCHES = 4;

// FP64 fallback lists of a context: calls with the fallback take them in turn, and a call
// whose list is still in use by an earlier one first waits for it; captured calls take
// lists of their own.
constexpr int FB_SLOTS = 16;
constexpr int FB_CAPTURE_SLOTS = 4;

const zb::KernelInfo *find_kernel(int nv, int lanes, int mixed, int jac);
const zb::KernelInfo *kernel_for(int nv, int lanes, int mixed, int method);

// Kernel method (METHOD_*) of validated options whose lu is resolved (not ZB_LU_AUTO).
inline int method_of(const zb_opts *o)
{
    if (!o) return zb::METHOD_BDF;
    if (o->integrator == ZB_RKC) return zb::METHOD_RKC;
    const bool vc = o->integrator == ZB_BDF_VARIABLE;
    if (o->lu == ZB_LU_MFMA) return vc ? zb::METHOD_BDF_VC_BLU : zb::METHOD_BDF_BLU;
    return o->jac_policy + (vc ? zb::METHOD_BDF_VC : zb::METHOD_BDF);
}
// zb_opts.lu against the rest of the options (precision prec).
zb_err check_lu(const zb_opts *o, int prec);
int lanes_for(zb_context *ctx, const zb_network *net, int prec, const zb_opts *o);
// zb_opts.lu for one network: ZB_LU_AUTO resolved from the context's tuning.
int lu_for(zb_context *ctx, const zb_network *net, int prec, const zb_opts *o);
// The options of one segment: lu resolved (lu_for).
zb_opts resolved_opts(zb_context *ctx, const zb_network *net, int prec, const zb_opts *o);
zb_err check_segment(zb_context *ctx, const zb_segment &s);
// Validates the segments and launches them (one persistent launch per kernel
// class) on `stream`.  ws = nullptr takes a rotating slot of the context.
zb_err burn_impl(zb_context *ctx, const zb_segment *segs, int n, const zb_opts *opts, void *stream,
                 int force_lanes = 0, float *ms_out = nullptr, const Workspace *ws = nullptr);
// Number of persistent launches (kernel classes) a call with these segments makes.
int count_launches(zb_context *ctx, const zb_segment *segs, int n, const zb_opts *opts, int *launches);
// Resident workgroups of kernel k per CU with the LDS a launch over networks of
// up to max_nr reactions needs (0 if it does not fit).
int blocks_per_cu(const zb::KernelInfo *k, int max_nr);

}  // namespace zbh

struct zb_context {
    int device = 0;
    int cus = 0;
    // [0] failed zones, then (QUEUE_SLOTS + QUEUE_CAPTURE_SLOTS) x MAXSEG queue counters
    unsigned long long *ws = nullptr;
    // (FB_SLOTS + FB_CAPTURE_SLOTS) x FB_STRIDE FP64 fallback lists
    unsigned long long *fb = nullptr;
    // slot rotation: each eager slot's event is recorded after the last launch that uses it
    std::mutex slot_mu;
    zbh::SlotRing qring, fbring;
    std::vector<hipEvent_t> qev, fbev;
    // this device's copy of the static scratch array (zb_burn_batch_noalloc)
    unsigned long long *static_scratch = nullptr;
    std::mutex mu;
    // autotuned choices keyed by (nv, nr, precision): lanes per zone with the vector LU, and
    // the fastest (lanes, LU) pair overall, for ZB_LU_AUTO
    using Tuned = zbh::TuneEntry;
    std::vector<Tuned> tuned;
    std::string arch;   // gcnArchName of the device, the key of saved tunings
    // side streams for calls that launch several kernel classes (default priority)
    std::mutex fork_mu;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
};

struct zb_network {
    zb_context *ctx = nullptr;
    zb::DevNet dn{};
    void *dmem = nullptr;
};
