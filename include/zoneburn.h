/*
 * zoneburn: per-zone stiff reaction-network burn on MI355X (gfx950).
 *
 * What is computed.  The paper ("Software design" section) describes
 * microphysics routines written for a single zone and looped over the zones of
 * a simulation, state kept in GPU memory for the whole run, a compile-time
 * selected reaction network that fixes the composition, a VODE-type stiff
 * integrator, and a step cap after which a failing zone is reported back to the
 * application instead of stopping the run.  zb_burn is that loop: every zone
 * independently integrates y' = f(y) over [0, dt], where y holds the species
 * abundances (and the temperature for a network with self-heating), with a
 * variable-order (1..5) BDF method in Nordsieck form, Newton iteration on a
 * dense LU of M = I - gamma J with the analytic Jacobian, and weighted-RMS
 * error, order and step control.  Zones never communicate.
 *
 * Conventions.  Every function returns a zb_err; nothing else crosses the
 * ABI.  Pointers documented as DEVICE must be device (or managed) memory of the
 * context's GPU; HOST pointers are ordinary host memory.  The caller owns every
 * buffer it passes; the library owns networks, servers and its workspaces.
 * Calls on one context from several host threads are safe except where noted.
 */
#ifndef ZONEBURN_H
#define ZONEBURN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ZB_OK = 0,
    ZB_EINVAL = 1,     /* bad argument; nothing was launched */
    ZB_ENOMEM = 2,     /* device or host allocation failed */
    ZB_EDEVICE = 3,    /* HIP runtime error (launch, copy, synchronize) */
    ZB_EZONES = 4,     /* zb_sync: at least one zone ended with a non-OK status */
    ZB_EBUSY = 5,      /* server: pending queue full; burn: no counter slot left for a captured call */
    ZB_ENOTFOUND = 6,  /* server: unknown ticket */
    ZB_EUNSUPPORTED = 7 /* no kernel for this (network size, mapping, precision) */
} zb_err;

/* Per-zone outcome (the paper: cap the steps and pass failures back). */
typedef enum {
    ZB_ZONE_OK = 0,
    ZB_ZONE_MAXSTEPS = 1,   /* max_steps accepted steps did not reach dt */
    ZB_ZONE_ERRTEST = 2,    /* ten consecutive error-test failures */
    ZB_ZONE_CONV = 3,       /* ten consecutive Newton failures */
    ZB_ZONE_HMIN = 4,       /* step size fell below the resolution of t */
    ZB_ZONE_NONFINITE = 5,  /* non-finite initial state or right-hand side */
    ZB_ZONE_OK_RETRY = 6,   /* failed, then reached dt on the zone-by-zone retry (valid result) */
    ZB_ZONE_OK_FP64 = 7     /* failed in mixed precision, then reached dt in FP64 (the
                               zb_opts.fp64_fallback run; valid result) */
} zb_zone_status;

/* Per-zone counters: accepted steps, RHS evaluations, Jacobians, LU factorizations,
   Newton iterations, error-test failures, Newton (convergence) failures. */
typedef struct { int32_t nst, nfe, nje, nlu, nni, netf, ncf; } zb_zone_stats;

/* Mass-action network with Arrhenius rates (the paper: a network, selected by the
   user, defines the composition).  Reaction r consumes reactant[r][0] and, unless it
   is -1, reactant[r][1]; it produces product[r][0] and, unless -1, product[r][1].
   Rate  k_r = exp(lnA + n ln T - E / T) * scale  when thermal, else exp(lnA) * scale;
   w_r = k_r Y_a Y_b (k_r Y_a for one reactant).  dY_i/dt = sum_r nu_ir w_r and, when
   thermal, dT/dt = sum_r q_r w_r.  Arrays are HOST pointers, copied by zb_network_create. */
typedef struct {
    int32_t n_species;         /* 1 .. 64 (63 when thermal); the burn kernels take
                                  n_species + thermal <= 48 (ZB_EUNSUPPORTED beyond) */
    int32_t thermal;           /* 0: T is passed through unchanged; 1: T is integrated */
    int32_t n_reactions;       /* 0 .. 4096 */
    const int32_t *reactant;   /* [n_reactions][2] */
    const int32_t *product;    /* [n_reactions][2] */
    const double *lnA, *n_exp, *E, *q;   /* [n_reactions] each; q unused unless thermal */
} zb_network_desc;

typedef struct zb_context zb_context;
typedef struct zb_network zb_network;
typedef struct zb_server zb_server;

enum { ZB_FP64 = 0, ZB_MIXED = 1 };               /* zb_opts.precision */
enum { ZB_MAP_AUTO = 0 };                          /* zb_opts.mapping: else lanes per zone 1..64 */
enum { ZB_JAC_EVERY_STEP = 0, ZB_JAC_REUSE = 1 };  /* zb_opts.jac_policy */
enum { ZB_BDF = 0, ZB_RKC = 1, ZB_BDF_VARIABLE = 2 };   /* zb_opts.integrator */
enum { ZB_RETRY_JAC_ANALYTIC = 0, ZB_RETRY_JAC_FD = 1 };   /* zb_opts.retry_jac */
enum { ZB_LU_VALU = 0, ZB_LU_MFMA = 1, ZB_LU_AUTO = 2 };   /* zb_opts.lu */

typedef struct {
    int32_t max_steps;   /* accepted steps per zone before ZB_ZONE_MAXSTEPS (<= 0: 100000) */
    int32_t precision;   /* ZB_FP64: everything in FP64.  ZB_MIXED: the iteration-matrix LU and
                            its triangular solves in FP32 (rows and columns scaled by the error
                            weights); RHS, Jacobian, residual, update, norms and control in FP64 */
    int32_t mapping;     /* ZB_MAP_AUTO or lanes per zone (1, 2, 4, 8, 16, 32, 64) */
    int32_t retry;       /* 1: zone-by-zone retry (the paper, Software design: a failing zone is
                            integrated again with different tolerances instead of stopping the
                            run).  A zone that ends with any failure status is integrated once
                            more from its input with retry_rtol, retry_atol and retry_max_steps;
                            success reports ZB_ZONE_OK_RETRY, a second failure that run's status;
                            its counters add up over both runs.  0: off */
    double retry_rtol, retry_atol;   /* > 0 when retry is on */
    int32_t retry_max_steps;         /* <= 0: the same as max_steps */
    int32_t jac_policy;  /* ZB_JAC_EVERY_STEP (0): Jacobian and LU on every step attempt.
                            ZB_JAC_REUSE (1): the VODE-style reuse (the integrator the paper
                            names, Brown-Byrne-Hindmarsh 1989): the factored iteration matrix is
                            kept across steps and re-formed when gamma = h l_0 moved by more than
                            30 % since it was factored, after 20 steps, or after a Newton failure
                            with a Jacobian from an earlier step (then J is refreshed at the same
                            prediction and Newton retried once); a re-formed matrix takes a fresh
                            J unless the saved one is younger than 50 steps and gamma moved by
                            less than 20 %; a lagged matrix's correction is scaled by
                            2 / (1 + gamma / gamma_M).  The Jacobian stays in the zone's LDS. */
    int32_t integrator;  /* ZB_BDF (0): the VODE-type BDF above.  ZB_RKC (1): the damped
                            second-order Runge-Kutta-Chebyshev method the paper names beside VODE
                            for mildly stiff zones (Sommeijer, Shampine & Verwer 1998; eps = 2/13,
                            stages from the Gershgorin bound of the Jacobian, at most 250; error
                            estimate (12 (y_n - y_{n+1}) + 6 h (F_n + F_{n+1})) / 15).  Same
                            statuses, start, end clamp, abundance constraint and retry; counters
                            nst, nfe, nje (one bound per attempt), netf.  FP64 only (no LU):
                            ZB_EINVAL with ZB_MIXED.  jac_policy does not apply.
                            ZB_BDF_VARIABLE (2): the BDF in VODE's variable-coefficient form:
                            with xi_i = (t_{n+1} - t_{n+1-i}) / h over the accepted steps, the
                            corrector coefficients are those of prod_{i<=q} (1 + x/xi_i) (l_1 =
                            1) and the error estimate divides by xi_{q+1}, so the step is the
                            BDF of the actual uneven grid; identical to ZB_BDF at constant steps
                            (order changes, which follow q+1 equal steps, use the same
                            coefficients).  Both precisions and both jac_policy values. */
    int32_t retry_jac;   /* the Jacobian of the retry run (the paper, Software design: a retry
                            may use another Jacobian approximation).  ZB_RETRY_JAC_ANALYTIC (0):
                            the analytic one, as in the first run.  ZB_RETRY_JAC_FD (1): forward
                            differences, column j = (f(y + d_j e_j) - f(y)) / d_j with
                            d_j = 2^-26 max(|y_j|, atol + rtol |y_j|) taken as (y_j + d_j) - y_j;
                            each one adds nv to the zone's nfe.  BDF only: ZB_EINVAL with ZB_RKC
                            when retry is on. */
    int32_t lu;          /* factorisation of the iteration matrix (the paper, Solvers: a dense LU).
                            ZB_LU_VALU (0): right-looking LU with partial pivoting on the vector
                            units, the default.  ZB_LU_MFMA (1): the same pivoting in 16-column
                            panels, each panel's update of the columns right of it done as one
                            FP32 product on the matrix cores (v_mfma_f32_32x32x2f32,
                            v_mfma_f32_16x16x4f32).  It needs ZB_MIXED, ZB_JAC_EVERY_STEP and a
                            BDF integrator (else ZB_EINVAL).  It applies to networks of 33 to 48
                            variables on 64 lanes per zone; other mappings keep ZB_LU_VALU.  On
                            MI355X the two run within 2 % of each other at these sizes.
                            ZB_LU_AUTO (2): per segment, the factorisation and lanes per zone
                            that zb_autotune timed fastest for its network and precision (with
                            mapping ZB_MAP_AUTO), where the other options allow ZB_LU_MFMA;
                            else ZB_LU_VALU and the mapping rules of ZB_LU_VALU. */
    int32_t fp64_fallback;   /* 1: with ZB_MIXED, a zone that fails (after the retry, if on) is
                            burned again from its input in FP64, by the FP64 kernel of its
                            class after the mixed-precision run, with the same options; success
                            reports ZB_ZONE_OK_FP64, a failure that run's status, and the
                            counters add up over both runs.  At most 1024 zones of each segment
                            of a call fall back (the others keep their failure status).  The
                            lists rotate over 16 slots per context; a call whose slot an
                            earlier call may still be using waits for that call on the host
                            first.  Ignored with ZB_FP64; ZB_EUNSUPPORTED in the server.
                            0: off. */
} zb_opts;

/* Create a context on HIP device `device` (allocates a small device workspace). */
zb_err zb_context_create(int device, zb_context **out);
zb_err zb_context_destroy(zb_context *ctx);

/* Copy a network to the device and precompute its per-row evaluation tables.
   ZB_EINVAL on out-of-range sizes or indices. */
zb_err zb_network_create(zb_context *ctx, const zb_network_desc *desc, zb_network **out);
zb_err zb_network_destroy(zb_network *net);
/* Number of integrated variables (n_species + thermal) and reactions. */
zb_err zb_network_info(const zb_network *net, int32_t *n_var, int32_t *n_reactions);

/* Burn `zones` zones in place over [0, dt] (the operator-split burn of one hydro step).
   state       DEVICE, row-major [zones][n_species + 1]: abundances, then T.  On return every
               zone holds its final state, or its last accepted state if it failed.
   rate_scale  DEVICE [zones][n_reactions] multipliers of k_r, or NULL for 1.
   zone_status DEVICE [zones] zb_zone_status, or NULL.
   stats       DEVICE [zones] counters, or NULL.
   stream      hipStream_t (as void*), NULL for the null stream.  The call is asynchronous:
               argument errors return at once, everything else surfaces in zb_sync.
               The call takes device counters from a ring of the context (1024 slots): when
               its slot may still be used by a call 1024 calls back, it first waits on the
               host for that call's launches.  A call captured into a graph on `stream`
               (stream capture) keeps counters of its own for the context's lifetime;
               64 such calls per context, ZB_EBUSY after that (zb_graph_create has its own).
   ZB_EINVAL: zones < 0, dt not finite or <= 0, rtol <= 0, atol <= 0 (or not finite),
   NULL state with zones > 0, buffers of another device, or invalid opts.
   ZB_EUNSUPPORTED: no kernel for the network size with this mapping and precision
   (n_species + thermal > 48, or a forced mapping whose LDS needs more than a CU has). */
zb_err zb_burn(zb_context *ctx, const zb_network *net, double *state, int64_t zones, double dt,
               double rtol, double atol, const double *rate_scale, const zb_opts *opts,
               int32_t *zone_status, zb_zone_stats *stats, void *stream);

/* Wait for `stream` and report: ZB_OK, ZB_EDEVICE, or ZB_EZONES if any zone of any burn on
   this context since the previous zb_sync ended with a non-OK status (the count is cleared). */
zb_err zb_sync(zb_context *ctx, void *stream, int64_t *n_failed_zones);

/* Several networks in one call (the paper's loop over zones, with the zones of different
   networks and tolerances batched).  Segments that use the same kernel (same padded size,
   lanes per zone and precision; up to 8 per launch) share ONE persistent launch with a device
   work queue per segment, so zones of uneven cost keep every wave busy.  Different kernel
   classes run as concurrent persistent launches on side streams forked from `stream` and
   joined back into it (costliest class first), so one class's tail is filled by the others.
   Each segment is burned exactly (bitwise) as zb_burn would burn it alone with the same opts
   and lanes per zone.  Errors as zb_burn; the call may be captured in a HIP graph. */
typedef struct {
    const zb_network *net;
    double *state;              /* DEVICE [zones][n_species+1] */
    int64_t zones;
    double dt, rtol, atol;
    const double *rate_scale;   /* DEVICE or NULL */
    int32_t *zone_status;       /* DEVICE or NULL */
    zb_zone_stats *stats;       /* DEVICE or NULL */
    const double *source;       /* DEVICE [zones][n_species+1] or NULL: a constant term added to
                                   each zone's right-hand side over the whole burn (the paper's
                                   spectral-deferred-correction coupling, Software design: the
                                   hydro's advective change per unit time enters the burn as a
                                   fixed source).  The T entry is used only with heating. */
} zb_segment;
zb_err zb_burn_batch(zb_context *ctx, const zb_segment *segs, int32_t n_seg, const zb_opts *opts,
                     void *stream);

/* zb_burn_batch for callers that cannot allocate device memory or other runtime resources
   while they burn (code under stream capture, tight serving loops, harnesses that forbid
   allocation): the call allocates nothing, creates no stream or event and never waits on the
   host.  Its zone-queue counters live in a static device array of the library (4 launches x
   8 counters, 256 bytes per GPU, held until the process ends) instead of the context's ring;
   the context (created beforehand) supplies the device and the failed-zone count of zb_sync.
   Every kernel class of the call runs on `stream`, one after another (no side streams).
   Results are bitwise those of zb_burn_batch with the same arguments.
   ZB_EINVAL as zb_burn_batch, and when the segments need more than 4 launches (kernel
   classes, 8 segments per launch).  ZB_EUNSUPPORTED with fp64_fallback in ZB_MIXED (its
   lists are not in the static array).  All such calls on one GPU share the array: calls that
   overlap in time on one GPU (other streams, other threads, other contexts) race; order them. */
zb_err zb_burn_batch_noalloc(zb_context *ctx, const zb_segment *segs, int32_t n_seg,
                             const zb_opts *opts, void *stream);

/* Fixed-shape repeats as a HIP graph: the burn of these segments (buffers, sizes, tolerances
   and options fixed at creation) is captured once and replayed by zb_graph_launch, each
   replay burning whatever the buffers then hold.  The graph owns its work-queue counters
   (cleared by a kernel inside the graph, no memset node); replays of one graph must not
   overlap in time (launch them on one stream, or order them).  Failed zones count towards
   zb_sync of the context.  The buffers must outlive the graph. */
typedef struct zb_graph zb_graph;
zb_err zb_graph_create(zb_context *ctx, const zb_segment *segs, int32_t n_seg, const zb_opts *opts,
                       zb_graph **out);
zb_err zb_graph_launch(zb_graph *graph, void *stream);
zb_err zb_graph_destroy(zb_graph *graph);

/* ------------------------------------------------------------------------------------------
   Serving: continuous batching of burn requests (the paper keeps simulation state resident in
   GPU memory and burns it there; here many independent requests of different networks, sizes
   and tolerances share one GPU).

   zb_server_submit copies the request's HOST input and queues it.  Requests are admitted
   first come, first served as soon as their device state (state, status, counters, scales)
   fits in the server's HBM budget, which is allocated once at creation (no device allocation
   per request).  A scheduler thread cuts admitted requests into slices of zones and keeps
   persistent launches in flight on several streams; a launch holds slices of up to 8
   requests that use the same kernel class, taken shortest remaining work first (estimated
   from zones left and the network's size), and a request arriving while others run joins
   the next launch, its kernels overlapping the launches in flight.  Results stay in device memory
   until zb_server_fetch copies them out and frees the memory.  Every zone is burned exactly
   (bitwise) as zb_burn would burn it with opts = zb_server_opts.burn, so a request's result
   is the same alone and in any mix.  Latencies are measured on the host from submit.
   ------------------------------------------------------------------------------------------ */
typedef struct {
    size_t hbm_budget_bytes;       /* device bytes for resident requests (>= 1 MiB), allocated once */
    int32_t streams;               /* concurrent launch streams, 0 = 4 (1..8) */
    int32_t launches_per_stream;   /* launches queued per stream, 0 = 2 (1..4) */
    int64_t slice_zones;           /* zones per slice, 0 = the GPU's resident zones for the
                                      request's kernel (a launch holds two slices) */
    int32_t max_pending;           /* requests waiting for admission before ZB_EBUSY, 0 = 1024 */
    int32_t reserved;
    zb_opts burn;                  /* precision, mapping and max_steps of every request */
} zb_server_opts;

typedef struct {
    int64_t zones, zones_ok;   /* zones_ok counts ZB_ZONE_OK, ZB_ZONE_OK_RETRY and ZB_ZONE_OK_FP64 */
    double queue_s;          /* submit -> admission (device memory granted) */
    double first_launch_s;   /* submit -> first slice launched */
    double latency_s;        /* submit -> last slice finished on the device */
} zb_request_info;

typedef struct {
    int64_t requests_done, zones_done, launches, pending, active, bytes_in_use, peak_bytes_in_use;
} zb_server_totals;

/* ZB_EINVAL on bad options; ZB_ENOMEM if the budget cannot be allocated. */
zb_err zb_server_create(zb_context *ctx, const zb_server_opts *opts, zb_server **out);
/* host_state: HOST [zones][n_species+1]; host_rate_scale: HOST [zones][n_reactions] or NULL.
   Both are copied before the call returns.  ZB_EINVAL for bad arguments or a request larger
   than the whole budget; ZB_EBUSY when max_pending requests are already waiting. */
zb_err zb_server_submit(zb_server *srv, const zb_network *net, const double *host_state,
                        int64_t zones, double dt, double rtol, double atol,
                        const double *host_rate_scale, uint64_t *ticket);
/* Wait up to timeout_s seconds (0: just test) for a request; *done = 1 when it has finished. */
zb_err zb_server_wait(zb_server *srv, uint64_t ticket, double timeout_s, int32_t *done);
/* Copy a finished request's results to HOST buffers (any may be NULL) and release it.
   ZB_EBUSY if it has not finished, ZB_ENOTFOUND for an unknown or already fetched ticket. */
zb_err zb_server_fetch(zb_server *srv, uint64_t ticket, double *host_state_out,
                       int32_t *zone_status_out, zb_zone_stats *stats_out, zb_request_info *info);
zb_err zb_server_stats(zb_server *srv, zb_server_totals *out);
/* Waits for the launches in flight, then frees everything; unfetched requests are dropped. */
zb_err zb_server_destroy(zb_server *srv);

/* Lanes per zone the library uses for (network, precision) when opts->mapping is AUTO. */
zb_err zb_get_mapping(zb_context *ctx, const zb_network *net, int32_t precision, int32_t *lanes);
/* Time every supported mapping on a DEVICE sample state [zones][ns+1] (copied, not modified)
   and use the fastest qualifying one for (network size, reactions, precision) on this context
   from now on, with the vector LU (ZB_LU_AUTO then resolves to ZB_LU_VALU as well).  A mapping qualifies when every sample zone ends with the status the first
   mapping gave it and at least 99% of the zones agree with that mapping to a gated relative
   1e-6 (the mappings differ only in the order of reductions).  The sample is burned once
   first for its step counts; each mapping is then timed on the sample ordered longest zone
   first and repeated (copies of a zone side by side, at most 16) until it fills the GPU's
   resident zones of that mapping 8 times over, so that the times follow the steady
   throughput rather than the ramp-down at the end.  times_ms (HOST, optional) receives one
   entry per lane count 1,2,4,...,64, per copy of the sample (negative when unsupported).
   Allocates device scratch for up to 32 copies of the sample and host memory for 17;
   synchronous. */
zb_err zb_autotune(zb_context *ctx, const zb_network *net, const double *sample_state,
                   int64_t zones, double dt, double rtol, double atol, int32_t precision,
                   int32_t *best_lanes, float *times_ms);

/* One candidate of zb_autotune_candidates. */
typedef struct {
    int32_t lanes;       /* lanes per zone */
    int32_t lu;          /* ZB_LU_VALU or ZB_LU_MFMA */
    float ms;            /* burn time per copy of the sample (see zb_autotune); < 0: not run */
    int32_t qualified;   /* 1: statuses equal to the first candidate's, >= 99 % of the zones
                            within a gated relative 1e-6 of it */
} zb_tune_candidate;

/* The autotuner over both tuned dimensions: every lanes-per-zone mapping with the vector LU,
   and, where a matrix-core LU kernel exists for the network (ZB_MIXED, 33 to 48 variables,
   64 lanes), that LU too; each is timed on the DEVICE sample state [zones][ns+1] (copied, not
   modified) with the Jacobian every step and the BDF integrator.  The fastest qualifying
   candidate then serves launches with zb_opts.lu = ZB_LU_AUTO and mapping ZB_MAP_AUTO; the
   fastest qualifying vector-LU one serves launches with ZB_LU_VALU and ZB_MAP_AUTO (what
   zb_autotune records).  out (HOST, max_out entries, optional) receives the candidates in the
   order tried, *n_out their number and *best (optional) the index of the chosen one.  Timed
   as in zb_autotune (ms per copy of the sample).  ZB_EUNSUPPORTED when no candidate ran.
   Allocates as zb_autotune does; synchronous. */
zb_err zb_autotune_candidates(zb_context *ctx, const zb_network *net, const double *sample_state,
                              int64_t zones, double dt, double rtol, double atol,
                              int32_t precision, zb_tune_candidate *out, int32_t max_out,
                              int32_t *n_out, int32_t *best);

/* The context's autotuned choices (zb_autotune, zb_autotune_candidates) as a JSON file at
   `path` (HOST string): one entry per (network size, reactions, precision) with the lanes per
   zone of the vector LU and the (lanes, LU) pair of ZB_LU_AUTO, keyed by the device's
   architecture name and the HIP runtime version.  The file is written beside `path` and
   renamed over it.  ZB_EINVAL when it cannot be written. */
zb_err zb_tune_save(zb_context *ctx, const char *path);
/* Adds the choices of a file written by zb_tune_save to this context's table (replacing
   entries of the same key); *loaded (optional) receives the number applied.  A file from
   another architecture or HIP runtime version applies nothing (*loaded = 0, ZB_OK), and
   entries naming a kernel this library does not hold are skipped.  ZB_EINVAL for a missing,
   unreadable, malformed or over-1-MiB file, or values out of range (the table is then left
   as it was). */
zb_err zb_tune_load(zb_context *ctx, const char *path, int32_t *loaded);

/* Human-readable name of an error code and the last error message of this thread. */
const char *zb_strerror(zb_err err);
const char *zb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ZONEBURN_H */
