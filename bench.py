"""Benchmark: zone-burns/s of the per-zone stiff BDF burn on one MI355X.

Workload (the 14-variable network the headline metric names): 13 species + T,
30 random two-body reactions with Arrhenius rates, 2^20 zones with
T ~ U(1e3, 5e3) and Dirichlet(1) abundances, dt = 1, rtol = 1e-8, atol = 1e-12.
A step is one complete burn of all 2^20 zones (device-resident state, reset to
the initial state before every step).  The mixed-precision burn (FP32 LU, FP64
everything else) is the reported value; the plain FP64 burn of the same input
is reported next to it.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload ...]

Prints one JSON line.  The default run (the headline) also carries, each from a
fixed small number of launches so that the whole run stays within a few minutes:
plain_fp64, jac_reuse and vode_form (other methods on the same input), roofline
(FP64 ALU bound of the burn kernel), cpu_baseline (the CPU oracle on a bounded
sample of the same zones, with all host threads and with one), accuracy_vs_oracle
(that sample, every GPU leg), batched (the four-network batch, FP64 / mixed /
blocked matrix-core LU, each against the oracle) and serving (a Poisson request
stream through the continuous-batching server: p50/p99 latency, per network).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
BAR = 1e-6                  # gated relative error bar at rtol = 1e-8
QNOM = 5                    # nominal order of the per-step flop count
EXTRA_STEPS, EXTRA_WARMUP = 2, 1     # timed / untimed launches of the secondary legs


def lu_flops(nv):
    return 2.0 * nv ** 3 / 3.0 - nv * nv / 2.0 - nv / 6.0


def burn_flops(nv, nr, stats, q=QNOM):
    """Algorithmic FP64 flops of the burns from the per-zone counters (summed over zones).

    Per step attempt: prediction q(q+1)/2 nv, correction and the weight, error and
    order-selection norms 2(q+1) nv + 12 nv; per Jacobian: 25 R + nv^2 (the entries and
    M = I - gamma J); per factorisation: 2 nv^3/3 - nv^2/2 - nv/6; per Newton iteration:
    12 R (the RHS) + 2 nv^2 - nv (forward and back substitution) + 7 nv (residual, update,
    norm).  q is taken at its nominal 5.  exp/log are counted apart (transcendentals())."""
    st = stats.astype(np.float64)
    nst, nje, nlu, nni, netf, ncf = (st[:, k].sum() for k in (0, 2, 3, 4, 5, 6))
    att = nst + netf + ncf
    per_att = q * (q + 1) / 2.0 * nv + 2.0 * (q + 1) * nv + 12.0 * nv
    return (att * per_att + nje * (25.0 * nr + nv * nv) + nlu * lu_flops(nv)
            + nni * (12.0 * nr + 2.0 * nv * nv - nv + 7.0 * nv))


def transcendentals(nr, thermal, stats):
    """exp per reaction and one log per RHS evaluation of a thermal network."""
    return stats[:, 1].astype(np.float64).sum() * ((nr + 1) if thermal else 0)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "burn_kernel_14x16_nv14_2p20zones_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2608_06466_amd", "csrc", f)
                  for f in ("zb_burn_kernel.h", "zb_internal.h", "zb_log.h", "zb_stepmath.h",
                            "zb_k14.hip")] + [
                  os.path.join(ROOT, "paper_2608_06466_amd", "build.py")]   # the compile flags


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(precision, zones):
    """HBM bytes per burn launch from the committed FETCH_SIZE/WRITE_SIZE profile.

    None unless the profile was taken on the current kernel sources and on the
    same zone count (the counters do not run inside this process)."""
    import re
    if zones != 1 << 20 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    txt = open(TRAFFIC_PROFILE).read()
    m = re.search(r"kernel_sources_sha256: ([0-9a-f]{64})", txt)
    t = re.search(rf"traffic_bytes_per_launch:.*\b{precision}=([0-9.e+]+)", txt)
    if not m or not t:
        return None
    return float(t.group(1)) if kernel_sources_sha256() == m.group(1) else None


def host_info():
    """CPU model, sockets and threads of the host the oracle runs on."""
    model, sockets = None, set()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model is None:
                model = line.split(":", 1)[1].strip()
            elif line.startswith("physical id"):
                sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "sockets": len(sockets) or None, "logical_cpus": os.cpu_count(),
            "cpus_available": avail, "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def oracle_threads():
    info = host_info()
    t = int(os.environ.get("OMP_NUM_THREADS", info["cpus_available"]))
    return max(1, min(t, info["cpus_available"]))


def accuracy(out, status, stats, ref, nv, rtol, atol, fine_fn=None, thermal=True):
    """GPU result against the oracle's on the same zones.

    gated: |d| / max(|y_ref|, atol/rtol); strict: |d| / max(|y_ref|, atol); T_raw: the
    relative error of T alone; lockstep: the share of zones whose seven counters equal the
    oracle's (the same step path).  Zones above the 1e-6 gated bar are listed with whether
    they kept the oracle's path and, from fine_fn (the oracle at rtol/100 on those zones),
    the oracle's own error there."""
    ref_state, ref_status, ref_stats = ref
    ok = (ref_status == 0) & (status == 0)
    d = np.abs(out[ok][:, :nv] - ref_state[ok][:, :nv])
    r = np.abs(ref_state[ok][:, :nv])
    gz = (d / np.maximum(r, atol / rtol)).max(1)
    sz = (d / np.maximum(r, atol)).max(1)
    lock = np.all(stats[ok] == ref_stats[ok], axis=1)
    res = {"sampled_zones": int(len(status)), "status_mismatches": int((status != ref_status).sum()),
           "max_gated_rel_err": float(gz.max()), "median_gated_rel_err": float(np.median(gz)),
           "max_strict_rel_err": float(sz.max()),
           "zones_over_1e-6": int((gz > BAR).sum()),
           "within_1e-6_fraction": float((gz <= BAR).sum() / max(1, len(status))),
           "lockstep_rate": float(lock.mean()),
           "max_gated_rel_err_lockstep": float(gz[lock].max()) if lock.any() else 0.0}
    if thermal:
        t = np.abs(out[ok][:, nv - 1] - ref_state[ok][:, nv - 1]) / np.abs(ref_state[ok][:, nv - 1])
        res["max_T_rel_err"] = float(t.max())
    over = np.nonzero(gz > BAR)[0]
    if over.size:
        zi = np.nonzero(ok)[0][over]
        e_orc = None
        if fine_fn is not None:
            fine = fine_fn(zi)
            e_orc = (np.abs(ref_state[zi][:, :nv] - fine[0][:, :nv])
                     / np.maximum(np.abs(fine[0][:, :nv]), atol / rtol)).max(1)
        res["over_bar"] = [{"err": float(gz[o]), "lockstep": bool(lock[o]),
                            "oracle_own_err": None if e_orc is None else float(e_orc[j])}
                           for j, o in enumerate(over[:16])]
    return res


def timed_launches(label, launch, reset, steps, warmup):
    """Runs reset(); launch() warmup + steps times; returns [(wall_s, kernel_ms)] of the timed
    launches and the failed-zone counts.  The HIP events bracket the launch on the stream it
    runs on (torch's current stream)."""
    import torch
    stream = torch.cuda.current_stream()
    out, fails = [], []
    for it in range(warmup + steps):
        reset()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        nf = launch()
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nf = nf() if callable(nf) else nf
        fails.append(nf)
        tag = f"step {it - warmup}" if it >= warmup else "warmup"
        print(f"[bench] {label} {tag}: {(t1 - t0) * 1e3:.1f} ms (kernel {e0.elapsed_time(e1):.1f} ms), "
              f"failed zones {nf}", file=sys.stderr, flush=True)
        if it >= warmup:
            out.append((t1 - t0, e0.elapsed_time(e1)))
    return out, fails


def headline(args):
    import torch
    from paper_2608_06466_amd import workloads as W
    from paper_2608_06466_amd import zoneburn as zb

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    cfg = W.nv14(args.zones or (1 << 20))
    net_d, state0_np = cfg["net"], cfg["state"]
    dt, rtol, atol = cfg["dt"], cfg["rtol"], cfg["atol"]
    zones = state0_np.shape[0]
    nv, nr = net_d["n_species"] + 1, len(net_d["lnA"])

    ctx = zb.Context(0)
    net = zb.Network(ctx, net_d)
    state0 = torch.tensor(state0_np, device=dev)
    work = torch.empty_like(state0)

    def run(label, precision, steps, warmup, jac_policy=0, integrator="bdf"):
        lanes = zb.get_mapping(ctx, net, precision)
        holder = {}

        def launch():
            holder["r"] = zb.burn(ctx, net, work, dt, rtol, atol, precision=precision,
                                  jac_policy=jac_policy, integrator=integrator)
            return lambda: zb.sync(ctx)

        times, _ = timed_launches(label, launch, lambda: work.copy_(state0), steps, warmup)
        status, stats = holder["r"]
        st, sts = stats.cpu().numpy(), status.cpu().numpy()
        wall = float(np.mean([t[0] for t in times]))
        kms = float(np.mean([t[1] for t in times]))
        return dict(lanes=lanes, wall_s=wall, kernel_ms=kms, stats=st, status=sts,
                    out=work.cpu().numpy(), steps=steps, warmup=warmup)

    res = {"mixed": run("mixed", "mixed", args.steps, args.warmup)}
    # the comparison legs: a fixed small number of launches each
    fsteps = min(args.steps, 5)
    res["fp64"] = run("fp64", "fp64", fsteps, min(args.warmup, 1))
    # VODE-style Jacobian/LU reuse, and VODE's own configuration (variable-coefficient form
    # with that reuse)
    res["reuse"] = run("mixed reuse", "mixed", EXTRA_STEPS, EXTRA_WARMUP, jac_policy=1)
    res["vode"] = run("mixed vode", "mixed", EXTRA_STEPS, EXTRA_WARMUP, jac_policy=1,
                      integrator="bdf_variable")

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 1 GiB read + 1 GiB written", file=sys.stderr, flush=True)
    net.close()
    ctx.close()
    del state0, work
    torch.cuda.empty_cache()

    def flops(r):
        return burn_flops(nv, nr, r["stats"])

    def roofline(r, precision):
        achieved = flops(r) / (r["kernel_ms"] * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(precision, zones),
                "flops_per_zone": round(flops(r) / zones, 1)}

    # ---- CPU oracle on a bounded sample (all host threads, then one) + accuracy ----
    cpu, acc = None, None
    within = {k: 1.0 for k in res}
    if not args.no_cpu:
        import oracle
        threads = oracle_threads()
        rng = np.random.default_rng(12345)
        pilot = np.sort(rng.choice(zones, 256, replace=False))
        t0 = time.perf_counter()
        oracle.burn(net_d, state0_np[pilot], dt, rtol, atol, nthreads=threads)
        pt = time.perf_counter() - t0
        n = int(min(zones, max(512, 256 * args.cpu_seconds / max(pt, 1e-3))))
        idx = np.sort(rng.choice(zones, n, replace=False))
        t0 = time.perf_counter()
        ref = oracle.burn(net_d, state0_np[idx], dt, rtol, atol, nthreads=threads)
        ct = time.perf_counter() - t0
        n1 = max(16, int(n * (args.cpu_seconds / 2.0) / (ct * threads)))
        idx1 = idx[:n1]
        t0 = time.perf_counter()
        oracle.burn(net_d, state0_np[idx1], dt, rtol, atol, nthreads=1)
        ct1 = time.perf_counter() - t0
        cpu = {"value": round(n / ct, 3), "unit": "zone-burns/s", "cores": threads, "kind": "oracle",
               "sample": f"{n} zones drawn uniformly (seed 12345) from the same {zones}-zone input, "
                         f"plain C FP64 oracle, OpenMP over zones, {ct:.1f} s wall",
               "one_thread": {"value": round(n1 / ct1, 3), "zones": n1, "wall_s": round(ct1, 2)},
               "host": host_info()}
        refs = {"mixed": ref, "fp64": ref,
                "reuse": oracle.burn(net_d, state0_np[idx], dt, rtol, atol, nthreads=threads,
                                     jac_policy=1),
                "vode": oracle.burn(net_d, state0_np[idx], dt, rtol, atol, nthreads=threads,
                                    jac_policy=1, form="variable")}
        okw = {"mixed": {}, "fp64": {}, "reuse": dict(jac_policy=1),
               "vode": dict(jac_policy=1, form="variable")}
        acc = {}
        for k in ("mixed", "fp64", "reuse", "vode"):
            fine_fn = (lambda zi, k=k: oracle.burn(net_d, state0_np[idx][zi], dt, rtol / 100,
                                                   atol / 100, max_steps=10000000,
                                                   nthreads=threads, **okw[k]))
            acc[k] = accuracy(res[k]["out"][idx], res[k]["status"][idx], res[k]["stats"][idx],
                              refs[k], nv, rtol, atol, fine_fn)
            within[k] = acc[k]["within_1e-6_fraction"]

    def summary(r, key):
        ok = int((r["status"] == 0).sum())
        return dict(value=ok * within[key] / r["wall_s"], ok_zones=ok,
                    ms_per_step=r["wall_s"] * 1e3, kernel_ms=r["kernel_ms"],
                    lanes_per_zone=r["lanes"], mean_steps=float(r["stats"][:, 0].mean()),
                    max_steps=int(r["stats"][:, 0].max()))

    sm, sf, sr, sv = (summary(res[k], k) for k in ("mixed", "fp64", "reuse", "vode"))
    line = {
        "metric": "zone-burns/sec at rel err \u22641e-6 (14-var net), mixed vs plain FP64; serving p99",
        "value": round(sm["value"], 1),
        "unit": "zone-burns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sm["ms_per_step"], 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (f32 LU)",
        "data": "synthetic",
        "config": {"workload": "14-var network: 13 species + T, 30 two-body Arrhenius reactions, "
                               f"{zones} zones, T~U(1e3,5e3), Dirichlet(1), dt=1, rtol=1e-8, atol=1e-12",
                   "zones": zones, "nv": nv, "reactions": nr, "precision": "mixed",
                   "lanes_per_zone": sm["lanes_per_zone"], "parallelism": "1 GPU"},
        "value_note": "zones with status OK per second, times the share of the oracle-sampled "
                      "zones within the 1e-6 gated bar",
        "ok_zones": sm["ok_zones"],
        "plain_fp64": {"value": round(sf["value"], 1), "ms_per_step": round(sf["ms_per_step"], 2),
                       "kernel_ms": round(sf["kernel_ms"], 2), "roofline": roofline(res["fp64"], "fp64"),
                       "lanes_per_zone": sf["lanes_per_zone"], "steps": res["fp64"]["steps"],
                       "warmup": res["fp64"]["warmup"]},
        "mixed_over_fp64": round(sm["value"] / sf["value"], 3),
        "jac_reuse": {"value": round(sr["value"], 1), "ms_per_step": round(sr["ms_per_step"], 2),
                      "kernel_ms": round(sr["kernel_ms"], 2), "precision": "mixed",
                      "failed_zones": int((res["reuse"]["status"] != 0).sum()),
                      "jacobians_per_zone": round(float(res["reuse"]["stats"][:, 2].mean()), 1),
                      "lus_per_zone": round(float(res["reuse"]["stats"][:, 3].mean()), 1),
                      "steps": EXTRA_STEPS, "warmup": EXTRA_WARMUP,
                      "note": "VODE-style reuse of the Jacobian and LU (jac_policy 1); accuracy "
                              "against the oracle's reuse policy"},
        "vode_form": {"value": round(sv["value"], 1), "ms_per_step": round(sv["ms_per_step"], 2),
                      "kernel_ms": round(sv["kernel_ms"], 2), "precision": "mixed",
                      "failed_zones": int((res["vode"]["status"] != 0).sum()),
                      "mean_steps": round(sv["mean_steps"], 1),
                      "jacobians_per_zone": round(float(res["vode"]["stats"][:, 2].mean()), 1),
                      "steps": EXTRA_STEPS, "warmup": EXTRA_WARMUP,
                      "note": "variable-coefficient BDF form with the Jacobian/LU reuse (integrator "
                              "bdf_variable, jac_policy 1); accuracy against the oracle's same "
                              "configuration"},
        "roofline": roofline(res["mixed"], "mixed"),
        "kernel_ms": round(sm["kernel_ms"], 2),
        "zone_steps": {"mean": round(sm["mean_steps"], 1), "max": sm["max_steps"]},
        "transcendentals_per_s": round(transcendentals(nr, 1, res["mixed"]["stats"])
                                       / (sm["kernel_ms"] * 1e-3), 1),
        "kernel_sources_sha256": kernel_sources_sha256()[:16],
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": acc,
    }
    del res
    if not args.no_extra:
        line["batched"] = batched(args, sub=True)
        line["serving"] = serving(args, sub=True)
    print(json.dumps(line), flush=True)


# ------------------------------------------------------------------ other workloads

def _common_line(metric, value, unit, args, ms, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def robertson(args):
    """Robertson's problem, 4096 zones, t in [0, 1e5] (latency-bound: 64 waves at 1 lane/zone)."""
    import torch
    import oracle
    from paper_2608_06466_amd import workloads as W
    from paper_2608_06466_amd import zoneburn as zb
    cfg = W.robertson(args.zones or 4096)
    zones = cfg["state"].shape[0]
    ctx = zb.Context(0)
    net = zb.Network(ctx, cfg["net"])
    s0 = torch.tensor(cfg["state"], device="cuda:0")
    sc = torch.tensor(cfg["scale"], device="cuda:0")
    best, tt = zb.autotune(ctx, net, s0, cfg["dt"], cfg["rtol"], cfg["atol"], "fp64")
    w = torch.empty_like(s0)
    holder = {}

    def launch():
        holder["r"] = zb.burn(ctx, net, w, cfg["dt"], cfg["rtol"], cfg["atol"], rate_scale=sc)
        return lambda: zb.sync(ctx)

    times, _ = timed_launches("robertson", launch, lambda: w.copy_(s0), args.steps, args.warmup)
    status, stats = (x.cpu().numpy() for x in holder["r"])
    ok = int((status == 0).sum())
    wall = float(np.mean([t[0] for t in times]))
    kms = float(np.mean([t[1] for t in times]))
    line = _common_line("zone-burns/s, Robertson (3 species, t = 0..1e5)", round(ok / wall, 1),
                        "zone-burns/s", args, round(wall * 1e3, 3), "f64",
                        {"workload": f"Robertson, {zones} zones, lognormal(0,0.1) rate scales, t=0..1e5, "
                                     "rtol=1e-8, atol=1e-12", "lanes_per_zone": best,
                         "autotune_ms_per_lane_count_1_to_64": [round(t, 3) for t in tt]})
    line["kernel_ms"] = round(kms, 3)
    line["zone_steps"] = {"mean": round(float(stats[:, 0].mean()), 1), "max": int(stats[:, 0].max())}
    fl = burn_flops(3, 3, stats)
    line["roofline"] = {"bound": "alu", "achieved": round(fl / (kms * 1e-3) / 1e12, 4),
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(fl / (kms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 5), "traffic": None}
    if not args.no_cpu:
        threads = oracle_threads()
        t0 = time.perf_counter()
        ref = oracle.burn(cfg["net"], cfg["state"], cfg["dt"], cfg["rtol"], cfg["atol"],
                          cfg["scale"], nthreads=threads)
        ct = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(zones / ct, 1), "unit": "zone-burns/s", "cores": threads,
                                "kind": "oracle", "sample": f"all {zones} zones", "host": host_info()}
        line["accuracy_vs_oracle"] = accuracy(w.cpu().numpy(), status, stats, ref, 3, cfg["rtol"],
                                              cfg["atol"], thermal=False)
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()


def batched(args, sub=False):
    """Four networks (nv 3, 14, 22, 48; 4:2:1:1 of 2^21 zones) in one zb_burn_batch call, FP64
    and with the FP32 LU, each against the oracle on a stratified sample.  The FP32 headline
    takes the autotuned (lanes, LU) pair of each network (lu='auto'); it runs again with the
    vector LU everywhere (lu='valu') and with the blocked matrix-core LU (lu='mfma': the
    48-variable class).  sub: one timed launch per leg, returned as a dict (the headline run's
    'batched' object)."""
    import torch
    import oracle
    from paper_2608_06466_amd import workloads as W
    from paper_2608_06466_amd import zoneburn as zb
    steps, warmup = (1, 0) if sub else (args.steps, args.warmup)
    segs_h = W.batched((args.batched_zones if sub else args.zones) or (1 << 21))
    ctx = zb.Context(0)
    nets = [zb.Network(ctx, s["net"]) for s in segs_h]
    total = sum(s["state"].shape[0] for s in segs_h)
    init = [torch.tensor(s["state"], device="cuda:0") for s in segs_h]
    work = [torch.empty_like(t) for t in init]
    scales = [None if s["scale"] is None else torch.tensor(s["scale"], device="cuda:0") for s in segs_h]
    status = [torch.empty(t.shape[0], dtype=torch.int32, device="cuda:0") for t in init]
    stats = [torch.empty((t.shape[0], 7), dtype=torch.int32, device="cuda:0") for t in init]
    segs = [dict(net=nets[k], state=work[k], dt=s["dt"], rtol=s["rtol"], atol=s["atol"],
                 rate_scale=scales[k], status=status[k], stats=stats[k]) for k, s in enumerate(segs_h)]

    def reset():
        for w, i0 in zip(work, init):
            w.copy_(i0)

    # autotuned zone-to-wavefront mapping: each network's lanes per zone (and, with the FP32
    # LU, the factorisation: vector or matrix-core), per precision, timed on 8192 zones drawn
    # from its own segment (zb_autotune, zb_autotune_candidates; the chosen pair then serves
    # every launch of that network in this context)
    tuned = {}
    rng_t = np.random.default_rng(99)
    for prec in ("fp64", "mixed"):
        for k, s in enumerate(segs_h):
            nz = s["state"].shape[0]
            pick = np.sort(rng_t.choice(nz, min(nz, 8192), replace=False))
            sample = torch.tensor(s["state"][pick], device="cuda:0")
            if prec == "fp64":
                best, tt = zb.autotune(ctx, nets[k], sample, s["dt"], s["rtol"], s["atol"], prec)
                t = {"lanes": best, "ms_per_lane_count_1_to_64": [round(v, 2) for v in tt]}
            else:
                cands, bi = zb.autotune_candidates(ctx, nets[k], sample, s["dt"], s["rtol"],
                                                   s["atol"], prec)
                t = {"lanes": cands[bi]["lanes"], "lu": cands[bi]["lu"],
                     "candidates_ms": {f"{c['lanes']}/{c['lu']}": round(c["ms"], 2)
                                       for c in cands if c["ms"] > 0}}
            tuned.setdefault(f"nv{nets[k].nv}", {})[prec] = t
            print(f"[bench] batched autotune nv{nets[k].nv} {prec}: lanes {t['lanes']}"
                  f"{' lu ' + t['lu'] if 'lu' in t else ''}", file=sys.stderr, flush=True)
            del sample

    res = {}
    for key, prec, lu in (("fp64", "fp64", "valu"), ("mixed", "mixed", "auto"),
                          ("mixed_valu", "mixed", "valu"), ("mixed_mfma", "mixed", "mfma")):
        def launch(prec=prec, lu=lu):
            zb.burn_batch(ctx, segs, precision=prec, lu=lu)
            return lambda: zb.sync(ctx)

        ts, _ = timed_launches(f"batched {key}", launch, reset, steps, warmup)
        r = {"wall_s": float(np.mean([t[0] for t in ts])), "kernel_ms": float(np.mean([t[1] for t in ts])),
             "out": [w.cpu().numpy() for w in work], "status": [s.cpu().numpy() for s in status],
             "stats": [s.cpu().numpy() for s in stats]}
        r["ok"] = int(sum((s == 0).sum() for s in r["status"]))
        r["flops"] = float(sum(burn_flops(n.nv, n.nr, st) for n, st in zip(nets, r["stats"])))
        res[key] = r
    per_class = []
    for k, s in enumerate(segs_h):
        st = res["fp64"]["stats"][k][:, 0]
        per_class.append({"nv": nets[k].nv, "reactions": nets[k].nr, "zones": int(st.shape[0]),
                          "steps_p1": float(np.percentile(st, 1)), "steps_median": float(np.median(st)),
                          "steps_max": int(st.max())})
    nv_r = [(n.nv, n.nr, n.thermal) for n in nets]
    for n in nets:
        n.close()
    ctx.close()
    del init, work, scales, status, stats, segs
    torch.cuda.empty_cache()

    def roof(r):
        a = r["flops"] / (r["kernel_ms"] * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(a, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(a / FP64_PEAK_TFLOPS, 4), "traffic": None}

    acc = None
    within = {k: 1.0 for k in res}
    if not args.no_cpu:
        threads = oracle_threads()
        rng = np.random.default_rng(4321)
        acc = {"fp64": [], "mixed": [], "mixed_valu": [], "mixed_mfma": []}
        cpu_time_per_zone = []
        for k, s in enumerate(segs_h):
            nz = s["state"].shape[0]
            n = min(nz, [256, 256, 128, 48][k])
            idx = np.sort(rng.choice(nz, n, replace=False))
            sc = None if s["scale"] is None else s["scale"][idx]
            t0 = time.perf_counter()
            ref = oracle.burn(s["net"], s["state"][idx], s["dt"], s["rtol"], s["atol"], sc,
                              nthreads=threads)
            cpu_time_per_zone.append((time.perf_counter() - t0) / n)
            fine_fn = (lambda zi, s=s, idx=idx, sc=sc: oracle.burn(
                s["net"], s["state"][idx][zi], s["dt"], s["rtol"] / 100, s["atol"] / 100,
                None if sc is None else sc[zi], max_steps=10000000, nthreads=threads))
            for prec in acc:
                a = accuracy(res[prec]["out"][k][idx], res[prec]["status"][k][idx],
                             res[prec]["stats"][k][idx], ref, nv_r[k][0], s["rtol"], s["atol"],
                             fine_fn, thermal=bool(nv_r[k][2]))
                a["nv"] = nv_r[k][0]
                acc[prec].append(a)
        # share within the bar: zone-weighted over the classes' samples
        for prec in acc:
            within[prec] = float(sum(a["within_1e-6_fraction"] * s["state"].shape[0]
                                     for a, s in zip(acc[prec], segs_h)) / total)
        est = total / sum(t * s["state"].shape[0] for t, s in zip(cpu_time_per_zone, segs_h))
        cpu = {"value": round(est, 1), "unit": "zone-burns/s", "cores": threads, "kind": "oracle",
               "sample": "256/256/128/48 zones of the nv 3/14/22/48 segments; whole-batch "
                         "rate extrapolated from the per-class time per zone"}
    else:
        cpu = None
    m, f, b, v = res["mixed"], res["fp64"], res["mixed_mfma"], res["mixed_valu"]
    val = {k: r["ok"] * within[k] / r["wall_s"] for k, r in res.items()}
    out = {"value": round(val["mixed"], 1), "unit": "zone-burns/s",
           "ms_per_step": round(m["wall_s"] * 1e3, 2), "kernel_ms": round(m["kernel_ms"], 2),
           "steps": steps, "warmup": warmup,
           "workload": f"Robertson : nv14 : nv22 : nv48 = 4:2:1:1 of {total} zones, T log-uniform on "
                       "[90, 2500] K, dt 1 (Robertson 1e5), rtol 1e-8, atol 1e-12, one zb_burn_batch "
                       "call (mixed precision), zone-to-wavefront mapping and LU autotuned per "
                       "network",
           "per_class": per_class, "autotuned_mapping": tuned, "roofline": roof(m),
           "plain_fp64": {"value": round(val["fp64"], 1), "ms_per_step": round(f["wall_s"] * 1e3, 2),
                          "roofline": roof(f)},
           "mixed_over_fp64": round(val["mixed"] / val["fp64"], 3),
           "valu_lu": {"value": round(val["mixed_valu"], 1), "ms_per_step": round(v["wall_s"] * 1e3, 2),
                       "note": "mixed precision with lu='valu': every class factors on the "
                               "vector units"},
           "mfma_lu": {"value": round(val["mixed_mfma"], 1), "ms_per_step": round(b["wall_s"] * 1e3, 2),
                       "over_valu_lu": round(val["mixed_mfma"] / val["mixed_valu"], 3),
                       "note": "mixed precision with lu='mfma': the 48-variable class factors with "
                               "the blocked LU (trailing updates as FP32 MFMA products), the others "
                               "keep the vector-unit LU"},
           "cpu_baseline": cpu, "accuracy_vs_oracle": acc}
    if sub:
        return out
    line = _common_line("zone-burns/s, four networks (nv 3, 14, 22, 48) in one call", out["value"],
                        "zone-burns/s", args, out["ms_per_step"], "f64 (f32 LU)",
                        {"workload": out["workload"], "per_class": per_class})
    for k in ("kernel_ms", "autotuned_mapping", "roofline", "plain_fp64", "mixed_over_fp64", "valu_lu", "mfma_lu",
              "cpu_baseline",
              "accuracy_vs_oracle"):
        line[k] = out[k]
    print(json.dumps(line), flush=True)


def _pct(x, p):
    return round(float(np.percentile(x, p)), 4) if len(x) else None


def serving(args, sub=False):
    """Poisson stream of burn requests (1k..256k zones, the four networks of the batched
    workload, rtol 1e-6 or 1e-8) through the continuous-batching server: throughput and
    request latency (arrival to result on the host), split per network into queueing
    (arrival to first launch) and service (first launch to result)."""
    import threading
    import torch
    from paper_2608_06466_amd import workloads as W
    from paper_2608_06466_amd import zoneburn as zb
    n_req = args.sub_requests if sub else args.requests
    ctx = zb.Context(0)
    nets_d = W.batched_networks()
    nets = [zb.Network(ctx, n) for n in nets_d]
    # capacity pilot: zone-burns/s of each network on launches that fill the GPU several times
    rate = []
    for k in range(4):
        st, sc, dt = W.request_inputs(nets_d, {"net": k, "zones": [1 << 19, 1 << 18, 1 << 17, 1 << 15][k],
                                               "seed": 99})
        t = torch.tensor(st, device="cuda:0")
        s = None if sc is None else torch.tensor(sc, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        zb.burn(ctx, nets[k], t, dt, 1e-8, 1e-12, rate_scale=s, precision=args.precision)
        zb.sync(ctx)
        rate.append(st.shape[0] / (time.perf_counter() - t0))
        print(f"[bench] serving pilot network {k}: {rate[-1]:.0f} zone-burns/s", file=sys.stderr,
              flush=True)
        del t, s
    lo, hi = math.log(1 << 10), math.log(1 << 18)
    mean_zones = ((1 << 18) - (1 << 10)) / (hi - lo)
    mean_cost = np.mean([mean_zones / r for r in rate])         # GPU seconds per request
    lam = args.load / mean_cost
    reqs = W.serving_requests(n_req, seed=501, rate_hz=lam)
    inputs = [W.request_inputs(nets_d, r) for r in reqs]
    print(f"[bench] serving: arrival rate {lam:.3f}/s, {n_req} requests, budget {args.budget_gib} GiB",
          file=sys.stderr, flush=True)
    srv = zb.Server(ctx, int(args.budget_gib * (1 << 30)), precision=args.precision)
    tickets = [None] * len(reqs)
    infos = [None] * len(reqs)
    done_evt = threading.Event()

    def collector():
        for i in range(len(reqs)):
            while tickets[i] is None:
                time.sleep(0.0005)
            while not srv.wait(tickets[i], timeout=1.0):
                pass
            out, status, stats, info = srv.fetch(tickets[i])
            infos[i] = info
            if (i + 1) % 8 == 0:
                print(f"[bench] serving: {i + 1} requests done", file=sys.stderr, flush=True)
        done_evt.set()

    th = threading.Thread(target=collector, daemon=True)
    th.start()
    t_start = time.perf_counter()
    for i, r in enumerate(reqs):
        delay = t_start + r["arrival"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        st, sc, dt = inputs[i]
        tickets[i] = srv.submit(nets[r["net"]], st, dt, r["rtol"], 1e-12, sc)
    done_evt.wait()
    th.join()
    t_end = time.perf_counter()
    tot = srv.stats()
    srv.close()
    for n in nets:
        n.close()
    ctx.close()
    torch.cuda.empty_cache()
    lat = np.array([i["latency_s"] for i in infos])
    queue = np.array([i["queue_s"] for i in infos])
    first = np.array([i["first_launch_s"] for i in infos])
    ok = sum(i["zones_ok"] for i in infos)
    zones = sum(r["zones"] for r in reqs)
    per_net = []
    for k in range(4):
        m = np.array([r["net"] == k for r in reqs])
        per_net.append({"nv": nets_d[k]["n_species"] + nets_d[k]["thermal"], "requests": int(m.sum()),
                        "latency_p50": _pct(lat[m], 50), "latency_p99": _pct(lat[m], 99),
                        "queue_p50": _pct(first[m], 50), "queue_p99": _pct(first[m], 99),
                        "service_p50": _pct(lat[m] - first[m], 50),
                        "service_p99": _pct(lat[m] - first[m], 99)})
    out = {"value": round(ok / (t_end - t_start), 1), "unit": "zone-burns/s",
           "latency_s": {"p50": _pct(lat, 50), "p99": _pct(lat, 99), "max": round(float(lat.max()), 4),
                         "mean": round(float(lat.mean()), 4)},
           "admission_wait_s": {"p50": _pct(queue, 50), "p99": _pct(queue, 99)},
           "queue_to_first_launch_s": {"p50": _pct(first, 50), "p99": _pct(first, 99)},
           "per_network": per_net,
           "requests": n_req, "zones": zones, "zones_ok": ok, "wall_s": round(t_end - t_start, 2),
           "workload": f"{n_req} Poisson requests (seed 501) at {lam:.3f}/s ({args.load} of the "
                       "measured capacity), 1k..256k zones log-uniform, networks nv 3/14/22/48, rtol "
                       f"1e-6 or 1e-8, HBM budget {args.budget_gib} GiB, precision {args.precision}",
           "capacity_zone_burns_per_s": [round(r, 1) for r in rate], "server": tot}
    if sub:
        return out
    line = _common_line("serving: zone-burns/s and request latency p50/p99 (Poisson burn requests)",
                        out["value"], "zone-burns/s", args, round((t_end - t_start) * 1e3, 1),
                        "f64 (f32 LU)" if args.precision == "mixed" else "f64",
                        {"workload": out["workload"], "precision": args.precision})
    line["steps"] = n_req
    for k in ("latency_s", "admission_wait_s", "queue_to_first_launch_s", "per_network", "zones",
              "zones_ok", "capacity_zone_burns_per_s", "server"):
        line[k] = out[k]
    print(json.dumps(line), flush=True)


def _reap_children():
    """End any child process this run left (none is started on purpose)."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    print(f"[bench] child processes at exit: {[(p.pid, p.name()) for p in kids]}", file=sys.stderr,
          flush=True)
    for p in kids:
        try:
            p.kill()
        except psutil.Error:
            pass


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "robertson", "batched", "serving"],
                    help="headline: 14-variable network, 2^20 zones, with the batched and serving "
                         "objects (the default); robertson: 4096 Robertson zones; batched: four "
                         "networks, 2^21 zones, one call, FP64 and mixed; serving: Poisson stream "
                         "of requests through the server")
    ap.add_argument("--zones", type=int, default=0, help="zones (0: the workload's own size)")
    ap.add_argument("--batched-zones", type=int, default=0,
                    help="zones of the headline run's batched object (0: 2^21)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the CPU-oracle baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the batched and serving objects")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--requests", type=int, default=500, help="serving: number of requests")
    ap.add_argument("--sub-requests", type=int, default=48,
                    help="requests of the headline run's serving object")
    ap.add_argument("--load", type=float, default=0.7, help="serving: offered load / capacity")
    ap.add_argument("--budget-gib", type=float, default=16.0, help="serving: HBM budget")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"],
                    help="serving: precision of every request")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: zones need no communication, and one MI355X is what "
              f"the library drives; --gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)
    {"headline": headline, "robertson": robertson, "batched": batched,
     "serving": serving}[args.workload](args)
    _reap_children()


if __name__ == "__main__":
    main()
