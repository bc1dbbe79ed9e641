"""Benchmark: zone-burns/s of the per-zone stiff BDF burn on one MI355X.

Workload (the 14-variable network the headline metric names): 13 species + T,
30 random two-body reactions with Arrhenius rates, 2^20 zones with
T ~ U(1e3, 5e3) and Dirichlet(1) abundances, dt = 1, rtol = 1e-8, atol = 1e-12.
A step is one complete burn of all 2^20 zones (device-resident state, reset to
the initial state before every step).  The mixed-precision burn (FP32 LU, FP64
everything else) is the reported value; the plain FP64 burn of the same input
is reported next to it.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  Extra keys: plain_fp64 (the FP64 path), roofline (FP64
ALU bound of the burn kernel), cpu_baseline (the CPU oracle on a bounded
sample of the same zones; the same sample gives the accuracy of both GPU paths).
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


def step_flops(nv, nr, thermal, stats):
    """Algorithmic FP64 flops of the burns, from the per-zone counters.

    Per Jacobian + LU (one per step attempt): Jacobian entries 37 per reaction
    (3 partials and their scatter into up to 5 rows), M = I - gamma J (2 nv^2),
    LU sum_m (m + 2 m^2) over m = nv-1..0, history prediction, weights, error
    norm and correction at a nominal order 3 (13 nv).  Per RHS: 14 per reaction.
    Per Newton iteration: forward/back solve 2 nv^2 - nv, residual, update and
    norm 9 nv.  exp/log are not counted (see transcendentals()).
    """
    nst, nfe, nje, nlu, nni = (stats[:, k].astype(np.float64).sum() for k in range(5))
    lu = sum(m + 2 * m * m for m in range(nv))
    per_att = 37 * nr + 2 * nv * nv + lu + 13 * nv
    per_rhs = 14 * nr
    per_it = 2 * nv * nv - nv + 9 * nv
    return nje * per_att + nfe * per_rhs + nni * per_it


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "burn_kernel_14x16_nv14_2p20zones_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2608_06466_amd", "csrc", f)
                  for f in ("zb_burn_kernel.h", "zb_internal.h", "zb_k14.hip")] + [
                  os.path.join(ROOT, "paper_2608_06466_amd", "build.py")]   # the compile flags


def measured_traffic(precision, zones):
    """HBM bytes per burn launch from the committed FETCH_SIZE/WRITE_SIZE profile.

    None unless the profile was taken on the current kernel sources and on the
    same zone count (the counters do not run inside this process)."""
    import hashlib
    import re
    if zones != 1 << 20 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    txt = open(TRAFFIC_PROFILE).read()
    m = re.search(r"kernel_sources_sha256: ([0-9a-f]{64})", txt)
    t = re.search(rf"traffic_bytes_per_launch:.*\b{precision}=([0-9.e+]+)", txt)
    if not m or not t:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return float(t.group(1)) if h.hexdigest() == m.group(1) else None


def transcendentals(nr, thermal, stats):
    return stats[:, 1].astype(np.float64).sum() * ((nr + 2) if thermal else 0)


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
    stream = torch.cuda.current_stream()

    def run(precision, steps, warmup, jac_policy=0, integrator="bdf"):
        lanes = zb.get_mapping(ctx, net, precision)
        times, kernel_ms = [], []
        status = stats = None
        for it in range(warmup + steps):
            work.copy_(state0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            status, stats = zb.burn(ctx, net, work, dt, rtol, atol, precision=precision,
                                    jac_policy=jac_policy, integrator=integrator)
            e1.record(stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            nfail = zb.sync(ctx)
            if it >= warmup:
                times.append(t1 - t0)
                kernel_ms.append(e0.elapsed_time(e1))
            print(f"[bench] {precision} jac {jac_policy} {integrator} "
                  f"step {it - warmup if it >= warmup else 'warmup'}: "
                  f"{(t1 - t0) * 1e3:.1f} ms (kernel {e0.elapsed_time(e1):.1f} ms), failed zones {nfail}",
                  file=sys.stderr, flush=True)
        st = stats.cpu().numpy()
        sts = status.cpu().numpy()
        return dict(lanes=lanes, wall_s=float(np.mean(times)), kernel_ms=float(np.mean(kernel_ms)),
                    stats=st, status=sts, out=work.cpu().numpy())

    res = {}
    for prec in ("mixed", "fp64"):
        res[prec] = run(prec, args.steps, args.warmup)
    # the VODE-style Jacobian/LU reuse (reported beside the headline method, which takes a
    # Jacobian and an LU on every step)
    res["reuse"] = run("mixed", args.steps, args.warmup, jac_policy=1)
    # VODE's own configuration: the variable-coefficient BDF form with that reuse
    res["vode"] = run("mixed", args.steps, args.warmup, jac_policy=1, integrator="bdf_variable")

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 1 GiB read + 1 GiB written", file=sys.stderr, flush=True)

    def summary(r):
        ok = int((r["status"] == 0).sum())
        fl = step_flops(nv, nr, 1, r["stats"])
        return dict(value=ok / r["wall_s"], ok_zones=ok, ms_per_step=r["wall_s"] * 1e3,
                    kernel_ms=r["kernel_ms"], flops=fl, lanes_per_zone=r["lanes"],
                    mean_steps=float(r["stats"][:, 0].mean()),
                    max_steps=int(r["stats"][:, 0].max()))

    sm, sf, sr = summary(res["mixed"]), summary(res["fp64"]), summary(res["reuse"])
    sv = summary(res["vode"])

    def roofline(s, precision):
        achieved = s["flops"] / (s["kernel_ms"] * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(precision, zones)}

    # ---- CPU oracle baseline on a bounded sample (rank 0, N=1 only) ----
    cpu = None
    accuracy = None
    if not args.no_cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        threads = max(1, min(threads, os.cpu_count() or 1))
        rng = np.random.default_rng(12345)
        pilot = np.sort(rng.choice(zones, 256, replace=False))
        t0 = time.perf_counter()
        oracle.burn(net_d, state0_np[pilot], dt, rtol, atol, nthreads=threads)
        pt = time.perf_counter() - t0
        n = int(min(zones, max(512, 256 * args.cpu_seconds / max(pt, 1e-3))))
        idx = np.sort(rng.choice(zones, n, replace=False))
        t0 = time.perf_counter()
        ref, ref_status, _ = oracle.burn(net_d, state0_np[idx], dt, rtol, atol, nthreads=threads)
        ct = time.perf_counter() - t0
        cpu = {"value": round(n / ct, 3), "unit": "zone-burns/s", "cores": threads, "kind": "oracle",
               "sample": f"{n} zones drawn uniformly (seed 12345) from the same 2^20-zone input, "
                         f"plain C FP64 oracle, OpenMP over zones, {ct:.1f} s wall"}
        accuracy = {}
        ref_r, ref_r_status, _ = oracle.burn(net_d, state0_np[idx], dt, rtol, atol, nthreads=threads,
                                             jac_policy=1)
        ref_v, ref_v_status, _ = oracle.burn(net_d, state0_np[idx], dt, rtol, atol, nthreads=threads,
                                             jac_policy=1, form="variable")
        refs = {"mixed": (ref, ref_status), "fp64": (ref, ref_status),
                "reuse": (ref_r, ref_r_status), "vode": (ref_v, ref_v_status)}
        for prec in ("mixed", "fp64", "reuse", "vode"):
            rs, rst = refs[prec]
            out = res[prec]["out"][idx][:, :nv]
            ok = (rst == 0) & (res[prec]["status"][idx] == 0)
            gated = np.abs(out[ok] - rs[ok, :nv]) / np.maximum(np.abs(rs[ok, :nv]), atol / rtol)
            gz = gated.max(1)
            accuracy[prec] = {"max_gated_rel_err": float(gz.max()),
                              "zones_over_1e-6": int((gz > 1e-6).sum()),
                              "median_gated_rel_err": float(np.median(gz)),
                              "status_mismatches": int((rst != res[prec]["status"][idx]).sum()),
                              "sampled_zones": n}

    line = {
        "metric": "zone-burns/sec at rel err <=1e-6 (14-var net), mixed vs plain FP64",
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
        "plain_fp64": {"value": round(sf["value"], 1), "ms_per_step": round(sf["ms_per_step"], 2),
                       "kernel_ms": round(sf["kernel_ms"], 2), "roofline": roofline(sf, "fp64"),
                       "lanes_per_zone": sf["lanes_per_zone"]},
        "mixed_over_fp64": round(sm["value"] / sf["value"], 3),
        "jac_reuse": {"value": round(sr["value"], 1), "ms_per_step": round(sr["ms_per_step"], 2),
                      "kernel_ms": round(sr["kernel_ms"], 2), "precision": "mixed",
                      "failed_zones": int((res["reuse"]["status"] != 0).sum()),
                      "jacobians_per_zone": round(float(res["reuse"]["stats"][:, 2].mean()), 1),
                      "lus_per_zone": round(float(res["reuse"]["stats"][:, 3].mean()), 1),
                      "note": "VODE-style reuse of the Jacobian and LU (jac_policy 1); value counts "
                              "OK zones; accuracy against the oracle's reuse policy"},
        "vode_form": {"value": round(sv["value"], 1), "ms_per_step": round(sv["ms_per_step"], 2),
                      "kernel_ms": round(sv["kernel_ms"], 2), "precision": "mixed",
                      "failed_zones": int((res["vode"]["status"] != 0).sum()),
                      "mean_steps": round(sv["mean_steps"], 1),
                      "jacobians_per_zone": round(float(res["vode"]["stats"][:, 2].mean()), 1),
                      "note": "variable-coefficient BDF form with the Jacobian/LU reuse (integrator "
                              "bdf_variable, jac_policy 1); value counts OK zones; accuracy against "
                              "the oracle's same configuration"},
        "roofline": roofline(sm, "mixed"),
        "kernel_ms": round(sm["kernel_ms"], 2),
        "zone_steps": {"mean": round(sm["mean_steps"], 1), "max": sm["max_steps"]},
        "transcendentals_per_s": round(transcendentals(nr, 1, res["mixed"]["stats"])
                                       / (sm["kernel_ms"] * 1e-3), 1),
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": accuracy,
    }
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()



# ------------------------------------------------------------------ other workloads

def _common_line(metric, value, unit, args, ms, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def _gated(out, ref, nv, rtol, atol):
    return (np.abs(out[:, :nv] - ref[:, :nv]) / np.maximum(np.abs(ref[:, :nv]), atol / rtol)).max(1)


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
    best, times = zb.autotune(ctx, net, s0, cfg["dt"], cfg["rtol"], cfg["atol"], "fp64")
    w = torch.empty_like(s0)
    stream = torch.cuda.current_stream()
    ts, ks = [], []
    for it in range(args.warmup + args.steps):
        w.copy_(s0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        status, stats = zb.burn(ctx, net, w, cfg["dt"], cfg["rtol"], cfg["atol"], rate_scale=sc)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        zb.sync(ctx)
        if it >= args.warmup:
            ts.append(t1 - t0)
            ks.append(e0.elapsed_time(e1))
    st = stats.cpu().numpy()
    ok = int((status.cpu().numpy() == 0).sum())
    wall = float(np.mean(ts))
    line = _common_line("zone-burns/s, Robertson (3 species, t = 0..1e5)", round(ok / wall, 1), "zone-burns/s", args,
                        round(wall * 1e3, 3), "f64",
                        {"workload": f"Robertson, {zones} zones, lognormal(0,0.1) rate scales, t=0..1e5, "
                                     "rtol=1e-8, atol=1e-12", "lanes_per_zone": best,
                         "autotune_ms_per_lane_count_1_to_64": [round(t, 3) for t in times]})
    line["kernel_ms"] = round(float(np.mean(ks)), 3)
    line["zone_steps"] = {"mean": round(float(st[:, 0].mean()), 1), "max": int(st[:, 0].max())}
    if not args.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        threads = max(1, min(threads, os.cpu_count() or 1))
        t0 = time.perf_counter()
        ref, rst, _ = oracle.burn(cfg["net"], cfg["state"], cfg["dt"], cfg["rtol"], cfg["atol"],
                                  cfg["scale"], nthreads=threads)
        ct = time.perf_counter() - t0
        out = w.cpu().numpy()
        g = _gated(out, ref, 3, cfg["rtol"], cfg["atol"])
        line["cpu_baseline"] = {"value": round(zones / ct, 1), "unit": "zone-burns/s", "cores": threads,
                                "kind": "oracle", "sample": f"all {zones} zones"}
        line["accuracy_vs_oracle"] = {"max_gated_rel_err": float(g.max()),
                                      "zones_over_1e-6": int((g > 1e-6).sum()),
                                      "status_mismatches": int((rst != status.cpu().numpy()).sum())}
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()


def batched(args):
    """Four networks (nv 3, 14, 22, 48; 4:2:1:1 of 2^21 zones) in one zb_burn_batch call, FP64
    and with the FP32 LU, each against the oracle on a stratified sample;
    the FP32 run again with the blocked matrix-core LU (lu='mfma': the 48-variable class)."""
    import torch
    import oracle
    from paper_2608_06466_amd import workloads as W
    from paper_2608_06466_amd import zoneburn as zb
    segs_h = W.batched(args.zones or (1 << 21))
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
    stream = torch.cuda.current_stream()
    res = {}
    for key, prec, lu in (("fp64", "fp64", "valu"), ("mixed", "mixed", "valu"),
                          ("mixed_mfma", "mixed", "mfma")):
        ts = []
        for it in range(args.warmup + args.steps):
            for w, i0 in zip(work, init):
                w.copy_(i0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            zb.burn_batch(ctx, segs, precision=prec, lu=lu)
            e1.record(stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            nf = zb.sync(ctx)
            print(f"[bench] batched {key} step {it}: {(t1 - t0) * 1e3:.1f} ms, failed zones {nf}",
                  file=sys.stderr, flush=True)
            if it >= args.warmup:
                ts.append((t1 - t0, e0.elapsed_time(e1)))
        r = {"wall_s": float(np.mean([t[0] for t in ts])), "kernel_ms": float(np.mean([t[1] for t in ts])),
             "out": [w.cpu().numpy() for w in work], "status": [s.cpu().numpy() for s in status],
             "stats": [s.cpu().numpy() for s in stats]}
        r["ok"] = int(sum((s == 0).sum() for s in r["status"]))
        r["flops"] = float(sum(step_flops(n.nv, n.nr, n.thermal, st) for n, st in zip(nets, r["stats"])))
        res[key] = r
    per_class = []
    for k, s in enumerate(segs_h):
        st = res["fp64"]["stats"][k][:, 0]
        per_class.append({"nv": nets[k].nv, "reactions": nets[k].nr, "zones": int(st.shape[0]),
                          "steps_p1": float(np.percentile(st, 1)), "steps_median": float(np.median(st)),
                          "steps_max": int(st.max())})

    def roof(r):
        a = r["flops"] / (r["kernel_ms"] * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(a, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(a / FP64_PEAK_TFLOPS, 4), "traffic": None}

    m, f = res["mixed"], res["fp64"]
    line = _common_line("zone-burns/s, four networks (nv 3, 14, 22, 48) in one call", round(m["ok"] / m["wall_s"], 1),
                        "zone-burns/s", args, round(m["wall_s"] * 1e3, 2), "f64 (f32 LU)",
                        {"workload": f"Robertson : nv14 : nv22 : nv48 = 4:2:1:1 of {total} zones, "
                                     "T log-uniform on [90, 2500] K, dt 1 (Robertson 1e5), rtol 1e-8, "
                                     "atol 1e-12", "per_class": per_class})
    line["plain_fp64"] = {"value": round(f["ok"] / f["wall_s"], 1), "ms_per_step": round(f["wall_s"] * 1e3, 2),
                          "roofline": roof(f)}
    line["roofline"] = roof(m)
    line["mixed_over_fp64"] = round((m["ok"] / m["wall_s"]) / (f["ok"] / f["wall_s"]), 3)
    b = res["mixed_mfma"]
    line["mfma_lu"] = {"value": round(b["ok"] / b["wall_s"], 1), "ms_per_step": round(b["wall_s"] * 1e3, 2),
                       "over_valu_lu": round((b["ok"] / b["wall_s"]) / (m["ok"] / m["wall_s"]), 3),
                       "note": "mixed precision with lu='mfma': the 48-variable class factors with the "
                               "blocked LU (trailing updates as FP32 MFMA products), the others keep "
                               "the vector-unit LU"}
    if not args.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        threads = max(1, min(threads, os.cpu_count() or 1))
        rng = np.random.default_rng(4321)
        acc = {"fp64": [], "mixed": [], "mixed_mfma": []}
        cpu_time_per_zone = []
        for k, s in enumerate(segs_h):
            nz = s["state"].shape[0]
            n = [256, 256, 128, 48][k]
            idx = np.sort(rng.choice(nz, n, replace=False))
            t0 = time.perf_counter()
            ref, rst, _ = oracle.burn(s["net"], s["state"][idx], s["dt"], s["rtol"], s["atol"],
                                      None if s["scale"] is None else s["scale"][idx], nthreads=threads)
            cpu_time_per_zone.append((time.perf_counter() - t0) / n)
            for prec in ("fp64", "mixed", "mixed_mfma"):
                out = res[prec]["out"][k][idx]
                ok = (rst == 0) & (res[prec]["status"][k][idx] == 0)
                g = _gated(out[ok], ref[ok], nets[k].nv, s["rtol"], s["atol"])
                acc[prec].append({"nv": nets[k].nv, "sampled": n, "max_gated_rel_err": float(g.max()),
                                  "zones_over_1e-6": int((g > 1e-6).sum()),
                                  "median_gated_rel_err": float(np.median(g)),
                                  "status_mismatches": int((rst != res[prec]["status"][k][idx]).sum())})
        est = total / sum(t * s["state"].shape[0] for t, s in zip(cpu_time_per_zone, segs_h))
        line["cpu_baseline"] = {"value": round(est, 1), "unit": "zone-burns/s", "cores": threads,
                                "kind": "oracle",
                                "sample": "256/256/128/48 zones of the nv 3/14/22/48 segments; whole-batch "
                                          "rate extrapolated from the per-class time per zone"}
        line["accuracy_vs_oracle"] = acc
    print(json.dumps(line), flush=True)
    for n in nets:
        n.close()
    ctx.close()


def serving(args):
    """Poisson stream of burn requests (1k..256k zones, the four networks of the batched workload, rtol 1e-6
    or 1e-8) through the continuous-batching server: throughput and request latency."""
    import threading
    import torch
    from paper_2608_06466_amd import workloads as W
    from paper_2608_06466_amd import zoneburn as zb
    ctx = zb.Context(0)
    nets_d = W.batched_networks()
    nets = [zb.Network(ctx, n) for n in nets_d]
    # capacity pilot: zone-burns/s of each network on a full GPU
    rate = []
    for k in range(4):
        st, sc, dt = W.request_inputs(nets_d, {"net": k, "zones": [1 << 16, 1 << 15, 1 << 14, 1 << 13][k],
                                               "seed": 99})
        t = torch.tensor(st, device="cuda:0")
        s = None if sc is None else torch.tensor(sc, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        zb.burn(ctx, nets[k], t, dt, 1e-8, 1e-12, rate_scale=s, precision=args.precision)
        zb.sync(ctx)
        rate.append(st.shape[0] / (time.perf_counter() - t0))
    lo, hi = math.log(1 << 10), math.log(1 << 18)
    mean_zones = ((1 << 18) - (1 << 10)) / (hi - lo)
    mean_cost = np.mean([mean_zones / r for r in rate])         # GPU seconds per request
    lam = args.load / mean_cost
    reqs = W.serving_requests(args.requests, seed=501, rate_hz=lam)
    inputs = [W.request_inputs(nets_d, r) for r in reqs]
    print(f"[bench] serving: capacity pilot {[round(r) for r in rate]} zone-burns/s per network, "
          f"arrival rate {lam:.3f}/s, {args.requests} requests", file=sys.stderr, flush=True)
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
    t_end = time.perf_counter()
    tot = srv.stats()
    srv.close()
    lat = np.array([i["latency_s"] for i in infos])
    queue = np.array([i["queue_s"] for i in infos])
    ok = sum(i["zones_ok"] for i in infos)
    zones = sum(r["zones"] for r in reqs)
    line = _common_line("serving: zone-burns/s and request latency p50/p99 (Poisson burn requests)",
                        round(ok / (t_end - t_start), 1), "zone-burns/s", args,
                        round((t_end - t_start) * 1e3, 1), "f64 (f32 LU)" if args.precision == "mixed" else "f64",
                        {"workload": f"{args.requests} Poisson requests at {lam:.3f}/s ({args.load} of the "
                                     "measured capacity), 1k..256k zones log-uniform, networks nv 3/14/22/48, "
                                     f"rtol 1e-6 or 1e-8, HBM budget {args.budget_gib} GiB",
                         "precision": args.precision})
    line["steps"] = args.requests
    line["latency_s"] = {"p50": round(float(np.percentile(lat, 50)), 4),
                         "p99": round(float(np.percentile(lat, 99)), 4),
                         "max": round(float(lat.max()), 4), "mean": round(float(lat.mean()), 4)}
    line["queue_s"] = {"p50": round(float(np.percentile(queue, 50)), 4), "p99": round(float(np.percentile(queue, 99)), 4)}
    line["zones"] = zones
    line["zones_ok"] = ok
    line["server"] = tot
    line["capacity_zone_burns_per_s"] = [round(r, 1) for r in rate]
    print(json.dumps(line), flush=True)
    for n in nets:
        n.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "robertson", "batched", "serving"],
                    help="headline: 14-variable network, 2^20 zones (the default); robertson: 4096 "
                         "Robertson zones; batched: four networks, 2^21 zones, one call, FP64 and "
                         "mixed; serving: Poisson stream of requests through the server")
    ap.add_argument("--zones", type=int, default=0, help="zones (0: the workload's own size)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the CPU-oracle baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--requests", type=int, default=48, help="serving: number of requests")
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


if __name__ == "__main__":
    main()
