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


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "burn_kernel_16x16_nv14_2p20zones_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2608_06466_amd", "csrc", f)
                  for f in ("zb_kernels.hip", "zb_internal.h")]


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--zones", type=int, default=1 << 20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the CPU-oracle baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the burn needs no communication between zones and this "
              f"build runs on a single MI355X; --gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_06466_amd import workloads as W
    from paper_2608_06466_amd import zoneburn as zb

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    cfg = W.config2(args.zones)
    net_d, state0_np = cfg["net"], cfg["state"]
    dt, rtol, atol = cfg["dt"], cfg["rtol"], cfg["atol"]
    zones = state0_np.shape[0]
    nv, nr = net_d["n_species"] + 1, len(net_d["lnA"])

    ctx = zb.Context(0)
    net = zb.Network(ctx, net_d)
    state0 = torch.tensor(state0_np, device=dev)
    work = torch.empty_like(state0)
    stream = torch.cuda.current_stream()

    def run(precision, steps, warmup):
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
            status, stats = zb.burn(ctx, net, work, dt, rtol, atol, precision=precision)
            e1.record(stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            nfail = zb.sync(ctx)
            if it >= warmup:
                times.append(t1 - t0)
                kernel_ms.append(e0.elapsed_time(e1))
            print(f"[bench] {precision} step {it - warmup if it >= warmup else 'warmup'}: "
                  f"{(t1 - t0) * 1e3:.1f} ms (kernel {e0.elapsed_time(e1):.1f} ms), failed zones {nfail}",
                  file=sys.stderr, flush=True)
        st = stats.cpu().numpy()
        sts = status.cpu().numpy()
        return dict(lanes=lanes, wall_s=float(np.mean(times)), kernel_ms=float(np.mean(kernel_ms)),
                    stats=st, status=sts, out=work.cpu().numpy())

    res = {}
    for prec in ("mixed", "fp64"):
        res[prec] = run(prec, args.steps, args.warmup)

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

    sm, sf = summary(res["mixed"]), summary(res["fp64"])

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
        for prec in ("mixed", "fp64"):
            out = res[prec]["out"][idx][:, :nv]
            ok = (ref_status == 0) & (res[prec]["status"][idx] == 0)
            gated = np.abs(out[ok] - ref[ok, :nv]) / np.maximum(np.abs(ref[ok, :nv]), atol / rtol)
            gz = gated.max(1)
            accuracy[prec] = {"max_gated_rel_err": float(gz.max()),
                              "zones_over_1e-6": int((gz > 1e-6).sum()),
                              "median_gated_rel_err": float(np.median(gz)),
                              "status_mismatches": int((ref_status != res[prec]["status"][idx]).sum()),
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


if __name__ == "__main__":
    main()
