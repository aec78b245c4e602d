#!/usr/bin/env python3
"""Benchmark of the collision-coalescence hot path on one MI355X.

Workload: one GPU's patch of a thunderstorm domain, 256 x 256 x 50 points,
33 mass-doubling bins of liquid drops, gravitational collection kernel
tabulated at 1000/750/500 hPa, 15% cloudy points with gamma spectra (seeded
synthetic inputs, see paper_2409_07232_amd/workloads.py).  One benchmark
step is one fsbm_coal_step call: cloudy-point compaction, 100 collision
steps of 2 s, scatter back.  The state evolves from call to call, like a
model integration; inputs are resident in HBM before timing starts.

Metric: grid-point collision updates per second (cloudy points x collision
steps / time) of the FP32-compensated path; the plain FP64 path is reported
beside it.  The roofline entry is for the dominant kernel (the collision
step kernel), timed with HIP events on the stream it runs on.  The CPU
baseline is the FP64 oracle on a bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per evaluated bin pair (FP32 and FP64 paths alike):
# 24 arithmetic operations + 2 divisions + 3 transcendentals, each counted
# as one floating-point operation.
FLOPS_PER_PAIR = 29
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64 (published)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 path beside the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=1 << 14)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--nz", type=int, default=50)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (the "
                         "reference kernel for scaling HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_path(w, precision, steps, warmup, N0, p):
    """Warm up, then time `steps` calls; returns a result dict."""
    import torch

    from paper_2409_07232_amd import _lib as L
    h = L.FsbmCoal.from_workload(w, precision=precision,
                                 flags=L.FLAG_PROFILE)
    N = N0.clone()
    for _ in range(warmup):
        h.step(N, p, w.dt, w.nsteps)
    torch.cuda.synchronize()
    st0 = h.stats()
    pairs = 0
    active = st0["active_points"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.step(N, p, w.dt, w.nsteps)
        st = h.stats()          # synchronises the stream
        pairs += st["pair_evals"]
        active = st["active_points"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = h.stats()
    launches = st1["kernel_launches"] - st0["kernel_launches"]
    kms = st1["kernel_ms"] - st0["kernel_ms"]
    h.close()
    secs = t1 - t0
    return {"secs": secs, "ms_per_step": 1e3 * secs / steps,
            "updates_per_s": active * w.nsteps * steps / secs,
            "active_points": active, "pair_evals": pairs,
            "kernel_launches": launches, "kernel_ms": kms,
            "kernel_avg_ms": kms / max(launches, 1),
            "limiter_steps": st1["limiter_steps"],
            "fallback_steps": st1["fp64_fallback_steps"]}


def roofline(res, peak):
    achieved = FLOPS_PER_PAIR * res["pair_evals"] / (res["kernel_ms"] * 1e-3)
    achieved /= 1e12
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 5),
            "traffic": None}


def cpu_baseline(w, npts, nsteps):
    import numpy as np

    import oracle
    from paper_2409_07232_amd import workloads as wl
    idx = wl.sample_active(w, npts, seed=11)
    sub = w.subset(idx)
    om = oracle.OracleModel(w.nbins, w.nspecies, w.tables, w.p_levels,
                            w.product, x1_g=w.x1_g, s=w.s, theta=w.theta)
    N = np.array(sub.N, copy=True)
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    om.run(N, sub.p, w.dt, nsteps, nthreads=cores)
    secs = time.perf_counter() - t0
    return {"value": round(len(idx) * nsteps / secs, 1),
            "unit": "grid-point collision updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d seeded cloudy points x %d steps of %.0f s of the "
                      "same workload, FP64, %.1f s" % (len(idx), nsteps,
                                                       w.dt, secs)}, idx, N


def parity(w, idx, Nref, nsteps):
    """GPU result on the CPU-baseline sample against the oracle's."""
    import numpy as np
    import torch

    from oracle import compare
    from paper_2409_07232_amd import _lib as L
    from paper_2409_07232_amd import workloads as wl
    sub = w.subset(idx)
    x = wl.bin_masses(w.nbins, w.s, w.x1_g)
    out = {}
    for name, prec in (("fp32c", L.FSBM_FP32C), ("fp64", L.FSBM_FP64)):
        h = L.FsbmCoal.from_workload(w, precision=prec)
        N = torch.from_numpy(np.array(sub.N, copy=True)).to("cuda")
        p = torch.from_numpy(np.array(sub.p, copy=True)).to("cuda")
        h.step(N, p, w.dt, nsteps)
        got = N.cpu().numpy()
        h.close()
        out[name] = {"rel_bin": float("%.3e" % compare.rel_bin(got, Nref, x)),
                     "drift": float("%.3e" % compare.drift(got, sub.N, x))}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the collision step has no "
              "cross-point exchange, so a multi-GPU run is N independent "
              "copies of this one; got --gpus %d" %
              args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2409_07232_amd import _lib as L
    from paper_2409_07232_amd import workloads as wl
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written":
                          n * 8, "dispatches": 3}), flush=True)
        return
    L.load()
    log("generating workload")
    w = wl.config2(nx=args.nx, ny=args.ny, nz=args.nz)
    N0 = torch.from_numpy(w.N).to("cuda")
    p = torch.from_numpy(w.p).to("cuda")
    log("timing fp32c: %d warmup + %d steps" % (args.warmup, args.steps))
    r32 = time_path(w, L.FSBM_FP32C, args.steps, args.warmup, N0, p)
    log("fp32c %.2f ms/step, %.3e updates/s" % (r32["ms_per_step"],
                                               r32["updates_per_s"]))
    r64 = None
    if not args.no_fp64:
        log("timing fp64")
        r64 = time_path(w, L.FSBM_FP64, args.steps, args.warmup, N0, p)
        log("fp64 %.2f ms/step, %.3e updates/s" % (r64["ms_per_step"],
                                                  r64["updates_per_s"]))
    del N0
    cpu = None
    par = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on %d points" % args.cpu_points)
        cpu, idx, Nref = cpu_baseline(w, args.cpu_points, args.cpu_steps)
        log("cpu %.3e updates/s on %d cores" % (cpu["value"], cpu["cores"]))
        par = parity(w, idx, Nref, args.cpu_steps)
    line = {
        "metric": "grid-point collision updates/s at 33 bins; FP32-comp vs "
                  "FP64, rel err <=1e-5",
        "value": round(r32["updates_per_s"], 1),
        "unit": "grid-point collision updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "thunderstorm_patch_%dx%dx%d_33bins_liquid" % (
                       args.nx, args.ny, args.nz),
                   "points": w.npoints, "cloudy_points": r32["active_points"],
                   "bins": w.nbins, "species": w.nspecies, "dt_s": w.dt,
                   "collision_steps_per_step": w.nsteps,
                   "kernel_tables": "gravitational, 3 pressure levels",
                   "parallelism": "single GPU"},
        "roofline": roofline(r32, PEAK_FP32_TFLOPS),
        "kernel": {"name": "lane_step_f32c<33>",
                   "avg_launch_ms": round(r32["kernel_avg_ms"], 4),
                   "launches": r32["kernel_launches"],
                   "pair_evals": r32["pair_evals"],
                   "flops_per_pair": FLOPS_PER_PAIR,
                   "fallback_steps": r32["fallback_steps"]},
    }
    if r64 is not None:
        line["fp64"] = {"value": round(r64["updates_per_s"], 1),
                        "ms_per_step": round(r64["ms_per_step"], 4),
                        "dtype": "f64",
                        "roofline": roofline(r64, PEAK_FP64_TFLOPS),
                        "avg_launch_ms": round(r64["kernel_avg_ms"], 4)}
    if cpu is not None:
        line["cpu_baseline"] = cpu
        line["parity_on_cpu_sample"] = par
    line["context"] = {
        "paper": "2.08x whole-WRF speedup, 16 A100 vs 16 EPYC cores "
                 "(CONUS-12km); collision kernel 29.11 ms per call on one "
                 "A100 for a ~398k-point patch (<= 1.37e7 point-updates/s); "
                 "other hardware, precision and workload: context only"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
