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

--workload selects the other measured shapes (each prints its own line with
the same fields; the default run prints the headline line only):
  four_species     2^20 points, liquid/ice/snow/graupel, 33 bins
  refined66|132|264  262,144 points, liquid + graupel, refined grids
  mixed            2^22 points, 10% cloudy, 33/66/132-bin grids in one
                   persistent launch (FP32C) beside per-grid FP64 launches
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
FP32C_TOL = 1e-5           # rel_bin bar of the FP32C path
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64 (published)

# HBM bytes per launch of a kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs scaled by the same counters on a 1 GiB device copy (the profile
# summary under profiles/ gives the commands).  They hold only for the
# kernel sources they were taken on: the SHA-256 of the concatenated files
# below must match, otherwise the traffic entry is reported as null.
TRAFFIC_SOURCES = ("kernels_lane.hip", "device_common.hpp")
MEASURED_TRAFFIC = {
    # kernel: (sources sha256, bytes per launch, profile summary)
    "lane_step_f32c<33>": (
        "ed6c3a8e7abf9b33ae7222591dcef7390d7643d0b4b8214941fb912fe061b844",
        4.305e+09, "profiles/lane_step_thunderstorm_256x256x50.md"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 path beside the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the sequential (in-place) form, timed beside "
                         "the headline on the thunderstorm workload")
    ap.add_argument("--workload", default="thunderstorm",
                    choices=["thunderstorm", "four_species", "refined66",
                             "refined132", "refined264", "mixed"])
    ap.add_argument("--points", type=int, default=0,
                    help="point count of the four_species, refined and "
                         "mixed workloads (default: the configuration's)")
    ap.add_argument("--collision-steps", type=int, default=0,
                    help="collision steps per call (default: the "
                         "workload's 100)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target oracle time of the CPU baseline sample")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps (default: the workload's)")
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--nz", type=int, default=50)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (the "
                         "reference kernel for scaling HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_name(st, precision, nbins):
    f32 = precision == 1
    if st["kernel"] == 2:
        return "lane_seq_f64<%d>" % nbins
    if st["kernel"] == 0:
        return "lane_step_%s<%d>" % ("f32c" if f32 else "f64", nbins)
    return "wave_step<%s>" % ("F32" if f32 else "F64")


def time_calls(run_once, handles, steps, warmup, nsteps):
    """Warm up, then time `steps` calls of run_once(); the first handle
    holds the launch timings and pair counters of a multi-grid call."""
    import torch
    for k in range(warmup):
        run_once()
        torch.cuda.synchronize()
        log("warm-up call %d done" % (k + 1))
    st0 = [h.stats() for h in handles]
    pairs = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        run_once()
        sts = [h.stats() for h in handles]   # synchronises the stream
        pairs += sum(st["pair_evals"] for st in sts)
        log("timed call %d done, %.1f s so far" % (k + 1,
                                                  time.perf_counter() - t0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st1 = [h.stats() for h in handles]
    launches = sum(b["kernel_launches"] - a["kernel_launches"]
                   for a, b in zip(st0, st1))
    kms = sum(b["kernel_ms"] - a["kernel_ms"] for a, b in zip(st0, st1))
    active = sum(st["active_points"] for st in st1)
    secs = t1 - t0
    return {"secs": secs, "ms_per_step": 1e3 * secs / steps,
            "updates_per_s": active * nsteps * steps / secs,
            "active_points": active, "pair_evals": pairs,
            "kernel_launches": launches, "kernel_ms": kms,
            "kernel_avg_ms": kms / max(launches, 1),
            "limiter_steps": sum(st["limiter_steps"] for st in st1),
            "fallback_steps": sum(st["fp64_fallback_steps"] for st in st1),
            "stats": st1[0]}


def time_path(w, precision, steps, warmup, N0, p, order=0):
    """One handle, one fsbm_coal_step per benchmark step."""
    from paper_2409_07232_amd import _lib as L
    h = L.FsbmCoal.from_workload(w, precision=precision,
                                 flags=L.FLAG_PROFILE, order=order)
    N = N0.clone()
    r = time_calls(lambda: h.step(N, p, w.dt, w.nsteps), [h], steps, warmup,
                   w.nsteps)
    h.close()
    return r


def time_multi(ws, precision, steps, warmup, N0s, ps, batched):
    """Several grids: one fsbm_coal_step_multi call (batched) or one
    fsbm_coal_step call per grid."""
    from paper_2409_07232_amd import _lib as L
    hs = [L.FsbmCoal.from_workload(w, precision=precision,
                                   flags=L.FLAG_PROFILE) for w in ws]
    Ns = [n.clone() for n in N0s]
    if batched:
        # the widest grid first, as the library expects its scratch to fit
        def run_once():
            L.step_multi(hs, Ns, ps, ws[0].dt, ws[0].nsteps)
    else:
        def run_once():
            for h, N, p, w in zip(hs, Ns, ps, ws):
                h.step(N, p, w.dt, w.nsteps)
    r = time_calls(run_once, hs, steps, warmup, ws[0].nsteps)
    for h in hs:
        h.close()
    return r


def measured_traffic(kernel):
    """Profiled HBM bytes per launch, or None if the kernel changed."""
    import hashlib
    entry = MEASURED_TRAFFIC.get(kernel)
    if entry is None:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2409_07232_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return entry[1] if h.hexdigest() == entry[0] else None


def roofline(res, peak, kernel=None):
    achieved = FLOPS_PER_PAIR * res["pair_evals"] / (res["kernel_ms"] * 1e-3)
    achieved /= 1e12
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 5),
            "traffic": measured_traffic(kernel) if kernel else None}


def _oracle_model(w, order=0):
    import oracle
    return oracle.OracleModel(w.nbins, w.nspecies, w.tables, w.p_levels,
                              w.product, x1_g=w.x1_g, s=w.s, theta=w.theta,
                              order=order)


def cpu_baseline(ws, seconds, nsteps, order=0):
    """The oracle on a seeded sample of cloudy points of each grid (sample
    sizes proportional to the grids' cloudy counts), grown until one run
    takes about `seconds`; the reported rate is that run's."""
    import numpy as np

    import oracle
    from paper_2409_07232_amd import workloads as wl
    cores = oracle.max_threads()
    ncloudy = [int(w.cloudy().sum()) for w in ws]
    share = [n / max(sum(ncloudy), 1) for n in ncloudy]
    # run full-length samples, rescaling the point count from each run's
    # time, until one takes at least a third of the target (or covers every
    # cloudy point); the last run is the one reported
    base = 16 * cores
    while True:
        npts = [min(nc, max(1, int(round(base * sh))))
                for sh, nc in zip(share, ncloudy)]
        samples = []
        t0 = time.perf_counter()
        for w, n in zip(ws, npts):
            idx = wl.sample_active(w, n, seed=11)
            sub = w.subset(idx)
            N = np.array(sub.N, copy=True)
            res = _oracle_model(w, order).run(N, sub.p, w.dt, nsteps,
                                              nthreads=cores)
            samples.append((idx, N, res["capped_per_point"] if order else
                            res["limiter_per_point"]))
        secs = time.perf_counter() - t0
        if secs >= seconds / 3 or all(n >= nc for n, nc in
                                      zip(npts, ncloudy)):
            break
        base = int(base * min(16.0, seconds / max(secs, 1e-3)))
    tot = sum(len(s[0]) for s in samples)
    desc = " + ".join("%d of %s" % (len(s[0]), w.name)
                      for s, w in zip(samples, ws))
    return {"value": round(tot * nsteps / secs, 1),
            "unit": "grid-point collision updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%s seeded cloudy points x %d steps of %.0f s of the "
                      "same workload, FP64%s, %.1f s" % (
                          desc, nsteps, ws[0].dt,
                          ", sequential form" if order else "", secs)}, \
        samples


def parity(ws, samples, nsteps, paths=None):
    """GPU results on the CPU-baseline sample against the oracle's (R15
    rel_bin; points the oracle limited judged with the 1e-3 floor)."""
    import numpy as np
    import torch

    from oracle import compare
    from paper_2409_07232_amd import _lib as L
    from paper_2409_07232_amd import workloads as wl
    out = {}
    if paths is None:
        paths = (("fp32c", L.FSBM_FP32C, 0), ("fp64", L.FSBM_FP64, 0))
    for name, prec, order in paths:
        err = drift = err_all = 0.0
        n_over = n_ill = 0
        for w, (idx, Nref, lim) in zip(ws, samples):
            sub = w.subset(idx)
            x = wl.bin_masses(w.nbins, w.s, w.x1_g)
            h = L.FsbmCoal.from_workload(w, precision=prec, order=order)
            N = torch.from_numpy(np.array(sub.N, copy=True)).to("cuda")
            p = torch.from_numpy(np.array(sub.p, copy=True)).to("cuda")
            h.step(N, p, w.dt, nsteps)
            got = N.cpu().numpy()
            h.close()
            floor = np.where(lim > 0, 1e-3, 1e-9)
            pe = compare.per_point_rel_bin(got, Nref, x, floor)
            if prec == L.FSBM_FP32C:
                # points over the FP32C tolerance whose own result is
                # unstable at FP32 precision (the oracle moves by more than
                # the tolerance under half-ulp input noise) are counted
                # apart; every other point is held to the tolerance
                over = np.nonzero(pe > FP32C_TOL)[0]
                n_over += len(over)
                if len(over):
                    unst = compare.unstable_points(
                        _oracle_model(w, order), sub.N[over], sub.p[over],
                        w.dt, nsteps, Nref[over], x, floor[over], FP32C_TOL)
                    n_ill += int(unst.sum())
                    err_all = max(err_all, float(pe.max()))
                    pe[over[unst]] = 0.0
            err = max(err, float(pe.max()) if pe.size else 0.0)
            drift = max(drift, compare.drift(got, sub.N, x))
        out[name] = {"rel_bin": float("%.3e" % err),
                     "drift": float("%.3e" % drift),
                     "limited_points": int(sum((s[2] > 0).sum()
                                               for s in samples)),
                     "points": int(sum(len(s[0]) for s in samples))}
        if prec == L.FSBM_FP32C:
            out[name].update({
                "points_over_tol": n_over,
                "ill_conditioned_at_fp32": n_ill,
                "rel_bin_incl_ill_conditioned": float(
                    "%.3e" % max(err, err_all))})
    return out


def make_workloads(args):
    """(workloads, config entry) of the selected benchmark workload."""
    from paper_2409_07232_amd import workloads as wl
    name = args.workload
    if name == "thunderstorm":
        ws = [wl.config2(nx=args.nx, ny=args.ny, nz=args.nz)]
        cfg = {"workload": "thunderstorm_patch_%dx%dx%d_33bins_liquid" % (
                   args.nx, args.ny, args.nz),
               "kernel_tables": "gravitational, 3 pressure levels"}
    elif name == "four_species":
        ws = [wl.config3(npoints=args.points or (1 << 20))]
        cfg = {"workload": "four_species_%dpts_33bins" % ws[0].npoints,
               "kernel_tables": "10 gravitational pair tables, 3 levels"}
    elif name.startswith("refined"):
        nb = int(name[len("refined"):])
        ws = [wl.config4(nbins=nb, npoints=args.points or 262144)]
        cfg = {"workload": "liquid_graupel_%dpts_%dbins" % (ws[0].npoints,
                                                             nb),
               "kernel_tables": "3 gravitational pair tables, 3 levels"}
    else:
        ws = wl.config5(npoints=args.points or (1 << 22))
        ws.sort(key=lambda w: -w.nspecies * w.nbins)
        cfg = {"workload": "mixed_grids_%dpts_10pct_cloudy_33_66_132bins" %
                           sum(w.npoints for w in ws),
               "kernel_tables": "per grid, 3 levels"}
    if args.collision_steps:
        for w in ws:
            w.nsteps = args.collision_steps
    return ws, cfg


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
    log("generating workload %s" % args.workload)
    ws, cfg = make_workloads(args)
    N0s = [torch.from_numpy(w.N).to("cuda") for w in ws]
    ps = [torch.from_numpy(w.p).to("cuda") for w in ws]
    multi = len(ws) > 1
    log("timing fp32c: %d warmup + %d steps" % (args.warmup, args.steps))
    if multi:
        r32 = time_multi(ws, L.FSBM_FP32C, args.steps, args.warmup, N0s, ps,
                         batched=True)
    else:
        r32 = time_path(ws[0], L.FSBM_FP32C, args.steps, args.warmup, N0s[0],
                        ps[0])
    log("fp32c %.2f ms/step, %.3e updates/s" % (r32["ms_per_step"],
                                               r32["updates_per_s"]))
    r64 = None
    if not args.no_fp64:
        log("timing fp64" + (" (per-grid launches)" if multi else ""))
        if multi:
            r64 = time_multi(ws, L.FSBM_FP64, args.steps, args.warmup, N0s,
                             ps, batched=False)
        else:
            r64 = time_path(ws[0], L.FSBM_FP64, args.steps, args.warmup,
                            N0s[0], ps[0])
        log("fp64 %.2f ms/step, %.3e updates/s" % (r64["ms_per_step"],
                                                  r64["updates_per_s"]))
    rsq = None
    if not args.no_sequential and not multi and ws[0].nspecies == 1:
        log("timing the sequential form (fp64)")
        rsq = time_path(ws[0], L.FSBM_FP64, args.steps, args.warmup, N0s[0],
                        ps[0], order=L.ORDER_SEQUENTIAL)
        log("sequential %.2f ms/step, %.3e updates/s" % (
            rsq["ms_per_step"], rsq["updates_per_s"]))
    del N0s
    nsteps = ws[0].nsteps
    cpu = par = None
    if not args.no_cpu_baseline:
        csteps = args.cpu_steps or nsteps
        log("cpu baseline (oracle), about %.0f s" % args.cpu_seconds)
        cpu, samples = cpu_baseline(ws, args.cpu_seconds, csteps)
        log("cpu %.3e updates/s on %d cores (%s)" % (cpu["value"],
                                                    cpu["cores"],
                                                    cpu["sample"]))
        par = parity(ws, samples, csteps)
        if rsq is not None:
            log("cpu baseline of the sequential form (oracle), about %.0f s"
                % (args.cpu_seconds / 3))
            cpu_sq, samples_sq = cpu_baseline(ws, args.cpu_seconds / 3,
                                              csteps, order=1)
            par_sq = parity(ws, samples_sq, csteps,
                            paths=(("fp64", L.FSBM_FP64, 1),))
    w0 = ws[0]
    cfg.update({"points": sum(w.npoints for w in ws),
                "cloudy_points": r32["active_points"],
                "bins": [w.nbins for w in ws] if multi else w0.nbins,
                "species": [w.nspecies for w in ws] if multi else
                w0.nspecies,
                "dt_s": w0.dt, "collision_steps_per_step": nsteps,
                "parallelism": "single GPU"})
    if multi:
        cfg["launch"] = ("fp32c: one persistent launch over all grids per "
                         "fused-step group; fp64: one call per grid")
    npts_all = sum(w.npoints for w in ws)

    def rates(r):
        # every grid point of the workload (cloud-free ones take no work)
        # and every evaluated bin pair, per second of the timed calls
        return {"all_points_per_s": round(npts_all * nsteps * args.steps /
                                          r["secs"], 1),
                "pairs_per_s": round(r["pair_evals"] / r["secs"], 1)}

    line = {
        "metric": "grid-point collision updates/s at 33 bins; FP32-comp vs "
                  "FP64, rel err <=1e-5",
        "value": round(r32["updates_per_s"], 1),
        "unit": "grid-point collision updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": cfg,
        "roofline": roofline(r32, PEAK_FP32_TFLOPS,
                             kernel_name(r32["stats"], 1, w0.nbins)),
        "kernel": {"name": kernel_name(r32["stats"], 1, w0.nbins),
                   "avg_launch_ms": round(r32["kernel_avg_ms"], 4),
                   "launches": r32["kernel_launches"],
                   "pair_evals": r32["pair_evals"],
                   "pairs_per_point_step": round(
                       r32["pair_evals"] / max(1, r32["active_points"] *
                                               nsteps * args.steps), 1),
                   "flops_per_pair": FLOPS_PER_PAIR,
                   "steps_per_launch": r32["stats"]["steps_per_launch"],
                   "limiter_steps": r32["limiter_steps"],
                   "fallback_steps": r32["fallback_steps"]},
        "rates": rates(r32),
    }
    if r64 is not None:
        line["fp64"] = {"value": round(r64["updates_per_s"], 1),
                        "ms_per_step": round(r64["ms_per_step"], 4),
                        "dtype": "f64",
                        "kernel": kernel_name(r64["stats"], 0, w0.nbins),
                        "roofline": roofline(r64, PEAK_FP64_TFLOPS),
                        "avg_launch_ms": round(r64["kernel_avg_ms"], 4),
                        "rates": rates(r64)}
    if rsq is not None:
        line["sequential"] = {
            "form": "Bott's in-place pair order, FP64",
            "value": round(rsq["updates_per_s"], 1),
            "unit": "grid-point collision updates/s",
            "ms_per_step": round(rsq["ms_per_step"], 4), "dtype": "f64",
            "kernel": kernel_name(rsq["stats"], 0, w0.nbins),
            "roofline": roofline(rsq, PEAK_FP64_TFLOPS),
            "avg_launch_ms": round(rsq["kernel_avg_ms"], 4),
            "pair_evals": rsq["pair_evals"],
            "capped_pairs": rsq["limiter_steps"],
            "rates": rates(rsq)}
        if cpu is not None:
            line["sequential"]["cpu_baseline"] = cpu_sq
            line["sequential"]["parity_on_cpu_sample"] = par_sq["fp64"]
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
