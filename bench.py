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
steps / time) of the FP32-compensated path, timed as the library runs by
default: each call replays its captured hipGraph on a non-default stream.
The plain FP64 path is reported beside it.  The roofline entry is for the
dominant kernel (the collision step kernel): a few more calls on separate
handles launch the kernels directly and time each collision-kernel launch
with HIP events on the stream it runs on; achieved = algorithmic flops of
the pairs those launches evaluated / their summed duration.  The CPU
baseline is the FP64 oracle on a bounded sample of the same workload.

The default run also measures the four-species workload (2^20 points,
liquid/ice/snow/graupel, 33 bins), the second 33-bin configuration, under
the key "four_species".

--workload selects the other measured shapes (each prints its own line with
the same fields):
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

# Algorithmic work per evaluated bin pair: 24 floating-point operations
# (interpolated kernel 2, collided masses 5, merged mass 1, neighbour ratio
# 2, slope 2, flux fraction 4, clamps 2, flux 1, net combine 2, per-bin
# accumulation 4: the operations of one pair's update as the method states
# it), plus 2 divisions and 3 transcendentals (log, exp, expm1) that are not
# counted as flops.  OPS_PER_PAIR_ALL counts each of those once as well.
FLOPS_PER_PAIR = 24
OPS_PER_PAIR_ALL = 29
FP32C_TOL = 1e-5           # rel_bin bar of the FP32C path
FLOOR = 1e-9               # rel_bin floor (fraction of the point's mass)
LIMITED_FLOOR = 1e-3       # floor of the bins the oracle's limiter scaled
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64 (published)

# HBM bytes per launch of a kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs scaled by the same counters on a 1 GiB device copy (the profile
# summary under profiles/ gives the commands).  They hold only for the
# kernel sources they were taken on: the SHA-256 of the concatenated files
# below must match, otherwise the traffic entry is reported as null.
LANE_SOURCES = ("kernels_lane.hip", "device_common.hpp", "fp64_math.hpp",
                "slow_path.hpp")
_PROF_LANE = "profiles/lane_step_thunderstorm_256x256x50.md"
_PROF_LIQ = "profiles/cond_brk_thunderstorm_256x256x50.md"
MEASURED_TRAFFIC = {
    # (kernel, workload): (sources, their sha256, HBM bytes per launch,
    # profile summary)
    ("lane_step_f32c<33>", "thunderstorm_patch_256x256x50_33bins_liquid"): (
        LANE_SOURCES,
        "f6d1ade88a1b6d690439e81f670bc3a8ae865d7d744d9f968b6162bb46b754b6",
        4.1020e9, _PROF_LANE),
    ("lane_step_f64<33>", "thunderstorm_patch_256x256x50_33bins_liquid"): (
        LANE_SOURCES,
        "f6d1ade88a1b6d690439e81f670bc3a8ae865d7d744d9f968b6162bb46b754b6",
        2.9020e9, _PROF_LANE),
    ("lane_seq_f64<33>", "thunderstorm_patch_256x256x50_33bins_liquid"): (
        ("kernels_seq.hip", "device_common.hpp", "fp64_math.hpp"),
        "e3d3533ecc1db38a43a7235d0aca79d908879dc407321d5ca9978f3076c4b3d9",
        2.671e8, _PROF_LANE),
    # the four launches (NS = 1..4) of a group of steps together
    ("lane_multi_f32c<33,NS=1..4>", "four_species_1048576pts_33bins"): (
        ("kernels_multi.hip", "device_common.hpp", "fp64_math.hpp"),
        "7af86f1ccac6ca324a79a6f47cb61d7cbb72de42e50dcc87239980aae7c326fe",
        1.7022e10,
        "profiles/lane_multi_four_species_1048576x33.md"),
    # the FP64 path's 10-step launches (scratch of spilled registers
    # included)
    ("wave_step<F64>", "four_species_1048576pts_33bins"): (
        ("kernels_wave.hip", "device_common.hpp", "fp64_math.hpp"),
        "236bf87b9101be5cc136069b4072f863b97c311810b25e69096d368f34ac0e4b",
        3.898e10,
        "profiles/lane_multi_four_species_1048576x33.md"),
    ("cond_steps<33>", "thunderstorm_patch_256x256x50_33bins_liquid_"
                       "prescribed_supersaturation"): (
        ("condense.hip", "device_common.hpp", "fp64_math.hpp"),
        "88378ab700895a482b5cf270ba2fd0056e0e5f61f2a23c8a4a6290a20f7d4518",
        4.0955e8, _PROF_LIQ),
    ("brk_steps<33>", "thunderstorm_patch_256x256x50_33bins_liquid_"
                      "spontaneous_breakup"): (
        ("breakup.hip", "condense.hip", "device_common.hpp",
         "fp64_math.hpp"),
        "838efcfb004611665b84befbef40e45b5ffc80ad4c8e9303b00fd9ef1bb45a17",
        3.2392e8, _PROF_LIQ),
    ("sed_steps<56>",
     "thunderstorm_patch_columns_256x256_50lev_33bins_liquid"): (
        ("sediment.hip", "device_common.hpp", "fp64_math.hpp"),
        "23565fac77e596e16f2e9df62d3c97ee586c471c80af0d8eecb610409c07c3d1",
        1.8177e9, "profiles/sed_steps_thunderstorm_columns_65536x50.md"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--profiled-calls", type=int, default=2,
                    help="calls with per-launch HIP-event timing after the "
                         "timed ones (kernel time of the roofline entry)")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 path beside the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the sequential (in-place) form, timed beside "
                         "the headline on the thunderstorm workload")
    ap.add_argument("--no-four-species", action="store_true",
                    help="skip the four-species entry of the default run")
    ap.add_argument("--no-sediment", action="store_true",
                    help="skip the sedimentation entry of the default run")
    ap.add_argument("--no-condense", action="store_true",
                    help="skip the condensation entry of the default run")
    ap.add_argument("--no-breakup", action="store_true",
                    help="skip the breakup entry of the default run")
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
    if st["kernel"] == 3:
        return "lane_multi_f32c<%d,NS=1..4>" % nbins
    return "wave_step<%s>" % ("F32" if f32 else "F64")


def _handles(ws, precision, order=0, flags=0):
    from paper_2409_07232_amd import _lib as L
    return [L.FsbmCoal.from_workload(w, precision=precision, order=order,
                                     flags=flags) for w in ws]


def _runner(hs, ws, Ns, ps, batched, stream):
    """One benchmark step: one fsbm_coal_step_multi call (batched) or one
    fsbm_coal_step call per grid, on `stream`."""
    from paper_2409_07232_amd import _lib as L
    if batched:
        def run_once():
            L.step_multi(hs, Ns, ps, ws[0].dt, ws[0].nsteps, stream=stream)
    else:
        def run_once():
            for h, N, p, w in zip(hs, Ns, ps, ws):
                h.step(N, p, w.dt, w.nsteps, stream=stream)
    return run_once


def measure(ws, precision, args, N0s, ps, batched=False, order=0,
            label=""):
    """Time `args.steps` calls (after `args.warmup`) through the library's
    default path: a captured hipGraph replayed on a non-default stream.
    Then `args.profiled_calls` more calls on separate handles with
    FSBM_FLAG_PROFILE (direct launches, each collision-kernel launch timed
    with HIP events on its stream), continuing from the same state, give
    the kernel time and the pairs those launches evaluated."""
    import torch
    nsteps = ws[0].nsteps
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    hs = _handles(ws, precision, order)
    Ns = [n.clone() for n in N0s]
    torch.cuda.synchronize()
    run_once = _runner(hs, ws, Ns, ps, batched, s)
    for k in range(args.warmup):
        run_once()
        s.synchronize()
        log("%s warm-up call %d done" % (label, k + 1))
    pairs = exact = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        run_once()
        sts = [h.stats() for h in hs]   # synchronises the stream
        pairs += sum(st["pair_evals"] for st in sts)
        exact += sum(st["exact_pair_evals"] for st in sts)
        log("%s timed call %d done, %.1f s so far" % (
            label, k + 1, time.perf_counter() - t0))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    sts = [h.stats() for h in hs]
    active = sum(st["active_points"] for st in sts)
    res = {"secs": secs, "ms_per_step": 1e3 * secs / args.steps,
           "updates_per_s": active * nsteps * args.steps / secs,
           "active_points": active, "pair_evals": pairs,
           "exact_pair_evals": exact,
           "limiter_steps": sum(st["limiter_steps"] for st in sts),
           "fallback_steps": sum(st["fp64_fallback_steps"] for st in sts),
           "graph_captures": sum(st["graph_captures"] for st in sts),
           "stats": sts[0]}
    for h in hs:
        h.close()
    # profiled calls: the timed ones' final state, launched directly
    from paper_2409_07232_amd import _lib as L
    hp = _handles(ws, precision, order, flags=L.FLAG_PROFILE)
    run_prof = _runner(hp, ws, Ns, ps, batched, s)
    ppairs = pexact = 0
    t0 = time.perf_counter()
    for k in range(args.profiled_calls):
        run_prof()
        sts = [h.stats() for h in hp]
        ppairs += sum(st["pair_evals"] for st in sts)
        pexact += sum(st["exact_pair_evals"] for st in sts)
    s.synchronize()
    psecs = time.perf_counter() - t0
    sts = [h.stats() for h in hp]
    launches = sum(st["kernel_launches"] for st in sts)
    kms = sum(st["kernel_ms"] for st in sts)
    res.update({"prof_calls": args.profiled_calls,
                "prof_updates_per_s": active * nsteps *
                args.profiled_calls / max(psecs, 1e-9),
                "prof_pair_evals": ppairs, "prof_exact_pair_evals": pexact,
                "kernel_launches": launches, "kernel_ms": kms,
                "kernel_avg_ms": kms / max(launches, 1)})
    for h in hp:
        h.close()
    return res


def measured_traffic(kernel, workload):
    """Profiled HBM bytes per launch of a kernel on a workload, or None if
    there is no such record or the kernel changed since."""
    import hashlib
    entry = MEASURED_TRAFFIC.get((kernel, workload))
    if entry is None:
        return None
    h = hashlib.sha256()
    for f in entry[0]:
        with open(os.path.join(ROOT, "paper_2409_07232_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return entry[2] if h.hexdigest() == entry[1] else None


def roofline(res, peak, kernel, workload):
    """The collision kernel's algorithmic rate over its profiled launches:
    pairs the fast kernel evaluated (the exact FP64 path's pairs left out)
    x FLOPS_PER_PAIR / summed launch time."""
    fast = res["prof_pair_evals"] - res["prof_exact_pair_evals"]
    secs = max(res["kernel_ms"], 1e-9) * 1e-3
    achieved = FLOPS_PER_PAIR * fast / secs / 1e12
    all_ops = OPS_PER_PAIR_ALL * fast / secs / 1e12
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 5),
            "traffic": measured_traffic(kernel, workload),
            "flops_per_pair": FLOPS_PER_PAIR,
            "ops_per_pair_incl_div_transc": OPS_PER_PAIR_ALL,
            "frac_incl_div_transc": round(all_ops / peak, 5),
            "pairs_per_launch": round(fast / max(res["kernel_launches"], 1))}


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
            per_point = (res["capped_per_point"] if order else
                         res["limiter_per_point"])
            samples.append((idx, N, per_point, res["limited_bins"]))
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
    rel_bin with the 1e-9 floor; only the bins the oracle's limiter scaled
    are judged with the 1e-3 floor).  FP32C points over the tolerance whose
    own result is unstable at FP32 precision are counted apart."""
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
        for w, (idx, Nref, lim, lim_bins) in zip(ws, samples):
            sub = w.subset(idx)
            x = wl.bin_masses(w.nbins, w.s, w.x1_g)
            h = L.FsbmCoal.from_workload(w, precision=prec, order=order)
            N = torch.from_numpy(np.array(sub.N, copy=True)).to("cuda")
            p = torch.from_numpy(np.array(sub.p, copy=True)).to("cuda")
            h.step(N, p, w.dt, nsteps)
            got = N.cpu().numpy()
            h.close()
            floor = np.where(lim_bins, LIMITED_FLOOR, FLOOR)
            pe = compare.per_point_rel_bin(got, Nref, x, floor)
            if prec == L.FSBM_FP32C:
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
                     "limited_bins": int(sum(s[3].sum() for s in samples)),
                     "points": int(sum(len(s[0]) for s in samples))}
        if prec == L.FSBM_FP32C:
            out[name].update({
                "points_over_tol": n_over,
                "ill_conditioned_at_fp32": n_ill,
                "rel_bin_incl_ill_conditioned": float(
                    "%.3e" % max(err, err_all))})
    return out


def make_workloads(args, name=None):
    """(workloads, config entry) of a benchmark workload."""
    from paper_2409_07232_amd import workloads as wl
    name = name or args.workload
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


def _rates(r, npts_all, nsteps, steps):
    # every grid point of the workload (cloud-free ones take no work) and
    # every evaluated bin pair, per second of the timed calls
    return {"all_points_per_s": round(npts_all * nsteps * steps /
                                      r["secs"], 1),
            "pairs_per_s": round(r["pair_evals"] / r["secs"], 1)}


def _kernel_entry(r, name, nsteps, steps):
    return {"name": name,
            "avg_launch_ms": round(r["kernel_avg_ms"], 4),
            "launches_profiled": r["kernel_launches"],
            "profiled_calls": r["prof_calls"],
            "pair_evals_timed_calls": r["pair_evals"],
            "exact_path_pair_evals_timed_calls": r["exact_pair_evals"],
            "pairs_per_point_step": round(
                r["pair_evals"] / max(1, r["active_points"] * nsteps *
                                      steps), 1),
            "steps_per_launch": r["stats"]["steps_per_launch"],
            "limiter_steps": r["limiter_steps"],
            "fallback_steps": r["fallback_steps"]}


def _timing_entry(r):
    return {"value_path": "captured hipGraph replayed on a non-default "
                          "stream (the library's default)",
            "graph_captures": r["graph_captures"],
            "profiled_path_updates_per_s": round(r["prof_updates_per_s"],
                                                 1)}


def run_workload(args, name, steps, warmup, cpu_seconds, with_seq):
    """Measure one workload: FP32C (headline), FP64, optionally the
    sequential form, the CPU baseline and parity on its sample.  Returns
    the entry of the JSON line (without the top-level keys)."""
    import torch

    from paper_2409_07232_amd import _lib as L

    class A:
        pass
    a = A()
    a.__dict__.update(vars(args))
    a.steps, a.warmup = steps, warmup
    log("generating workload %s" % name)
    ws, cfg = make_workloads(args, name)
    N0s = [torch.from_numpy(w.N).to("cuda") for w in ws]
    ps = [torch.from_numpy(w.p).to("cuda") for w in ws]
    multi = len(ws) > 1
    nsteps = ws[0].nsteps
    w0 = ws[0]
    npts_all = sum(w.npoints for w in ws)
    log("%s fp32c: %d warm-up + %d timed calls" % (name, warmup, steps))
    r32 = measure(ws, L.FSBM_FP32C, a, N0s, ps, batched=multi,
                  label=name + " fp32c")
    log("%s fp32c %.2f ms/call, %.3e updates/s" % (
        name, r32["ms_per_step"], r32["updates_per_s"]))
    r64 = None
    if not args.no_fp64:
        r64 = measure(ws, L.FSBM_FP64, a, N0s, ps, batched=False,
                      label=name + " fp64")
        log("%s fp64 %.2f ms/call, %.3e updates/s" % (
            name, r64["ms_per_step"], r64["updates_per_s"]))
    rsq = None
    if with_seq and not multi and w0.nspecies == 1:
        rsq = measure(ws, L.FSBM_FP64, a, N0s, ps, order=L.ORDER_SEQUENTIAL,
                      label=name + " sequential")
        log("%s sequential %.2f ms/call, %.3e updates/s" % (
            name, rsq["ms_per_step"], rsq["updates_per_s"]))
    del N0s
    cfg.update({"points": npts_all,
                "cloudy_points": r32["active_points"],
                "bins": [w.nbins for w in ws] if multi else w0.nbins,
                "species": [w.nspecies for w in ws] if multi else
                w0.nspecies,
                "dt_s": w0.dt, "collision_steps_per_step": nsteps,
                "accumulate": "fp64 (FP32 pair amounts summed per bin in "
                              "FP64, FP64 totals and update)",
                "parallelism": "single GPU"})
    if multi:
        cfg["launch"] = ("fp32c: one persistent launch over all grids per "
                         "fused-step group; fp64: one call per grid")
    k32 = kernel_name(r32["stats"], 1, w0.nbins)
    ent = {"value": round(r32["updates_per_s"], 1),
           "ms_per_step": round(r32["ms_per_step"], 4),
           "config": cfg,
           "roofline": roofline(r32, PEAK_FP32_TFLOPS, k32, cfg["workload"]),
           "kernel": _kernel_entry(r32, k32, nsteps, steps),
           "timing": _timing_entry(r32),
           "rates": _rates(r32, npts_all, nsteps, steps)}
    if r64 is not None:
        k64 = kernel_name(r64["stats"], 0, w0.nbins)
        ent["fp64"] = {"value": round(r64["updates_per_s"], 1),
                       "ms_per_step": round(r64["ms_per_step"], 4),
                       "dtype": "f64",
                       "roofline": roofline(r64, PEAK_FP64_TFLOPS, k64,
                                            cfg["workload"]),
                       "kernel": _kernel_entry(r64, k64, nsteps, steps),
                       "timing": _timing_entry(r64),
                       "rates": _rates(r64, npts_all, nsteps, steps)}
    if rsq is not None:
        ksq = kernel_name(rsq["stats"], 0, w0.nbins)
        ent["sequential"] = {
            "form": "Bott's in-place pair order, FP64",
            "value": round(rsq["updates_per_s"], 1),
            "unit": "grid-point collision updates/s",
            "ms_per_step": round(rsq["ms_per_step"], 4), "dtype": "f64",
            "roofline": roofline(rsq, PEAK_FP64_TFLOPS, ksq,
                                 cfg["workload"]),
            "kernel": _kernel_entry(rsq, ksq, nsteps, steps),
            "capped_pairs": rsq["limiter_steps"],
            "timing": _timing_entry(rsq),
            "rates": _rates(rsq, npts_all, nsteps, steps)}
    if not args.no_cpu_baseline:
        csteps = args.cpu_steps or nsteps
        log("%s cpu baseline (oracle), about %.0f s" % (name, cpu_seconds))
        cpu, samples = cpu_baseline(ws, cpu_seconds, csteps)
        log("%s cpu %.3e updates/s on %d cores (%s)" % (
            name, cpu["value"], cpu["cores"], cpu["sample"]))
        ent["cpu_baseline"] = cpu
        ent["parity_on_cpu_sample"] = parity(ws, samples, csteps)
        if rsq is not None:
            log("%s cpu baseline of the sequential form, about %.0f s" % (
                name, cpu_seconds / 3))
            cpu_sq, samples_sq = cpu_baseline(ws, cpu_seconds / 3, csteps,
                                              order=1)
            ent["sequential"]["cpu_baseline"] = cpu_sq
            ent["sequential"]["parity_on_cpu_sample"] = parity(
                ws, samples_sq, csteps,
                paths=(("fp64", L.FSBM_FP64, 1),))["fp64"]
    return ent


def _sed_level_updates(geo, dt, nsteps):
    """(column, species-bin, level) updates of a sedimentation call,
    sub-steps included (the kernel's own count of sub-steps)."""
    import numpy as np
    c = (geo["v_cm_s"].reshape(1, 1, -1) * geo["vfac"][:, :, None] * dt /
         geo["dz_cm"][None, :, None]).max(axis=1)       # [ncols][S*B]
    nsub = np.maximum(np.ceil(c), 1.0)
    return float(nsub.sum()) * nsteps * geo["nlev"]


def run_sediment(args, steps, warmup):
    """Sedimentation of the thunderstorm patch's 65,536 columns of 50
    levels (the vertical term of eq. (1)), one call of the workload's 100
    steps of 2 s per benchmark step, FP64, timed like the collision path;
    kernel time from HIP events on the call's stream; the oracle on a
    sample of columns on the host cores."""
    import numpy as np
    import torch

    import oracle
    from paper_2409_07232_amd import _lib as L
    from paper_2409_07232_amd import workloads as wl
    w = wl.config2(nx=args.nx, ny=args.ny, nz=args.nz)
    geo = wl.sediment_geometry(w)
    dt, nsteps = w.dt, w.nsteps
    h = L.FsbmCoal.from_workload(w, precision=0)
    N = torch.from_numpy(w.N).to("cuda")
    dz = torch.from_numpy(geo["dz_cm"]).to("cuda")
    v = torch.from_numpy(geo["v_cm_s"]).to("cuda")
    vf = torch.from_numpy(geo["vfac"]).to("cuda")
    pr = torch.zeros((geo["ncols"], 1, w.nbins), dtype=torch.float64,
                     device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())

    def call():
        h.sediment(N, geo["ncols"], geo["nlev"], geo["col_stride"],
                   geo["lev_stride"], dz, v, vf, dt, nsteps, pr, stream=s)
    for _ in range(warmup):
        call()
    s.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        call()
    e1.record(s)
    s.synchronize()
    secs = time.perf_counter() - t0
    kms = e0.elapsed_time(e1) / max(steps, 1)
    npts = w.npoints
    upd = _sed_level_updates(geo, dt, nsteps)
    flops = 6.0 * upd                      # per level update: 3 mul, sub,
    bytes_ = 16.0 * npts * w.nbins + 8.0 * npts + \
        16.0 * geo["ncols"] * w.nbins      # (div, add); state, factors,
    log("sedimentation %.3f ms/call" % (1e3 * secs / steps))  # precip
    ent_workload = "thunderstorm_patch_columns_%dx%d_%dlev_33bins_liquid" % (
        args.nx, args.ny, args.nz)
    # the kernel's register array of levels
    sed_kernel = "sed_steps<%d>" % (32 if args.nz <= 32 else
                                    (56 if args.nz <= 56 else 64))
    ent = {"form": "first-order upwind flux form, still air, sub-stepped "
                   "to Courant numbers <= 1, FP64",
           "value": round(npts * nsteps * steps / secs, 1),
           "unit": "grid-point sedimentation updates/s",
           "ms_per_step": round(1e3 * secs / steps, 4), "dtype": "f64",
           "config": {"workload": ent_workload,
                      "columns": geo["ncols"], "levels": geo["nlev"],
                      "dt_s": dt, "steps_per_call": nsteps,
                      "level_updates_per_call": upd},
           "kernel": {"name": sed_kernel, "avg_call_ms": round(kms, 4)},
           "roofline": {"bound": "alu", "achieved":
                        round(flops / (kms * 1e-3) / 1e12, 4),
                        "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(flops / (kms * 1e-3) / 1e12 /
                                      PEAK_FP64_TFLOPS, 5),
                        "traffic": measured_traffic(sed_kernel,
                                                    ent_workload),
                        "flops_per_level_update": 6,
                        "hbm_bytes_per_call_algorithmic": bytes_,
                        "hbm_gbs_algorithmic": round(bytes_ / (kms * 1e-3)
                                                     / 1e9, 1)}}
    h.close()
    if not args.no_cpu_baseline:
        # the oracle on seeded columns, grown to about 5 s
        rng = np.random.default_rng(12)
        cores = oracle.max_threads()
        ncol = 64
        while True:
            cols = np.sort(rng.choice(geo["ncols"], ncol, replace=False))
            idx = cols[:, None] + np.arange(geo["nlev"])[None, :] * \
                geo["lev_stride"]
            sub = np.ascontiguousarray(w.N[idx]).reshape(-1, 1, w.nbins)
            t0 = time.perf_counter()
            oracle.sediment(sub, geo["dz_cm"], geo["v_cm_s"], dt, nsteps,
                            vfac=geo["vfac"][cols], col_stride=geo["nlev"],
                            lev_stride=1)
            cs = time.perf_counter() - t0
            if cs >= 1.5 or ncol >= geo["ncols"]:
                break
            ncol = min(geo["ncols"], ncol * 4)
        ent["cpu_baseline"] = {
            "value": round(ncol * geo["nlev"] * nsteps / cs, 1),
            "unit": "grid-point sedimentation updates/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d seeded columns x %d levels x %d steps, %.1f s" % (
                ncol, geo["nlev"], nsteps, cs)}
    return ent


def run_condense(args, steps, warmup):
    """Condensation/evaporation of the thunderstorm patch's drop spectra at
    the seeded supersaturation mix (fsbm_coal_condense), one call of the
    workload's 100 steps of 2 s per benchmark step, FP64, timed like the
    collision path; call time from HIP events on the call's stream; the
    oracle on a sample of cloudy points on one host core."""
    import numpy as np
    import torch

    import oracle
    from paper_2409_07232_amd import _lib as L
    from paper_2409_07232_amd import workloads as wl
    w = wl.config2(nx=args.nx, ny=args.ny, nz=args.nz)
    ssat, g = wl.condensation_inputs(w)
    dt, nsteps = w.dt, w.nsteps
    h = L.FsbmCoal.from_workload(w, precision=0)
    N0 = torch.from_numpy(w.N).to("cuda")
    N = N0.clone()
    sd = torch.from_numpy(ssat).to("cuda")
    gd = torch.from_numpy(g).to("cuda")
    ev = torch.zeros(w.npoints, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())

    def call():
        h.condense(N, sd, gd, dt, nsteps, ev, stream=s)
    for _ in range(warmup):
        call()
    s.synchronize()
    # the timed calls continue one another from the workload's state
    N.copy_(N0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        call()
    e1.record(s)
    s.synchronize()
    secs = time.perf_counter() - t0
    kms = e0.elapsed_time(e1) / max(steps, 1)
    act = w.cloudy() & (g * ssat != 0.0)
    nact = int(act.sum())
    # all 33 bins of a cloudy point hold drops (untruncated gamma spectra)
    bins = float(np.count_nonzero(w.N[act, 0, :]))
    flops = 12.0 * bins * nsteps
    # state and evaporated mass of the active points read and written, s
    # and G of every point read, the rows of the dry points scanned
    bytes_ = 16.0 * (w.nbins + 1) * nact + 16.0 * w.npoints + \
        8.0 * w.nbins * (w.npoints - nact)
    h.close()
    log("condensation %.3f ms/call" % (1e3 * secs / steps))
    ent_workload = ("thunderstorm_patch_%dx%dx%d_33bins_liquid_prescribed_"
                    "supersaturation" % (args.nx, args.ny, args.nz))
    ent = {"form": "r dr/dt = G s growth, number- and mass-keeping "
                   "remapping onto the bin grid, FP64",
           "value": round(nact * nsteps * steps / secs, 1),
           "unit": "grid-point condensation updates/s",
           "ms_per_step": round(1e3 * secs / steps, 4), "dtype": "f64",
           "config": {"workload": ent_workload,
                      "points": w.npoints, "active_points": nact,
                      "dt_s": dt, "steps_per_call": nsteps},
           "kernel": {"name": "cond_steps<33>", "avg_call_ms": round(kms, 4)},
           "roofline": {"bound": "alu", "achieved":
                        round(flops / (kms * 1e-3) / 1e12, 4),
                        "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(flops / (kms * 1e-3) / 1e12 /
                                      PEAK_FP64_TFLOPS, 5),
                        "traffic": measured_traffic(
                            "cond_steps<33>", ent_workload),
                        "flops_per_bin_update": 12,
                        "hbm_bytes_per_call_algorithmic": bytes_}}
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(13)
        pts = np.flatnonzero(act)
        n = 256
        while True:
            idx = np.sort(rng.choice(pts, min(n, pts.size), replace=False))
            sub = np.ascontiguousarray(w.N[idx])
            t0 = time.perf_counter()
            oracle.condense(sub, ssat[idx], g[idx], dt, nsteps, s=w.s,
                            x1_g=w.x1_g)
            cs = time.perf_counter() - t0
            if cs >= 1.5 or n >= pts.size:
                break
            n = min(pts.size, n * 4)
        ent["cpu_baseline"] = {
            "value": round(idx.size * nsteps / cs, 1),
            "unit": "grid-point condensation updates/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d seeded cloudy points x %d steps, %.1f s" % (
                idx.size, nsteps, cs)}
    return ent


def run_breakup(args, steps, warmup):
    """Spontaneous breakup of the thunderstorm patch's drop spectra
    (fsbm_coal_breakup) with the seeded rate and fragment tables, one call
    of the workload's 100 steps of 2 s per benchmark step, FP64, timed like
    the collision path; the oracle on a sample of cloudy points on one host
    core."""
    import numpy as np
    import torch

    import oracle
    from paper_2409_07232_amd import _lib as L
    from paper_2409_07232_amd import workloads as wl
    w = wl.config2(nx=args.nx, ny=args.ny, nz=args.nz)
    rate, Q = wl.breakup_tables(w.nbins, w.s, w.x1_g)
    dt, nsteps = w.dt, w.nsteps
    h = L.FsbmCoal.from_workload(w, precision=0)
    h.set_breakup(rate, Q)
    N0 = torch.from_numpy(w.N).to("cuda")
    N = N0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())

    def call():
        h.breakup(N, dt, nsteps, stream=s)
    for _ in range(warmup):
        call()
    s.synchronize()
    # the timed calls continue one another from the workload's state
    N.copy_(N0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        call()
    e1.record(s)
    s.synchronize()
    secs = time.perf_counter() - t0
    kms = e0.elapsed_time(e1) / max(steps, 1)
    h.close()
    act = (w.N[:, 0, 1:] != 0.0).any(axis=1)
    nact = int(act.sum())
    B = w.nbins
    # per point-step: B products b_l N_l, B differences, B (B - 1) / 2
    # multiply-add pairs of the fragment sums
    flops = float(B * B + B) * nact * nsteps
    bytes_ = 16.0 * B * nact + 8.0 * B * (w.npoints - nact)
    log("breakup %.3f ms/call" % (1e3 * secs / steps))
    ent_workload = ("thunderstorm_patch_%dx%dx%d_33bins_liquid_spontaneous_"
                    "breakup" % (args.nx, args.ny, args.nz))
    ent = {"form": "linear spontaneous breakup, share 1 - exp(-P dt) of "
                   "each bin per step into a fragment table, FP64",
           "value": round(nact * nsteps * steps / secs, 1),
           "unit": "grid-point breakup updates/s",
           "ms_per_step": round(1e3 * secs / steps, 4), "dtype": "f64",
           "config": {"workload": ent_workload,
                      "points": w.npoints, "active_points": nact,
                      "dt_s": dt, "steps_per_call": nsteps},
           "kernel": {"name": "brk_steps<33>", "avg_call_ms": round(kms, 4)},
           "roofline": {"bound": "alu", "achieved":
                        round(flops / (kms * 1e-3) / 1e12, 4),
                        "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(flops / (kms * 1e-3) / 1e12 /
                                      PEAK_FP64_TFLOPS, 5),
                        "traffic": measured_traffic(
                            "brk_steps<33>", ent_workload),
                        "flops_per_point_step": B * B + B,
                        "hbm_bytes_per_call_algorithmic": bytes_}}
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(14)
        pts = np.flatnonzero(act)
        n = 256
        while True:
            idx = np.sort(rng.choice(pts, min(n, pts.size), replace=False))
            sub = np.ascontiguousarray(w.N[idx])
            t0 = time.perf_counter()
            oracle.breakup(sub, rate, Q, dt, nsteps)
            cs = time.perf_counter() - t0
            if cs >= 1.5 or n >= pts.size:
                break
            n = min(pts.size, n * 4)
        ent["cpu_baseline"] = {
            "value": round(idx.size * nsteps / cs, 1),
            "unit": "grid-point breakup updates/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d seeded cloudy points x %d steps, %.1f s" % (
                idx.size, nsteps, cs)}
    return ent


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
    ent = run_workload(args, args.workload, args.steps, args.warmup,
                       args.cpu_seconds, not args.no_sequential)
    line = {
        "metric": "grid-point collision updates/s at 33 bins; FP32-comp vs "
                  "FP64, rel err <=1e-5",
        "value": ent.pop("value"),
        "unit": "grid-point collision updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ent.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": ent.pop("config"),
        "roofline": ent.pop("roofline"),
    }
    if "cpu_baseline" in ent:
        line["cpu_baseline"] = ent.pop("cpu_baseline")
    line.update(ent)
    if args.workload == "thunderstorm" and not args.no_sediment:
        line["sedimentation"] = run_sediment(args, args.steps, args.warmup)
    if args.workload == "thunderstorm" and not args.no_condense:
        line["condensation"] = run_condense(args, args.steps, args.warmup)
    if args.workload == "thunderstorm" and not args.no_breakup:
        line["breakup"] = run_breakup(args, args.steps, args.warmup)
    if args.workload == "thunderstorm" and not args.no_four_species:
        # the second 33-bin configuration: fewer calls (each is seconds)
        fs = run_workload(args, "four_species", min(args.steps, 2), 1,
                          min(args.cpu_seconds, 8.0), False)
        fs["dtype"] = "f32"
        line["four_species"] = fs
    line["context"] = {
        "paper": "2.08x whole-WRF speedup, 16 A100 vs 16 EPYC cores "
                 "(CONUS-12km); collision kernel 29.11 ms per call on one "
                 "A100 for a ~398k-point patch (<= 1.37e7 point-updates/s); "
                 "other hardware, precision and workload: context only"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
