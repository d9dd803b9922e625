"""Benchmark: particle-steps/s of the boosted-frame PIC step on one MI355X.

Prints ONE JSON line.  The timed region is K full steps of ``pic_step`` (every
step: injection, periodic sort, gather/push/deposit, current fold + filter,
Yee update) on the gamma_boost = 130, 8192 x 512 cell, 8 particles/cell
workload (33.5 M electrons with implicit ion partners) in the FP32 split
precision form, all inputs resident in HBM.  K defaults to the workload's
whole run (5000 steps): the cost of a step grows as the wake forms and pulls
electrons away from their partners, so a short window at the start would
overstate the rate.

The particles are re-sorted every `sort_interval` steps.  A window of K steps
holds floor-ish K / interval sorts; when it holds fewer than K / interval (a
short window), the missing share is added at the cost of one sort timed right
after the window, so that `ms_per_step` and `value` carry the sort at its
real rate.  `timed_window` gives the window's own figures.

Beside it: the same run in FP64 and in the deterministic mode; per-kernel
HIP-event times of the dominant kernel against the HBM roofline; the
gamma_boost = 13 (2048 x 256) and 3D gamma_boost = 100 (512 x 128 x 128,
quadratic) workloads with their own rooflines (the 3D one also against the
FP32 vector ALU peak); the whole-run figure of the committed profile while
the sources match it; and the FP64 oracle timed on the host cores, on all of
them (OpenMP) over the full geometry and on one over a slab.
"""
import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor nominal
VALU_FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 vector
# Algorithmic bytes (compulsory traffic) of the gather-push-deposit kernel:
# each particle's state read and written once, each field array of the
# particle step read once and the current written once.
BYTES_PER_PARTICLE = {(2, "fp32"): 52.0, (2, "fp64"): 96.0,   # 2D: read 28 + write 24 (FP32)
                      (3, "fp32"): 60.0, (3, "fp64"): 112.0}  # 3D: read 32 + write 28 (FP32)
BYTES_PER_CELL_GPD = {"fp32": 36.0, "fp64": 72.0}   # E, B read (24) + J write (12)
BYTES_PER_CELL_STEP = {"fp32": 72.0, "fp64": 144.0}  # whole step: E, B r+w, J w+r
# FP32 flops per particle of the 3D quadratic gather-push-deposit (162 gather
# products over 27 nodes x 6 components, the Boris push, and the Esirkepov
# weights and prefix sums over 4^3 nodes x 3 components): about 2300
FLOPS_PER_PARTICLE_3D_QUADRATIC = 2300.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 over the HIP sources and the C header (sorted by name)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1011_0917_amd", "csrc", "*")) +
                   [os.path.join(ROOT, "include", "bfpic.h")])
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the summary is missing or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters: reads and writes mib MiB three times."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"bench: copy calibration {mib} MiB x 3")


def whole_run_profile(workload):
    """Whole-run figures of the committed profile summary, or None when it is
    missing or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"step_{workload}_whole_run.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return {"steps": int(vals["steps"]), "ms_per_step": float(vals["ms_per_step"]),
                "particle_steps_per_s": float(vals["particle_steps_per_s"]),
                "step_roofline_frac": float(vals["step_roofline_frac"]),
                "source": os.path.relpath(path, ROOT)}
    except (KeyError, ValueError):
        return None


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "cpu_model": model}


def run_gpu(name, precision, steps, warmup, sort_interval, with_kernel_times=True, det=0):
    import torch
    import paper_1011_0917_amd as P
    from workloads import WORKLOADS, resolve_gpu
    W = WORKLOADS[name]
    cfg, init, _ = resolve_gpu(W, precision=precision, sort_interval=sort_interval)
    cfg.deterministic = det
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], n_uniform=init["n_lab"], laser=init["laser"])
    sim.pic_step(warmup)
    d0 = sim.diagnostics()
    torch.cuda.synchronize()
    if with_kernel_times:
        sim.kernel_timing(True)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    sim.pic_step(steps)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    kt = {}
    if with_kernel_times:
        for k in P.TIMER:
            t, n = sim.kernel_time(k)
            kt[k] = {"ms": t, "launches": n}
    # one sort timed on its own, right after the window
    sim.kernel_timing(True)
    sim.sort()
    sort_ms, _ = sim.kernel_time("sort")
    d1 = sim.diagnostics()
    cells = W["nz"] * W["nx"] * W.get("ny", 1)
    nparts = 0.5 * (d0["live"] + d1["live"])
    sim.close()
    del sim
    torch.cuda.empty_cache()
    # sorts the window held: steps s in (warmup, warmup + steps] with s % interval == 0
    held = 0
    if sort_interval > 0:
        held = (warmup + steps) // sort_interval - warmup // sort_interval
    due = steps / sort_interval if sort_interval > 0 else 0.0
    extra = max(0.0, due - held) * sort_ms
    return {"ms": ms, "steps": steps, "particles": nparts, "cells": cells, "kernels": kt,
            "diag_end": d1, "W": W, "sort_ms": sort_ms, "sorts_held": held, "sorts_due": due,
            "ms_amortised": ms + extra}


def gpd_roofline(r, precision="fp32"):
    """Roofline object of the tiled gather-push-deposit kernel of a run."""
    W = r["W"]
    dim = W["dim"]
    kt = r["kernels"]["gpd_tiled"]
    gpd_ms = kt["ms"] / max(kt["launches"], 1)
    nbytes = BYTES_PER_PARTICLE[(dim, precision)] * r["particles"] + \
        BYTES_PER_CELL_GPD[precision] * r["cells"]
    achieved = nbytes / (gpd_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes": nbytes,
            "kernel": "k_gpd_tiled", "kernel_ms": gpd_ms}


# Steps of a side workload's default run: its whole run, except where the
# configuration goes numerically unstable and its fields overflow before the
# end (gamma_b = 13: from step ~550 the field energy grows ~1e12 per 100 steps
# and FP32 overflows near step 1000), where only the stable part is timed.
SIDE_STEPS = {"boost13_2d": 500}


def side_workload(name, steps, warmup, sort_interval):
    """FP32 line of another configuration: rates, kernel split and rooflines."""
    from workloads import WORKLOADS
    r = run_gpu(name, "fp32", steps or SIDE_STEPS.get(name, WORKLOADS[name]["steps"]), warmup,
                sort_interval)
    W = r["W"]
    dim = W["dim"]
    ms = r["ms_amortised"] / r["steps"]
    step_bytes = BYTES_PER_PARTICLE[(dim, "fp32")] * r["particles"] + \
        BYTES_PER_CELL_STEP["fp32"] * r["cells"]
    out = {"workload": name, "grid": [W["nz"], W["nx"]] + ([W["ny"]] if dim == 3 else []),
           "ppc": W["ppc"], "gamma_boost": W["gamma_b"], "shape_order": W["order"],
           "particles": int(r["particles"]), "steps": r["steps"], "warmup": warmup,
           "value": r["particles"] / (ms * 1e-3), "unit": "particle-steps/s",
           "ms_per_step": ms, "cell_updates_per_s": r["cells"] / (ms * 1e-3),
           "step_roofline_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "roofline": gpd_roofline(r),
           "kernel_ms_per_step": {k: v["ms"] / r["steps"] for k, v in r["kernels"].items()}}
    out["roofline"]["traffic"] = measured_traffic("k_gpd_tiled", name, "fp32")
    if dim == 3 and W["order"] == 2:
        kms = out["roofline"]["kernel_ms"]
        tf = FLOPS_PER_PARTICLE_3D_QUADRATIC * r["particles"] / (kms * 1e-3) / 1e12
        out["roofline_valu"] = {"bound": "alu", "achieved": tf, "peak": VALU_FP32_PEAK_TFLOPS,
                                "unit": "TFLOP/s", "frac": tf / VALU_FP32_PEAK_TFLOPS,
                                "flops_per_particle": FLOPS_PER_PARTICLE_3D_QUADRATIC,
                                "kernel": "k_gpd_tiled"}
    return out


def run_adjoint(name="adjoint_2d", precision="fp32"):
    """Taped forward and reverse sweep of the adjoint configuration, timed."""
    import torch
    import paper_1011_0917_amd as P
    from workloads import WORKLOADS, adjoint_setup, resolve_gpu
    W = WORKLOADS[name]
    cfg, init, nst = resolve_gpu(W, precision=precision, sort_interval=0)
    dt = P.yee_dt(2, cfg.dz, cfg.dx, 1.0, cfg.cfl)
    a = adjoint_setup(W, cfg.dz, P.beta, dt)
    sim = P.Simulation(cfg, capacity=init["capacity"])
    sim.init_boosted_plasma(init["gamma_b"], knots_z=a["knots_z"], knots_n=a["knots_n"],
                            laser=init["laser"])
    n0 = sim.num_slots()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = sim.forward_loss(nst, a["interval"], a["window"][0], a["window"][1], a["box"])
    t1 = time.perf_counter()
    da0, dn = sim.adjoint(len(a["knots_n"]))
    t2 = time.perf_counter()
    sim.close()
    return {"workload": name, "precision": precision, "steps": nst,
            "checkpoint_interval": a["interval"], "particles": n0, "loss": loss,
            "dL_da0": da0, "forward_ms_per_step": (t1 - t0) * 1e3 / nst,
            "adjoint_ms_per_step": (t2 - t1) * 1e3 / nst,
            "adjoint_particle_steps_per_s": n0 * nst / (t2 - t1)}


def cpu_single(name, nz_sample=256, steps=20):
    """The FP64 oracle, single-threaded, on a slab of the same workload."""
    import oracle as O
    from workloads import resolve_oracle, small
    W = small(name, nz=nz_sample, steps=steps)
    kw, init = resolve_oracle(W)
    s = O.Sim(**kw)
    s.init(n_uniform=init["n_lab"], laser=init["laser"])
    s.step(1)
    n = s.num_pairs()
    t = time.perf_counter()
    s.step(steps)
    el = time.perf_counter() - t
    return {"value": n * steps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{name} physics on a {nz_sample} x {W['nx']} cell slab "
                      f"({n} electrons + partners), {steps} steps, {el:.1f} s, 1 thread"}


def cpu_baseline(name, steps=2):
    """The FP64 oracle on every usable host core (OpenMP particle loop with
    per-thread currents), on the workload's full geometry: one untimed step,
    then `steps` timed steps; beside it the single-threaded slab timing."""
    import oracle as O
    from workloads import WORKLOADS, resolve_oracle
    host = host_info()
    threads = max(1, min(host["nproc"] or 1, O.max_threads()))
    W = WORKLOADS[name]
    kw, init = resolve_oracle(W)
    s = O.Sim(**kw)
    s.set_threads(threads)
    s.init(n_uniform=init["n_lab"], laser=init["laser"])
    s.step(1)
    n = s.num_pairs()
    t = time.perf_counter()
    s.step(steps)
    el = time.perf_counter() - t
    del s
    cells = W["nz"] * W["nx"] * W.get("ny", 1)
    out = {"value": n * steps / el, "unit": "particle-steps/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{name} full geometry ({W['nz']} x {W['nx']} cells, {n} electrons + "
                     f"partners), {steps} steps after one untimed step, {el:.1f} s, "
                     f"{threads} threads",
           "cell_updates_per_s": cells * steps / el, "host": host}
    out["single_thread"] = cpu_single(name)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's whole run)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="boost130_2d")
    ap.add_argument("--sort-interval", type=int, default=50)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip timing the adjoint configuration's reverse sweep")
    ap.add_argument("--no-deterministic", action="store_true",
                    help="skip timing the deterministic (fixed-point current) FP32 form")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the gamma_boost = 13 and 3D workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X "
              "(sharding across GPUs is described, not built)", file=sys.stderr)
        sys.exit(2)
    from workloads import WORKLOADS
    explicit_steps = args.steps
    if args.steps is None:
        args.steps = WORKLOADS[args.workload]["steps"]
    import torch
    torch.cuda.set_device(0)
    log(f"bench: {args.workload} fp32 split, {args.warmup} warmup + {args.steps} timed steps")
    r32 = run_gpu(args.workload, "fp32", args.steps, args.warmup, args.sort_interval)
    dim = r32["W"]["dim"]
    ms_step = r32["ms_amortised"] / r32["steps"]
    pps = r32["particles"] / (ms_step * 1e-3)
    cups = r32["cells"] / (ms_step * 1e-3)
    # dominant kernel: tiled gather-push-deposit
    roof = gpd_roofline(r32)
    roof["traffic"] = measured_traffic("k_gpd_tiled", args.workload, "fp32")
    roof["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)"
    step_bytes = BYTES_PER_PARTICLE[(dim, "fp32")] * r32["particles"] + \
        BYTES_PER_CELL_STEP["fp32"] * r32["cells"]
    out = {
        "metric": "particle-steps/s (FP32 split boosted-frame PIC step) + % HBM roofline",
        "value": pps, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded SplitMix64 plasma, analytic laser)",
        "config": {"workload": args.workload, "grid": [r32["W"]["nz"], r32["W"]["nx"]],
                   "ppc": r32["W"]["ppc"], "gamma_boost": r32["W"]["gamma_b"],
                   "particles": int(r32["particles"]), "sort_interval": args.sort_interval,
                   "parallelism": "1 GPU"},
        "cell_updates_per_s": cups,
        "step_roofline_frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        # the whole step's algorithmic bytes at the HBM peak bound both rates
        "step_roofline_rates": {
            "particle_steps_per_s": r32["particles"] * HBM_PEAK_GBS * 1e9 / step_bytes,
            "cell_updates_per_s": r32["cells"] * HBM_PEAK_GBS * 1e9 / step_bytes},
        "roofline": roof,
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in r32["kernels"].items()},
        "timed_window": {
            "ms_per_step": r32["ms"] / r32["steps"],
            "particle_steps_per_s": r32["particles"] * r32["steps"] / (r32["ms"] * 1e-3),
            "sorts_held": r32["sorts_held"], "sorts_due": r32["sorts_due"],
            "sort_ms": r32["sort_ms"],
            "note": "ms_per_step and value add (sorts_due - sorts_held) x sort_ms to the "
                    "window's time when the window holds fewer sorts than its steps owe"},
        "whole_run": whole_run_profile(args.workload),
    }
    if not args.no_fp64:
        log("bench: fp64 plain form")
        r64 = run_gpu(args.workload, "fp64", args.steps, args.warmup, args.sort_interval,
                      with_kernel_times=False)
        ms64 = r64["ms_amortised"] / r64["steps"]
        pps64 = r64["particles"] / (ms64 * 1e-3)
        out["fp64"] = {"value": pps64, "unit": "particle-steps/s", "ms_per_step": ms64}
        out["fp32_over_fp64"] = pps / pps64
    if not args.no_deterministic:
        log("bench: fp32 deterministic (int64 fixed-point currents)")
        rd = run_gpu(args.workload, "fp32", args.steps, args.warmup, args.sort_interval,
                     with_kernel_times=False, det=1)
        msd = rd["ms_amortised"] / rd["steps"]
        out["deterministic"] = {"value": rd["particles"] / (msd * 1e-3),
                                "unit": "particle-steps/s", "ms_per_step": msd}
    if not args.no_side:
        out["other_workloads"] = {}
        for name in ("boost13_2d", "boost100_3d"):
            if name == args.workload:
                continue
            log(f"bench: {name} fp32 split")
            out["other_workloads"][name] = side_workload(name, explicit_steps, args.warmup,
                                                         args.sort_interval)
    if not args.no_adjoint:
        log("bench: adjoint_2d taped forward + reverse sweep (fp32)")
        out["adjoint"] = run_adjoint()
    if not args.no_cpu_baseline:
        log("bench: oracle cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.workload)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
