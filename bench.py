#!/usr/bin/env python3
"""Benchmark of the reconstruction solve on one MI355X.

Workload (one "step"): the whole hot path on a 512^3 periodic mesh with a seeded lognormal
overdensity (sigma_g = 1.0, Gaussian-cut power-law spectrum with R_c = 2 cells, seed 1002),
already resident in HBM: the FP64 FAS V-cycle solve to relative residual 1e-10 and, beside it
on the same input, the mixed-precision solve to the same FP64 residual.

Headline value: the finest-mesh FP64 red-black NGS sweep throughput (Gcell-updates/s), from HIP
events recorded by the library around every finest-mesh sweep (its red and black launches) inside
the timed region, on the launches' own stream. The roofline entry prices that kernel at its
algorithmic 24 bytes per cell update (theta read + write, delta read) against the 8 TB/s HBM
peak; "traffic" is the HBM traffic per sweep measured with rocprofv3 counters (committed
summary), over the same sweep time.

Also reported: time to solution of both 512^3 solves (medians over the timed steps; the mixed
solve with npre = npost = 2, at most 4 FP32 V-cycles per outer step and 8 sweeps on the inner
coarsest mesh) and the largest difference
of the two solutions relative to max |theta|; one adjoint solve at 512^3; the CIC deposit of 256^3
particles onto a 256^3 mesh; and the batched form on 64 boxes of {64, 96, 128}^3 (mixed precision
to 1e-8), each timed after an untimed run. The CPU baseline times the oracle on bounded samples.

Prints ONE JSON line. --gpus N > 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_PER_UPDATE = 24.0  # theta read + theta write + delta read, FP64
PROFILE_PMC = os.path.join(ROOT, "profiles", "sweep64_512_pmc.txt")
KERNEL_SOURCES = ["paper_1709_06350_amd/csrc/sweep.hip", "paper_1709_06350_amd/csrc/mr_device.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(schedule: str):
    """HBM bytes per finest sweep from the committed PMC summary, if it was taken on the same kernel
    source and the same finest-level schedule as this run."""
    if not os.path.exists(PROFILE_PMC):
        return None
    txt = open(PROFILE_PMC).read()
    m = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_sweep:\s*([0-9.eE+]+)", txt)
    c = re.search(r"schedule:\s*([0-9,]+)", txt)
    if not m or not b or not c or m.group(1) != kernel_hash() or c.group(1) != schedule:
        return None
    return float(b.group(1))


SCHED_KERNEL = {0: "half_sweep_tiled", 1: "half_sweep_pipe", 2: "sweep_fused"}
# options of the mixed-precision solve
MIXED_OPTS = {"npre": 2, "npost": 2, "inner_cycles": 4, "ncoarse": 8}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(full: bool = False, reps: int = 5):
    """The oracle (numpy, FP64, one thread) on the host cores, on bounded samples of the workload:
    the red-black sweep at 32^3 and 128^3 (medians of `reps` runs) and at 256^3 (median of 3), and
    the whole solve to 1e-10 at 32^3 (median of `reps`), inputs of the same recipe (lognormal,
    sigma_g = 1.0, R_c = 2 cells, seed 1002) at the sample size. Times to solution at 128^3, 256^3 and
    512^3 are extrapolated from the 32^3 solve's sweep-equivalents (solve time / sweep time) and the
    measured sweep time at that size (512^3: the 256^3 sweep time scaled by the cell count), and
    labelled so; with full=True the 128^3 solve is run once and reported as measured."""
    import statistics

    import numpy as np

    import inputs
    from oracle import multigrid as omg

    def med(fn, k):
        ts = []
        out = None
        for _ in range(k):
            t0 = time.perf_counter()
            out = fn()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts), out

    sweep_s, solve = {}, {}
    for s, k in ((32, reps), (128, reps), (256, 3)):
        d = inputs.lognormal(s, 1.0, 2.0, 1002)
        th = np.zeros_like(d)
        if s < 256:   # one untimed sweep first (the 256^3 median of 3 absorbs a slow first run)
            omg.rb_sweep(th, d, None, 1.0)
        sweep_s[s], _ = med(lambda: omg.rb_sweep(th, d, None, 1.0), k)
        del d, th
    d32 = inputs.lognormal(32, 1.0, 2.0, 1002)
    t32, (_, info32) = med(lambda: omg.solve(d32, tol=1e-10), reps)
    solve["32"] = {"seconds": round(t32, 3), "cycles": info32["cycles"], "kind": "measured", "runs": reps}
    equiv = t32 / sweep_s[32]
    for s in (128, 256):
        solve[str(s)] = {"seconds": round(equiv * sweep_s[s], 1), "kind": "extrapolated",
                         "how": f"32^3 solve in sweep-equivalents x {s}^3 sweep time"}
    if full:
        d128 = inputs.lognormal(128, 1.0, 2.0, 1002)
        t0 = time.perf_counter()
        _, info128 = omg.solve(d128, tol=1e-10)
        solve["128"] = {"seconds": round(time.perf_counter() - t0, 1), "cycles": info128["cycles"],
                        "kind": "measured", "runs": 1}
    solve["512"] = {"seconds": round(equiv * sweep_s[256] * 8, 0), "kind": "extrapolated",
                    "how": "32^3 solve in sweep-equivalents x 256^3 sweep time x 8 (cells)"}
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {
        "value": round(256 ** 3 / sweep_s[256] / 1e9, 5),
        "unit": "Gcell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle red-black sweep at 256^3 (median of 3: {sweep_s[256]:.2f} s), 128^3 (median of {reps}: "
                  f"{sweep_s[128]:.3f} s) and 32^3 ({sweep_s[32]:.4f} s); oracle solve to 1e-10 at 32^3 (median of "
                  f"{reps}); numpy, one thread; times to solution above 32^3 extrapolated unless marked measured",
        "sweep_seconds": {"32": round(sweep_s[32], 5), "128": round(sweep_s[128], 4), "256": round(sweep_s[256], 3)},
        "time_to_1e-10_s": solve,
        "host": {"cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(), "affinity_cpus": affinity},
    }


def copy_calibration(nbytes: int, reps: int):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def stream_probe(nbytes: int = 1 << 30, reps: int = 5, configs=None):
    """Achievable HBM bandwidth from the library's hand-written streaming kernels (mr_hbm_stream):
    copy (16 B per element), read (8 B) and triad (24 B: the relaxation update's two reads and one
    write), plain and non-temporal, several grid sizes; the median of `reps` launches each."""
    import statistics

    import torch

    from paper_1709_06350_amd import mr

    count = nbytes // 8
    a = torch.ones(count, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    per_elem = {mr.MR_STREAM_COPY: 16, mr.MR_STREAM_READ: 8, mr.MR_STREAM_TRIAD: 24}
    names = {mr.MR_STREAM_COPY: "copy", mr.MR_STREAM_READ: "read", mr.MR_STREAM_TRIAD: "triad"}
    configs = configs or [(k, nt, bpc) for k in per_elem for nt in (False, True) for bpc in (4, 8, 16)]
    out = {}
    for kind, nt, bpc in configs:
        mr.hbm_stream(kind, a, c, b, nt, bpc)
        ms = statistics.median(mr.hbm_stream(kind, a, c, b, nt, bpc) for _ in range(reps))
        key = f"{names[kind]}{'_nt' if nt else ''}_{bpc}"
        out[key] = round(per_elem[kind] * count / (ms * 1e-3) / 1e9, 1)
    best = {names[k]: max(v for kk, v in out.items() if kk.startswith(names[k] + "_")) for k in per_elem}
    return {"GBps": out, "best_GBps": best, "bytes_per_array": nbytes, "reps": reps}


def _timed_batch(mr, deltas, thetas, **kw):
    """A reusable batch: created (allocation, tiles, graph capture) and solved once untimed, then
    one timed solve. Returns (seconds, infos)."""
    import torch

    with mr.Batch([d.shape[0] for d in deltas], **kw) as b:
        b.solve(deltas, thetas)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos = b.solve(deltas, thetas)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos


def batched_run():
    """64 boxes of {64, 96, 128}^3, mixed precision to 1e-8, on a reusable batch (no device
    allocation in the timed solve); the one-shot call (allocation and capture included) beside it."""
    import torch

    import inputs
    from paper_1709_06350_amd import mr

    spec = inputs.batched_boxes()
    deltas = [torch.from_numpy(inputs.lognormal(n, s, 4.0, seed)).cuda() for n, s, seed in spec]
    thetas = [torch.zeros_like(d) for d in deltas]
    cells = sum(n ** 3 for n, _, _ in spec)
    dt, infos = _timed_batch(mr, deltas, thetas, tol=1e-8)
    mr.solve_batched(deltas, thetas, tol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mr.solve_batched(deltas, thetas, tol=1e-8)
    torch.cuda.synchronize()
    d1 = time.perf_counter() - t0
    da, ia = _timed_batch(mr, deltas, thetas, tol=1e-8, anderson=True)
    cyc = [i.cycles for i in infos]
    cya = [i.cycles for i in ia]
    return {
        "boxes": len(spec),
        "cells": cells,
        "seconds": round(dt, 4),
        "mcells_solved_per_s": round(cells / dt / 1e6, 2),
        "outer_iterations": [min(cyc), max(cyc)],
        "worst_rel_residual": max(i.rel_residual for i in infos),
        "tol": 1e-8,
        "one_shot_seconds": round(d1, 4),
        "note": "timed solve on a reusable batch (mr_batch_solve: no device allocation, graph captured at "
                "creation); one_shot_seconds: mr_solve_batched with allocation and capture",
        "anderson": {"seconds": round(da, 4), "mcells_solved_per_s": round(cells / da / 1e6, 2),
                     "outer_iterations": [min(cya), max(cya)],
                     "worst_rel_residual": max(i.rel_residual for i in ia),
                     "status": max(i.status for i in ia)},
    }


def cic_run():
    """Deposits of 256^3 Zel'dovich-displaced particles onto a 256^3 mesh (particles resident): NGP,
    CIC and TSC for the catalogue in lattice order and randomly permuted, by the default path (tile
    sort for CIC and TSC) and by the atomic scatter kernels (MR_FLAG_DEPOSIT_SCATTER); medians of 5
    launches after one untimed. Then the Lagrangian mapping of the same particles."""
    import numpy as np
    import torch

    import inputs
    from paper_1709_06350_amd import mr

    n = 256
    pos_np = inputs.zeldovich_particles(n, 4.0, 1001)
    pos = torch.from_numpy(pos_np).cuda()
    perm = np.random.default_rng(1002).permutation(pos_np.shape[0])
    shuf = torch.from_numpy(np.ascontiguousarray(pos_np[perm])).cuda()
    theta = torch.from_numpy(40.0 * inputs.grf(n, 4.0, 1006)).cuda()   # a smooth synthetic potential
    npart = pos.shape[0]
    reps = 5

    def timed(c, p, scheme, out):
        c.deposit(p, 1.0, scheme, out=out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            c.deposit(p, 1.0, scheme, out=out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    with mr.Context(n) as c:
        out = c.deposit(pos, 1.0, "cic")
        ref = out.clone()
        res = {}
        for flags, tag in ((0, ""), (mr.MR_FLAG_DEPOSIT_SCATTER, "scatter_")):
            c.set_opts(flags=flags)
            for scheme in ("ngp", "cic", "tsc"):
                res[f"{tag}{scheme}"] = timed(c, pos, scheme, out)
                res[f"{tag}{scheme}_shuffled"] = timed(c, shuf, scheme, out)
        c.set_opts(flags=0)
        c.deposit(shuf, 1.0, "cic", out=out)
        same = bool(torch.equal(out, ref))
        # Lagrangian mapping of the same particles (mesh displacement + CIC gather), and without the
        # mesh field (the differences formed at the particles from theta)
        disp, psi = c.lagrangian(theta, pos, want_psi=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c.lagrangian(theta, pos, want_psi=True, out=disp)
        torch.cuda.synchronize()
        dl = (time.perf_counter() - t0) / reps
        c.lagrangian(theta, pos, out=disp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c.lagrangian(theta, pos, out=disp)
        torch.cuda.synchronize()
        dn = (time.perf_counter() - t0) / reps
    dt = res["cic"]
    cic = {"particles": npart, "mesh": n, "seconds": round(dt, 5), "gparticles_per_s": round(npart / dt / 1e9, 3),
           "ngp_seconds": round(res["ngp"], 5), "tsc_seconds": round(res["tsc"], 5),
           "shuffled_seconds": {k: round(res[f"{k}_shuffled"], 5) for k in ("ngp", "cic", "tsc")},
           "scatter_kernels_seconds": {k: round(res[f"scatter_{k}"], 5) for k in ("ngp", "cic", "tsc")},
           "scatter_kernels_shuffled_seconds": {k: round(res[f"scatter_{k}_shuffled"], 5) for k in ("ngp", "cic", "tsc")},
           "shuffled_equals_lattice_bitwise": same,
           "note": "CIC and TSC sort the particles by 16 x 16 x 32 mesh tile (no global atomics); NGP and the "
                   "scatter_kernels entries use 64-bit atomics; medians of 5"}
    lag = {"particles": npart, "mesh": n, "seconds": round(dl, 5), "gparticles_per_s": round(npart / dl / 1e9, 3),
           "note": "mesh displacement grad(theta) into a caller buffer + CIC gather to the particles",
           "without_mesh_field_seconds": round(dn, 5)}
    return cic, lag


def adjoint_run(ctx, delta, theta):
    """One adjoint solve (gradient of a loss through the solve) at the bench mesh, after the solve."""
    import torch

    g = theta - theta.mean()
    ctx.set_opts(tol=1e-8)
    out, info = ctx.adjoint_solve(delta, theta, g, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, info = ctx.adjoint_solve(delta, theta, g, out=out, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same with Anderson mixing of lambda between cycles (depth 3, the fastest for the adjoint)
    ctx.adjoint_solve(delta, theta, g, out=out, check=False, anderson_depth=3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out, info_a = ctx.adjoint_solve(delta, theta, g, out=out, check=False, anderson_depth=3)
    torch.cuda.synchronize()
    da = time.perf_counter() - t1
    ctx.set_opts(tol=1e-10)
    return {"seconds": round(dt, 4), "cycles": info.cycles, "rel_residual": info.rel_residual, "tol": 1e-8,
            "status": info.status, "g": "theta - <theta> (dL/dtheta of L = |theta|^2 / 2)",
            "anderson3": {"seconds": round(da, 4), "cycles": info_a.cycles, "rel_residual": info_a.rel_residual,
                          "status": info_a.status}}


def order4_run(ctx, delta, theta, rb_cycles):
    """The same FP64 solve with the 4-class sub-sweep ordering (one untimed and one timed run)."""
    import torch

    from paper_1709_06350_amd import mr

    ctx.set_opts(flags=mr.MR_FLAG_ORDER4)
    try:
        ctx.solve(delta, theta, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = ctx.solve(delta, theta, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        ctx.set_opts(flags=0)
    return {"seconds": round(dt, 4), "cycles": info.cycles, "red_black_cycles": rb_cycles,
            "rel_residual": info.rel_residual, "status": info.status,
            "note": "4 conflict-free class sub-sweeps per sweep (row-filtered tiled launches)"}


def anderson_run(ctx, delta, theta, rb_cycles, depth=2):
    """The same FP64 solve with Anderson-accelerated V-cycles (one untimed and one timed run)."""
    import torch

    ctx.solve_anderson(delta, theta, depth=depth, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = ctx.solve_anderson(delta, theta, depth=depth, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"seconds": round(dt, 4), "cycles": info.cycles, "plain_cycles": rb_cycles, "depth": depth,
            "rel_residual": info.rel_residual, "status": info.status}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the CIC and adjoint timings")
    ap.add_argument("--no-order4", action="store_true", help="skip the 4-class ordering solve")
    ap.add_argument("--particles-only", action="store_true",
                    help="only time the deposits and the Lagrangian mapping (256^3 mesh, 256^3 particles)")
    ap.add_argument("--schedule", default="", metavar="KIND,TM,TJ,NCHUNKS",
                    help="pin the finest-level FP64 relaxation schedule (mr_set_schedule) instead of the timed one")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only measure the achievable HBM bandwidth with the library's streaming kernels")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched 64-box workload (for profiling its kernels)")
    ap.add_argument("--mixed-only", action="store_true",
                    help="only run the mixed-precision solve (steps times, untimed; for counter runs)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also run the oracle's 128^3 solve to 1e-10 once for the CPU baseline (minutes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a device copy of BYTES bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch

    import inputs
    from paper_1709_06350_amd import mr

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, 3)
        return
    if args.stream_probe:
        print(json.dumps({"hbm_stream": stream_probe()}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_run()}), flush=True)
        return
    if args.particles_only:
        cic, lag = cic_run()
        print(json.dumps({"deposit": cic, "lagrangian": lag}), flush=True)
        return
    n = args.n
    delta_np = inputs.config2_delta(n)
    delta = torch.from_numpy(delta_np).cuda()
    theta = torch.zeros_like(delta)
    theta_m = torch.zeros_like(delta)
    ctx = mr.Context(n, tol=1e-10, max_cycles=100)
    if args.schedule:
        ctx.set_schedule(0, tuple(int(x) for x in args.schedule.split(",")))
    sched = ctx.get_schedule(0)
    sched_str = ",".join(str(x) for x in sched)
    run_mixed = not args.no_mixed or args.mixed_only
    ctxm = None
    if run_mixed:
        ctxm = mr.Context(n, tol=1e-10, max_cycles=100, precision=mr.PREC_MIXED, **MIXED_OPTS)
        ctxm.solve(delta, theta_m)
    if args.mixed_only:
        # the mixed-precision solve alone (for counter runs of its kernels)
        for _ in range(args.steps):
            ctxm.solve(delta, theta_m)
        torch.cuda.synchronize()
        print(json.dumps({"mixed_only": True, "n": n, "steps": args.steps}), flush=True)
        return

    def step():
        _, i64 = ctx.solve(delta, theta)
        im = None
        if run_mixed:
            _, im = ctxm.solve(delta, theta_m)
        return i64, im

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    ts64, tsm = [], []
    info64 = infom = None
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        _, info64 = ctx.solve(delta, theta)
        torch.cuda.synchronize()
        b = time.perf_counter()
        ts64.append(b - a)
        if run_mixed:
            _, infom = ctxm.solve(delta, theta_m)
            torch.cuda.synchronize()
            tsm.append(time.perf_counter() - b)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    tim = ctx.timing_read()
    ctx.timing_enable(False)
    t64 = statistics.median(ts64)
    tm = statistics.median(tsm) if run_mixed else 0.0
    theta_err = None
    if run_mixed:
        # both solutions carry the zero-mean gauge
        theta_err = float((theta_m - theta).abs().max() / theta.abs().max())

    avg_sweep_s = tim["sweep64_ms"] / max(1, tim["sweep64_launches"]) * 1e-3
    cells = float(n) ** 3
    gcups = cells / avg_sweep_s / 1e9
    achieved = SWEEP_BYTES_PER_UPDATE * cells / avg_sweep_s / 1e9
    traffic = measured_traffic(sched_str)
    out = {
        "metric": "NGS smoother Gcell-updates/s (% HBM peak); 512^3 time-to-1e-10, mixed vs FP64",
        "value": round(gcups, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_total / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"lognormal delta on a periodic {n}^3 mesh (sigma_g=1.0, R_c=2 cells, seed 1002): "
                        "FP64 FAS V-cycle solve to rel. residual 1e-10"
                        + (" plus the mixed-precision solve on the same input" if run_mixed else ""),
            "n": n,
            "tol": 1e-10,
            "npre": 2,
            "npost": 2,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / avg_sweep_s / 1e9, 1),
            "kernel": f"{SCHED_KERNEL[sched[0]]}<{sched[1]},{sched[2]}> (finest-mesh FP64 red-black sweep"
                      + (", one launch" if sched[0] == 2 else ": red + black launch") + f", {sched[3]} chunks)",
            "schedule": sched_str,
            "sweep_us": round(avg_sweep_s * 1e6, 2),
            "algorithmic_bytes_per_sweep": SWEEP_BYTES_PER_UPDATE * cells,
            "traffic_bytes_per_sweep": traffic,
            "sweeps_timed": tim["sweep64_launches"],
        },
        "time_to_solution_s": {
            "fp64": round(t64, 4),
            "mixed": round(tm, 4) if run_mixed else None,
            "ratio_mixed_over_fp64": round(tm / t64, 4) if run_mixed and t64 > 0 else None,
            "statistic": f"median of {args.steps} timed solves each (after {args.warmup} untimed)",
            "fp64_all": [round(x, 4) for x in ts64],
            "mixed_all": [round(x, 4) for x in tsm],
            "mixed_opts": dict(MIXED_OPTS, note="flexible GMRES inner solve of at most inner_cycles FP32 "
                                                 "V-cycles per outer FP64 step, ncoarse sweeps on the inner "
                                                 "coarsest mesh; FP64 solve at npre = npost = 2, ncoarse = 20"),
            "theta_max_rel_diff_mixed_vs_fp64": theta_err,
        },
        "cycles": {"fp64": info64.cycles if info64 else None,
                   "mixed": infom.cycles if infom else None},
        "rel_residual": {"fp64": info64.rel_residual if info64 else None,
                         "mixed": infom.rel_residual if infom else None},
        "paper_context": "CPU code of the paper: 8 V-cycles, < 1 min on 64 CPUs (128^3) and about 6 min on "
                         "360 CPUs (512^3), absolute rms residual 1e-8; other hardware and inputs, not a target",
    }
    if not args.no_extra:
        out["adjoint"] = adjoint_run(ctx, delta, theta)
        out["cic"], out["lagrangian"] = cic_run()
        if not args.no_order4:
            out["order4"] = order4_run(ctx, delta, theta, info64.cycles if info64 else None)
        out["anderson"] = {"fp64": anderson_run(ctx, delta, theta, info64.cycles if info64 else None)}
        if run_mixed:
            out["anderson"]["mixed"] = anderson_run(ctxm, delta, theta_m, infom.cycles if infom else None)
            if t64 > 0:
                out["anderson"]["mixed_over_plain_fp64"] = round(
                    out["anderson"]["mixed"]["seconds"] / t64, 4)
    if not args.no_batched:
        out["batched"] = batched_run()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(full=args.cpu_full)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
