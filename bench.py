"""Throughput of the P3M gravity step on one MI355X.

A step is one kick-drift-kick leapfrog step of the whole force path:
kick(dt/2) with the force of the previous step and drift(dt) (one fused
pass), the P3M force (binning; then the CIC deposit and FFT Poisson solve on
the plan's second stream beside the pair sum; then gradient + interpolation,
which adds the two parts) and kick(dt/2), ordered on one HIP stream with the
particles resident in HBM. Workload: 128^3 particles on a Zel'dovich-displaced lattice
(P(k) ~ k^-2, rms displacement 0.3 spacing), 128^3 PM grid, r_s = 1.25 cells,
r_c = 4.5 r_s, Plummer softening 0.03 spacing, G = 1, FP32 force arithmetic
with FP64 positions, momenta, kick and drift.

Prints one JSON line: particles/s over the timed steps (whole job), the pair
interaction rate of the short-range kernel, its roofline figures measured
with HIP events around every pair-kernel launch of the timed region, the same
step in FP64, and the CPU oracle timed on a bounded sample of the same input
(with the force error of both GPU precisions against it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "zeldovich128"
FLOP_PER_PAIR = 41          # 37 FP32 arithmetic flops + 4 transcendentals per pair
FP32_PEAK_TFLOPS = 157.3    # MI355X published FP32 vector peak
FP64_PEAK_TFLOPS = 78.6     # MI355X published FP64 vector peak
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 step timing")
    ap.add_argument("--cpu-sample", type=int, default=20000,
                    help="particles whose short-range force the CPU oracle evaluates")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the force timing and error legs of the 32^3 and 256^3 workloads")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward timing of the differentiable leapfrog")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device (a plain copy "
                         "of known size, to scale memory counters in a profiled run)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pairs_zeldovich128_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "k_pairs_zeldovich128_valu.json")
PAIR_SOURCE = os.path.join(ROOT, "paper_1510_07621_amd", "csrc", "pair.hip")


def counter_record(path):
    """A committed counter summary of k_pairs, or None when the pair kernel's
    source changed after the counters were taken."""
    import hashlib
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(PAIR_SOURCE, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("pair_source_sha256") != digest:
        return None
    return rec


def measured_traffic():
    """HBM bytes per k_pairs launch (FETCH_SIZE and WRITE_SIZE passes)."""
    rec = counter_record(TRAFFIC_FILE)
    return rec.get("bytes_per_launch") if rec else None


def measured_valu():
    """VALU issue and lane utilisation of k_pairs (SQ and GRBM counter pass)."""
    rec = counter_record(VALU_FILE)
    if not rec:
        return None
    return {k: rec[k] for k in ("valu_issue_util", "valu_lane_util", "valu_issue_per_cu_clock",
                                "valu_issue_ceiling_per_cu_clock", "clock_ghz")}


def run_steps(binding, plan, x, p, F, m, dt, box, steps):
    """KDK steps; F holds the force at x on entry and on exit."""
    for _ in range(steps):
        binding.kick_drift(x, p, F, m, 0.5 * dt, dt, box)    # kick, then drift, one pass
        plan.force(x, m, out=F)
        binding.kick(p, F, 0.5 * dt)


def time_precision(binding, torch, w, pos0, precision, steps, warmup, dt):
    plan = binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, rs_cells=w.rs_cells,
                                       cutoff_rs=w.cutoff_rs, softening=w.softening,
                                       G=w.G, precision=precision), w.n)
    x = torch.as_tensor(pos0, device="cuda").contiguous()
    p = torch.zeros_like(x)
    F = torch.empty_like(x)
    m = w.mass
    plan.force(x, m, out=F)
    run_steps(binding, plan, x, p, F, m, dt, w.box, warmup)
    pairs_before = plan.pair_count(x)
    torch.cuda.synchronize()
    plan.set_timing(steps)
    t0 = time.perf_counter()
    run_steps(binding, plan, x, p, F, m, dt, w.box, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    calls, stage_ms = plan.stage_times()
    plan.set_timing(0)
    pairs_after = plan.pair_count(x)
    plan.close()
    assert calls == steps, (calls, steps)
    return {
        "seconds": t1 - t0,
        "stage_ms_per_step": {k: v / steps for k, v in stage_ms.items()},
        "pairs": 0.5 * (pairs_before + pairs_after),
        "pairs_before": pairs_before, "pairs_after": pairs_after,
    }


def adjoint_leg(binding, torch, name, precision, segment=None, keep_grad=False):
    """Forward and backward time of the differentiable leapfrog: the
    workload's KDK steps from its positions at rest, loss = sum of squared
    final displacements (minimum image, from the initial positions), gradient
    with respect to the initial positions through autodiff.leapfrog with
    checkpoints every `segment` steps (default ceil(sqrt(steps))). One
    untimed warm-up pass."""
    import math
    from paper_1510_07621_amd import autodiff, ics
    w = ics.workload(name)
    x0 = torch.as_tensor(w.positions(), device="cuda").contiguous()
    p0 = torch.zeros_like(x0)
    seg = segment or max(1, math.ceil(math.sqrt(w.steps)))
    P = binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, rs_cells=w.rs_cells,
                                    cutoff_rs=w.cutoff_rs, softening=w.softening, G=w.G,
                                    precision=precision, adjoint=True), w.n)

    def run():
        x = x0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xT, _ = autodiff.leapfrog(P, x, p0, w.mass, w.dt, w.box, w.steps, seg)
        d = xT - x0
        d = d - w.box * torch.round(d / w.box)
        loss = (d * d).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (g,) = torch.autograd.grad(loss, x)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, float(loss.detach()), g

    run()
    tf, tb, loss, g = run()
    P.close()
    if keep_grad:
        return g
    return {"workload": name, "n_particles": w.n, "grid_n": w.grid_n, "steps": w.steps,
            "dt": w.dt, "precision": precision, "checkpoint_segment": seg,
            "forward_s": tf, "backward_s": tb, "ratio": tb / tf, "loss": loss,
            "grad_rms": float(torch.sqrt((g * g).sum(0).mean()))}


def powerspec_leg(binding, torch, w, pos, calls=20):
    """Time of one power-spectrum call (binning, CIC deposit, forward FFT with
    shell binning) on the workload, FP32, grid_n / 2 shells, sigma at 8 cells,
    and its rate against HBM: algorithmic bytes 60 N (sort and pack 40 N,
    deposit reads 20 N) + 24 M (deposit write 4 M, z pass 4 + 4 M, y pass
    4 + 4 M, x pass 4 M; M = grid cells, 4-byte reals)."""
    P = binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, rs_cells=w.rs_cells,
                                    cutoff_rs=w.cutoff_rs, softening=w.softening, G=w.G,
                                    precision="fp32"), w.n)
    x = torch.as_tensor(pos, device="cuda").contiguous()
    R = 8.0 * w.h
    for _ in range(3):
        P.power_spectrum(x, w.mass, r_tophat=R)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(calls):
        k, p, m, sig = P.power_spectrum(x, w.mass, r_tophat=R)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    P.close()
    nbytes = 60.0 * w.n + 24.0 * w.grid_n ** 3
    return {"workload": w.name, "ms_per_call": ms, "algorithmic_bytes": nbytes,
            "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "sigma_8cells": float(sig)}


def config_leg(binding, torch, name, precisions=("fp32", "fp64"), calls=5, n_targets=512):
    """One force evaluation of a named workload per precision: time (HIP
    events, mean over `calls` after one warm-up), particles/s and pair
    interactions/s. Also returns the forces at `n_targets` sampled particles,
    which the CPU leg compares with the oracle."""
    from paper_1510_07621_amd import ics
    w = ics.workload(name)
    pos = w.positions()
    tg = np.sort(np.random.default_rng(99).choice(w.n, size=min(n_targets, w.n),
                                                  replace=False))
    x = torch.as_tensor(pos, device="cuda").contiguous()
    out = {"workload": name, "n_particles": w.n, "grid_n": w.grid_n}
    sampled = {}
    for prec in precisions:
        P = binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, rs_cells=w.rs_cells,
                                        cutoff_rs=w.cutoff_rs, softening=w.softening,
                                        G=w.G, precision=prec), w.n)
        F = P.force(x, w.mass)
        pairs = P.pair_count(x)
        P.set_timing(calls)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(calls):
            P.force(x, w.mass, out=F)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / calls
        ncall, st = P.stage_times()
        sampled[prec] = F.cpu().numpy()[:, tg]
        P.close()
        out[prec] = {"ms_per_force": ms, "particles_per_s": w.n / (ms * 1e-3),
                     "pairs": pairs, "pair_ms": st["pp"] / ncall,
                     "pair_interactions_per_s": pairs / (st["pp"] / ncall * 1e-3)}
    return out, (w, pos, tg, sampled)


def config_errors(out, sample):
    """CPU leg for one named workload: the RMS / max per-particle force error
    of each precision against the oracle (O-PP at the sampled particles +
    O-PM), written into that workload's entry."""
    from oracle import metrics
    from oracle import pm as o_pm
    from oracle import pp as o_pp
    w, pos, tg, sampled = sample
    ref = (o_pp.pp_accel(pos, w.mass, w.box, w.r_s, w.r_c, w.softening, w.G, targets=tg) +
           o_pm.pm_accel(pos, w.mass, w.box, w.grid_n, w.r_s, w.G, targets=tg)) * w.mass
    for prec, F in sampled.items():
        err = metrics.force_errors(F, ref)
        out[prec]["force_err_rms"] = err["rms"]
        out[prec]["force_err_max"] = err["max"]
        out[prec]["force_err_particles"] = int(tg.size)


def ewald_leg(binding, torch, calls=5):
    """All-pairs PP force with the tabulated Ewald correction (64^3 table) on
    the 32^3 uniform workload, FP64: time per call and ordered pairs/s."""
    from paper_1510_07621_amd import ics
    w = ics.workload("uniform32")
    P = binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, softening=w.softening, G=w.G,
                                    precision="fp64", ewald_gridsize=64), w.n)
    x = torch.as_tensor(w.positions(), device="cuda").contiguous()
    F = P.pp_ewald_force(x, w.mass)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(calls):
        P.pp_ewald_force(x, w.mass, out=F)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    P.close()
    pairs = float(w.n) * (w.n - 1)
    return {"workload": w.name, "ewald_gridsize": 64, "ms_per_call": ms,
            "pairs_per_s": pairs / (ms * 1e-3)}


def cpu_leg(binding, torch, w, pos, n_sample):
    """CPU oracle timed on a bounded sample, plus the GPU force error against it."""
    from oracle import metrics
    from oracle import pm as o_pm
    from oracle import pp as o_pp

    rng = np.random.default_rng(77)
    tg = np.sort(rng.choice(w.n, size=n_sample, replace=False))
    t0 = time.perf_counter()
    a_pm = o_pm.pm_accel(pos, w.mass, w.box, w.grid_n, w.r_s, w.G)          # all particles
    t1 = time.perf_counter()
    a_pp = o_pp.pp_accel(pos, w.mass, w.box, w.r_s, w.r_c, w.softening, w.G, targets=tg)
    t2 = time.perf_counter()
    t_pm, t_pp = t1 - t0, t2 - t1
    t_full = t_pm + t_pp * w.n / n_sample
    ref = (a_pp + a_pm[:, tg]) * w.mass
    errs = {}
    x = torch.as_tensor(pos, device="cuda")
    for prec in ("fp32", "fp64"):
        with binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, rs_cells=w.rs_cells,
                                         cutoff_rs=w.cutoff_rs, softening=w.softening,
                                         G=w.G, precision=prec), w.n) as P:
            F = P.force(x, w.mass)
            torch.cuda.synchronize()
            errs[prec] = metrics.force_errors(F.cpu().numpy()[:, tg], ref)
    return {
        "value": w.n / t_full,
        "unit": "particles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"O-PM on all {w.n} particles ({t_pm:.2f} s) + O-PP on {n_sample} "
                   f"sampled particles ({t_pp:.2f} s), PP time scaled by N/{n_sample}; "
                   "single-threaded NumPy/SciPy FP64"),
        "seconds_measured": t_pm + t_pp,
    }, errs


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the force path runs on one GPU; --gpus {args.gpus} is not "
              "supported (only --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1510_07621_amd import binding, ics

    w = ics.workload(WORKLOAD)
    pos = w.positions()
    r32 = time_precision(binding, torch, w, pos, "fp32", args.steps, args.warmup, args.dt)
    ms_step = 1e3 * r32["seconds"] / args.steps
    value = w.n * args.steps / r32["seconds"]
    pp_ms = r32["stage_ms_per_step"]["pp"]
    pairs = r32["pairs"]
    achieved = pairs * FLOP_PER_PAIR / (pp_ms * 1e-3) / 1e12
    out = {
        "metric": "P3M particles/s + pair-int/s, FP32 vs FP64 at stated force err; "
                  "adjoint/fwd ratio",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Zel'dovich lattice, PCG64 seed 2)",
        "config": {
            "workload": "zeldovich128: N=128^3 Zel'dovich-displaced lattice P(k)~k^-2 "
                        "rms 0.3 spacing, PM grid 128^3, r_s=1.25 cells, r_c=4.5 r_s, "
                        "eps=0.03 spacing, G=1, one KDK leapfrog step (dt=%g) per step"
                        % args.dt,
            "n_particles": w.n, "grid_n": w.grid_n, "precision": "fp32 force, fp64 x/p",
        },
        "pair_interactions_per_s": pairs / (pp_ms * 1e-3),
        "pairs_per_step": pairs,
        "stage_ms_per_step": r32["stage_ms_per_step"],
        "roofline": {
            "kernel": "k_pairs<float> (short-range pair loop)",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": measured_traffic(),
            "valu": measured_valu(),
            "flop_per_pair": FLOP_PER_PAIR,
            "avg_launch_ms": pp_ms,
        },
        "adjoint_fwd_ratio": None,
    }
    if not args.no_fp64:
        r64 = time_precision(binding, torch, w, pos, "fp64", args.fp64_steps, 1, args.dt)
        pp64 = r64["stage_ms_per_step"]["pp"]
        out["fp64"] = {
            "value": w.n * args.fp64_steps / r64["seconds"],
            "ms_per_step": 1e3 * r64["seconds"] / args.fp64_steps,
            "steps": args.fp64_steps,
            "pair_interactions_per_s": r64["pairs"] / (pp64 * 1e-3),
            "stage_ms_per_step": r64["stage_ms_per_step"],
            "pp_frac_of_fp64_peak": r64["pairs"] * FLOP_PER_PAIR / (pp64 * 1e-3) / 1e12
                                    / FP64_PEAK_TFLOPS,
        }
    if not args.no_configs:
        cfg_legs = [config_leg(binding, torch, name) for name in ("uniform32", "plummer256")]
        out["configs"] = [leg for leg, _ in cfg_legs]
    out["powerspec"] = powerspec_leg(binding, torch, w, pos)
    out["pp_ewald"] = ewald_leg(binding, torch)
    if not args.no_adjoint:
        legs = [adjoint_leg(binding, torch, "zeldovich64_kdk", "fp64", segment=1),
                adjoint_leg(binding, torch, "plummer128_kdk", "fp32")]
        out["adjoint_fwd_ratio"] = {leg["workload"]: leg["ratio"] for leg in legs}
        out["adjoint"] = legs
        # FP32-pair gradient of the clustered run against the FP64 path's, on
        # a 16^3 subset of particles (per-particle relative error of dL/dx0)
        g32 = adjoint_leg(binding, torch, "plummer128_kdk", "fp32", keep_grad=True)
        g64 = adjoint_leg(binding, torch, "plummer128_kdk", "fp64", keep_grad=True)
        sub = np.random.default_rng(16).choice(g64.shape[1], size=16 ** 3, replace=False)
        a = g32[:, sub].cpu().numpy()
        b = g64[:, sub].cpu().numpy()
        rel = np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)
        legs[1]["grad_err_vs_fp64_subset"] = {"rms": float(np.sqrt(np.mean(rel ** 2))),
                                              "median": float(np.median(rel)),
                                              "max": float(rel.max()), "particles": 16 ** 3}
    if not args.no_cpu:
        base, errs = cpu_leg(binding, torch, w, pos, args.cpu_sample)
        out["cpu_baseline"] = base
        out["force_err_vs_oracle"] = {k: {"rms": v["rms"], "max": v["max"]}
                                      for k, v in errs.items()}
        if not args.no_configs:
            for leg, sample in cfg_legs:
                config_errors(leg, sample)
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
    print(json.dumps(out))


if __name__ == "__main__":
    main()
