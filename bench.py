"""Throughput of the P3M gravity step on one MI355X.

A step is one kick-drift-kick leapfrog step of the whole force path:
kick(dt/2) with the force of the previous step and drift(dt) (one fused
pass), the P3M force (binning, work list and the reaction prepass; the CIC
deposit, FFT Poisson solve and gradient + interpolation on the plan's second
stream beside the short-range pair sum; then the gather of the pair sum's
reactions, which adds the mesh part and writes the force) and kick(dt/2),
ordered on one HIP stream with the particles resident in HBM.

Headline workload (default): 256^3 particles, 70 % in 2000 Plummer spheres
(scale radii log-uniform in 0.002-0.02 box) and 30 % uniform, 256^3 PM grid,
r_s = 1.25 cells, r_c = 4.5 r_s, Plummer softening 0.03 spacing, G = 1,
m = 1/N; FP32 force arithmetic with FP64 positions, momenta, kick and drift;
pairs between dense groups evaluated once (pair_partials 80).

Prints one JSON line: particles/s over the timed steps (whole job), the pair
interaction rate, the roofline of the pair kernel (and of the pair stage, the
pair kernel and the gather of its reactions) from HIP events recorded around
every launch of the timed region, the mesh stages timed alone against HBM, FP64 and FP32 force
timings and errors on the other workloads (median of repeated calls after
three warm-ups), the adjoint legs, and the CPU oracle on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 41          # 37 FP32 arithmetic flops + 4 transcendentals per pair
FP32_PEAK_TFLOPS = 157.3    # MI355X published FP32 vector peak
FP64_PEAK_TFLOPS = 78.6     # MI355X published FP64 vector peak
HBM_PEAK_GBS = 8000.0
HEADLINE_PARTIALS = 80      # one-sided pair sum between dense groups (clustered set)


PROFILES = os.path.join(ROOT, "profiles")
PAIR_SOURCES = ("pair.hip", "react.hip", "p3m_internal.h")


def counter_record(name):
    """A committed counter summary of the pair stage (profiles/<name>.json),
    or None when the source of the pair kernel, of the gather or of the
    constants they share changed after the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(PROFILES, name + ".json")) as f:
            rec = json.load(f)
        digest = {}
        for src in PAIR_SOURCES:
            with open(os.path.join(ROOT, "paper_1510_07621_amd", "csrc", src), "rb") as f:
                digest[src] = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    return rec if rec.get("source_sha256") == digest else None


def log(msg):
    """Progress of the legs on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dt", type=float, default=0.001)
    ap.add_argument("--workload", default="plummer256", choices=["plummer256", "zeldovich128"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-workload force timings and errors")
    ap.add_argument("--no-mesh", action="store_true", help="skip the mesh-stage timings")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward timing of the differentiable leapfrog")
    ap.add_argument("--cpu-targets", type=int, default=16384,
                    help="particles whose short-range force the CPU oracle evaluates")
    ap.add_argument("--mesh-only", action="store_true",
                    help="time only the mesh stages (pm_force with nothing beside it) and "
                         "print them as one JSON line (the mesh stages' profiling command)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device (a plain copy "
                         "of known size, to scale memory counters in a profiled run)")
    return ap.parse_args()


def plan_for(binding, w, precision, pair_partials=0, adjoint=False):
    return binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, rs_cells=w.rs_cells,
                                       cutoff_rs=w.cutoff_rs, softening=w.softening, G=w.G,
                                       precision=precision, pair_partials=pair_partials,
                                       adjoint=adjoint), w.n)


def run_steps(binding, plan, st, m, dt, box, steps):
    """KDK steps on the state st (x, p, F, ids, order, and spare buffers x2,
    p2, ids2); F holds the force at x on entry and on exit. The particles are
    kept in the cell order of each force call: the force comes in that order
    and the second half-kick moves positions, momenta and ids into it, so the
    next binning reads nearly sorted input and the force's stores are in
    order."""
    for _ in range(steps):
        binding.kick_drift(st["x"], st["p"], st["F"], m, 0.5 * dt, dt, box)   # one pass
        plan.force_cell_order(st["x"], m, out=st["F"], order=st["order"])
        binding.kick_reorder(st["order"], st["x"], st["p"], st["F"], 0.5 * dt, ids=st["ids"],
                             out=(st["x2"], st["p2"], st["ids2"], None))
        for k in ("x", "p", "ids"):
            st[k], st[k + "2"] = st[k + "2"], st[k]


def time_steps(binding, torch, w, pos0, precision, steps, warmup, dt, pair_partials):
    plan = plan_for(binding, w, precision, pair_partials)
    x = torch.as_tensor(pos0, device="cuda").contiguous()
    st = {"x": x, "p": torch.zeros_like(x), "F": torch.empty_like(x),
          "ids": torch.arange(w.n, dtype=torch.int64, device="cuda"),
          "order": torch.empty(w.n, dtype=torch.int32, device="cuda"),
          "x2": torch.empty_like(x), "p2": torch.empty_like(x),
          "ids2": torch.empty(w.n, dtype=torch.int64, device="cuda")}
    m = w.mass
    # the initial force, and the particles into its cell order
    plan.force_cell_order(st["x"], m, out=st["F"], order=st["order"])
    binding.kick_reorder(st["order"], st["x"], st["p"], st["F"], 0.0, ids=st["ids"],
                         out=(st["x2"], st["p2"], st["ids2"], None))
    for k in ("x", "p", "ids"):
        st[k], st[k + "2"] = st[k + "2"], st[k]
    run_steps(binding, plan, st, m, dt, w.box, warmup)
    x = st["x"]
    pairs_before = plan.pair_count(x)
    torch.cuda.synchronize()
    plan.set_timing(steps)
    t0 = time.perf_counter()
    run_steps(binding, plan, st, m, dt, w.box, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x = st["x"]
    calls, stage_ms = plan.stage_times()
    plan.set_timing(0)
    pairs_after = plan.pair_count(x)
    plan.close()
    assert calls == steps, (calls, steps)
    return {"seconds": t1 - t0,
            "stage_ms_per_step": {k: v / steps for k, v in stage_ms.items()},
            "pairs": 0.5 * (pairs_before + pairs_after)}


def median_calls(torch, fn, warmup=3, runs=20):
    """Median wall time (ms, HIP events) of fn over `runs` calls after `warmup`."""
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), ts


def sample_targets(n, size, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(size, n), replace=False))


def force_leg(binding, torch, name, runs, legs, tg=None, w=None, pos=None):
    """Force evaluations of a named workload: per (precision, pair_partials)
    the median time of `runs` calls after 3 warm-ups, particles/s, pair
    interactions/s over the pair stage, and the forces at the sampled
    particles `tg` (default 512 of them) for the CPU error leg."""
    from paper_1510_07621_amd import ics
    if w is None:
        w = ics.workload(name)
        pos = w.positions()
    if tg is None:
        tg = sample_targets(w.n, 512, 99)
    x = torch.as_tensor(pos, device="cuda").contiguous()
    out = {"workload": name, "n_particles": w.n, "grid_n": w.grid_n}
    sampled = {}
    for prec, pp in legs:
        key = prec if pp == 0 else f"{prec}_one_sided"
        P = plan_for(binding, w, prec, pp)
        F = P.force(x, w.mass)
        pairs = P.pair_count(x)
        ms, _ = median_calls(torch, lambda: P.force(x, w.mass, out=F), runs=runs)
        P.set_timing(runs)
        for _ in range(runs):
            P.force(x, w.mass, out=F)
        ncall, st = P.stage_times()
        P.set_timing(0)
        sampled[key] = F.cpu().numpy()[:, tg]
        P.close()
        pair_ms = (st["pp"] + st["react"]) / ncall
        out[key] = {"ms_per_force": ms, "runs": runs, "particles_per_s": w.n / (ms * 1e-3),
                    "pairs": pairs, "pair_stage_ms": pair_ms,
                    "pair_interactions_per_s": pairs / (pair_ms * 1e-3),
                    "pair_frac_of_peak": pairs * FLOP_PER_PAIR / (pair_ms * 1e-3) / 1e12 /
                    (FP32_PEAK_TFLOPS if prec == "fp32" else FP64_PEAK_TFLOPS)}
    return out, (w, pos, tg, sampled)


def mesh_leg(binding, torch, name, precision, runs=10):
    """The long-range force alone (pm_force: binning, CIC deposit, FFT
    Poisson solve, gradient + interpolation) with nothing beside it: median
    stage times and their rates against HBM. Algorithmic bytes per stage
    (N particles, M grid cells, r bytes per real): binning 24N read + 24N
    written (sorted records in FP32, index, cell) + 8M (cell starts);
    deposit 16N + rM; FFT two passes per transform, each reading and writing
    the half-complex grid: 8 rM; gradient + interpolation 24N + rM read, 24N
    written."""
    from paper_1510_07621_amd import ics
    w = ics.workload(name)
    x = torch.as_tensor(w.positions(), device="cuda").contiguous()
    P = plan_for(binding, w, precision)
    F = P.pm_force(x, w.mass)
    for _ in range(3):
        P.pm_force(x, w.mass, out=F)
    per = {k: [] for k in ("bin", "deposit", "fft", "interp")}
    for _ in range(runs):
        P.set_timing(1)
        P.pm_force(x, w.mass, out=F)
        _, st = P.stage_times()
        for k in per:
            per[k].append(st[k])
    P.set_timing(0)
    P.close()
    n, M = w.n, w.grid_n ** 3
    r = 4 if precision == "fp32" else 8
    nbytes = {"bin": 48.0 * n + 8.0 * M, "deposit": 16.0 * n + r * M, "fft": 8.0 * r * M,
              "interp": 48.0 * n + r * M}
    out = {"workload": name, "precision": precision}
    for k, v in per.items():
        ms = float(np.median(v))
        gbs = nbytes[k] / (ms * 1e-3) / 1e9
        out[k] = {"ms": ms, "algorithmic_bytes": nbytes[k], "achieved_GBs": gbs,
                  "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    return out


def config_errors(out, sample, ref=None):
    """CPU side of a force leg: RMS / max per-particle force error of each
    timed case against the oracle (O-PP at the sampled particles + O-PM),
    or against `ref`, the oracle's forces at those particles."""
    from oracle import metrics
    from oracle import pm as o_pm
    from oracle import pp as o_pp
    w, pos, tg, sampled = sample
    if ref is None:
        ref = (o_pp.pp_accel(pos, w.mass, w.box, w.r_s, w.r_c, w.softening, w.G, targets=tg) +
               o_pm.pm_accel(pos, w.mass, w.box, w.grid_n, w.r_s, w.G, targets=tg)) * w.mass
    for key, F in sampled.items():
        err = metrics.force_errors(F, ref)
        out[key]["force_err_rms"] = err["rms"]
        out[key]["force_err_max"] = err["max"]
        out[key]["force_err_particles"] = int(tg.size)
    return ref


def ewald_leg(binding, torch, runs=5):
    """All-pairs PP force with the tabulated Ewald correction (64^3 table) on
    the 32^3 uniform workload, FP64: median time per call, ordered pairs/s."""
    from paper_1510_07621_amd import ics
    w = ics.workload("uniform32")
    P = binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, softening=w.softening, G=w.G,
                                    precision="fp64", ewald_gridsize=64), w.n)
    x = torch.as_tensor(w.positions(), device="cuda").contiguous()
    F = P.pp_ewald_force(x, w.mass)
    ms, _ = median_calls(torch, lambda: P.pp_ewald_force(x, w.mass, out=F), runs=runs)
    P.close()
    return {"workload": w.name, "ewald_gridsize": 64, "ms_per_call": ms,
            "pairs_per_s": float(w.n) * (w.n - 1) / (ms * 1e-3)}


def powerspec_leg(binding, torch, name="zeldovich128", runs=20):
    """One power-spectrum call (binning, CIC deposit, forward FFT with shell
    binning), FP32, grid_n / 2 shells, sigma at 8 cells: median time and the
    rate of its algorithmic bytes, 60 N (sort and pack 40 N, deposit reads
    20 N) + 24 M (deposit write 4 M, z pass 4 + 4 M, y pass 4 + 4 M, x pass
    4 M; M grid cells), against HBM."""
    from paper_1510_07621_amd import ics
    w = ics.workload(name)
    x = torch.as_tensor(w.positions(), device="cuda").contiguous()
    P = plan_for(binding, w, "fp32")
    R = 8.0 * w.h
    ms, _ = median_calls(torch, lambda: P.power_spectrum(x, w.mass, r_tophat=R), runs=runs)
    _, _, _, sig = P.power_spectrum(x, w.mass, r_tophat=R)
    P.close()
    nbytes = 60.0 * w.n + 24.0 * w.grid_n ** 3
    return {"workload": name, "ms_per_call": ms, "algorithmic_bytes": nbytes,
            "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "sigma_8cells": float(sig)}


def adjoint_leg(binding, torch, name, precision, segment=None, keep_grad=False, pair_partials=0):
    """Forward and backward time of the differentiable leapfrog: the
    workload's KDK steps from its positions at rest, loss = sum of squared
    final displacements (minimum image, from the initial positions), gradient
    with respect to the initial positions through autodiff.leapfrog with
    checkpoints every `segment` steps (default ceil(sqrt(steps))). One
    untimed warm-up pass."""
    from paper_1510_07621_amd import autodiff, ics
    w = ics.workload(name)
    x0 = torch.as_tensor(w.positions(), device="cuda").contiguous()
    p0 = torch.zeros_like(x0)
    seg = segment or max(1, math.ceil(math.sqrt(w.steps)))
    P = plan_for(binding, w, precision, pair_partials, adjoint=True)

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
            "pair_partials": pair_partials,
            "forward_s": tf, "backward_s": tb, "ratio": tb / tf, "loss": loss,
            "grad_rms": float(torch.sqrt((g * g).sum(0).mean()))}


_CPU_SHARED = {}     # inherited by the forked pool workers (not pickled per task)


def _pp_chunk(tg):
    """One worker of the CPU baseline: the oracle's short-range sum at its
    share of the sampled particles (the oracle builds its own k-d tree of all
    particles in every call)."""
    from oracle import pp as o_pp
    pos, w_args = _CPU_SHARED["pos"], _CPU_SHARED["w_args"]
    t0 = time.perf_counter()
    a = o_pp.pp_accel(pos, *w_args, targets=tg, chunk=128)
    return a, time.perf_counter() - t0


def cpu_leg(w, pos, tg):
    """The CPU oracle (FP64 P3M) on the host's cores (at most 16): O-PM on
    all particles (NumPy, one process), then O-PP at the sampled particles
    `tg` over a pool of processes. One pool task evaluates a single particle,
    which times the k-d tree build under the same load; the other tasks split
    the sample. Full O-PP is extrapolated as one tree build plus the sample's
    evaluation time x N / sample x (tasks on the sample) / (pool size), that
    is, with the evaluation spread over every core."""
    import multiprocessing as mp
    from oracle import pm as o_pm
    cores = max(2, min(16, len(os.sched_getaffinity(0))))
    w_args = (w.mass, w.box, w.r_s, w.r_c, w.softening, w.G)
    t0 = time.perf_counter()
    a_pm = o_pm.pm_accel(pos, w.mass, w.box, w.grid_n, w.r_s, w.G, targets=tg)
    t_pm = time.perf_counter() - t0
    chunks = [tg[:1]] + np.array_split(tg, cores - 1)
    _CPU_SHARED.update(pos=pos, w_args=w_args)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_pp_chunk, chunks, chunksize=1)
    t_pool = time.perf_counter() - t0
    _CPU_SHARED.clear()
    t_build = res[0][1]
    t_eval = max(r[1] for r in res[1:]) - t_build
    a_pp = np.concatenate([r[0] for r in res[1:]], axis=1)
    t_pp_full = t_build + max(t_eval, 0.0) * (w.n / tg.size) * (cores - 1) / cores
    t_full = t_pm + t_pp_full
    return {
        "value": w.n / t_full,
        "unit": "particles/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"O-PM on all {w.n} particles ({t_pm:.1f} s, 1 process), then O-PP at "
                   f"{tg.size} random particles split over {cores - 1} of a pool of {cores} "
                   f"processes ({t_pool:.1f} s wall; k-d tree build {t_build:.1f} s, timed by "
                   f"the pool's one-particle task; evaluation {t_eval:.1f} s); full O-PP "
                   f"extrapolated as one build + evaluation x N/{tg.size} spread over "
                   f"{cores} processes ({t_pp_full:.0f} s); NumPy/SciPy FP64"),
        "seconds_measured": t_pm + t_pool,
        "seconds_full_extrapolated": t_full,
    }, (a_pp + a_pm) * w.mass


def ewald_cpu_leg(torch, binding, n_targets=64):
    """The direct Ewald sum (O-EW, the accuracy truth) on the 32^3 uniform
    workload: time per target particle (and the full N extrapolated), and the
    P3M method error, oracle and GPU (FP64), against it at those targets."""
    from oracle import ewald, metrics
    from oracle import p3m as o_p3m
    from paper_1510_07621_amd import ics
    w = ics.workload("uniform32")
    pos = w.positions()
    tg = np.arange(0, w.n, w.n // n_targets)[:n_targets]
    t0 = time.perf_counter()
    truth = ewald.ewald_accel(pos, w.mass, w.box, eps=w.softening, targets=tg)
    t_ew = time.perf_counter() - t0
    ref = o_p3m.p3m_accel(pos, w.mass, w.box, w.grid_n, w.rs_cells, w.cutoff_rs,
                          w.softening, targets=tg)
    x = torch.as_tensor(pos, device="cuda").contiguous()
    with plan_for(binding, w, "fp64") as P:
        F = P.force(x, w.mass).cpu().numpy() / w.mass
    return {"workload": w.name, "targets": int(tg.size), "seconds": t_ew,
            "extrapolated_full_s": t_ew * w.n / tg.size,
            "p3m_method_err_oracle": metrics.force_errors(ref, truth),
            "p3m_method_err_gpu": metrics.force_errors(F[:, tg], truth)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the force path runs on one GPU; --gpus {args.gpus} is not "
              "supported (only --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1510_07621_amd import binding, ics

    if args.mesh_only:
        out = {"mesh": [mesh_leg(binding, torch, name, prec)
                        for name in ("zeldovich128", "plummer256") for prec in ("fp32", "fp64")]}
        copy_calibration(torch, args, out)
        print(json.dumps(out))
        return
    w = ics.workload(args.workload)
    pos = w.positions()
    partials = HEADLINE_PARTIALS if args.workload == "plummer256" else 0
    log(f"{args.workload}: {w.n} particles, timing {args.steps} steps")
    r = time_steps(binding, torch, w, pos, "fp32", args.steps, args.warmup, args.dt, partials)
    log(f"headline {1e3 * r['seconds'] / args.steps:.2f} ms/step")
    ms_step = 1e3 * r["seconds"] / args.steps
    st = r["stage_ms_per_step"]
    pairs = r["pairs"]
    pair_ms = st["pp"] + st["react"]
    # the dominant kernel: the pair kernel (every pair evaluation; in the
    # one-sided sum the gather after it only sums partials and, in the P3M
    # force, adds the mesh part and writes the force)
    achieved = pairs * FLOP_PER_PAIR / (st["pp"] * 1e-3) / 1e12
    desc = {"plummer256": "plummer256: N=256^3, 70% in 2000 Plummer spheres (scale radii "
                          "log-uniform 0.002-0.02 box), 30% uniform, PM grid 256^3",
            "zeldovich128": "zeldovich128: N=128^3 Zel'dovich-displaced lattice P(k)~k^-2 "
                            "rms 0.3 spacing, PM grid 128^3"}[args.workload]
    out = {
        "metric": "P3M particles/s + pair-int/s, FP32 vs FP64 at stated force err; "
                  "adjoint/fwd ratio",
        "value": w.n * args.steps / r["seconds"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded, PCG64)",
        "config": {
            "workload": desc + ", r_s=1.25 cells, r_c=4.5 r_s, eps=0.03 spacing, G=1, one KDK "
                               "leapfrog step (dt=%g) per step" % args.dt,
            "n_particles": w.n, "grid_n": w.grid_n, "precision": "fp32 force, fp64 x/p",
            "pair_partials": partials,
            "particle_order": "cell order of the last force call (ids carried along)",
        },
        "pair_interactions_per_s": pairs / (pair_ms * 1e-3),
        "pairs_per_step": pairs,
        "stage_ms_per_step": st,
        "roofline": {
            "kernel": "k_pairs<float> (short-range pair sum)",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": None,
            "valu": None,
            "flop_per_pair": FLOP_PER_PAIR,
            "avg_launch_ms": st["pp"],
            "pair_stage": {
                "kernels": "k_pairs + k_react_gather (the gather also adds the mesh part and "
                           "writes the force)" if partials else "k_pairs",
                "avg_ms": pair_ms,
                "frac": pairs * FLOP_PER_PAIR / (pair_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                "avg_launch_ms_parts": {"k_pairs": st["pp"], "k_react_gather": st["react"]},
            },
        },
        "adjoint_fwd_ratio": None,
    }
    if args.workload == "plummer256":
        # HBM bytes per launch of the pair stage and its VALU issue, from the
        # committed counter runs of this workload (null once the sources changed)
        rec = counter_record("pair_stage_plummer256_traffic")
        if rec:
            out["roofline"]["traffic"] = rec["k_pairs"]["fetch_bytes"] + rec["k_pairs"]["write_bytes"]
            out["roofline"]["pair_stage"]["traffic"] = rec["bytes_per_launch"]
        rec = counter_record("pair_stage_plummer256_valu")
        if rec:
            out["roofline"]["valu"] = {k: {q: v[q] for q in ("valu_issue_util", "valu_lane_util",
                                                              "valu_issue_per_cu_clock",
                                                              "clock_ghz")}
                                       for k, v in rec["kernels"].items()}
    tg_head = sample_targets(w.n, args.cpu_targets, 77)
    cfg = []
    if not args.no_configs:
        cfg.append(force_leg(binding, torch, "uniform32", 20,
                             legs=(("fp64", 0), ("fp32", 0))))
        cfg.append(force_leg(binding, torch, "zeldovich128", 20,
                             legs=(("fp32", 0), ("fp64", 0))))
        cfg.append(force_leg(binding, torch, "plummer256", 5,
                             legs=(("fp32", HEADLINE_PARTIALS), ("fp32", 0),
                                   ("fp64", HEADLINE_PARTIALS), ("fp64", 0)),
                             tg=tg_head if args.workload == "plummer256" else None,
                             w=w if args.workload == "plummer256" else None,
                             pos=pos if args.workload == "plummer256" else None))
        out["configs"] = [c for c, _ in cfg]
        log("force legs done")
    if not args.no_mesh:
        out["mesh"] = [mesh_leg(binding, torch, name, prec)
                       for name in ("zeldovich128", "plummer256") for prec in ("fp32", "fp64")]
        log("mesh legs done")
    out["powerspec"] = powerspec_leg(binding, torch)
    out["pp_ewald"] = ewald_leg(binding, torch)
    if not args.no_adjoint:
        legs = [adjoint_leg(binding, torch, "zeldovich64_kdk", "fp64", segment=1),
                adjoint_leg(binding, torch, "plummer128_kdk", "fp32")]
        out["adjoint_fwd_ratio"] = {leg["workload"]: leg["ratio"] for leg in legs}
        out["adjoint"] = legs
        log("adjoint legs done")
        g32 = adjoint_leg(binding, torch, "plummer128_kdk", "fp32", keep_grad=True)
        g64 = adjoint_leg(binding, torch, "plummer128_kdk", "fp64", keep_grad=True)
        sub = np.random.default_rng(16).choice(g64.shape[1], size=16 ** 3, replace=False)
        a = g32[:, sub].cpu().numpy()
        b = g64[:, sub].cpu().numpy()
        rel = np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)
        legs[1]["grad_fp32_vs_fp64_gpu_subset"] = {"rms": float(np.sqrt(np.mean(rel ** 2))),
                                                  "median": float(np.median(rel)),
                                                  "max": float(rel.max()), "particles": 16 ** 3}
    if not args.no_cpu:
        from oracle import metrics
        # the headline's force path (both precisions) at the sampled particles
        x = torch.as_tensor(pos, device="cuda").contiguous()
        head = {}
        for prec, pp in (("fp32", partials), ("fp64", 0)):
            with plan_for(binding, w, prec, pp) as P:
                head[prec] = P.force(x, w.mass).cpu().numpy()[:, tg_head]
        del x
        log("CPU oracle leg")
        base, ref = cpu_leg(w, pos, tg_head)
        log(f"CPU oracle leg done ({base['seconds_measured']:.0f} s)")
        out["cpu_baseline"] = base
        out["force_err_vs_oracle"] = {}
        for prec, F in head.items():
            e = metrics.force_errors(F, ref)
            out["force_err_vs_oracle"][prec] = {"rms": e["rms"], "max": e["max"],
                                                "particles": int(tg_head.size)}
        for leg, sample in cfg:
            config_errors(leg, sample, ref if leg["workload"] == args.workload else None)
        out["ewald"] = ewald_cpu_leg(torch, binding)
        log("Ewald leg done")
    copy_calibration(torch, args, out)
    print(json.dumps(out))


def copy_calibration(torch, args, out):
    """A plain device-to-device copy of known size after the run, whose memory
    counters scale those of the kernels in a profiled run."""
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes


if __name__ == "__main__":
    main()
