#!/usr/bin/env python3
"""Throughput of the PIC-MCC/PPPM hot path on one MI355X.

One step = the whole hot path once for every particle of the workload: RHS,
Poisson (FFT in x,y + tridiagonal in z), E, the fused gather / leapfrog /
electrode and grain absorption / PPPM sub-cycling / null-collision MCC /
CIC deposit kernel for both species, and the periodic cell sort.

Default workload: 64x64x256 cells of 50 um, 32 macro-particles per cell per
species (6.7e7 particles), 8 grains with a 3-cell PPPM cutoff.  The
FP32-refined form is the headline `value`; the plain FP64 form runs on the
same input for the speedup.  Particles are loaded in HBM before timing starts.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s + % HBM roofline, FP32-refined/batched vs FP64 at stated err"
HBM_PEAK_GBS = 8000.0
RECORD_BYTES = {"fp32r": 32, "fp64": 52}      # per particle: read once, written once
NODE_BYTES = {"fp32r": 16 + 8, "fp64": 32 + 8}  # per node and step: E read, rho written
# one Coulomb-collision pass, per alive particle: cell read to count and to
# scatter, id read, order key and slot written, then read, id read, velocity
# read and written (FP64: three position doubles instead of the packed cell,
# double velocities); per cell and species: the count cleared, scanned, its
# cursor cleared, its range read
COULOMB_BYTES = {"fp32r": 64, "fp64": 128}
COULOMB_CELL_BYTES = 48


TRAFFIC_PROFILES = {
    "push_fp32r": os.path.join(ROOT, "profiles", "hbm_traffic_push_f32r_full_64x64x256_ppc32.md"),
    "push_fp64": os.path.join(ROOT, "profiles", "hbm_traffic_push_f64_full_64x64x256_ppc32.md"),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1801_00972_amd", "csrc", f)
                  for f in ("particles.hip", "device_common.hpp", "pic_types.hpp")]


def traffic_per_particle_step(kernel, workload):
    """HBM bytes per particle-step of the push kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE record, if it was taken on the current
    kernel sources and this workload (else None)."""
    import hashlib
    path = TRAFFIC_PROFILES.get(kernel)
    if path is None or not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-record:"):
            rec = json.loads(line.split(":", 1)[1])
    if rec is None or rec.get("workload") != workload:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["fetch_bytes_per_particle_step"] + rec["write_bytes_per_particle_step"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _alive(sim):
    return sum(sum(sim.counters(r)["n_alive"]) for r in range(len(sim.wls)))


def _counter_sum_scalar(sim, key):
    return sum(sim.counters(r)[key] for r in range(len(sim.wls)))


def _counter_sum(sim, key):
    return sum(sum(sim.counters(r)[key]) for r in range(len(sim.wls)))


def fine_box(wl, h=0.08, cells=200):
    """The paper's diagnostic grid: cells^3 cells of h dx (200 of 0.08 dx cover
    16 PIC cells) around the centre of the grain cluster, inside the domain."""
    import numpy as np
    span = h * cells
    centre = np.asarray(wl["grain_pos"]).mean(axis=0) if len(wl["grain_pos"]) else \
        np.array([wl["nx"], wl["ny"], wl["nz"]]) / 2.0
    lim = np.array([wl["nx"], wl["ny"], wl["nz"]]) - span
    origin = np.clip(np.floor(centre - span / 2), 0, lim)
    return origin, h, (cells, cells, cells)


def run_form(wls, steps, warmup, sort_interval=8, autotune=True, label=None, average=0,
             fine=False):
    """Times one arithmetic form on one context (a list of replica workloads:
    one for the single-run forms, several for the batched ensemble)."""
    import torch

    from paper_1801_00972_amd.pic import (PIC_PROF_COULOMB, PIC_PROF_FIELD, PIC_PROF_LISTS,
                                          PIC_PROF_PUSH, PIC_PROF_SORT, Simulation,
                                          pic_profile_enable, pic_profile_read)

    label = label or wls[0]["name"]
    log(f"[bench] init {label} ({len(wls)} replica(s))")
    t_init = time.perf_counter()
    sim = Simulation(wls, sort_interval=sort_interval)
    torch.cuda.synchronize()
    log(f"[bench] init took {time.perf_counter() - t_init:.1f} s")
    tuning, trials = sim.tuning(), []
    if autotune:
        log("[bench] autotune (live steps)")
        tuning, trials = sim.autotune(trial_steps=48)
        log(f"[bench] settings {tuning} after {len(trials)} trials")
    if fine:
        for r, w in enumerate(wls):
            sim.set_fine_grid(*fine_box(w), replica=r)
    if average:
        # rf-phase-resolved averages (4 bins) sampled every `average` steps
        sim.average(average, 4)
    log(f"[bench] warmup {warmup} steps")
    sim.step(warmup)
    torch.cuda.synchronize()
    steps_before = sim.counters(0)["step"]
    # timed window 1: direct launches with every kernel class bracketed by events
    n_start = _alive(sim)
    md0, coll0 = _counter_sum(sim, "md_particles"), _counter_sum(sim, "n_collisions")
    fall0 = sum(sim.counters(r)["tile_fallback"] for r in range(len(wls)))
    coul0 = _counter_sum_scalar(sim, "n_coulomb")
    pic_profile_enable(sim.ctx, True)
    torch.cuda.synchronize()
    log(f"[bench] timing {steps} steps (direct launches, kernel events)")
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_end = _alive(sim)
    push_ms, push_n = pic_profile_read(sim.ctx, PIC_PROF_PUSH)
    field_ms, _ = pic_profile_read(sim.ctx, PIC_PROF_FIELD)
    sort_ms, sort_n = pic_profile_read(sim.ctx, PIC_PROF_SORT)
    lists_ms, _ = pic_profile_read(sim.ctx, PIC_PROF_LISTS)
    coul_ms, coul_n = pic_profile_read(sim.ctx, PIC_PROF_COULOMB)
    coul_pairs = _counter_sum_scalar(sim, "n_coulomb") - coul0
    pic_profile_enable(sim.ctx, False)
    md1, coll1 = _counter_sum(sim, "md_particles"), _counter_sum(sim, "n_collisions")
    fall1 = sum(sim.counters(r)["tile_fallback"] for r in range(len(wls)))
    # timed window 2: the same number of steps as a user runs them (the tuned
    # settings, no kernel events: replays of the captured step graph unless
    # the tuner found direct launches faster)
    log(f"[bench] timing {steps} steps (tuned path)")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    n_end2 = _alive(sim)
    tuned_ps = 0.5 * (n_end + n_end2) * steps
    particle_steps = 0.5 * (n_start + n_end) * steps
    wall = t1 - t0
    prec = wls[0]["precision"]
    nn = sum(w["nx"] * w["ny"] * (w["nz"] + 1) for w in wls)
    alg_bytes = particle_steps * 2 * RECORD_BYTES[prec] + steps * nn * NODE_BYTES[prec]
    achieved = alg_bytes / (push_ms * 1e-3) / 1e9 if push_ms > 0 else 0.0
    kernel = "push_batch_f32r" if tuning.get("batch_push") else "push_" + prec
    tpps = traffic_per_particle_step(kernel, wls[0]["name"] if len(wls) == 1 else "ensemble")
    traffic = tpps * particle_steps / max(push_n, 1) if tpps else None
    res = dict(
        value=tuned_ps / (t3 - t2),
        ms_per_step=1e3 * (t3 - t2) / steps,
        n_start=n_start, n_end=n_end2, replicas=len(wls),
        particles_loaded=sum(2 * w["nx"] * w["ny"] * w["nz"] * w["ppc"] for w in wls),
        settings=tuning,
        autotune_trials=[dict(t, ms_per_step=round(ms, 4)) for t, ms in trials],
        steps_before_timing=steps_before,
        direct_with_kernel_events=dict(value=particle_steps / wall, ms_per_step=1e3 * wall / steps),
        push_ms_per_launch=push_ms / max(push_n, 1),
        push_launches=push_n,
        field_ms_per_step=field_ms / steps,
        lists_ms_per_step=lists_ms / steps,
        sort_ms_total=sort_ms, sort_launches=sort_n,
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4),
                      traffic=round(traffic) if traffic else None,
                      traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE, WRITE_SIZE, calibrated)",
                      kernel=kernel, bytes_per_launch=alg_bytes / max(push_n, 1)),
        refine_residual=sim.counters(0)["refine_residual"] if prec == "fp32r" else None,
        tile_fallback_blocks=fall1 - fall0,
        md_particle_steps=md1 - md0,
        collisions=coll1 - coll0,
    )
    if average:
        res["averages"] = dict(interval=average, phase_bins=4,
                               fine_nodes=sim.fine_nodes if fine else None,
                               samples=sim.averages(0, -1, what=0)["samples"])
    if coul_n:
        # the pass runs at the start of a step on the particles alive then
        ncell = sum(w["nx"] * w["ny"] * w["nz"] for w in wls)
        per_pass = 0.5 * (n_start + n_end) * COULOMB_BYTES[prec] + ncell * COULOMB_CELL_BYTES
        gbs = per_pass * coul_n / (coul_ms * 1e-3) / 1e9
        res["coulomb"] = dict(interval=wls[0].get("coulomb_interval", 0), passes=coul_n,
                              ms_per_pass=coul_ms / coul_n, pairings=coul_pairs,
                              roofline=dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS,
                                            unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
                                            bytes_per_pass=per_pass))
        log(f"[bench] {label}: Coulomb pass {res['coulomb']['ms_per_pass']:.3f} ms "
            f"({coul_n} passes), {gbs:.0f} GB/s algorithmic")
    log(f"[bench] {label}: {res['value']:.3e} particle-steps/s, {res['ms_per_step']:.3f} ms/step "
        f"(direct with events {res['direct_with_kernel_events']['ms_per_step']:.3f} ms/step), "
        f"push {res['push_ms_per_launch']:.3f} ms/launch, {achieved:.0f} GB/s")
    sim.close()
    return res


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of nbytes (read nbytes + write nbytes),
    timed with HIP events: the HBM bandwidth this machine reaches, and the
    known-size kernel that calibrates the HBM byte counters."""
    import torch

    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return dict(bytes_per_copy=2 * nbytes, ms=ms, GBs=2 * nbytes / (ms * 1e-3) / 1e9)


def cpu_baseline(wl, steps=6):
    """The oracle, as it stands, on the same workload: loading untimed, then a
    bounded number of full steps timed on the host cores."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"[bench] cpu baseline: oracle, {steps} steps of {wl['name']} on {threads} threads")
    o = oracle.Oracle(dict(wl, precision="fp64"))
    o.init_particles()
    o._units()
    n0 = o.n_alive(0) + o.n_alive(1)
    t0 = time.perf_counter()
    o.step(steps)
    t1 = time.perf_counter()
    n1 = o.n_alive(0) + o.n_alive(1)
    ps = 0.5 * (n0 + n1) * steps
    res = dict(value=ps / (t1 - t0), unit="particle-steps/s", cores=threads, kind="oracle",
               sample=f"{steps} full FP64 oracle steps of {wl['name']} ({n0} particles) "
                      f"from the oracle's own loading, {t1 - t0:.1f} s",
               cpu_model=_cpu_model())
    # the same oracle on one thread, one more step of the same run
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        n2 = o.n_alive(0) + o.n_alive(1)
        t2 = time.perf_counter()
        o.step(1)
        t3 = time.perf_counter()
        n3 = o.n_alive(0) + o.n_alive(1)
        gomp.omp_set_num_threads(threads)
        res["single_thread"] = dict(value=0.5 * (n2 + n3) / (t3 - t2), unit="particle-steps/s",
                                    sample=f"step {steps + 1} of the same run, {t3 - t2:.1f} s")
    except OSError:
        res["single_thread"] = None
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def form_workloads(form, workload, coulomb=0, xs=False):
    wls = _form_workloads(form, workload)
    if xs:
        from paper_1801_00972_amd import workloads as W
        # energy-dependent cross sections from synthetic stand-in tables
        wls = [dict(w, xs=W.stand_in_xs()) for w in wls]
    if coulomb:
        # Coulomb collisions every `coulomb` steps, Coulomb logarithm 10
        wls = [dict(w, coulomb_interval=coulomb, coulomb_lnL=10.0) for w in wls]
    return wls


def _form_workloads(form, workload):
    from paper_1801_00972_amd import workloads as W
    if workload == "large":
        if form != "fp32r":
            raise SystemExit("the large workload (128x128x512, 16 ppc, 64 grains) is FP32R only")
        return [W.large_fp32r()]
    if form == "batched":
        return W.ensemble() if workload == "full" else W.small_ensemble()
    return [W.full_fp64(form) if workload == "full" else dict(W.small_fp64(), precision=form)]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=["full", "small", "large"], default="full")
    ap.add_argument("--forms", default="fp32r,fp64,batched")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--sort-interval", type=int, default=8)
    ap.add_argument("--average", type=int, default=0,
                    help="sample the time averages every N steps (0: off)")
    ap.add_argument("--fine", action="store_true",
                    help="with --average: also the 200^3 grid of 0.08 dx over the grain cluster")
    ap.add_argument("--xs", action="store_true",
                    help="energy-dependent cross sections (synthetic stand-in tables)")
    ap.add_argument("--coulomb", type=int, default=0,
                    help="Coulomb collisions every N steps (0: off, the default workloads)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", flush=True)
        sys.exit(2)

    import torch

    from paper_1801_00972_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if args.workload == "large":
        forms = ["fp32r"]
    results = {}
    for form in forms:
        wls = form_workloads(form, args.workload, args.coulomb, args.xs)
        results[form] = run_form(wls, args.steps, args.warmup, args.sort_interval,
                                 autotune=not args.no_autotune, average=args.average,
                                 fine=args.fine and args.average > 0,
                                 label=f"{form} {wls[0]['name']}" if len(wls) == 1 else
                                 f"batched ensemble of {len(wls)}")
    head = "fp32r" if "fp32r" in results else forms[0]
    wl = form_workloads(head, args.workload)[0]
    R = results[head]
    line = {
        "metric": METRIC,
        "value": R["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head in ("fp32r", "batched") else "f64",
        "data": "synthetic",
        "config": {
            "workload": wl["name"] if head != "batched" else "ensemble",
            "precision": head,
            "grid": [wl["nx"], wl["ny"], wl["nz"]],
            "ppc_per_species": wl["ppc"],
            "particles": 2 * wl["nx"] * wl["ny"] * wl["nz"] * wl["ppc"],
            "grains": int(len(wl["grain_pos"])),
            "pp_cutoff_cells": wl["cutoff"],
            "stated_err": {"fp32r": 1e-5, "fp64": 1e-12},
            "coulomb_interval": args.coulomb,
            "cross_section_tables": bool(args.xs),
            "average_interval": args.average,
            "fine_grid": bool(args.fine and args.average),
            "settings": R["settings"],
        },
        "roofline": R["roofline"],
        "forms": {k: {kk: v for kk, v in r.items() if kk != "roofline"} | {"roofline": r["roofline"]}
                  for k, r in results.items()},
    }
    if "fp64" in results and "fp32r" in results:
        line["speedup_fp32r_vs_fp64"] = results["fp32r"]["value"] / results["fp64"]["value"]
    if "fp64" in results and "batched" in results:
        line["speedup_batched_vs_fp64"] = results["batched"]["value"] / results["fp64"]["value"]
    cb = copy_bandwidth()
    line["copy_bandwidth"] = cb
    line["roofline"]["frac_of_measured_copy"] = round(R["roofline"]["achieved"] / cb["GBs"], 4)
    if args.workload == "large":
        # 2.7e8 FP64 oracle particles take ~15 GB and minutes per step: not a bounded sample
        line["cpu_baseline"] = None
    elif not args.no_cpu_baseline:
        cb = cpu_baseline(W.full_fp64("fp64") if args.workload == "full" else W.small_fp64())
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
