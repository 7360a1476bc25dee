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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(wl, steps, warmup, sort_interval=16):
    import torch

    from paper_1801_00972_amd.pic import (PIC_PROF_FIELD, PIC_PROF_LISTS, PIC_PROF_PUSH,
                                          PIC_PROF_SORT, Simulation, pic_profile_enable,
                                          pic_profile_read)

    log(f"[bench] init {wl['name']}")
    sim = Simulation(wl, sort_interval=sort_interval)
    torch.cuda.synchronize()
    log(f"[bench] warmup {warmup} steps")
    sim.step(warmup)
    torch.cuda.synchronize()
    c0 = sim.counters()
    pic_profile_enable(sim.ctx, True)
    torch.cuda.synchronize()
    log(f"[bench] timing {steps} steps")
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = sim.counters()
    push_ms, push_n = pic_profile_read(sim.ctx, PIC_PROF_PUSH)
    field_ms, _ = pic_profile_read(sim.ctx, PIC_PROF_FIELD)
    sort_ms, sort_n = pic_profile_read(sim.ctx, PIC_PROF_SORT)
    lists_ms, _ = pic_profile_read(sim.ctx, PIC_PROF_LISTS)
    pic_profile_enable(sim.ctx, False)
    n_start, n_end = sum(c0["n_alive"]), sum(c1["n_alive"])
    particle_steps = 0.5 * (n_start + n_end) * steps
    wall = t1 - t0
    nn = wl["nx"] * wl["ny"] * (wl["nz"] + 1)
    prec = wl["precision"]
    alg_bytes = particle_steps * 2 * RECORD_BYTES[prec] + steps * nn * NODE_BYTES[prec]
    achieved = alg_bytes / (push_ms * 1e-3) / 1e9 if push_ms > 0 else 0.0
    res = dict(
        value=particle_steps / wall,
        ms_per_step=1e3 * wall / steps,
        n_start=n_start, n_end=n_end,
        push_ms_per_launch=push_ms / max(push_n, 1),
        push_launches=push_n,
        field_ms_per_step=field_ms / steps,
        lists_ms_per_step=lists_ms / steps,
        sort_ms_total=sort_ms, sort_launches=sort_n,
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                      kernel="push_" + prec, bytes_per_launch=alg_bytes / max(push_n, 1)),
        refine_residual=c1["refine_residual"] if prec == "fp32r" else None,
        tile_fallback_blocks=c1["tile_fallback"] - c0["tile_fallback"],
        md_particle_steps=sum(c1["md_particles"]) - sum(c0["md_particles"]),
        collisions=sum(c1["n_collisions"]) - sum(c0["n_collisions"]),
    )
    log(f"[bench] {prec}: {res['value']:.3e} particle-steps/s, {res['ms_per_step']:.3f} ms/step, "
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


def cpu_baseline(wl, steps=2):
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
    return dict(value=ps / (t1 - t0), unit="particle-steps/s", cores=threads, kind="oracle",
                sample=f"{steps} full FP64 oracle steps of {wl['name']} ({n0} particles) "
                       f"from the oracle's own loading, {t1 - t0:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=["full", "small"], default="full")
    ap.add_argument("--forms", default="fp32r,fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sort-interval", type=int, default=16)
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
    results = {}
    for form in forms:
        wl = W.full_fp64(form) if args.workload == "full" else dict(W.small_fp64(), precision=form)
        results[form] = run_form(wl, args.steps, args.warmup, args.sort_interval)
    head = "fp32r" if "fp32r" in results else forms[0]
    wl = W.full_fp64(head) if args.workload == "full" else dict(W.small_fp64(), precision=head)
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
        "dtype": "f32" if head == "fp32r" else "f64",
        "data": "synthetic",
        "config": {
            "workload": wl["name"],
            "precision": head,
            "grid": [wl["nx"], wl["ny"], wl["nz"]],
            "ppc_per_species": wl["ppc"],
            "particles": 2 * wl["nx"] * wl["ny"] * wl["nz"] * wl["ppc"],
            "grains": int(len(wl["grain_pos"])),
            "pp_cutoff_cells": wl["cutoff"],
            "stated_err": {"fp32r": 1e-5, "fp64": 1e-12},
            "sort_interval": args.sort_interval,
        },
        "roofline": R["roofline"],
        "forms": {k: {kk: v for kk, v in r.items() if kk != "roofline"} | {"roofline": r["roofline"]}
                  for k, r in results.items()},
    }
    if "fp64" in results and "fp32r" in results:
        line["speedup_fp32r_vs_fp64"] = results["fp32r"]["value"] / results["fp64"]["value"]
    cb = copy_bandwidth()
    line["copy_bandwidth"] = cb
    line["roofline"]["frac_of_measured_copy"] = round(R["roofline"]["achieved"] / cb["GBs"], 4)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(W.full_fp64("fp64") if args.workload == "full" else W.small_fp64())
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
