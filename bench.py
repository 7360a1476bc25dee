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
RECORD_WRITTEN = {"fp32r": 28, "fp64": 48}    # of which the push writes back (not the id)
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
             fine=False, keep_state=False, persistent=False):
    """Times one arithmetic form on one context (a list of replica workloads:
    one for the single-run forms, several for the batched ensemble).
    keep_state: also return the state after the timed windows, its fields and
    the state one more step later (for the CPU baseline's comparison).
    persistent: for an ensemble whose tuner did not choose the persistent
    push, also time the steps with it (batch_push = 1)."""
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
    moved = alg_bytes - particle_steps * (RECORD_BYTES[prec] - RECORD_WRITTEN[prec])
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
                      kernel=kernel, bytes_per_launch=alg_bytes / max(push_n, 1),
                      frac_of_bytes_written=round(moved / (push_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                      if push_ms > 0 else 0.0,
                      note="frac_of_bytes_written: the same time against the bytes the "
                           "kernel must move (the id is read, never written back)"),
        refine_residual=sim.counters(0)["refine_residual"] if prec == "fp32r" else None,
        tile_fallback_blocks=fall1 - fall0,
        md_particle_steps=md1 - md0,
        collisions=coll1 - coll0,
    )
    res["push_form"] = ("one persistent launch for every replica and species"
                        if tuning.get("batch_push") else
                        "one launch per replica and species" if len(wls) > 1 else
                        "one launch per species")
    if persistent and len(wls) > 1 and not tuning.get("batch_push"):
        # the persistent one-launch push, timed on the same live run
        sim.set_tuning(batch_push=1)
        pic_profile_enable(sim.ctx, True)
        n0p = _alive(sim)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        n1p = _alive(sim)
        pms, pn = pic_profile_read(sim.ctx, PIC_PROF_PUSH)
        pic_profile_enable(sim.ctx, False)
        pps = 0.5 * (n0p + n1p) * steps
        pbytes = pps * 2 * RECORD_BYTES[prec] + steps * nn * NODE_BYTES[prec]
        pach = pbytes / (pms * 1e-3) / 1e9 if pms > 0 else 0.0
        res["persistent_launch"] = dict(
            value=pps / (t5 - t4), ms_per_step=1e3 * (t5 - t4) / steps,
            note="direct launches with kernel events, batch_push = 1",
            push_ms_per_launch=pms / max(pn, 1),
            roofline=dict(bound="hbm", achieved=round(pach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(pach / HBM_PEAK_GBS, 4), kernel="push_batch_f32r"))
        log(f"[bench] {label}: persistent push {res['persistent_launch']['value']:.3e} "
            f"particle-steps/s, {res['persistent_launch']['ms_per_step']:.3f} ms/step")
    if keep_state:
        from paper_1801_00972_amd.pic import PIC_E, PIC_PHI, PIC_RHO_FIXED
        before = sim.get_state()
        flds = sim.fields(0, PIC_PHI | PIC_E | (PIC_RHO_FIXED if prec == "fp32r" else 0))
        sim.step(1)
        res["_snapshot"] = dict(before=before, fields=flds, after=sim.get_state())
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


def _native_oracle():
    """The oracle built for this host (-O3 -march=native, OpenMP, no fast-math),
    with the threads bound close (read when its OpenMP runtime loads)."""
    import tempfile

    import oracle
    os.environ.setdefault("OMP_PROC_BIND", "close")
    out = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle_native.so")
    oracle.build(native=True, out=out)
    oracle.use_library(out)
    return oracle


def fp32r_error(wl, snap, o):
    """Per-quantity error of the FP32R form against the FP64 oracle: the
    fields of one state and one step of every particle from it (the oracle
    `o` holds that state and moves it in its own field)."""
    import numpy as np

    from tests.parity_util import compare_step_all
    f_o = o.fields(fixed_point=True)
    g = snap["fields"]
    V = max(abs(o.rf_voltage(snap["before"]["step"])), 1e-300)
    err = dict(
        rho_fixed_bit_exact=bool(np.array_equal(g["rho_fixed"], f_o["rho_fixed"])),
        phi=float(np.abs(g["phi"] - f_o["phi"]).max() / max(np.abs(f_o["phi"]).max(), V)),
        E=float(np.abs(g["E"] - f_o["E"]).max() / np.abs(f_o["E"]).max()),
    )
    o.step_in_field(f_o["E"])
    after = snap["after"]
    rep = compare_step_all(wl, after, o, 1.0, 1.0, 1e-5)
    err.update(position_cells=rep["max_dpos"], velocity=rep["max_dvel"],
               discrete_flips=rep["flips"], particles=rep["n"],
               grain_count_diff=int(np.abs(after["grain_count"] - o.grain_count).sum()),
               grain_counts=after["grain_count"].tolist())
    return err


def divergence(wl, steps, warmup):
    """How far the FP32R form drifts from the FP64 form over `steps` steps: the
    FP32R state after `warmup` steps is loaded exactly into an FP64 context,
    both step on, and particles, potential and grain counts are compared."""
    import numpy as np

    from paper_1801_00972_amd.pic import PIC_PHI, Simulation
    a = Simulation(dict(wl, precision="fp32r"))
    a.step(warmup)
    b = Simulation(dict(wl, precision="fp64"))
    b.set_state(a.get_state())
    out = dict(start_step=warmup, steps=steps, checkpoints=[])
    done = 0
    for k in sorted({1, 10, 100, steps}):
        if k > steps:
            continue
        a.step(k - done)
        b.step(k - done)
        done = k
        sa, sb = a.get_state(), b.get_state()
        row = dict(after=k)
        for s, name in ((0, "electrons"), (1, "ions")):
            ia, ib = sa[s]["id"], sb[s]["id"]
            common, ka, kb = np.intersect1d(ia, ib, assume_unique=True, return_indices=True)
            d = sa[s]["pos"][ka] - sb[s]["pos"][kb]
            for ax, n in ((0, wl["nx"]), (1, wl["ny"])):
                d[:, ax] -= n * np.round(d[:, ax] / n)
            dist = np.sqrt((d * d).sum(axis=1))
            dv = np.abs(sa[s]["vel"][ka] - sb[s]["vel"][kb]).max(axis=1)
            vs = np.abs(sb[s]["vel"][kb]).max(axis=1)
            row[name] = dict(alive_fp32r=int(len(ia)), alive_fp64=int(len(ib)),
                             only_one_form=int(len(ia) + len(ib) - 2 * len(common)),
                             pos_cells_median=float(np.median(dist)),
                             pos_cells_p99=float(np.quantile(dist, 0.99)),
                             pos_cells_max=float(dist.max()),
                             vel_rel_median=float(np.median(dv / vs)),
                             vel_rel_p99=float(np.quantile(dv / vs, 0.99)))
        fa, fb = a.fields(0, PIC_PHI), b.fields(0, PIC_PHI)
        row["phi_rel"] = float(np.abs(fa["phi"] - fb["phi"]).max() / np.abs(fb["phi"]).max())
        ga, gb = a.grain_charges()[0], b.grain_charges()[0]
        row["grain_net_fp32r"] = (ga[:, 1] - ga[:, 0]).tolist()
        row["grain_net_fp64"] = (gb[:, 1] - gb[:, 0]).tolist()
        log(f"[bench] divergence after {k} steps: {row}")
        out["checkpoints"].append(row)
    a.close()
    b.close()
    del np
    return out


def cpu_baseline(wl, snap=None, steps=12):
    """The oracle, as it stands, timed on the host cores on the benchmark's own
    state (the FP32R state after the timed windows, read back exactly), a
    bounded number of full steps; with that state also the per-quantity error
    of the FP32R form's step against the oracle's."""
    import numpy as np
    oracle = _native_oracle()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    wl64 = dict(wl, precision="fp64")
    res = dict(unit="particle-steps/s", cores=threads, kind="oracle", cpu_model=_cpu_model(),
               nproc=nproc, omp_proc_bind=os.environ.get("OMP_PROC_BIND"),
               build="gcc -O3 -march=native -fopenmp -ffp-contract=off (no fast-math)")
    if snap is not None:
        log(f"[bench] cpu baseline: FP32R error of one step against the oracle")
        o = oracle.Oracle(wl64)
        st = snap["before"]
        for s in range(2):
            o.set_particles(s, st[s]["pos"], st[s]["vel"], st[s]["id"])
        o.set_counts(grain_count=st["grain_count"], wall_count=st["wall_count"], step=st["step"])
        res["fp32r_error"] = fp32r_error(wl, snap, o)
        log(f"[bench] FP32R error: {res['fp32r_error']}")
        src = ("the benchmark's FP32R state after its timed steps, read back exactly "
               f"(step {st['step']})")
        o = oracle.Oracle(wl64)
        for s in range(2):
            o.set_particles(s, st[s]["pos"], st[s]["vel"], st[s]["id"])
        o.set_counts(grain_count=st["grain_count"], wall_count=st["wall_count"], step=st["step"])
        o.compact()
    else:
        o = oracle.Oracle(wl64)
        o.init_particles()
        src = "the oracle's own loading"
    o._units()
    log(f"[bench] cpu baseline: oracle, {steps} steps of {wl['name']} on {threads} threads")
    n0 = o.n_alive(0) + o.n_alive(1)
    t0 = time.perf_counter()
    o.step(steps)
    t1 = time.perf_counter()
    n1 = o.n_alive(0) + o.n_alive(1)
    res["value"] = 0.5 * (n0 + n1) * steps / (t1 - t0)
    res["sample"] = (f"{steps} full FP64 oracle steps of {wl['name']} ({n0} particles) from "
                     f"{src}, {t1 - t0:.1f} s")
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
    del np
    return res


def _cpu_model():
    """The host CPU's model name, as lscpu gives it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
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
    ap.add_argument("--divergence", type=int, default=0,
                    help="only measure how far FP32R drifts from FP64 over N steps "
                         "(from the state after --warmup FP32R steps) and print it as JSON")
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
    if args.divergence > 0:
        wl = W.full_fp64("fp32r") if args.workload == "full" else W.small_fp64()
        print(json.dumps(dict(metric="fp32r_vs_fp64_divergence", workload=wl["name"],
                              **divergence(wl, args.divergence, args.warmup))), flush=True)
        return
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if args.workload == "large":
        forms = ["fp32r"]
    results = {}
    head = "fp32r" if "fp32r" in forms else forms[0]
    want_cpu = not args.no_cpu_baseline and args.workload != "large"
    for form in forms:
        wls = form_workloads(form, args.workload, args.coulomb, args.xs)
        results[form] = run_form(wls, args.steps, args.warmup, args.sort_interval,
                                 autotune=not args.no_autotune, average=args.average,
                                 fine=args.fine and args.average > 0,
                                 keep_state=want_cpu and form == "fp32r" and form == head,
                                 persistent=form == "batched",
                                 label=f"{form} {wls[0]['name']}" if len(wls) == 1 else
                                 f"batched ensemble of {len(wls)}")
        if form == "batched":
            # the plain FP64 form on the same replicas, for the batched form's speedup
            wls64 = [dict(w, precision="fp64") for w in wls]
            r64 = run_form(wls64, args.steps, args.warmup, args.sort_interval, autotune=False,
                           label=f"fp64 ensemble of {len(wls64)}")
            results["batched"]["fp64_same_replicas"] = {
                k: r64[k] for k in ("value", "ms_per_step", "push_ms_per_launch", "settings")}
    wl = form_workloads(head, args.workload)[0]
    snap = results.get(head, {}).pop("_snapshot", None)
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
    if "batched" in results:
        # the same 16 replicas stepped in the plain FP64 form
        line["speedup_batched_vs_fp64"] = (results["batched"]["value"] /
                                           results["batched"]["fp64_same_replicas"]["value"])
    cb = copy_bandwidth()
    line["copy_bandwidth"] = cb
    line["roofline"]["frac_of_measured_copy"] = round(R["roofline"]["achieved"] / cb["GBs"], 4)
    if args.workload == "large":
        # 2.7e8 FP64 oracle particles take ~15 GB and minutes per step: not a bounded sample
        line["cpu_baseline"] = None
    elif not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, snap)
        if "fp32r_error" in line["cpu_baseline"]:
            line["fp32r_error"] = line["cpu_baseline"]["fp32r_error"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
