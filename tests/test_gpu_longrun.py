"""Long-run statistics: each GPU form against the FP64 oracle as distributions.

The column workload (16x16x128 cells of 50 um, 4 ppc, two grains in the rf
sheath) runs 2000 steps from loading.  The oracle side is 32 runs with seeds
1000..1031, stored in tests/golden/longrun_oracle_column.json by
tests/golden/make_longrun_oracle.py (which calls only the oracle); the GPU
side is 32 runs with seeds 0..31 per form: FP64, FP32R, and FP32R as one
batched context of the 32 replicas.  Disjoint seeds make the two sides
independent samples of one distribution, so the comparison is a genuine
two-sample test rather than a check that identical trajectories stay
identical.  Per quantity (each grain's absorbed electrons and ions and its
net count averaged over the last fifth of the steps, the surviving electrons
at half time and at the end, the surviving ions, the four electrode tallies,
and the laterally averaged potential over the last fifth at three planes)
the means must agree within three standard errors of their difference,
|mean_gpu - mean_oracle| <= 3 sqrt(s_gpu^2 / S_gpu + s_oracle^2 / S_oracle).
"""
import json
import os

import numpy as np
import pytest

from paper_1801_00972_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "longrun_oracle_column.json")
SEEDS = 32


def _golden():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    assert g["workload"] == W.column()["name"]
    return g


def _names(ng, planes):
    names = []
    for g in range(ng):
        names += [f"grain{g}_e", f"grain{g}_i", f"q_tail{g}"]
    names += ["alive_e_half", "alive_e_end", "alive_i_end", "wall0_e", "wall0_i", "wall1_e", "wall1_i"]
    names += [f"phi_z{p}" for p in planes]
    return names


def _row(grain_e, grain_i, q_tail, alive_e, alive_i, wall, phi_planes):
    r = []
    for g in range(len(grain_e)):
        r += [grain_e[g], grain_i[g], q_tail[g]]
    r += list(alive_e) + [alive_i, wall[0][0], wall[0][1], wall[1][0], wall[1][1]]
    return r + list(phi_planes)


def _oracle_rows(gold):
    return np.array([_row(r["grain_e"], r["grain_i"], r["q_tail"], r["alive_e"], r["alive_i"],
                          r["wall"], r["phi_planes"]) for r in gold["rows"]], float)


def _gpu_rows(prec, batched, gold):
    from paper_1801_00972_amd.pic import PIC_PHI, Simulation
    steps, tail, planes = gold["steps"], gold["tail"], gold["planes"]
    wls = [W.column(seed, prec) for seed in range(SEEDS)]
    sims = [Simulation(wls)] if batched else [Simulation(w) for w in wls]
    reps = [(sim, r) for sim in sims for r in range(len(sim.wls))]
    nx, ny, nz = wls[0]["nx"], wls[0]["ny"], wls[0]["nz"]
    ng = len(wls[0]["grain_pos"])
    alive_half = np.zeros(len(reps))
    for sim in sims:
        sim.step(steps // 2)
    for i, (sim, r) in enumerate(reps):
        alive_half[i] = sim.counters(r)["n_alive"][0]
    for sim in sims:
        sim.step(steps // 2 - tail)
        sim.average(1, 1)  # phi_k of the last `tail` steps
    q = np.zeros((len(reps), ng))
    for _ in range(tail):
        for sim in sims:
            sim.step(1)
        for i, (sim, r) in enumerate(reps):
            counts, _ = sim.grain_charges(r)
            q[i] += counts[:, 1] - counts[:, 0]
    rows = []
    for i, (sim, r) in enumerate(reps):
        c = sim.counters(r)
        counts, _ = sim.grain_charges(r)
        av = sim.averages(r, -1, PIC_PHI)
        assert av["samples"] == tail
        phi_z = av["phi"].reshape(nz + 1, ny, nx).mean(axis=(1, 2))
        rows.append(_row(counts[:, 0], counts[:, 1], q[i] / tail, [alive_half[i], c["n_alive"][0]],
                         c["n_alive"][1], c["wall_count"], [phi_z[p] for p in planes]))
    for sim in sims:
        sim.close()
    return np.array(rows, float)


@pytest.mark.parametrize("form", ["fp64", "fp32r", "fp32r_batched"])
def test_long_run_distributions_match_oracle(form):
    gold = _golden()
    prec = "fp64" if form == "fp64" else "fp32r"
    print(f"[case] {form}: {SEEDS} seeds x {gold['steps']} steps of {gold['workload']}", flush=True)
    g = _gpu_rows(prec, form.endswith("batched"), gold)
    o = _oracle_rows(gold)
    ng = len(W.column()["grain_pos"])
    names = _names(ng, gold["planes"])
    assert g.shape[1] == o.shape[1] == len(names)
    print("  per-seed rows (first 4 of each side):", flush=True)
    for k in range(4):
        print(f"    gpu seed {k:4d}: {np.array2string(g[k], precision=3, max_line_width=250)}")
        print(f"    oracle {gold['rows'][k]['seed']:4d}: "
              f"{np.array2string(o[k], precision=3, max_line_width=250)}", flush=True)
    # the samples are samples: the seeds' rows differ within each side and
    # no GPU row repeats an oracle row
    assert len({tuple(r) for r in g}) > SEEDS // 2
    assert not any(np.array_equal(r, s) for r in g for s in o)
    bad = []
    for k, name in enumerate(names):
        mg, mo = g[:, k].mean(), o[:, k].mean()
        se = np.sqrt(g[:, k].var(ddof=1) / len(g) + o[:, k].var(ddof=1) / len(o))
        flag = abs(mg - mo) > 3 * se + 1e-9 * max(abs(mo), 1.0)
        print(f"  {name:13s} gpu {mg:12.4f} (sd {g[:, k].std(ddof=1):9.4f})  oracle {mo:12.4f} "
              f"(sd {o[:, k].std(ddof=1):9.4f})  |diff| {abs(mg - mo):9.4f}  3se {3 * se:9.4f}"
              f"{'  <--' if flag else ''}", flush=True)
        if flag:
            bad.append(name)
    assert not bad, f"means differ beyond 3 standard errors: {bad}"
    # every particle is accounted for in every run
    n0 = 16 * 16 * 128 * 4
    for rows in (g, o):
        e = sum(rows[:, 3 * i] for i in range(ng)) + rows[:, 3 * ng + 1] + rows[:, 3 * ng + 3] + \
            rows[:, 3 * ng + 5]
        i_ = sum(rows[:, 3 * i + 1] for i in range(ng)) + rows[:, 3 * ng + 2] + rows[:, 3 * ng + 4] + \
            rows[:, 3 * ng + 6]
        assert np.all(e == n0) and np.all(i_ == n0)
