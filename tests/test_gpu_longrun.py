"""Long-run statistics: GPU forms against the oracle over many seeds.

The step is chaotic, so after a few hundred steps single trajectories of two
correct implementations part.  What must agree is the distribution: for each
of 16 seeds of the small box (16x16x32 cells, 8 ppc, one grain on a node),
500 steps of the oracle (FP64) and of each GPU form (FP64; FP32R; FP32R as one
batched context of 16 replicas) give the grain's electron and ion counts, the
survivors per species and the electrode tallies at the end, and the grain
charge averaged over the last 100 steps.  Per quantity the seed means must
agree within three standard errors of their difference,
|mean_gpu - mean_oracle| <= 3 sqrt(s_gpu^2 / S + s_oracle^2 / S).
"""
import numpy as np
import pytest

import oracle
from paper_1801_00972_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SEEDS = 16
STEPS = 500
TAIL = 100
NAMES = ["grain_e", "grain_i", "alive_e", "alive_i", "wall0_e", "wall0_i", "wall1_e", "wall1_i",
         "Q_tail"]


def _wl(seed, prec):
    return dict(W.small_fp64(), precision=prec, seed=seed, name=f"small_seed{seed}")


def _row(gc, alive, wall, q_tail):
    return [gc[0, 0], gc[0, 1], alive[0], alive[1], wall[0][0], wall[0][1], wall[1][0], wall[1][1],
            q_tail]


@pytest.fixture(scope="module")
def oracle_runs():
    rows = []
    for seed in range(SEEDS):
        o = oracle.Oracle(_wl(seed, "fp64"))
        o.init_particles()
        o.step(STEPS - TAIL)
        q = 0.0
        for _ in range(TAIL):
            o.step(1)
            q += float(o.grain_count[0, 1] - o.grain_count[0, 0])
        rows.append(_row(o.grain_count, [o.n_alive(0), o.n_alive(1)], o.wall_count, q / TAIL))
        print(f"[oracle] seed {seed}: {rows[-1]}", flush=True)
    return np.array(rows, float)


def _gpu_runs(prec, batched):
    from paper_1801_00972_amd.pic import Simulation
    wls = [_wl(seed, prec) for seed in range(SEEDS)]
    sims = [Simulation(wls)] if batched else [Simulation(w) for w in wls]
    reps = [(sim, r) for sim in sims for r in range(len(sim.wls))]
    for sim in sims:
        sim.step(STEPS - TAIL)
    q = np.zeros(SEEDS)
    for _ in range(TAIL):
        for sim in sims:
            sim.step(1)
        for i, (sim, r) in enumerate(reps):
            counts, _ = sim.grain_charges(r)
            q[i] += float(counts[0, 1] - counts[0, 0])
    rows = []
    for i, (sim, r) in enumerate(reps):
        c = sim.counters(r)
        counts, _ = sim.grain_charges(r)
        rows.append(_row(counts, c["n_alive"], c["wall_count"], q[i] / TAIL))
    for sim in sims:
        sim.close()
    return np.array(rows, float)


@pytest.mark.parametrize("form", ["fp64", "fp32r", "fp32r_batched"])
def test_long_run_statistics_match_oracle(form, oracle_runs):
    prec = "fp64" if form == "fp64" else "fp32r"
    print(f"[case] {form}: {SEEDS} seeds x {STEPS} steps of the 16x16x32 box", flush=True)
    g = _gpu_runs(prec, batched=form.endswith("batched"))
    o = oracle_runs
    bad = []
    for k, name in enumerate(NAMES):
        mg, mo = g[:, k].mean(), o[:, k].mean()
        se = np.sqrt(g[:, k].var(ddof=1) / SEEDS + o[:, k].var(ddof=1) / SEEDS)
        print(f"  {name:8s} gpu {mg:12.3f}  oracle {mo:12.3f}  |diff| {abs(mg - mo):9.3f}  3se {3 * se:9.3f}",
              flush=True)
        if abs(mg - mo) > 3 * se + 1e-9 * max(abs(mo), 1.0):
            bad.append(name)
    assert not bad, f"means differ beyond 3 standard errors: {bad}"
    # every particle is accounted for in every run
    n0 = 16 * 16 * 32 * 8
    for rows in (g, o):
        assert np.all(rows[:, 0] + rows[:, 2] + rows[:, 4] + rows[:, 6] == n0)
        assert np.all(rows[:, 1] + rows[:, 3] + rows[:, 5] + rows[:, 7] == n0)
