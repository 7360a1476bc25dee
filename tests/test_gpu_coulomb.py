"""Coulomb collisions (Table I: e-e, e-Ar+, Ar+-Ar+; binary pairing model)
through the C ABI against the oracle.

The pass runs at the start of a step on the state both sides share, so the
cells, pairing order and draws are the same; one step of the GPU is compared
with one oracle step, particle by particle (FP64 1e-12, FP32R 1e-5), and the
number of pairings is exact.  The dense box puts more particles in many
cells than a cell's shared-memory stage holds, so cells of both kinds run.  A large Coulomb logarithm makes the collisions
turn velocities by O(1) angles so that a missing or misplaced pass cannot
hide inside the FP32R tolerance.
"""
import numpy as np
import pytest

from paper_1801_00972_amd import workloads as W
from tests.parity_util import compare_step, oracle_from_state

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32r": 1e-5}


def _wl(box, prec, interval=1, lnL=2.0e5):
    if box == "small":
        wl = dict(W.small_fp64(), precision=prec)
    elif box == "ragged":  # 3 particles per cell: many cells with 0, 1, odd counts
        wl = W.tiny(nx=12, ny=10, nz=17, ppc=3, grains=[[0.3, 9.6, 8.5]], cutoff=2, precision=prec,
                    seed=5)
    else:  # dense: a quarter of the cells hold over 128 electrons; an odd cell count
        wl = W.tiny(nx=5, ny=3, nz=9, ppc=124, precision=prec, seed=9)
    wl["coulomb_interval"] = interval
    wl["coulomb_lnL"] = lnL
    return wl


def _copy(st):
    """The oracle works on the arrays it is given: each oracle gets its own."""
    return {k: ({q: a.copy() for q, a in v.items()} if k in (0, 1) else v) for k, v in st.items()}


def _step_vs_oracle(sim, wl, prec, check_count=True):
    st = sim.get_state()
    orc = oracle_from_state(wl, _copy(st))
    due = wl["coulomb_interval"] > 0 and st["step"] % wl["coulomb_interval"] == 0
    n_expect = oracle_from_state(wl, _copy(st)).coulomb() if due else 0
    before = sim.counters()["n_coulomb"]
    orc.step(1)
    sim.step(1)
    after = sim.get_state()
    n_gpu = sim.counters()["n_coulomb"] - before
    rep = compare_step(wl, after, orc, TOL[prec], TOL[prec], TOL[prec])
    print(f"  step {st['step']}: pass {due}, pairings gpu {n_gpu} oracle {n_expect}, "
          f"dpos {rep['max_dpos']:.2e} dvel {rep['max_dvel']:.2e} flips {rep['flips']}", flush=True)
    if check_count:
        assert n_gpu == n_expect
    assert rep["flips"] <= 2
    return st, after


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
@pytest.mark.parametrize("box", ["small", "ragged", "dense"])
def test_coulomb_step_matches_oracle(prec, box):
    from paper_1801_00972_amd.pic import Simulation
    wl = _wl(box, prec)
    print(f"[case] coulomb {box} {prec} lnL {wl['coulomb_lnL']}", flush=True)
    sim = Simulation(wl)
    sim.step(2)
    st, after = _step_vs_oracle(sim, wl, prec)
    assert sim.counters()["n_coulomb"] > 0
    # the pass changed the velocities by far more than the tolerance: without
    # it the oracle's step would not match (checked by stepping it without)
    w0 = dict(wl, coulomb_interval=0)
    orc0 = oracle_from_state(w0, _copy(st))
    orc0.step(1)
    with pytest.raises(AssertionError):
        compare_step(w0, after, orc0, TOL[prec], TOL[prec], TOL[prec])
    sim.close()


def test_coulomb_every_third_step_fp64():
    from paper_1801_00972_amd.pic import Simulation
    wl = _wl("ragged", "fp64", interval=3)
    print("[case] coulomb every 3rd step, ragged fp64", flush=True)
    sim = Simulation(wl)
    sim.step(1)
    for _ in range(3):  # steps 1 and 2 without a pass, step 3 with one
        _step_vs_oracle(sim, wl, "fp64")
    sim.close()


def test_coulomb_physical_log_fp64():
    from paper_1801_00972_amd.pic import Simulation
    wl = _wl("small", "fp64", lnL=10.0)
    print("[case] coulomb small fp64 lnL 10", flush=True)
    sim = Simulation(wl)
    sim.step(1)
    _step_vs_oracle(sim, wl, "fp64")
    sim.close()


def _by_id(st):
    """A species' arrays in id order (slot order depends on re-binning atomics)."""
    out = {}
    for s in range(2):
        o = np.argsort(st[s]["id"])
        out[s] = {k: st[s][k][o] for k in ("pos", "vel", "id")}
    return out


def test_coulomb_fp32r_is_deterministic_and_batched_equals_alone():
    from paper_1801_00972_amd.pic import Simulation
    wls = [_wl("small", "fp32r"), _wl("ragged", "fp32r")]
    print("[case] coulomb fp32r determinism and ensemble", flush=True)
    alone = []
    for wl in wls:
        runs = []
        for _ in range(2):
            sim = Simulation(wl)
            sim.step(4)
            runs.append(_by_id(sim.get_state()))
            sim.close()
        for s in range(2):
            for k in ("pos", "vel", "id"):
                assert np.array_equal(runs[0][s][k], runs[1][s][k])
        alone.append(runs[0])
    for batch in (1, 0):
        ens = Simulation(wls)
        ens.set_tuning(batch_push=batch)
        ens.step(4)
        for r in range(2):
            st = _by_id(ens.get_state(r))
            for s in range(2):
                for k in ("pos", "vel", "id"):
                    assert np.array_equal(st[s][k], alone[r][s][k]), (batch, r, s, k)
        ens.close()


def test_coulomb_config_is_checked():
    from paper_1801_00972_amd.pic import PicError, Simulation
    for interval, lnL in ((-1, 10.0), (1, 0.0), (2, float("nan"))):
        with pytest.raises(PicError):
            Simulation(dict(W.small_fp32r(), coulomb_interval=interval, coulomb_lnL=lnL))
