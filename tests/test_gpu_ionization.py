"""Electron-impact ionisation (Table I: e + Ar -> Ar+ + 2e) on the GPU against
the oracle, through the C ABI.

Hot electrons (10 eV) and a stand-in ionisation table scaled up so that a step
of the 16x16x32 box makes hundreds of pairs.  From the same state, one GPU
step and one oracle step give the same particles by id -- the new ones
included, whose ids follow their parents' ids on both sides -- at the stated
tolerances, and the same number of ionisations; over several coupled steps
(the oracle re-synchronised each step) the new particles are pushed through
the padding tile's global-memory paths and re-binned.  A batched ensemble
gives each replica's FP32R state bitwise as stepped alone, a checkpoint
resumes bitwise, and a run that outgrows max_particles counts its drops.
"""
import numpy as np
import pytest

from paper_1801_00972_amd import workloads as W
from tests.parity_util import compare_step, oracle_from_state
from tests.test_gpu_parity import TOL

pytestmark = pytest.mark.gpu


def _wl(prec, seed=0, **kw):
    xs = W.stand_in_xs(ionization=True)
    xs["e_iz"] = xs["e_iz"] * 40.0
    wl = dict(W.small_fp64(), precision=prec, seed=seed, Te_eV=10.0, xs=xs,
              name=f"ionizing_{prec}_{seed}")
    wl.update(kw)
    return wl


def _sim(wl, **kw):
    from paper_1801_00972_amd.pic import Simulation
    names = [w["name"] for w in (wl if isinstance(wl, list) else [wl])]
    print(f"[case] {names} {kw}", flush=True)
    return Simulation(wl, **kw)


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
def test_ionization_steps_match_oracle(prec):
    wl = _wl(prec)
    sim = _sim(wl, sort_interval=2)
    sim.set_tuning(ion_sort_interval=3)
    tol = TOL[prec]
    made = 0
    for k in range(6):
        st = sim.get_state()
        orc = oracle_from_state(wl, st)
        c0 = sim.counters()
        sim.step(1)
        orc.step(1)
        after = sim.get_state()
        c1 = sim.counters()
        rep = compare_step(wl, after, orc, tol["pos"], tol["vel"], tol["margin"])
        n_iz = c1["n_ionizations"] - c0["n_ionizations"]
        print(f"  step {k}: {n_iz} ionisations (oracle {orc.n_ionizations}), flips {rep['flips']}, "
              f"dpos {rep['max_dpos']:.1e} dvel {rep['max_dvel']:.1e}", flush=True)
        assert abs(n_iz - orc.n_ionizations) <= rep["flips"]
        assert rep["flips"] <= 3
        made += n_iz
        for s in range(2):
            assert c1["n_alive"][s] == len(after[s]["id"])
    assert made > 300
    assert sim.counters()["iz_dropped"] == 0
    sim.close()


def test_ionization_batched_checkpoint_and_room(tmp_path):
    wls = [_wl("fp32r", seed=s, name=f"ion_r{s}") for s in range(3)]
    ens = _sim(wls)
    assert ens.tuning()["batch_push"] == 1
    alone = [_sim(w) for w in wls]
    ens.step(8)
    for sim in alone:
        sim.step(8)
    for r, sim in enumerate(alone):
        a, b = ens.get_state(r), sim.get_state()
        for s in range(2):
            oa, ob = np.argsort(a[s]["id"]), np.argsort(b[s]["id"])
            assert np.array_equal(a[s]["id"][oa], b[s]["id"][ob])
            assert np.array_equal(a[s]["pos"][oa], b[s]["pos"][ob])
            assert np.array_equal(a[s]["vel"][oa], b[s]["vel"][ob])
        assert ens.counters(r)["n_ionizations"] == sim.counters()["n_ionizations"] > 0
    # checkpoint mid-run, resume in a new context
    path = str(tmp_path / "iz.ckpt")
    alone[0].save(path)
    alone[0].step(6)
    resumed = _sim(wls[0])
    resumed.load(path)
    resumed.step(6)
    a, b = alone[0].get_state(), resumed.get_state()
    for s in range(2):
        oa, ob = np.argsort(a[s]["id"]), np.argsort(b[s]["id"])
        assert np.array_equal(a[s]["id"][oa], b[s]["id"][ob])
        assert np.array_equal(a[s]["pos"][oa], b[s]["pos"][ob])
    assert resumed.counters()["n_ionizations"] == alone[0].counters()["n_ionizations"]
    for sim in alone + [ens, resumed]:
        sim.close()
    # no room: the loaded count as the limit; once the slots run out the pairs
    # of a step are dropped and counted, and the run goes on
    n_load = 16 * 16 * 32 * 8
    full = _sim(dict(wls[0], max_particles=n_load, name="no_room"))
    full.step(12)
    c = full.counters()
    print(f"  no room: {c['n_ionizations']} made, {c['iz_dropped']} dropped", flush=True)
    assert c["iz_dropped"] > 0
    assert c["n_alive"][1] == n_load - sum(c["wall_count"][w][1] for w in range(2)) - \
        int(full.grain_charges()[0][:, 1].sum()) + c["n_ionizations"]
    full.close()
