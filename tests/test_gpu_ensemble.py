"""The batched ensemble form and the launch settings, through the C ABI.

 - replicas of uneven sizes stepped together (every push of every replica and
   species in one persistent launch, inside the captured step graph) give, per
   replica, bitwise the FP32R state of the same replica stepped alone;
 - one step of each replica of a batched context against the oracle;
 - changing the launch settings between steps (tile margin, persistent grid,
   batching, sort interval, graphs) leaves FP32R results bitwise unchanged;
 - the autotuner's live steps are ordinary steps, and its cache is reused.
"""
import numpy as np
import pytest

from paper_1801_00972_amd import workloads as W
from tests.parity_util import compare_step, oracle_from_state
from tests.test_gpu_parity import TOL, _random_state

pytestmark = pytest.mark.gpu


def _ensemble(prec="fp32r"):
    return [
        dict(W.small_fp64(), precision=prec, seed=11, name="r0_16x16x32"),
        W.tiny(nx=12, ny=10, nz=17, ppc=3, grains=[[0.3, 9.6, 8.5]], cutoff=2, precision=prec,
               seed=12, name="r1_12x10x17"),
        W.tiny(nx=24, ny=24, nz=20, ppc=2, cutoff=1, precision=prec, seed=13, name="r2_24x24x20",
               grains=[[4.5, 4.5, 6.2], [16.5, 18.3, 12.7], [12.1, 5.5, 9.9]]),
    ]


def _sim(wls, **kw):
    from paper_1801_00972_amd.pic import Simulation
    names = [w["name"] for w in (wls if isinstance(wls, list) else [wls])]
    print(f"[case] {names} {kw}", flush=True)
    return Simulation(wls, **kw)


def _same_state(sa, sb, bitwise=True):
    assert sa["step"] == sb["step"]
    assert np.array_equal(sa["grain_count"], sb["grain_count"])
    assert np.array_equal(sa["wall_count"], sb["wall_count"])
    for s in range(2):
        oa, ob = np.argsort(sa[s]["id"]), np.argsort(sb[s]["id"])
        assert np.array_equal(sa[s]["id"][oa], sb[s]["id"][ob])
        if bitwise:
            assert np.array_equal(sa[s]["pos"][oa], sb[s]["pos"][ob])
            assert np.array_equal(sa[s]["vel"][oa], sb[s]["vel"][ob])
        else:
            assert np.max(np.abs(sa[s]["pos"][oa] - sb[s]["pos"][ob]), initial=0) < 1e-9


def test_batched_ensemble_matches_replicas_alone():
    from paper_1801_00972_amd.pic import PIC_PHI, pic_profile_enable
    wls = _ensemble()
    ens = _sim(wls, sort_interval=4)
    t = ens.tuning()
    assert t["batch_push"] == 1 and t["use_graphs"] == 1
    alone = [_sim(w, sort_interval=4) for w in wls]
    for sim in [ens] + alone:
        sim.set_tuning(ion_sort_interval=5)
    for seg in range(5):
        if seg == 3:  # direct launches of the batched step (kernel timing forces them)
            pic_profile_enable(ens.ctx, True)
        ens.step(3)
        for r, a in enumerate(alone):
            a.step(3)
            _same_state(ens.get_state(r), a.get_state())
            assert np.array_equal(ens.fields(r, PIC_PHI)["phi"], a.fields(0, PIC_PHI)["phi"])
            ce, ca = ens.counters(r), a.counters()
            for k in ("n_alive", "n_collisions", "md_particles", "cap_violation"):
                assert ce[k] == ca[k], k
    assert sum(ens.counters(r)["md_particles"][0] for r in range(3)) > 0
    ens.close()
    for a in alone:
        a.close()


@pytest.mark.parametrize("prec", ["fp32r", "fp64"])
def test_ensemble_one_step_against_oracle(prec):
    wls = _ensemble(prec)
    ens = _sim(wls)
    orcs = []
    for r, wl in enumerate(wls):
        ng = len(wl["grain_pos"])
        st = _random_state(wl, 1500 + 300 * r, 1200 + 100 * r, seed=40 + r,
                           grain_count=[[2 * r, r]] * ng, step=9 * r, near_grain=300)
        ens.set_state(st, r)
        orcs.append(oracle_from_state(wl, ens.get_state(r)))
    assert ens.tuning()["batch_push"] == (1 if prec == "fp32r" else 0)
    ens.step(1)
    tol = TOL[prec]
    for r, (wl, orc) in enumerate(zip(wls, orcs)):
        orc.step(1)
        after = ens.get_state(r)
        rep = compare_step(wl, after, orc, tol["pos"], tol["vel"], tol["margin"])
        print(f"  replica {r}: n={rep['n']} flips={rep['flips']} dpos={rep['max_dpos']:.2e} "
              f"dvel={rep['max_dvel']:.2e}", flush=True)
        assert rep["flips"] <= 2
        assert np.abs(after["grain_count"] - orc.grain_count).sum() <= rep["flips"]
        assert np.abs(after["wall_count"] - orc.wall_count).sum() <= rep["flips"]
        assert after["step"] == orc.step_index
    ens.close()


def test_settings_leave_fp32r_results_unchanged():
    wls = _ensemble()[:2]
    ref = _sim(wls, sort_interval=16)
    sim = _sim(wls, sort_interval=16)
    plan = [dict(tile_margin=0, ion_tile_margin=0), dict(tile_margin=3, batch_blocks=8),
            dict(batch_push=0, ion_sort_interval=2), dict(batch_push=1, sort_interval=1, tile_margin=1),
            dict(sort_interval=3, ion_sort_interval=5, use_graphs=0, ion_tile_margin=3),
            dict(sort_interval=0, ion_sort_interval=0, use_graphs=1, batch_blocks=1024)]
    for kw in plan:
        sim.set_tuning(**kw)
        t = sim.tuning()
        assert all(t[k] == v for k, v in kw.items())
        print(f"  settings {t}", flush=True)
        sim.step(4)
        ref.step(4)
        for r in range(2):
            _same_state(sim.get_state(r), ref.get_state(r))
    ref.close()
    sim.close()


def test_bad_settings_are_rejected():
    from paper_1801_00972_amd.pic import PicError
    fp64 = _sim(dict(W.small_fp64(), name="fp64"))
    with pytest.raises(PicError):
        fp64.set_tuning(batch_push=1)
    fp64.close()
    sim = _sim(dict(W.small_fp32r(), name="fp32r"))
    for kw in (dict(tile_margin=4), dict(ion_tile_margin=-1), dict(batch_blocks=12), dict(batch_blocks=0),
               dict(sort_interval=-1), dict(ion_sort_interval=-2)):
        with pytest.raises(PicError):
            sim.set_tuning(**kw)
    sim.step(1)  # the context still works
    sim.close()


def test_autotune_steps_are_ordinary_steps(tmp_path):
    wls = _ensemble()[:2]
    tuned = _sim(wls)
    best, trials = tuned.autotune(trial_steps=4, cache=str(tmp_path / "tune.json"))
    print(f"  {len(trials)} trials, best {best}", flush=True)
    assert len(trials) >= 8
    assert best in [t for t, _ in trials]
    assert all(ms > 0 for _, ms in trials)
    steps = tuned.counters()["step"]
    assert steps == len(trials) * (2 + 4)
    plain = _sim(wls)
    plain.step(steps)
    for r in range(2):
        _same_state(tuned.get_state(r), plain.get_state(r))
    # a second context of the same shapes takes the cached settings without trials
    again = _sim(wls)
    best2, trials2 = again.autotune(trial_steps=4, cache=str(tmp_path / "tune.json"))
    assert trials2 == [] and best2 == best
    assert again.counters()["step"] == 0
    for s in (tuned, plain, again):
        s.close()


@pytest.mark.slow
def test_benchmark_ensemble_against_oracle():
    """The ensemble the benchmark times (16 replicas of 32^2x128 to 64^2x256
    cells, 16-32 ppc, 1-32 grains, 5.2e8 particles), stepped by the one
    persistent push launch: per replica the fixed-point charge density
    bit-exact and phi, E to 1e-5 against the oracle's fields of the same
    state, then one step of a sample of every replica's particles (uniform,
    near grains, near the electrodes) moved by the oracle in its own field."""
    import oracle
    from paper_1801_00972_amd.pic import PIC_E, PIC_PHI, PIC_RHO_FIXED
    from tests.parity_util import rel_inf
    from tests.test_gpu_fullsize import _select
    wls = W.ensemble()
    ens = _sim(wls)
    ens.set_tuning(batch_push=1)
    assert ens.tuning()["batch_push"] == 1
    ens.step(3)
    rng = np.random.default_rng(21)
    smalls = []
    for r, wl in enumerate(wls):
        st = ens.get_state(r)
        orc = oracle_from_state(wl, st)
        g = ens.fields(r, PIC_PHI | PIC_E | PIC_RHO_FIXED)
        o = orc.fields(fixed_point=True)
        assert np.array_equal(g["rho_fixed"], o["rho_fixed"]), wl["name"]
        e_phi = rel_inf(g["phi"], o["phi"], floor=abs(orc.rf_voltage(st["step"])))
        e_E = rel_inf(g["E"], o["E"])
        assert e_phi <= 1e-5 and e_E <= 1e-5, (wl["name"], e_phi, e_E)
        small = oracle.Oracle(wl)
        for s in range(2):
            idx = _select(st[s]["pos"], wl["grain_pos"], wl["nz"], rng, 600, 400, 100)
            small.set_particles(s, st[s]["pos"][idx], st[s]["vel"][idx], st[s]["id"][idx])
        small.set_counts(grain_count=st["grain_count"], step=st["step"])
        small.step_in_field(o["E"])
        smalls.append(small)
        print(f"  {wl['name']}: phi {e_phi:.1e} E {e_E:.1e}", flush=True)
        del st, orc, g, o
    ens.step(1)
    for r, wl in enumerate(wls):
        after = ens.get_state(r)
        sub = {}
        for s in range(2):
            keep = np.isin(after[s]["id"], smalls[r].id[s])
            sub[s] = {k: after[s][k][keep] for k in ("pos", "vel", "id")}
        rep = compare_step(wl, sub, smalls[r], 1e-5, 1e-5, 1e-5)
        assert rep["n"] > 1000 and rep["flips"] <= 2, (wl["name"], rep)
    print(f"  {len(wls)} replicas: one sampled step each within 1e-5", flush=True)
    ens.close()
