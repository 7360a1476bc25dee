"""Energy-dependent cross sections in the null-collision method (Table I:
e-Ar elastic and excitation, Ar+-Ar charge exchange and elastic) through the
C ABI against the oracle.

The tables are analytic stand-ins (the paper's LxCat data are not part of
this code), scaled up and with a low cap and a low excitation threshold so
that one step has thousands of collisions of every kind.  One GPU step is
compared with one oracle step from the same state, particle by particle
(FP64 1e-12, FP32R 1e-5), with the collision counts.
"""
import numpy as np
import pytest

from paper_1801_00972_amd import workloads as W
from tests.parity_util import compare_step, oracle_from_state

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32r": 1e-5}


def _tables():
    E = np.array([0.0, 0.5, 2.0, 4.0, 8.0, 20.0, 60.0])
    return dict(E=E,
                e_el=2e-18 * np.array([0.3, 1.0, 0.8, 0.6, 0.5, 0.4, 0.3]),
                e_ex=np.array([0.0, 0.0, 0.0, 0.0, 4e-19, 8e-19, 6e-19]),
                i_cx=3e-15 * np.array([1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4]),
                i_el=1e-15 * np.array([1.0, 1.0, 0.9, 0.8, 0.7, 0.6, 0.5]),
                E_ex=4.0)


def _wl(prec, box="small"):
    if box == "small":
        wl = dict(W.small_fp64(), precision=prec)
    else:
        wl = W.tiny(nx=12, ny=10, nz=17, ppc=3, grains=[[0.3, 9.6, 8.5]], cutoff=2, precision=prec,
                    seed=7)
    wl["xs"] = _tables()
    wl["E_cap_eV"] = 100.0
    return wl


def _copy(st):
    return {k: ({q: a.copy() for q, a in v.items()} if k in (0, 1) else v) for k, v in st.items()}


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
@pytest.mark.parametrize("box", ["small", "ragged"])
def test_xs_step_matches_oracle(prec, box):
    from paper_1801_00972_amd.pic import Simulation
    wl = _wl(prec, box)
    print(f"[case] cross-section tables {box} {prec}", flush=True)
    sim = Simulation(wl)
    sim.step(2)
    st = sim.get_state()
    orc = oracle_from_state(wl, _copy(st))
    c0 = sim.counters()
    orc.step(1)
    sim.step(1)
    after = sim.get_state()
    c1 = sim.counters()
    rep = compare_step(wl, after, orc, TOL[prec], TOL[prec], TOL[prec])
    gpu_coll = [c1["n_collisions"][s] - c0["n_collisions"][s] for s in range(2)]
    print(f"  collisions gpu {gpu_coll} oracle {orc.n_collisions}, dpos {rep['max_dpos']:.2e} "
          f"dvel {rep['max_dvel']:.2e} flips {rep['flips']}", flush=True)
    assert min(orc.n_collisions) > (500 if box == "small" else 50)
    assert rep["flips"] <= 2
    for s in range(2):
        assert abs(gpu_coll[s] - orc.n_collisions[s]) <= rep["flips"]
    sim.close()


def test_xs_fp32r_ensemble_equals_alone():
    from paper_1801_00972_amd.pic import Simulation
    wls = [_wl("fp32r"), _wl("fp32r", "ragged")]
    print("[case] cross-section tables, ensemble", flush=True)

    def by_id(st):
        return {s: {k: st[s][k][np.argsort(st[s]["id"])] for k in ("pos", "vel", "id")} for s in range(2)}

    alone = []
    for wl in wls:
        sim = Simulation(wl)
        sim.step(3)
        alone.append(by_id(sim.get_state()))
        sim.close()
    for batch in (1, 0):
        ens = Simulation(wls)
        ens.set_tuning(batch_push=batch)
        ens.step(3)
        for r in range(2):
            st = by_id(ens.get_state(r))
            for s in range(2):
                for k in ("pos", "vel", "id"):
                    assert np.array_equal(st[s][k], alone[r][s][k]), (batch, r, s, k)
        ens.close()


def test_xs_tables_are_checked():
    from paper_1801_00972_amd.pic import PicError, Simulation
    good = _tables()
    bad = [dict(good, E=good["E"][:1], e_el=good["e_el"][:1], i_cx=good["i_cx"][:1], e_ex=None,
                i_el=None),
           dict(good, E=good["E"][::-1].copy()),
           dict(good, e_el=-good["e_el"]),
           dict(good, E_ex=-1.0)]
    for xs in bad:
        with pytest.raises(PicError):
            Simulation(dict(W.small_fp32r(), xs=xs))
