"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Same particle state on both sides (pic_set_state / the oracle's arrays), then
 - the mesh quantities at step k: rho bit-exact in fixed point (FP32R) or to
   1e-12 (FP64); phi and E to 1e-12 (FP64) or 1e-5 (FP32R), relative to the
   largest value (phi: to max(|phi|, |V|));
 - one full step: positions to 1e-12 / 1e-5 cells, velocities to 1e-12 /
   1e-5 of max(|v|, v_th), survivors, electrode and grain tallies exact, except
   where a discrete decision sits within the oracle's recorded margin.
"""
import numpy as np
import pytest

import oracle
from paper_1801_00972_amd import workloads as W
from tests.parity_util import compare_step, oracle_from_state, rel_inf

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(field=1e-12, pos=1e-12, vel=1e-12, margin=1e-12),
       "fp32r": dict(field=1e-5, pos=1e-5, vel=1e-5, margin=1e-5)}


def _sim(wl, **kw):
    from paper_1801_00972_amd.pic import Simulation
    print(f"[case] {wl['name']} {wl['precision']} {wl['nx']}x{wl['ny']}x{wl['nz']} ppc={wl['ppc']}",
          flush=True)
    return Simulation(wl, **kw)


def _random_state(wl, n_e, n_i, seed, grain_count=None, step=0, near_grain=0):
    """Seeded synthetic state: uniform positions, Maxwellian velocities, some
    particles placed inside MD cubes and next to the electrodes."""
    rng = np.random.default_rng(seed)
    box = np.array([wl["nx"], wl["ny"], wl["nz"]], float)
    e, me, mi = 1.602176634e-19, 9.1093837015e-31, 39.948 * 1.66053906660e-27
    st = {}
    for s, (n, T, m) in enumerate(((n_e, wl["Te_eV"], me), (n_i, wl["Ti_eV"], mi))):
        pos = rng.random((n, 3)) * box
        g = np.asarray(wl["grain_pos"]).reshape(-1, 3)
        if near_grain and len(g):
            k = min(near_grain, n)
            pos[:k] = g[rng.integers(0, len(g), k)] + rng.uniform(-2.5, 2.5, (k, 3))
            pos[:k, 0] %= box[0]
            pos[:k, 1] %= box[1]
        pos[-max(n // 20, 1):, 2] = rng.random(max(n // 20, 1)) * 0.2  # close to z = 0
        if wl["precision"] == "fp32r":  # positions exactly representable as cell + float32 offset
            c = np.floor(pos)
            pos = c + (pos - c).astype(np.float32).astype(np.float64)
            pos = np.where(pos >= box, c, pos)
        vel = np.sqrt(T * e / m) * rng.standard_normal((n, 3))
        if wl["precision"] == "fp32r":
            vel = vel.astype(np.float32).astype(np.float64)
        st[s] = dict(pos=pos, vel=vel, id=rng.permutation(n).astype(np.uint32) + 7)
    ng = len(np.asarray(wl["grain_pos"]).reshape(-1, 3))
    st["grain_count"] = np.zeros((ng, 2), np.int64) if grain_count is None else np.asarray(grain_count)
    st["wall_count"] = np.zeros((2, 2), np.int64)
    st["step"] = step
    return st


def _check_fields(wl, sim, orc):
    tol = TOL[wl["precision"]]
    fixed = wl["precision"] == "fp32r"
    from paper_1801_00972_amd.pic import PIC_E, PIC_PHI, PIC_RHO, PIC_RHO_FIXED
    what = PIC_PHI | PIC_E | PIC_RHO | (PIC_RHO_FIXED if fixed else 0)
    g = sim.fields(0, what)
    o = orc.fields(fixed_point=fixed)
    if fixed:
        assert np.array_equal(g["rho_fixed"], o["rho_fixed"]), "fixed-point deposit is not bit-exact"
    assert rel_inf(g["rho"], o["rho"]) <= (1e-12 if not fixed else 1e-15)
    V = abs(orc.rf_voltage(orc.step_index))
    e_phi = rel_inf(g["phi"], o["phi"], floor=V)
    e_E = rel_inf(g["E"], o["E"])
    print(f"  fields: phi {e_phi:.2e}  E {e_E:.2e}", flush=True)
    assert e_phi <= tol["field"]
    assert e_E <= tol["field"]
    return g, o


CASES = [
    # (workload factory, n_e, n_i, grain counts, step)
    ("small", lambda p: dict(W.small_fp64(), precision=p), 3000, 2500, [[40, 7]], 123),
    ("ragged", lambda p: W.tiny(nx=12, ny=10, nz=17, ppc=2, grains=[[0.3, 9.6, 8.5]], cutoff=2,
                                precision=p), 1001, 777, [[3, 11]], 5),
    ("no_grains", lambda p: W.tiny(nx=16, ny=48, nz=9, ppc=1, precision=p), 4097, 255, None, 0),
    # three separated grains: the near-grain lookup box has cells outside every cube
    ("gaps", lambda p: W.tiny(nx=24, ny=24, nz=20, ppc=2, cutoff=1, precision=p,
                              grains=[[4.5, 4.5, 6.2], [16.5, 18.3, 12.7], [12.1, 5.5, 9.9]]),
     6000, 5000, [[5, 1], [0, 2], [9, 9]], 77),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fields_and_one_step(case, prec):
    name, make, n_e, n_i, gc, step = case
    wl = make(prec)
    sim = _sim(wl)
    st = _random_state(wl, n_e, n_i, seed=sum(map(ord, name)), grain_count=gc, step=step,
                       near_grain=400)
    sim.set_state(st)
    back = sim.get_state()
    # FP32R: the state the library actually holds (cell + float32 offset) is exact in FP64
    orc = oracle_from_state(wl, back)
    _check_fields(wl, sim, orc)
    sim.step(1)
    orc.step(1)
    after = sim.get_state()
    tol = TOL[prec]
    rep = compare_step(wl, after, orc, tol["pos"], tol["vel"], tol["margin"])
    print(f"  step: n={rep['n']} flips={rep['flips']} dpos={rep['max_dpos']:.2e} "
          f"dvel={rep['max_dvel']:.2e}", flush=True)
    assert rep["flips"] <= 2
    assert np.abs(after["wall_count"] - orc.wall_count).sum() <= rep["flips"]
    assert np.abs(after["grain_count"] - orc.grain_count).sum() <= rep["flips"]
    assert after["step"] == orc.step_index
    c = sim.counters()
    assert c["md_particles"][0] + c["md_particles"][1] > 0 or not len(wl["grain_pos"])
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
def test_loading_matches_oracle(prec):
    wl = dict(W.small_fp64(), precision=prec)
    sim = _sim(wl, sort_interval=0)
    g = sim.get_state()
    o = oracle.Oracle(wl)
    o.init_particles()
    for s in range(2):
        order = np.argsort(g[s]["id"])
        assert np.array_equal(g[s]["id"][order], o.id[s])
        # offsets are 24-bit multiples: exact in both forms
        assert np.array_equal(g[s]["pos"][order], o.pos[s])
        v, ov = g[s]["vel"][order], o.vel[s]
        if prec == "fp64":
            assert np.max(np.abs(v - ov) / np.abs(ov).max()) < 1e-14
        else:
            assert np.max(np.abs(v - ov.astype(np.float32))) <= np.max(np.spacing(np.abs(ov).astype(np.float32)))
    d_g, d_o = sim.derived(), o.derived()
    assert d_g["Qp"] == d_o["Qp"] and d_g["T_null"] == d_o["T_null"]
    assert d_g["w"] == d_o["w"]
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
def test_ten_steps_from_loading(prec):
    """Ten coupled steps from the same loaded state (rho, phi, push feed back),
    each compared at the stated tolerances (1e-12 FP64, 1e-5 FP32R) after the
    oracle takes the GPU's state, so that each step starts from the same
    particles on both sides."""
    wl = dict(W.small_fp64(), precision=prec)
    sim = _sim(wl)
    st = sim.get_state()
    orc = oracle_from_state(wl, st)
    tol = TOL[prec]
    worst = [0.0, 0.0]
    for k in range(10):
        sim.step(1)
        orc.step(1)
        after = sim.get_state()
        rep = compare_step(wl, after, orc, tol["pos"], tol["vel"], tol["margin"])
        worst = [max(worst[0], rep["max_dpos"]), max(worst[1], rep["max_dvel"])]
        assert rep["flips"] <= 3
        orc = oracle_from_state(wl, after)
    print(f"  ten steps: largest dpos {worst[0]:.2e} cells, dvel {worst[1]:.2e}", flush=True)
    c = sim.counters()
    n0 = 16 * 16 * 32 * 8
    for s in range(2):
        tot = c["n_alive"][s] + c["wall_count"][0][s] + c["wall_count"][1][s]
        counts, _ = sim.grain_charges()
        assert tot + counts[:, s].sum() == n0
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
@pytest.mark.parametrize("rebin", [0, 3])
def test_density_and_flux_moments(prec, rebin):
    """n and flux of both species on the nodes (pic_fields PIC_N | PIC_FLUX)
    against the oracle's moments of the same state, with particles drifting
    out of their tiles (no re-binning) or re-binned every 3 steps."""
    from paper_1801_00972_amd.pic import PIC_FLUX, PIC_N
    wl = dict(W.small_fp64(), precision=prec)
    sim = _sim(wl)
    sim.set_tuning(sort_interval=rebin, ion_sort_interval=rebin)
    for seg in range(3):
        sim.step(4)
        st = sim.get_state()
        n, flux = oracle_from_state(wl, st).moments()
        g = sim.fields(0, PIC_N | PIC_FLUX)
        e_n, e_f = rel_inf(g["n"], n), rel_inf(g["flux"], flux)
        print(f"  step {st['step']}: n {e_n:.2e} flux {e_f:.2e}", flush=True)
        assert e_n <= 1e-13 and e_f <= 1e-12
        # number of particles: sum of n dx^3 / w
        w, vol = sim.derived()["w"], wl["dx"] ** 3
        for s in range(2):
            assert g["n"][s].sum() * vol / w == pytest.approx(len(st[s]["id"]), rel=1e-12)
    sim.close()


def _inside(pos, origin, h, cells):
    u = (pos - np.asarray(origin)) / h
    return np.all((u >= 0.0) & (u < np.asarray(cells, np.float64)), axis=1)


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
@pytest.mark.parametrize("box", ["grain", "ragged", "unit"])
def test_fine_grid_moments(prec, box):
    """Densities and fluxes on the fine diagnostic grid (pic_fields
    PIC_FINE_N | PIC_FINE_FLUX) against the oracle's fine moments of the same
    state: 0.08-cell cells around the grain, a ragged box of half cells that
    spans x and touches both electrodes, and unit cells off the PIC nodes;
    particles drift out of their tiles (no re-binning).  The number of
    particles inside the box is exact."""
    from paper_1801_00972_amd.pic import PIC_FINE_FLUX, PIC_FINE_N, PIC_FINE_PHI
    origin, h, cells = {"grain": ((7.0, 7.0, 15.0), 0.08, (25, 25, 25)),
                        "ragged": ((0.0, 3.25, 0.0), 0.5, (32, 17, 64)),
                        "unit": ((2.5, 3.25, 4.75), 1.0, (10, 9, 20))}[box]
    print(f"[case] {prec} fine grid {box}: origin {origin} h {h} cells {cells}", flush=True)
    wl = dict(W.small_fp64(), precision=prec)
    sim = _sim(wl)
    sim.set_tuning(sort_interval=0, ion_sort_interval=0)
    sim.set_fine_grid(origin, h, cells)
    w, vol = sim.derived()["w"], (h * wl["dx"]) ** 3
    for seg in range(2):
        sim.step(3)
        st = sim.get_state()
        orc = oracle_from_state(wl, st)
        n, flux = orc.fine_moments(origin, h, cells)
        phi_o = orc.fine_phi(orc.fields(fixed_point=prec == "fp32r")["phi"], origin, h, cells)
        g = sim.fields(0, PIC_FINE_N | PIC_FINE_FLUX | PIC_FINE_PHI)
        e_n, e_f = rel_inf(g["fine_n"], n), rel_inf(g["fine_flux"], flux)
        e_p = rel_inf(g["fine_phi"], phi_o, floor=abs(orc.rf_voltage(st["step"])))
        print(f"  fine phi {e_p:.2e}", flush=True)
        assert e_p <= (1e-12 if prec == "fp64" else 1e-5)
        inside = [int(_inside(st[s]["pos"], origin, h, cells).sum()) for s in range(2)]
        print(f"  step {st['step']}: {inside} particles inside, n {e_n:.2e} flux {e_f:.2e}", flush=True)
        assert min(inside) > 0
        assert e_n <= 1e-12 and e_f <= 1e-12
        for s in range(2):
            assert g["fine_n"][s].sum() * vol / w == pytest.approx(inside[s], rel=1e-12)
    sim.close()


def test_fine_grid_arguments_are_checked():
    from paper_1801_00972_amd.pic import PIC_FINE_N, PIC_N, PicError
    wl = W.small_fp32r()
    sim = _sim(wl)
    with pytest.raises(PicError):
        sim.fields(0, PIC_FINE_N)  # no fine grid
    for origin, h, cells in (((0, 0, 0), 0.0, (4, 4, 4)), ((0, 0, 0), -1.0, (4, 4, 4)),
                             ((0, 0, 0), 0.5, (0, 4, 4)), ((-0.1, 0, 0), 0.5, (4, 4, 4)),
                             ((12.0, 0, 0), 0.5, (9, 4, 4)), ((0, 0, 30.0), 1.0, (1, 1, 3)),
                             ((0, 0, 0), float("nan"), (4, 4, 4)),
                             ((0, 0, 0), 1e-3, (1000, 1000, 1000))):
        with pytest.raises(PicError):
            sim.set_fine_grid(origin, h, cells)
    sim.set_fine_grid((0, 0, 0), 0.5, (32, 32, 64))  # the whole domain
    sim.average(1, 2)
    with pytest.raises(PicError):
        sim.set_fine_grid((1, 1, 1), 0.5, (4, 4, 4))  # averaging is running
    sim.step(2)
    assert sim.averages(0, -1, what=PIC_FINE_N)["samples"] == 2
    sim.average(0)
    sim.set_fine_grid((1, 1, 1), 0.5, (4, 4, 4))
    with pytest.raises(PicError):
        sim.averages(0, -1, what=PIC_FINE_N)  # the sums were of the old box
    assert sim.averages(0, -1, what=PIC_N)["samples"] == 2
    sim.set_fine_grid(None)
    with pytest.raises(PicError):
        sim.fields(0, PIC_FINE_N)
    sim.close()


def test_fixed_point_total_charge_is_exact():
    wl = W.small_fp32r()
    sim = _sim(wl)
    sim.step(20)
    from paper_1801_00972_amd.pic import PIC_RHO_FIXED
    f = sim.fields(0, PIC_RHO_FIXED)
    c = sim.counters()
    Qp = sim.derived()["Qp"]
    lost = c["wall_count"][0][1] + c["wall_count"][1][1] - c["wall_count"][0][0] - c["wall_count"][1][0]
    assert int(f["rho_fixed"].sum()) == -lost * Qp
    sim.close()


def test_fp32r_refinement_reaches_tolerance():
    """The refinement stops at ||b - A phi|| <= refine_tol ||b|| (1e-10), within
    max_refine sweeps; a solve that cannot reach it is counted; refine_tol 0
    always takes every sweep."""
    wl = W.small_fp32r()
    sim = _sim(wl, max_refine=3)
    sim.step(3)
    c = sim.counters()
    print("  refine residual", c["refine_residual"], "sweeps", c["refine_sweeps"])
    assert c["refine_residual"] <= 1e-10
    assert 1 <= c["refine_sweeps"] <= 3
    assert c["refine_unconverged"] == 0
    sim.close()
    # one FP32 sweep from psi = 0 (residual ~1e-7) does not reach 1e-10: counted
    sim = _sim(wl, max_refine=1)
    sim.step(1)
    c = sim.counters()
    assert c["refine_sweeps"] == 1 and c["refine_unconverged"] == 1
    assert c["refine_residual"] > 1e-10
    sim.close()
    sim = _sim(dict(wl, refine_tol=0.0), max_refine=3)
    sim.step(2)
    c = sim.counters()
    assert c["refine_sweeps"] == 3 and c["refine_unconverged"] == 2
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
def test_md_margin_counter_matches_oracle(prec):
    """Plain pushes that move at least cutoff cells in one step (a grain could
    be crossed outside its MD cube) are counted, as the oracle counts them:
    hot electrons and a 20 ps step make most of them that fast at cutoff 1."""
    wl = W.tiny(nx=12, ny=10, nz=14, ppc=2, grains=[[6.0, 5.0, 7.0]], cutoff=1, Te_eV=30.0,
                dt=2e-11, precision=prec)
    sim = _sim(wl)
    st = _random_state(wl, 3000, 500, seed=11)
    sim.set_state(st)
    orc = oracle_from_state(wl, sim.get_state())
    sim.step(1)
    orc.step(1)
    c = sim.counters()
    print("  md_margin", c["md_margin"], "oracle", orc.md_margin, flush=True)
    assert c["md_margin"][0] > 500
    assert c["md_margin"] == orc.md_margin
    sim.close()
    # without grains nothing is counted
    wl0 = dict(wl, grain_pos=np.zeros((0, 3)))
    sim = _sim(wl0)
    sim.set_state(_random_state(wl0, 3000, 500, seed=11))
    sim.step(1)
    assert sim.counters()["md_margin"] == [0, 0]
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
def test_md_particles_that_left_their_windows(prec):
    """Near-grain particles found wherever they are: hot electrons and a 20 ps
    step move about a cell per step, there is no re-binning, so after a few
    steps many particles sit outside their push block's window, and some of
    those inside an MD cube (the FP32R list scan finds them through the
    blocks' stray flags).  Every step is compared with the oracle (a particle
    left out of the MD list would not move), and a change of window margin in
    the middle (every block then counts as stray) changes nothing."""
    wl = W.tiny(nx=16, ny=16, nz=16, ppc=2, grains=[[5.5, 6.5, 8.0], [12.0, 11.0, 7.5]], cutoff=2,
                Te_eV=30.0, dt=2e-11, precision=prec)
    sim = _sim(wl, sort_interval=0)
    sim.set_tuning(ion_sort_interval=0)
    sim.set_state(_random_state(wl, 6000, 1500, seed=23, near_grain=600))
    tol = TOL[prec]
    md = 0
    for k in range(8):
        if k == 4:
            sim.set_tuning(tile_margin=1)
        st = sim.get_state()
        orc = oracle_from_state(wl, st)
        c0 = sim.counters()["md_particles"]
        sim.step(1)
        orc.step(1)
        rep = compare_step(wl, sim.get_state(), orc, tol["pos"], tol["vel"], tol["margin"])
        d = [a - b for a, b in zip(sim.counters()["md_particles"], c0)]
        md += sum(d)
        print(f"  step {k}: MD particles {d}, flips {rep['flips']}, dpos {rep['max_dpos']:.1e}",
              flush=True)
        assert rep["flips"] <= 3
    assert md > 500
    sim.close()


def test_weight_just_below_the_fixed_point_bound_runs():
    """w = n0 dx^3 / ppc just under 128 (macro charge just under 2^39 in
    2^-32 e): accepted, and the fixed-point deposit stays exact."""
    wl = W.tiny(nx=8, ny=8, nz=10, ppc=1, precision="fp32r")
    wl["n0"] = 128.0 * (1 - 1e-9) / wl["dx"] ** 3
    sim = _sim(wl)
    sim.step(2)
    from paper_1801_00972_amd.pic import PIC_RHO_FIXED
    orc = oracle_from_state(wl, sim.get_state())
    g = sim.fields(0, PIC_RHO_FIXED)
    assert np.array_equal(g["rho_fixed"], orc.fields(fixed_point=True)["rho_fixed"])
    sim.close()


def test_determinism_fp32r_bitwise():
    wl = W.small_fp32r()
    a, b = _sim(wl), _sim(wl)
    a.step(15)
    b.step(15)
    sa, sb = a.get_state(), b.get_state()
    for s in range(2):
        oa, ob = np.argsort(sa[s]["id"]), np.argsort(sb[s]["id"])
        assert np.array_equal(sa[s]["pos"][oa], sb[s]["pos"][ob])
        assert np.array_equal(sa[s]["vel"][oa], sb[s]["vel"][ob])
    a.close()
    b.close()


def test_empty_species_and_bad_inputs():
    from paper_1801_00972_amd.pic import PicError
    wl = W.tiny(nx=8, ny=8, nz=10, ppc=1)
    sim = _sim(wl)
    st = _random_state(wl, 0, 5, seed=1)
    sim.set_state(st)
    sim.step(2)
    assert sim.counters()["n_alive"][0] == 0
    bad = _random_state(wl, 3, 0, seed=2)
    bad[0]["pos"][1, 2] = wl["nz"] + 0.5
    with pytest.raises(PicError):
        sim.set_state(bad)
    sim.close()


@pytest.mark.parametrize("prec", ["fp32r", "fp64"])
def test_graph_replay_matches_direct_launches(prec):
    """The captured step graph, replayed with eager work and synchronisations
    between replays, against direct launches of the same step (kernel timing on
    forces direct launches).  FP32R is bitwise deterministic; FP64 deposits
    with floating-point atomics, so it agrees to round-off."""
    from paper_1801_00972_amd.pic import PIC_PHI, pic_profile_enable
    wl = dict(W.small_fp64(), precision=prec)
    a, b = _sim(wl, sort_interval=4), _sim(wl, sort_interval=4)
    for sim in (a, b):  # the ions are re-binned on their own interval
        sim.set_tuning(ion_sort_interval=5)
    pic_profile_enable(b.ctx, True)
    for rep in range(6):  # crosses two sorts and both buffer phases
        a.step(3)
        b.step(3)
        fa, fb = a.fields(0, PIC_PHI), b.fields(0, PIC_PHI)
        sa, sb = a.get_state(), b.get_state()
        assert sa["step"] == sb["step"] == 3 * (rep + 1)
        for s in range(2):
            oa, ob = np.argsort(sa[s]["id"]), np.argsort(sb[s]["id"])
            assert np.array_equal(sa[s]["id"][oa], sb[s]["id"][ob])
            if prec == "fp32r":
                assert np.array_equal(sa[s]["pos"][oa], sb[s]["pos"][ob])
                assert np.array_equal(sa[s]["vel"][oa], sb[s]["vel"][ob])
            else:
                assert np.max(np.abs(sa[s]["pos"][oa] - sb[s]["pos"][ob])) < 1e-10
        if prec == "fp32r":
            assert np.array_equal(fa["phi"], fb["phi"])
        assert np.array_equal(sa["grain_count"], sb["grain_count"])
    a.close()
    b.close()


def test_library_grain_placement_matches_oracle():
    """grain_pos NULL: the library places the grains (seeded rejection in a
    sphere with a minimum separation); the same positions, bit for bit, as the
    oracle's own placement, then one step on them against the oracle."""
    from paper_1801_00972_amd.pic import PIC_ECONFIG, PicError, Simulation
    cases = [
        dict(W.tiny(nx=24, ny=24, nz=30, ppc=2, cutoff=2, seed=5), grain_pos=None,
             cluster=dict(n=6, center=(12.0, 12.0, 18.5), radius=5.0, min_sep=3.0)),
        dict(W.full_fp64("fp32r"), grain_pos=None,
             cluster=dict(n=8, center=(32.0, 32.0, 231.6), radius=10.0, min_sep=4.0)),
    ]
    for wl in cases:
        o = oracle.Oracle(wl)
        sim = Simulation(wl)
        g = sim.grain_positions()
        assert g.shape == (wl["cluster"]["n"], 3)
        assert np.array_equal(g, o.grain_pos)
        sim.close()
    wl = dict(cases[0], precision="fp64")
    sim = _sim(dict(wl, name="placed"))
    st = _random_state(dict(wl, grain_pos=oracle.Oracle(wl).grain_pos), 3000, 2000, seed=3,
                       near_grain=400)
    sim.set_state(st)
    orc = oracle_from_state(wl, sim.get_state())
    _check_fields(dict(wl, name="placed"), sim, orc)
    sim.step(1)
    orc.step(1)
    rep = compare_step(wl, sim.get_state(), orc, 1e-12, 1e-12, 1e-12)
    assert rep["flips"] <= 2
    sim.close()
    with pytest.raises(PicError) as e:
        Simulation(dict(cases[0], cluster=dict(n=40, center=(12.0, 12.0, 18.5), radius=1.0,
                                               min_sep=1.0)))
    assert e.value.code == PIC_ECONFIG


@pytest.mark.parametrize("prec", ["fp64", "fp32r"])
def test_energy_diagnostic_matches_state(prec):
    """pic_energy against the same sums over the state and the field that
    pic_get_state and pic_fields return, and the kinetic energy of the loaded
    Maxwellians against (3/2) N kT w (3 sigma of the chi-square spread)."""
    from paper_1801_00972_amd.pic import PIC_E
    wl = dict(W.small_fp64(), precision=prec)
    sim = _sim(wl)
    en0 = sim.energy()
    e, me, mi = 1.602176634e-19, 9.1093837015e-31, 39.948 * 1.66053906660e-27
    w = sim.derived()["w"]
    n = 16 * 16 * 32 * 8
    for s, (m, T) in enumerate(((me, wl["Te_eV"]), (mi, wl["Ti_eV"]))):
        want = 1.5 * n * T * e * w
        assert abs(en0[("kinetic_e", "kinetic_i")[s]] / want - 1) < 3 * np.sqrt(2.0 / (3 * n))
    sim.step(7)
    en = sim.energy()
    st = sim.get_state()
    E = sim.fields(0, PIC_E)["E"]
    for s, (m, key) in enumerate(((me, "kinetic_e"), (mi, "kinetic_i"))):
        want = 0.5 * m * w * np.sum(st[s]["vel"] ** 2)
        assert abs(en[key] / want - 1) < 1e-12, (key, en[key], want)
    nxy = 16 * 16
    vol = np.full(E.shape[1], wl["dx"] ** 3)
    vol[:nxy] *= 0.5
    vol[-nxy:] *= 0.5
    want = 0.5 * 8.8541878128e-12 * np.sum(vol * np.sum(E ** 2, axis=0))
    assert abs(en["field"] / want - 1) < 1e-12
    assert en["total"] == en["kinetic_e"] + en["kinetic_i"] + en["field"]
    assert sim.energy() == en  # repeatable
    sim.close()
