"""Parity at the benchmark's full size (64x64x256 cells, 32 ppc, 8 grains, the
launch configuration bench.py times): all mesh quantities of a state the GPU
produced after a few steps, the densities and fluxes of that state, one step of
every particle moved by the oracle in its own field and compared by id, the
charge density the step's fused deposit leaves (bit-exact in fixed point).
Plus exact particle conservation."""
import numpy as np
import pytest

import oracle
from paper_1801_00972_amd import workloads as W
from tests.parity_util import compare_step, compare_step_all, rel_inf

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = {"fp64": 1e-12, "fp32r": 1e-5}


def _select(pos, grains, nz, rng, n_uniform=2000, n_grain=1500, n_wall=500):
    n = len(pos)
    pick = [rng.choice(n, size=min(n_uniform, n), replace=False)]
    grains = np.asarray(grains)
    box = np.flatnonzero(np.all((pos >= grains.min(0) - 3.5) & (pos <= grains.max(0) + 3.5), axis=1))
    d2 = np.full(len(box), np.inf)
    for g in grains:
        d = pos[box] - g
        d2 = np.minimum(d2, np.sum(d * d, axis=1))
    near = box[d2 < 3.5 ** 2]
    if len(near):
        pick.append(rng.choice(near, size=min(n_grain, len(near)), replace=False))
    wall = np.flatnonzero((pos[:, 2] < 0.3) | (pos[:, 2] > nz - 0.3))
    if len(wall):
        pick.append(rng.choice(wall, size=min(n_wall, len(wall)), replace=False))
    return np.unique(np.concatenate(pick))


@pytest.mark.parametrize("prec", ["fp32r", "fp64"])
def test_fullsize_fields_and_step(prec):
    from paper_1801_00972_amd.pic import PIC_E, PIC_PHI, PIC_RHO, PIC_RHO_FIXED, Simulation
    wl = W.full_fp64(prec)
    print(f"[case] {wl['name']}", flush=True)
    sim = Simulation(wl)  # the benchmark's configuration (sort every 16 steps)
    sim.step(3)
    st = sim.get_state()
    n0 = 64 * 64 * 256 * 32
    c = sim.counters()
    counts, _ = sim.grain_charges()
    for s in range(2):
        assert len(st[s]["id"]) == c["n_alive"][s]
        assert c["n_alive"][s] + sum(c["wall_count"][w][s] for w in range(2)) + counts[:, s].sum() == n0
    # all mesh quantities of this state
    fixed = prec == "fp32r"
    orc = oracle.Oracle(wl)
    for s in range(2):
        orc.set_particles(s, st[s]["pos"], st[s]["vel"], st[s]["id"])
    orc.set_counts(grain_count=st["grain_count"], wall_count=st["wall_count"], step=st["step"])
    g = sim.fields(0, PIC_PHI | PIC_E | PIC_RHO | (PIC_RHO_FIXED if fixed else 0))
    o = orc.fields(fixed_point=fixed)
    if fixed:
        assert np.array_equal(g["rho_fixed"], o["rho_fixed"])
    else:
        assert rel_inf(g["rho"], o["rho"]) <= 1e-12
    e_phi = rel_inf(g["phi"], o["phi"], floor=abs(orc.rf_voltage(st["step"])))
    e_E = rel_inf(g["E"], o["E"])
    print(f"  fields: phi {e_phi:.2e} E {e_E:.2e}", flush=True)
    assert e_phi <= TOL[prec] and e_E <= TOL[prec]
    # densities and fluxes of the same state
    from paper_1801_00972_amd.pic import PIC_FLUX, PIC_N
    gm = sim.fields(0, PIC_N | PIC_FLUX)
    n_o, flux_o = orc.moments()
    e_n, e_f = rel_inf(gm["n"], n_o), rel_inf(gm["flux"], flux_o)
    print(f"  moments: n {e_n:.2e} flux {e_f:.2e}", flush=True)
    assert e_n <= 1e-12 and e_f <= 1e-12
    del gm, n_o, flux_o
    # the fine grid of 200^3 cells of 0.08 dx over the grain cluster
    from paper_1801_00972_amd.pic import PIC_FINE_FLUX, PIC_FINE_N, PIC_FINE_PHI
    h, cells = 0.08, (200, 200, 200)
    centre = np.asarray(wl["grain_pos"]).mean(axis=0)
    origin = np.clip(np.floor(centre - 8.0), 0, [wl["nx"] - 16, wl["ny"] - 16, wl["nz"] - 16])
    sim.set_fine_grid(origin, h, cells)
    gf = sim.fields(0, PIC_FINE_N | PIC_FINE_FLUX | PIC_FINE_PHI)
    fn_o, ff_o = orc.fine_moments(origin, h, cells)
    e_n, e_f = rel_inf(gf["fine_n"], fn_o), rel_inf(gf["fine_flux"], ff_o)
    fp_o = orc.fine_phi(o["phi"], origin, h, cells)
    e_p = rel_inf(gf["fine_phi"], fp_o, floor=abs(orc.rf_voltage(st["step"])))
    print(f"  fine grid at {origin}: n {e_n:.2e} flux {e_f:.2e} phi {e_p:.2e}", flush=True)
    assert np.any(fn_o) and e_n <= 1e-12 and e_f <= 1e-12 and e_p <= TOL[prec]
    sim.set_fine_grid(None)
    del gf, fn_o, ff_o, fp_o
    # one step of every particle (6.7e7), moved by the oracle in its own field
    del st
    print("  oracle step of every particle", flush=True)
    orc.step_in_field(o["E"])
    sim.step(1)
    after = sim.get_state()
    print("  comparing by id", flush=True)
    rep = compare_step_all(wl, after, orc, TOL[prec], TOL[prec], TOL[prec])
    print(f"  full step: n={rep['n']} flips={rep['flips']} dpos={rep['max_dpos']:.2e} "
          f"dvel={rep['max_dvel']:.2e}", flush=True)
    assert rep["n"] > 0.99 * n0 and rep["flips"] <= 20
    assert np.array_equal(after["grain_count"], orc.grain_count) or rep["flips"] > 0
    # the deposit fused into the step: rho_{k+1} of the GPU's own new state
    dep = oracle.Oracle(wl)
    for s in range(2):
        dep.set_particles(s, after[s]["pos"], after[s]["vel"], after[s]["id"])
    dep.set_counts(grain_count=after["grain_count"], step=after["step"])
    g1 = sim.fields(0, PIC_RHO_FIXED if fixed else PIC_RHO)
    if fixed:
        assert np.array_equal(g1["rho_fixed"], dep.deposit_fixed())
    else:
        assert rel_inf(g1["rho"], dep.deposit()) <= 1e-12
    print("  rho_{k+1} of the fused deposit checked", flush=True)
    sim.close()


def test_fullsize_fields_after_sheath_formation():
    """The FP32R fields on a developed state (1,300 steps: sheaths formed, grains
    charged; the refinement sweeps until the residual is below its tolerance)
    against the oracle's fields of that state."""
    from paper_1801_00972_amd.pic import PIC_E, PIC_PHI, PIC_RHO_FIXED, Simulation
    wl = W.full_fp64("fp32r")
    print(f"[case] {wl['name']} after 1300 steps", flush=True)
    sim = Simulation(wl)
    for k in range(13):
        sim.step(100)
        print(f"  step {(k + 1) * 100}", flush=True)
    st = sim.get_state()
    g = sim.fields(0, PIC_PHI | PIC_E | PIC_RHO_FIXED)
    res = sim.counters()["refine_residual"]
    orc = oracle.Oracle(wl)
    for s in range(2):
        orc.set_particles(s, st[s]["pos"], st[s]["vel"], st[s]["id"])
    orc.set_counts(grain_count=st["grain_count"], wall_count=st["wall_count"], step=st["step"])
    o = orc.fields(fixed_point=True)
    assert np.array_equal(g["rho_fixed"], o["rho_fixed"])
    e_phi = rel_inf(g["phi"], o["phi"], floor=abs(orc.rf_voltage(st["step"])))
    e_E = rel_inf(g["E"], o["E"])
    print(f"  residual {res:.2e}: phi {e_phi:.2e} E {e_E:.2e}", flush=True)
    assert e_phi <= TOL["fp32r"] and e_E <= TOL["fp32r"]
    sim.close()


def _pairings(cells_e, cells_i, ncell):
    """Binary collisions of one Coulomb pass by the pairing rule, from the cells."""
    ne, ni = np.bincount(cells_e, minlength=ncell), np.bincount(cells_i, minlength=ncell)
    total = 0
    for n in (ne, ni):
        odd = (n >= 3) & (n % 2 == 1)
        total += int(np.sum(np.where(odd, 3 + (n - 3) // 2, np.where(n >= 2, n // 2, 0))))
    return total + int(np.sum(np.where((ne > 0) & (ni > 0), np.maximum(ne, ni), 0)))


def test_fullsize_coulomb_and_cross_section_tables():
    """A step at the benchmark's full size with Coulomb collisions and the
    synthetic cross-section tables.  A pass pairs the particles of each cell
    only, so the oracle runs it on 16 whole z-planes around the grains; a
    sample of those particles, with their post-pass velocities, is then moved
    by the oracle in the full state's field and compared with the GPU step.
    The GPU's pairing count over the whole box equals the pairing rule's
    count from the cells.  A large Coulomb logarithm makes the pass turn
    velocities visibly at the FP32R tolerance."""
    from paper_1801_00972_amd.pic import Simulation
    wl = dict(W.full_fp64("fp32r"), coulomb_interval=1, coulomb_lnL=1.0e6, xs=W.stand_in_xs())
    print(f"[case] {wl['name']} with Coulomb collisions and cross-section tables", flush=True)
    sim = Simulation(wl)
    sim.step(3)
    st = sim.get_state()
    c0 = sim.counters()["n_coulomb"]
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    cells = [(np.floor(st[s]["pos"]).astype(np.int64) * [1, nx, nx * ny]).sum(axis=1) for s in range(2)]
    full = oracle.Oracle(wl)
    for s in range(2):
        full.set_particles(s, st[s]["pos"], st[s]["vel"], st[s]["id"])
    full.set_counts(grain_count=st["grain_count"], wall_count=st["wall_count"], step=st["step"])
    E = full.fields(fixed_point=True)["E"]
    del full
    print("  oracle fields done", flush=True)
    # 16 whole z-planes around the grains
    z0 = int(np.floor(np.asarray(wl["grain_pos"])[:, 2].mean())) - 8
    sub = oracle.Oracle(wl)
    rows = []
    for s in range(2):
        r = np.flatnonzero((st[s]["pos"][:, 2] >= z0) & (st[s]["pos"][:, 2] < z0 + 16))
        rows.append(r)
        sub.set_particles(s, st[s]["pos"][r].copy(), st[s]["vel"][r].copy(), st[s]["id"][r])
    sub.set_counts(grain_count=st["grain_count"], step=st["step"])
    pairs_sub = sub.coulomb()
    sub_cells = [cells[s][rows[s]] for s in range(2)]
    assert pairs_sub == _pairings(sub_cells[0], sub_cells[1], nx * ny * nz)
    print(f"  oracle Coulomb pass on planes {z0}..{z0 + 15}: {pairs_sub} pairings", flush=True)
    changed = sum(int(np.count_nonzero(np.any(sub.vel[s] != st[s]["vel"][rows[s]], axis=1)))
                  for s in range(2))
    rng = np.random.default_rng(12)
    small = oracle.Oracle(dict(wl, coulomb_interval=0))
    for s in range(2):
        idx = _select(sub.pos[s], wl["grain_pos"], nz, rng)
        small.set_particles(s, sub.pos[s][idx], sub.vel[s][idx], sub.id[s][idx])
    small.set_counts(grain_count=st["grain_count"], step=st["step"])
    small.step_in_field(E)
    sim.step(1)
    after = sim.get_state()
    assert sim.counters()["n_coulomb"] - c0 == _pairings(cells[0], cells[1], nx * ny * nz)
    gsub = {}
    for s in range(2):
        keep = np.isin(after[s]["id"], small.id[s])
        gsub[s] = {k: after[s][k][keep] for k in ("pos", "vel", "id")}
    rep = compare_step(wl, gsub, small, TOL["fp32r"], TOL["fp32r"], TOL["fp32r"])
    print(f"  sampled step: n={rep['n']} flips={rep['flips']} dpos={rep['max_dpos']:.2e} "
          f"dvel={rep['max_dvel']:.2e}; the pass changed {changed} of "
          f"{len(rows[0]) + len(rows[1])} velocities", flush=True)
    assert changed > 0.5 * (len(rows[0]) + len(rows[1]))
    assert rep["n"] > 3000 and rep["flips"] <= 3
    sim.close()
