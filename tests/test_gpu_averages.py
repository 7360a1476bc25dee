"""Time- and rf-phase-averaged diagnostics (pic_average, pic_average_read)
through the C ABI, against the oracle, with and without the fine grid.

The GPU samples phi_k and the particle moments inside pic_step (in the
captured step graph, in direct launches, and in the batched step of an
ensemble).  The test reads the GPU state at every sampled step, lets the
oracle compute phi and the moments of that state, puts them in the same
rf-phase bin and averages: phi within the field tolerance, the moments to
1e-12, sample counts exact.  A stopped average takes no more samples.
"""
import numpy as np
import pytest

from paper_1801_00972_amd import workloads as W
from tests.parity_util import oracle_from_state, rel_inf

pytestmark = pytest.mark.gpu

FIELD_TOL = {"fp64": 1e-12, "fp32r": 1e-5}


def _phase_bin(k, f_rf, dt, nbins):
    x = f_rf * (float(k) * dt)
    return min(max(int((x - np.floor(x)) * nbins), 0), nbins - 1)


def _wls(form):
    prec = "fp64" if form == "fp64" else "fp32r"
    base = dict(W.small_fp64(), precision=prec)
    # an rf period of 6.5 steps, so a dozen steps fill every phase bin
    base["f_rf"] = 1.0 / (6.5 * base["dt"])
    if form != "batched":
        return [base]
    other = W.tiny(nx=12, ny=10, nz=17, ppc=3, grains=[[0.3, 9.6, 8.5]], cutoff=2, precision=prec,
                   seed=12, f_rf=base["f_rf"])
    return [base, other]


# fine grids of the replicas (origin, h, cells): 0.08-cell cells around the
# small box's grain, and half cells over the second replica's grain
FINE = [((7.0, 7.0, 15.0), 0.08, (25, 25, 25)), ((0.0, 8.0, 7.0), 0.5, (8, 4, 5))]


@pytest.mark.parametrize("form,graphs,interval,bins,fine", [
    ("fp64", 1, 2, 3, 0), ("fp32r", 1, 3, 4, 1), ("fp32r", 0, 1, 2, 0), ("fp64", 0, 1, 2, 1),
    ("batched", 1, 2, 3, 1)])
def test_averages_match_oracle(form, graphs, interval, bins, fine):
    from paper_1801_00972_amd.pic import (PIC_FINE_FLUX, PIC_FINE_N, PIC_FINE_PHI, PIC_FLUX, PIC_N,
                                          PIC_PHI, Simulation)
    wls = _wls(form)
    prec = wls[0]["precision"]
    print(f"[case] {form} graphs={graphs} interval={interval} bins={bins} fine={fine}", flush=True)
    sim = Simulation(wls if form == "batched" else wls[0])
    sim.set_tuning(use_graphs=graphs)
    if form == "batched":
        assert sim.tuning()["batch_push"] == 1
    R = len(wls)
    if fine:
        for r in range(R):
            sim.set_fine_grid(*FINE[r], replica=r)
    what = PIC_PHI | PIC_N | PIC_FLUX | ((PIC_FINE_N | PIC_FINE_FLUX | PIC_FINE_PHI) if fine else 0)
    sim.step(2)
    sim.average(interval, bins)
    acc = [[dict(phi=0.0, n=0.0, flux=0.0, fine_n=0.0, fine_flux=0.0, fine_phi=0.0, count=0, V=0.0)
            for _ in range(bins)] for _ in range(R)]
    for s in range(13):
        if s % interval == 0:
            for r in range(R):
                st = sim.get_state(r)
                orc = oracle_from_state(wls[r], st)
                f = orc.fields()
                n, flux = orc.moments()
                a = acc[r][_phase_bin(st["step"], wls[r]["f_rf"], wls[r]["dt"], bins)]
                a["phi"] = a["phi"] + f["phi"]
                a["n"] = a["n"] + n
                a["flux"] = a["flux"] + flux
                if fine:
                    fn_, ff_ = orc.fine_moments(*FINE[r])
                    a["fine_n"] = a["fine_n"] + fn_
                    a["fine_flux"] = a["fine_flux"] + ff_
                    a["fine_phi"] = a["fine_phi"] + orc.fine_phi(f["phi"], *FINE[r])
                a["count"] += 1
                a["V"] = max(a["V"], abs(orc.rf_voltage(st["step"])))
        sim.step(1)
    for r in range(R):
        total = dict(phi=0.0, n=0.0, flux=0.0, fine_n=0.0, fine_flux=0.0, fine_phi=0.0, count=0, V=0.0)
        for b in range(bins):
            a = acc[r][b]
            g = sim.averages(r, b, what=what)
            assert g["samples"] == a["count"]
            for k in ("phi", "n", "flux", "fine_n", "fine_flux", "fine_phi"):
                total[k] = total[k] + a[k]
            total["count"] += a["count"]
            total["V"] = max(total["V"], a["V"])
            if a["count"] == 0:
                assert not np.any(g["phi"]) and not np.any(g["n"])
                continue
            e_phi = rel_inf(g["phi"], a["phi"] / a["count"], floor=a["V"])
            e_n = rel_inf(g["n"], a["n"] / a["count"])
            e_f = rel_inf(g["flux"], a["flux"] / a["count"])
            print(f"  replica {r} bin {b}: {a['count']} samples, phi {e_phi:.2e} n {e_n:.2e} "
                  f"flux {e_f:.2e}", flush=True)
            assert e_phi <= FIELD_TOL[prec] and e_n <= 1e-12 and e_f <= 1e-12
            if fine:
                e_fn = rel_inf(g["fine_n"], a["fine_n"] / a["count"])
                e_ff = rel_inf(g["fine_flux"], a["fine_flux"] / a["count"])
                e_fp = rel_inf(g["fine_phi"], a["fine_phi"] / a["count"], floor=a["V"])
                print(f"    fine grid: n {e_fn:.2e} flux {e_ff:.2e} phi {e_fp:.2e}", flush=True)
                assert np.any(a["fine_n"]) and e_fn <= 1e-12 and e_ff <= 1e-12
                assert e_fp <= FIELD_TOL[prec]
        g = sim.averages(r, -1, what=what)
        assert g["samples"] == total["count"] == len(range(0, 13, interval))
        assert rel_inf(g["n"], total["n"] / total["count"]) <= 1e-12
        assert rel_inf(g["phi"], total["phi"] / total["count"], floor=total["V"]) <= FIELD_TOL[prec]
        if fine:
            assert rel_inf(g["fine_n"], total["fine_n"] / total["count"]) <= 1e-12
            assert rel_inf(g["fine_flux"], total["fine_flux"] / total["count"]) <= 1e-12
            assert rel_inf(g["fine_phi"], total["fine_phi"] / total["count"],
                           floor=total["V"]) <= FIELD_TOL[prec]
    # stopped: the sums stay as they are
    sim.average(0)
    sim.step(3)
    assert sim.averages(0, -1)["samples"] == total["count"]
    sim.close()


def test_average_arguments_are_checked():
    from paper_1801_00972_amd.pic import PIC_E, PicError, Simulation
    sim = Simulation(W.small_fp32r())
    with pytest.raises(PicError):
        sim.averages(0, -1)  # never started
    for args in ((-1, 1), (1, 0), (1, 65)):
        with pytest.raises(PicError):
            sim.average(*args)
    sim.average(1, 2)
    sim.step(2)
    with pytest.raises(PicError):
        sim.averages(0, 2)
    with pytest.raises(PicError):
        sim.averages(0, -1, what=PIC_E)
    assert sim.averages(0, 1)["samples"] + sim.averages(0, 0)["samples"] == 2
    sim.close()
