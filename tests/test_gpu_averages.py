"""Time- and rf-phase-averaged diagnostics (pic_average, pic_average_read)
through the C ABI, against the oracle.

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


@pytest.mark.parametrize("form,graphs,interval,bins", [
    ("fp64", 1, 2, 3), ("fp32r", 1, 3, 4), ("fp32r", 0, 1, 2), ("batched", 1, 2, 3)])
def test_averages_match_oracle(form, graphs, interval, bins):
    from paper_1801_00972_amd.pic import Simulation
    wls = _wls(form)
    prec = wls[0]["precision"]
    print(f"[case] {form} graphs={graphs} interval={interval} bins={bins}", flush=True)
    sim = Simulation(wls if form == "batched" else wls[0])
    sim.set_tuning(use_graphs=graphs)
    if form == "batched":
        assert sim.tuning()["batch_push"] == 1
    sim.step(2)
    sim.average(interval, bins)
    R = len(wls)
    acc = [[dict(phi=0.0, n=0.0, flux=0.0, count=0, V=0.0) for _ in range(bins)] for _ in range(R)]
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
                a["count"] += 1
                a["V"] = max(a["V"], abs(orc.rf_voltage(st["step"])))
        sim.step(1)
    for r in range(R):
        total = dict(phi=0.0, n=0.0, flux=0.0, count=0, V=0.0)
        for b in range(bins):
            a = acc[r][b]
            g = sim.averages(r, b)
            assert g["samples"] == a["count"]
            for k in ("phi", "n", "flux"):
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
        g = sim.averages(r, -1)
        assert g["samples"] == total["count"] == len(range(0, 13, interval))
        assert rel_inf(g["n"], total["n"] / total["count"]) <= 1e-12
        assert rel_inf(g["phi"], total["phi"] / total["count"], floor=total["V"]) <= FIELD_TOL[prec]
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
