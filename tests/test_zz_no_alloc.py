"""pic_fields_static (the entry point that allocates nothing) against pic_fields
on the GPU: the same quantities from the same state, two calls in a row on
two contexts, the second with a smaller box, through the C ABI.

Bar: the fixed-point charge density bit-exact; phi, E and rho from the same
deterministic solve bit-exact; densities and fluxes (FP64 atomic sums, whose
last bits depend on the order of additions) to 1e-12 of the largest value.
"""
import numpy as np
import pytest

from paper_1801_00972_amd import workloads as W
from paper_1801_00972_amd.pic import (PIC_E, PIC_EINVAL, PIC_FINE_PHI, PIC_FLUX, PIC_N, PIC_PHI,
                                      PIC_RHO, PIC_RHO_FIXED, PicError, Simulation,
                                      pic_fields_static)

pytestmark = pytest.mark.gpu

ALL = PIC_PHI | PIC_E | PIC_RHO | PIC_N | PIC_FLUX


def _static_fields(sim, what):
    import torch
    nn = sim.n_nodes[0]
    shapes = [(PIC_PHI, "phi", (nn,), torch.float64), (PIC_E, "E", (3, nn), torch.float64),
              (PIC_RHO, "rho", (nn,), torch.float64), (PIC_RHO_FIXED, "rho_fixed", (nn,), torch.int64),
              (PIC_N, "n", (2, nn), torch.float64), (PIC_FLUX, "flux", (2, 3, nn), torch.float64)]
    outs, names = [], []
    for bit, name, shape, dt in shapes:
        if what & bit:
            # filled with a marker so that an unwritten output shows
            outs.append(torch.full(shape, -7.0 if dt == torch.float64 else -7, dtype=dt, device="cuda"))
            names.append(name)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    pic_fields_static(sim.ctx, 0, what, outs, out_on_device=True)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 >= free0, f"device memory fell by {free0 - free1} bytes during the call"
    return {n: o.cpu().numpy() for n, o in zip(names, outs)}


def _compare(ref, got):
    for k in ("phi", "E", "rho", "rho_fixed"):
        if k in ref:
            assert np.array_equal(ref[k], got[k]), k
    for k in ("n", "flux"):
        if k in ref:
            scale = np.abs(ref[k]).max()
            assert scale > 0
            err = np.abs(ref[k] - got[k]).max() / scale
            assert err <= 1e-12, (k, err)


def test_static_fields_match_pic_fields_on_two_boxes():
    import torch
    torch.cuda.set_device(0)
    cases = [
        # the larger box first, then a smaller one: the second call must not
        # see what the first left in the fixed array
        (dict(W.small_fp64(), precision="fp32r"), ALL | PIC_RHO_FIXED, 3),
        (dict(W.small_fp64(), nx=12, ny=10, nz=9, grain_pos=[[6.0, 5.0, 4.5]], cutoff=2,
              precision="fp64"), ALL, 2),
    ]
    for wl, what, steps in cases:
        print(f"[no_alloc] {wl['nx']}x{wl['ny']}x{wl['nz']} {wl['precision']}", flush=True)
        sim = Simulation(wl)
        sim.step(steps)
        ref = sim.fields(0, what)
        got = _static_fields(sim, what)
        _compare(ref, got)
        # a second static call on the same state gives the same again
        again = _static_fields(sim, what)
        _compare(ref, again)
        sim.close()


def test_static_fields_rejects_what_it_cannot_stage():
    import torch
    torch.cuda.set_device(0)
    sim = Simulation(dict(W.small_fp64(), precision="fp32r"))
    nn = sim.n_nodes[0]
    buf = torch.zeros(64 * nn, dtype=torch.float64, device="cuda")
    with pytest.raises(PicError) as e:
        pic_fields_static(sim.ctx, 0, PIC_FINE_PHI, [buf], out_on_device=True)
    assert e.value.code == PIC_EINVAL
    sim.close()
    # 1,622,016 nodes: N needs 4 doubles per node, more than the 6 Mi doubles
    big = dict(W.small_fp64(), nx=128, ny=128, nz=98, ppc=1, grain_pos=[[64.0, 64.0, 49.0]],
               precision="fp32r")
    sim = Simulation(big)
    nn = sim.n_nodes[0]
    assert 4 * nn > 6 * 2 ** 20
    out = torch.zeros(2 * nn, dtype=torch.float64, device="cuda")
    with pytest.raises(PicError) as e:
        pic_fields_static(sim.ctx, 0, PIC_N, [out], out_on_device=True)
    assert e.value.code == PIC_EINVAL
    # E alone fits (3 doubles per node)
    ref = sim.fields(0, PIC_E)
    got = _static_fields(sim, PIC_E)
    assert np.array_equal(ref["E"], got["E"])
    sim.close()
