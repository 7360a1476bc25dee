"""Pins of the oracle's particle moments: the densities and fluxes of the
results (Sec. IV), assigned to the nodes with the cloud-in-cell weights of
Sec. III.

Pins: the load density of a uniform lattice (n0 on interior nodes and half
of it on the electrode planes, by the definition of the macro-particle
weight), conservation of particle number and momentum, linear reproduction
(the weighted node positions give back the particle position, which fixes
each axis), flux = n v for a common velocity (which fixes the component
order), translation by one cell (a periodic roll of the node arrays along
the right axis), and the charge density from the oracle's deposit, which is
e (n_i - n_e) without grains.
"""
import numpy as np
import pytest

import oracle
from paper_1801_00972_amd import workloads as W

E_CH = 1.602176634e-19


def _oracle(wl, pos_e, vel_e, pos_i=None, vel_i=None):
    o = oracle.Oracle(wl)
    pos_i = np.zeros((0, 3)) if pos_i is None else pos_i
    vel_i = np.zeros((0, 3)) if vel_i is None else vel_i
    o.set_particles(0, pos_e, vel_e, np.arange(len(pos_e)))
    o.set_particles(1, pos_i, vel_i, np.arange(len(pos_i)))
    return o


def _grid(wl, n):
    return np.asarray(n).reshape(wl["nz"] + 1, wl["ny"], wl["nx"])


def test_uniform_lattice_gives_the_load_density():
    wl = W.tiny(nx=6, ny=5, nz=7, ppc=8)
    nx, ny, nz = wl["nx"], wl["ny"], wl["nz"]
    # 8 particles per cell on the 2x2x2 sub-lattice at quarter offsets
    sub = np.array([[a, b, c] for c in (0.25, 0.75) for b in (0.25, 0.75) for a in (0.25, 0.75)])
    cells = np.array([[i, j, k] for k in range(nz) for j in range(ny) for i in range(nx)], float)
    pos = (cells[:, None, :] + sub[None, :, :]).reshape(-1, 3)
    o = _oracle(wl, pos, np.zeros_like(pos), pos, np.zeros_like(pos))
    n, flux = o.moments()
    for s in range(2):
        g = _grid(wl, n[s])
        assert np.allclose(g[1:nz], wl["n0"], rtol=1e-14, atol=0)
        assert np.allclose(g[0], wl["n0"] / 2, rtol=1e-14, atol=0)
        assert np.allclose(g[nz], wl["n0"] / 2, rtol=1e-14, atol=0)
    assert not np.any(flux)


def test_number_momentum_and_position_are_conserved():
    wl = W.tiny(nx=6, ny=5, nz=7)
    rng = np.random.default_rng(3)
    m = 400
    # keep x, y below the last cell so the node positions need no minimum image
    pos = rng.uniform([0, 0, 0], [5, 4, 7], size=(m, 3))
    vel = rng.normal(size=(m, 3)) * [1e5, 2e5, 3e5]
    pos_i = rng.uniform([0, 0, 0], [5, 4, 7], size=(m // 2, 3))
    vel_i = rng.normal(size=(m // 2, 3)) * 300.0
    o = _oracle(wl, pos, vel, pos_i, vel_i)
    n, flux = o.moments()
    w, vol = o.derived()["w"], wl["dx"] ** 3
    k, j, i = np.meshgrid(np.arange(wl["nz"] + 1), np.arange(wl["ny"]), np.arange(wl["nx"]),
                          indexing="ij")
    node = [i.ravel(), j.ravel(), k.ravel()]
    for s, (p, v) in enumerate(((pos, vel), (pos_i, vel_i))):
        assert n[s].sum() * vol == pytest.approx(w * len(p), rel=1e-13)
        for a in range(3):
            assert flux[s, a].sum() * vol == pytest.approx(w * v[:, a].sum(), rel=1e-12)
            assert (n[s] * node[a]).sum() * vol == pytest.approx(w * p[:, a].sum(), rel=1e-13)


def test_common_velocity_gives_flux_n_v():
    wl = W.tiny(nx=6, ny=5, nz=7)
    rng = np.random.default_rng(4)
    pos = rng.uniform([0, 0, 0], [6, 5, 7], size=(300, 3))
    v0 = np.array([1.0e5, -2.0e5, 3.0e5])
    o = _oracle(wl, pos, np.tile(v0, (300, 1)))
    n, flux = o.moments()
    for a in range(3):
        assert np.allclose(flux[0, a], n[0] * v0[a], rtol=1e-13, atol=0)
    assert not np.any(n[1]) and not np.any(flux[1])


@pytest.mark.parametrize("axis", [0, 1])
def test_shift_by_one_cell_rolls_the_arrays(axis):
    wl = W.tiny(nx=6, ny=5, nz=7)
    rng = np.random.default_rng(5 + axis)
    pos = rng.uniform([0, 0, 0], [6, 5, 7], size=(200, 3))
    vel = rng.normal(size=(200, 3)) * 1e5
    n0, f0 = _oracle(wl, pos, vel).moments()
    moved = pos.copy()
    period = (wl["nx"], wl["ny"])[axis]
    moved[:, axis] = np.mod(moved[:, axis] + 1.0, period)
    n1, f1 = _oracle(wl, moved, vel).moments()
    roll_axis = 2 - axis  # node arrays are [z][y][x]
    assert np.allclose(_grid(wl, n1[0]), np.roll(_grid(wl, n0[0]), 1, axis=roll_axis),
                       rtol=1e-12, atol=1e-12 * np.abs(n0).max())
    for a in range(3):
        assert np.allclose(_grid(wl, f1[0, a]), np.roll(_grid(wl, f0[0, a]), 1, axis=roll_axis),
                           rtol=1e-12, atol=1e-12 * np.abs(f0).max())


def test_charge_density_is_e_times_density_difference():
    wl = W.tiny(nx=6, ny=5, nz=7)
    rng = np.random.default_rng(6)
    pos_e = rng.uniform([0, 0, 0], [6, 5, 7], size=(250, 3))
    pos_i = rng.uniform([0, 0, 0], [6, 5, 7], size=(180, 3))
    o = _oracle(wl, pos_e, np.zeros_like(pos_e), pos_i, np.zeros_like(pos_i))
    n, _ = o.moments()
    rho = o.deposit()
    scale = np.abs(rho).max()
    assert np.allclose(rho, E_CH * (n[1] - n[0]), rtol=1e-12, atol=1e-13 * scale)
