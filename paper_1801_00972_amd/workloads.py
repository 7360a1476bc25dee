"""Seeded synthetic workloads of the rf-sheath dust-cluster problem.

This module holds inputs only -- box, species, gas, rf drive, time step and the
fixed grain positions -- and none of the method's arithmetic.  Both the HIP
library (through its Python binding) and the CPU oracle take the same dicts.

Keys (SI units, temperatures as kT in eV, positions of grains in cell units):
  nx, ny, nz        cells; x,y periodic, z from the grounded wall (z=0) to the rf electrode
  dx, dt            cell edge (m), time step (s)
  ppc               macro-particles per cell per species at load
  n0                plasma density (m^-3) that sets the macro-particle weight
  Te_eV, Ti_eV      load temperatures
  p_gas, T_gas      neutral argon reservoir (Pa, K)
  sigma_e, sigma_i  e-Ar elastic and Ar+-Ar charge-exchange cross sections (m^2)
  V_dc, V_rf, f_rf  rf electrode potential V_dc + V_rf sin(2 pi f_rf t)
  grain_radius      m
  grain_pos         (n_grains, 3) float64, cell units
  cutoff            MD cube half-width in cells
  md_sub            sub-steps per step inside the MD region
  seed              Philox key of the replica
  E_cap_eV          null-collision cap on the relative kinetic energy
  precision         "fp64" or "fp32r"
  steps             length of the run the workload is quoted for

The paper's own cluster (44 grains at measured positions) exists only in a
figure, and its cross sections come from a database that is not available, so
these workloads stand in for it with the same structure: a box that is periodic
laterally and bounded by two electrodes along the discharge axis, a fixed
cluster of micron-size absorbing grains in the sheath, Maxwellian electrons and
ions, and a neutral argon reservoir.
"""
from __future__ import annotations

import numpy as np

_BASE = dict(
    dx=50e-6, dt=5e-12, ppc=8, n0=1e15, Te_eV=3.0, Ti_eV=0.03,
    p_gas=10.0, T_gas=300.0, sigma_e=1e-19, sigma_i=5e-19,
    V_dc=-60.0, V_rf=40.0, f_rf=13.56e6, grain_radius=4e-6,
    cutoff=3, md_sub=40, seed=0, E_cap_eV=1000.0, precision="fp64",
)


def place_grains(n: int, center, radius_cells: float, min_sep_cells: float, seed: int,
                 max_tries: int = 1_000_000) -> np.ndarray:
    """Uniform positions inside a sphere (cell units), rejecting any candidate
    closer than min_sep_cells to an accepted one.  Seeded numpy PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    center = np.asarray(center, np.float64)
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise ValueError("grain placement failed: cluster too dense")
        p = center + radius_cells * (2.0 * rng.random(3) - 1.0)
        if np.sum((p - center) ** 2) > radius_cells ** 2:
            continue
        if any(np.sum((p - q) ** 2) < min_sep_cells ** 2 for q in out):
            continue
        out.append(p)
    return np.array(out, dtype=np.float64).reshape(n, 3)


def sheath_center_z(nz: int, dx: float, frac: float = 0.4, sheath_m: float = 3.05e-3) -> float:
    """Height (cell units) of the cluster centre: `frac` of an estimated sheath
    width below the rf electrode at z = nz (Child-law estimate at 60 V, 3 eV)."""
    return nz - frac * sheath_m / dx


def small_fp64() -> dict:
    """16x16x32 cells of 50 um, 8 ppc, one grain exactly on node (8, 8, 16)."""
    wl = dict(_BASE, nx=16, ny=16, nz=32, ppc=8, steps=500,
              grain_pos=np.array([[8.0, 8.0, 16.0]]))
    wl["name"] = "small_fp64_16x16x32_ppc8"
    return wl


def small_fp32r() -> dict:
    wl = small_fp64()
    wl["precision"] = "fp32r"
    wl["name"] = "small_fp32r_16x16x32_ppc8"
    return wl


def full_fp64(precision: str = "fp64") -> dict:
    """64x64x256 cells of 50 um, 32 ppc (~6.7e7 particles), 8 grains in a
    0.5 mm sphere (min separation 200 um) at 40% of the sheath height below
    the rf electrode, PPPM cutoff 3 cells."""
    nx, ny, nz, dx = 64, 64, 256, 50e-6
    g = place_grains(8, (nx / 2, ny / 2, sheath_center_z(nz, dx)), 0.5e-3 / dx, 200e-6 / dx, seed=1)
    wl = dict(_BASE, nx=nx, ny=ny, nz=nz, ppc=32, steps=20000, grain_pos=g, cutoff=3,
              precision=precision)
    wl["name"] = f"full_{precision}_64x64x256_ppc32_8grains"
    return wl


def large_fp32r() -> dict:
    """128x128x512 cells of 25 um, 16 ppc (~2.7e8 particles), 64 grains in a
    1 mm sphere, PPPM cutoff 4 cells."""
    nx, ny, nz, dx = 128, 128, 512, 25e-6
    g = place_grains(64, (nx / 2, ny / 2, sheath_center_z(nz, dx)), 1.0e-3 / dx, 200e-6 / dx, seed=5)
    wl = dict(_BASE, nx=nx, ny=ny, nz=nz, dx=dx, ppc=16, steps=10000, grain_pos=g, cutoff=4,
              precision="fp32r")
    wl["name"] = "large_fp32r_128x128x512_ppc16_64grains"
    return wl


def ensemble(n_replicas: int = 16, seed: int = 4) -> list:
    """Uneven replicas: grid from {32x32x128, 48x48x192, 64x64x256} at 50 um,
    16-32 ppc, 1-32 grains placed as for the full-size run, FP32-refined."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grids = [(32, 32, 128), (48, 48, 192), (64, 64, 256)]
    out = []
    for r in range(n_replicas):
        nx, ny, nz = grids[int(rng.integers(0, 3))]
        ppc = int(rng.integers(16, 33))
        ng = int(rng.integers(1, 33))
        dx = 50e-6
        g = place_grains(ng, (nx / 2, ny / 2, sheath_center_z(nz, dx)), min(0.5e-3 / dx, nx / 2 - 5),
                         200e-6 / dx, seed=100 + r)
        wl = dict(_BASE, nx=nx, ny=ny, nz=nz, ppc=ppc, steps=5000, grain_pos=g, cutoff=3,
                  seed=r, precision="fp32r")
        wl["name"] = f"replica{r}_{nx}x{ny}x{nz}_ppc{ppc}_{ng}grains"
        out.append(wl)
    return out


def column(seed: int = 0, precision: str = "fp64") -> dict:
    """16x16x128 cells of 50 um (0.8 x 0.8 x 6.4 mm), 4 ppc (262,144
    particles), two grains one above the other in the rf sheath at (8, 8,
    100) and (8, 8, 108): a narrow column tall enough for a bulk plasma
    between the two sheaths, for long statistical runs over many seeds."""
    wl = dict(_BASE, nx=16, ny=16, nz=128, ppc=4, steps=2000, cutoff=3, seed=seed,
              grain_pos=np.array([[8.0, 8.0, 100.0], [8.0, 8.0, 108.0]]), precision=precision)
    wl["name"] = f"column_{precision}_16x16x128_ppc4_2grains"
    return wl


def small_ensemble() -> list:
    """Three uneven small FP32-refined replicas (a quick form of the ensemble)."""
    out = []
    for r, (nx, ny, nz, ppc, g) in enumerate(((16, 16, 32, 8, [[8.0, 8.0, 16.0]]),
                                              (24, 24, 48, 6, [[12.0, 12.0, 30.5], [6.2, 17.9, 28.0]]),
                                              (32, 16, 40, 4, [[10.5, 8.5, 20.0]]))):
        wl = dict(_BASE, nx=nx, ny=ny, nz=nz, ppc=ppc, steps=500, cutoff=2, seed=r,
                  grain_pos=np.asarray(g, np.float64), precision="fp32r")
        wl["name"] = f"replica{r}_{nx}x{ny}x{nz}_ppc{ppc}"
        out.append(wl)
    return out


def tiny(nx=8, ny=8, nz=12, ppc=2, grains=None, **kw) -> dict:
    """Small boxes for parity cases that still span several tiles."""
    wl = dict(_BASE, nx=nx, ny=ny, nz=nz, ppc=ppc, steps=10,
              grain_pos=np.zeros((0, 3)) if grains is None else np.asarray(grains, np.float64))
    wl.update(kw)
    wl["name"] = f"tiny_{nx}x{ny}x{nz}_ppc{ppc}"
    return wl


def stand_in_xs(ionization: bool = False) -> dict:
    """Synthetic cross-section tables for the energy-dependent collision path:
    smooth analytic shapes of roughly argon-like magnitude (NOT measured data),
    on one grid of projectile energies (eV), for timing and tests; with
    `ionization`, also an ionisation table above a 15.76 eV threshold."""
    E = np.concatenate([[0.0], np.geomspace(1e-2, 1e3, 63)])
    e_el = 1.0e-19 * (0.4 + 0.6 * E / (1.0 + E)) / np.sqrt(1.0 + E / 200.0)
    E_ex = 11.5
    e_ex = np.where(E > E_ex, 3.0e-20 * (1.0 - E_ex / np.maximum(E, E_ex)), 0.0)
    i_cx = 5.0e-19 / (1.0 + E) ** 0.1
    i_el = 3.0e-19 / (1.0 + E) ** 0.2
    out = dict(E=E, e_el=e_el, e_ex=e_ex, i_cx=i_cx, i_el=i_el, E_ex=E_ex)
    if ionization:
        E_iz = 15.76
        out["e_iz"] = np.where(E > E_iz, 2.5e-20 * np.log(np.maximum(E, E_iz) / E_iz)
                               / (1.0 + np.log(np.maximum(E, E_iz) / E_iz)), 0.0)
        out["E_iz"] = E_iz
    return out
