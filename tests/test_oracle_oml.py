"""Pin of the oracle's near-grain motion against the orbit-motion-limited (OML)
charging currents of an isolated grain (grain charging, Sec. IV.B; the MD
step of Eq. (5)-(6) with dt_MD = dt/40 is what collects the particles).

Test mode (the oracle's orc_oml_collect): mesh off, collisions off, the
grain's charge frozen, its field cut off outside a sphere of radius R_c =
40 a (the potential shifted to zero there), and particles injected across
that sphere with the flux-weighted Maxwellian of an unperturbed plasma.
Re-inserting each absorbed or escaping particle at R_c, as a steady state
would, is the same as injecting independent test particles, which is what
is done.  For a Coulomb potential the effective potential has no barrier
between a and R_c for either sign of charge, so OML theory is exact for this
setup: a particle of kinetic energy E entering with impact parameter b is
absorbed iff b^2 <= a^2 (1 - q dphi / E), dphi = Q/(4 pi eps0) (1/a - 1/R_c).
With b^2 uniform on [0, B^2] (flux-weighted directions, B <= R_c) and E
Gamma(2, kT) (flux-weighted energies), the absorbed fraction is
  P = E_E[min(1, (a/B)^2 max(0, 1 - q dphi / E))],
which the test integrates numerically.  Without the R_c cap it reduces to
the textbook OML currents: I_i = pi a^2 e n <v_i> (1 + e|dphi|/kT_i) for
attracted ions and I_e = pi a^2 e n <v_e> exp(-e|dphi|/kT_e) for repelled
electrons (checked first).  The grain's charge is the floating charge of
the textbook currents at T_e = 3 eV, T_i = 0.03 eV in argon, which puts the
grain at -7.23 V (Q ~ -2.0e4 e at a = 4 um).

Electrons are injected only with b <= 1.5 a: a repelled particle with b > a
can never reach the grain (angular momentum), so the flux outside that
bound contributes nothing and is left out (importance sampling).
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

import oracle
from paper_1801_00972_amd import workloads as W

E_CH = 1.602176634e-19
M_E = 9.1093837015e-31
M_AR = 39.948 * 1.66053906660e-27
EPS0 = 8.8541878128e-12
A = 4e-6          # grain radius (m)
TE, TI = 3.0, 0.03  # eV


def _mean_speed(T_eV, m):
    return np.sqrt(8.0 * T_eV * E_CH / (np.pi * m))


def _floating_potential():
    """Textbook OML: electron and ion currents equal at the grain surface."""
    ve, vi = _mean_speed(TE, M_E), _mean_speed(TI, M_AR)
    return brentq(lambda phi: ve * np.exp(phi / TE) - vi * (1.0 - phi / TI), -50.0, 0.0)


def _absorbed_fraction(q_sign, Q, R_c, B, T, cap=True):
    """E_E[min(1, (a/B)^2 max(0, 1 - q dphi / E))] for E ~ Gamma(2, kT) (eV)."""
    dphi = Q / (4.0 * np.pi * EPS0) * (1.0 / A - 1.0 / R_c)
    qd = q_sign * dphi  # eV

    def p(E):
        x = (A / B) ** 2 * max(0.0, 1.0 - qd / E)
        return min(1.0, x) if cap else x

    pts = [abs(qd)] + ([-qd / ((B / A) ** 2 - 1.0)] if qd < 0 and B > A else [])
    return quad(lambda E: E / T ** 2 * np.exp(-E / T) * p(E), 0.0, 80.0 * T, points=pts,
                limit=400)[0]


def test_textbook_oml_limits():
    """The integral without the cap is the textbook OML current in units of
    pi a^2 n <v> (as B^2 / a^2 times the fraction); the floating potential
    of 3 eV electrons and 0.03 eV argon ions is -7.23 V."""
    phi = _floating_potential()
    assert abs(phi - (-7.23)) < 0.01
    Q = 4.0 * np.pi * EPS0 * A * phi
    big = 1e6  # R_c -> infinity
    for q_sign, T, want in ((+1, TI, 1.0 - phi / TI), (-1, TE, np.exp(phi / TE))):
        got = _absorbed_fraction(q_sign, Q, big, A, T, cap=False)
        assert abs(got / want - 1.0) < 1e-6, (q_sign, got, want)


def _inject(rng, n, T, m, centre, R_c_cells, B_cells):
    """n particles on the sphere of R_c cells around `centre`, moving inward
    with flux-weighted Maxwellian speeds and impact parameters b <= B."""
    E = rng.gamma(2.0, T, n) * E_CH
    v = np.sqrt(2.0 * E / m)
    nh = rng.standard_normal((n, 3))
    nh /= np.linalg.norm(nh, axis=1)[:, None]
    s2 = rng.random(n) * (B_cells / R_c_cells) ** 2
    sin_t, cos_t = np.sqrt(s2), np.sqrt(1.0 - s2)
    t1 = np.cross(nh, [0.0, 0.0, 1.0])
    flat = np.linalg.norm(t1, axis=1) < 1e-6
    t1[flat] = np.cross(nh[flat], [1.0, 0.0, 0.0])
    t1 /= np.linalg.norm(t1, axis=1)[:, None]
    t2 = np.cross(nh, t1)
    psi = rng.random(n) * 2.0 * np.pi
    vel = v[:, None] * (-cos_t[:, None] * nh
                        + sin_t[:, None] * (np.cos(psi)[:, None] * t1 + np.sin(psi)[:, None] * t2))
    pos = np.asarray(centre) + nh * R_c_cells * (1.0 - 1e-9)
    return pos, vel


@pytest.mark.slow
def test_oml_currents_of_a_floating_grain():
    phi_f = _floating_potential()
    Q = 4.0 * np.pi * EPS0 * A * phi_f
    dx, c = 50e-6, 4
    R_c_cells = 3.2                      # 160 um = 40 a, inside the 9-cell MD cube
    R_c = R_c_cells * dx
    centre = [8.0, 8.0, 8.0]
    wl = W.tiny(nx=16, ny=16, nz=16, ppc=1, grains=[centre], cutoff=c, md_sub=1, grain_radius=A)
    flags = oracle.NO_MESH | oracle.NO_MCC | oracle.FROZEN_Q
    rng = np.random.default_rng(2024)
    currents = {}
    #           species, T, mass, charge sign, injected, B (cells), MD sub-step (s)
    for sp, T, m, q_sign, n, B_cells, h in ((1, TI, M_AR, +1, 20000, R_c_cells, 2e-11),
                                           (0, TE, M_E, -1, 100000, 1.5 * A / dx, 1.25e-13)):
        o = oracle.Oracle(dict(wl, dt=h), flags=flags, Q_frozen_e=Q / E_CH)
        pos, vel = _inject(rng, n, T, m, centre, R_c_cells, B_cells)
        hits, out, still = o.oml_collect(sp, R_c_cells, pos, vel, max_calls=2_000_000)
        assert still == 0 and hits + out == n
        p = _absorbed_fraction(q_sign, Q, R_c, B_cells * dx, T)
        f = hits / n
        sigma = np.sqrt(p * (1.0 - p) / n)
        print(f"  species {sp}: absorbed {hits}/{n} = {f:.5f}, OML {p:.5f}, z = {(f - p) / sigma:+.2f}")
        # 3 sigma, plus 0.5 % for the sub-step's end-point test near the surface
        assert abs(f - p) <= 3.0 * sigma + 0.005 * p
        # current per unit density: e <v> / 4 through the injection disc pi B^2 ... times P
        currents[sp] = E_CH * _mean_speed(T, m) * np.pi * (B_cells * dx) ** 2 * f
    # the grain floats: with R_c -> infinity the currents balance; at 40 a the
    # potential drop is (1 - a/R_c) of it, which the finite-R_c theory gives
    want = (_mean_speed(TE, M_E) * np.pi * (1.5 * A) ** 2 * _absorbed_fraction(-1, Q, R_c, 1.5 * A, TE)) / \
           (_mean_speed(TI, M_AR) * np.pi * R_c ** 2 * _absorbed_fraction(+1, Q, R_c, R_c, TI))
    ratio = currents[0] / currents[1]
    print(f"  I_e / I_i = {ratio:.4f} (finite-R_c OML {want:.4f})")
    assert abs(ratio / want - 1.0) < 0.08
