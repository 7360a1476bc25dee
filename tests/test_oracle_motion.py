"""Pins of the oracle's particle motion: the leapfrog of Eq. (1)-(2) with the
CIC field gather, the PPPM near-grain field of Eq. (5)-(6) with dt/40
sub-cycling, the electrodes and grains as perfect absorbers, and exact
particle / charge bookkeeping.
"""
import numpy as np
import pytest

import oracle
from paper_1801_00972_amd import workloads as W

E_CH, EPS0, ME = 1.602176634e-19, 8.8541878128e-12, 9.1093837015e-31
M_AR = 39.948 * 1.66053906660e-27


def _state(wl, flags, e_pos=(), e_vel=(), i_pos=(), i_vel=(), Q=0.0):
    o = oracle.Oracle(wl, flags=flags, Q_frozen_e=Q)
    for s, (p, v) in enumerate(((e_pos, e_vel), (i_pos, i_vel))):
        p = np.asarray(p, np.float64).reshape(-1, 3)
        v = np.asarray(v, np.float64).reshape(-1, 3)
        o.set_particles(s, p, v, np.arange(len(p)))
    return o


def _uniform_E(wl, Ez):
    n = wl["nx"] * wl["ny"] * (wl["nz"] + 1)
    E = np.zeros((3, n))
    E[2] = Ez
    return E


def test_constant_field_parabola():
    wl = W.tiny(nx=4, ny=4, nz=40)
    E0 = 100.0
    v0 = np.array([2e5, -1e5, 1e5])
    o = _state(wl, oracle.NO_MCC, e_pos=[[1.5, 2.5, 12.25]], e_vel=[v0])
    n = 100
    o.step_in_field(_uniform_E(wl, E0), n)
    a = -E_CH / ME * E0
    dt, dx = wl["dt"], wl["dx"]
    z = 12.25 + (n * v0[2] * dt + a * dt * dt * n * (n + 1) / 2) / dx
    x = (1.5 + n * v0[0] * dt / dx) % 4
    assert o.pos[0][0, 2] == pytest.approx(z, rel=1e-12)
    assert o.pos[0][0, 0] == pytest.approx(x, rel=1e-12)
    assert o.vel[0][0, 2] == pytest.approx(v0[2] + n * a * dt, rel=1e-12)


def test_harmonic_leapfrog_closed_form():
    # linear E_z about zc: CIC reproduces it exactly, so the leapfrog obeys
    # Y_{k+1} - 2 Y_k + Y_{k-1} = -(w dt)^2 Y_k, solved by A cos + B sin of
    # the discrete frequency sin(w~ dt/2) = w dt/2
    wl = W.tiny(nx=4, ny=4, nz=40)
    dt, dx = wl["dt"], wl["dx"]
    zc = 20.0
    wdt = 0.1
    kappa = (wdt / dt) ** 2 * ME * dx / (-E_CH)  # V/m per cell
    nn = 4 * 4 * 41
    k = np.repeat(np.arange(41), 16)
    E = np.zeros((3, nn))
    E[2] = -kappa * (k - zc)
    A = 2.0
    o = _state(wl, oracle.NO_MCC, e_pos=[[1.2, 2.7, zc + A]], e_vel=[[0, 0, 0]])
    wt = 2 * np.arcsin(wdt / 2)
    B = -A * wdt ** 2 / (2 * np.sin(wt))
    for step in range(1, 301):
        o.step_in_field(E, 1)
        Y = A * np.cos(wt * step) + B * np.sin(wt * step)
        assert o.pos[0][0, 2] - zc == pytest.approx(Y, abs=1e-11)


def test_electrodes_absorb_and_tally():
    wl = W.tiny(nx=4, ny=4, nz=10)
    dt, dx = wl["dt"], wl["dx"]
    v = 0.5 * dx / dt
    o = _state(wl, oracle.NO_MCC | oracle.NO_MESH,
               e_pos=[[1, 1, 0.4], [1, 1, 9.6], [1, 1, 5.0]],
               e_vel=[[0, 0, -v], [0, 0, v], [0, 0, v]],
               i_pos=[[2, 2, 9.5]], i_vel=[[0, 0, v]])
    o.step(1)
    assert o.alive[0].tolist() == [0, 0, 1]
    assert o.alive[1].tolist() == [0]  # z = 10.0 exactly is on the electrode: absorbed
    assert o.wall_count.tolist() == [[1, 0], [1, 1]]


def test_periodic_wrap_is_exact_translation():
    wl = W.tiny(nx=5, ny=4, nz=10)
    dt, dx = wl["dt"], wl["dx"]
    o = _state(wl, oracle.NO_MCC | oracle.NO_MESH,
               e_pos=[[4.75, 0.25, 5.0]], e_vel=[[0.5 * dx / dt, -0.5 * dx / dt, 0]])
    o.step(1)
    assert o.pos[0][0].tolist() == [0.25, 3.75, 5.0]


def test_md_substeps_constant_field_parabola():
    # M sub-steps of dt/M in a uniform field, zero grain charge
    wl = W.tiny(nx=8, ny=8, nz=12, grains=[[4.5, 4.5, 6.5]], cutoff=1, md_sub=40)
    v0 = np.array([1e5, 0, 2e5])
    o = _state(wl, oracle.NO_MCC | oracle.FROZEN_Q, e_pos=[[4.1, 4.2, 6.1]], e_vel=[v0], Q=0.0)
    E0 = 50.0
    o.step_in_field(_uniform_E(wl, E0), 1)
    M = 40
    h = wl["dt"] / M
    a = -E_CH / ME * E0
    z = 6.1 + (M * v0[2] * h + a * h * h * M * (M + 1) / 2) / wl["dx"]
    assert o.pos[0][0, 2] == pytest.approx(z, rel=1e-13)


def test_md_single_substep_equals_plain_step():
    rng = np.random.default_rng(7)
    wl0 = W.tiny(nx=8, ny=8, nz=12, md_sub=1, cutoff=1)
    wl1 = W.tiny(nx=8, ny=8, nz=12, grains=[[4.5, 4.5, 6.5]], cutoff=1, md_sub=1)
    pos = np.c_[3 + 3 * rng.random((200, 2)), 5 + 3 * rng.random(200)]
    vel = 3e5 * rng.standard_normal((200, 3))
    E = 1e3 * rng.standard_normal((3, 8 * 8 * 13))
    a = _state(wl0, oracle.NO_MCC, e_pos=pos, e_vel=vel)
    b = _state(wl1, oracle.NO_MCC | oracle.FROZEN_Q, e_pos=pos, e_vel=vel, Q=0.0)
    a.step_in_field(E, 1)
    b.step_in_field(E, 1)
    keep = b.alive[0] == 1  # particles that hit the grain only exist in b's outcome
    assert np.array_equal(a.pos[0][keep], b.pos[0][keep])
    assert np.array_equal(a.vel[0][keep], b.vel[0][keep])


def test_md_coulomb_kick_without_mesh():
    # an ion at rest 2 cells from a fixed grain of charge Q: during one step it
    # hardly moves, so v = (q/m) Q r / (4 pi eps0 r^3) dt
    Q = -1e4
    wl = W.tiny(nx=8, ny=8, nz=12, grains=[[4.5, 4.5, 6.5]], cutoff=2)
    o = _state(wl, oracle.NO_MCC | oracle.NO_MESH | oracle.FROZEN_Q,
               i_pos=[[4.5, 4.5, 4.5]], i_vel=[[0, 0, 0]], Q=Q)
    o.step(1)
    r = -2 * wl["dx"]
    Ez = Q * E_CH * r / (4 * np.pi * EPS0 * abs(r) ** 3)
    vz = E_CH / M_AR * Ez * wl["dt"]
    assert vz > 0  # attracted towards the negative grain above it
    assert o.vel[1][0, 2] == pytest.approx(vz, rel=1e-7)
    assert abs(o.vel[1][0, 0]) < 1e-12 * abs(vz) and abs(o.vel[1][0, 1]) < 1e-12 * abs(vz)


def test_pppm_removes_the_grains_own_mesh_field():
    # only the grain's own charge on the mesh, rf off: inside the MD cube the
    # corrected field E_PIC - Q U + Coulomb must be the bare Coulomb field
    Q = -1e4
    # n0 tiny: the test ion's own charge on the mesh (its image force) is negligible
    base = dict(V_dc=0.0, V_rf=0.0, n0=1.0)
    wl = W.tiny(nx=10, ny=10, nz=14, grains=[[5.3, 4.6, 7.2]], cutoff=2, **base)
    p = [[5.3, 4.6, 5.7]]
    with_mesh = _state(wl, oracle.NO_MCC | oracle.FROZEN_Q, i_pos=p, i_vel=[[0, 0, 0]], Q=Q)
    no_mesh = _state(wl, oracle.NO_MCC | oracle.FROZEN_Q | oracle.NO_MESH, i_pos=p,
                     i_vel=[[0, 0, 0]], Q=Q)
    with_mesh.step(1)
    no_mesh.step(1)
    v1, v0 = with_mesh.vel[1][0], no_mesh.vel[1][0]
    assert np.max(np.abs(v1 - v0)) < 1e-9 * np.max(np.abs(v0))
    # and outside every cube the grain acts through the mesh alone
    far = [[0.5, 0.5, 7.0]]
    a = _state(wl, oracle.NO_MCC | oracle.FROZEN_Q, i_pos=far, i_vel=[[0, 0, 0]], Q=Q)
    a.step(1)
    E = oracle.Oracle(wl, flags=oracle.FROZEN_Q, Q_frozen_e=Q)
    E.set_particles(0, np.zeros((0, 3)), np.zeros((0, 3)), [])
    E.set_particles(1, np.zeros((0, 3)), np.zeros((0, 3)), [])
    f = E.fields()
    # CIC gather at (0.5, 0.5, 7.0) is the mean of the 4 nodes around it in k = 7
    nodes = [(0, 0), (1, 0), (0, 1), (1, 1)]
    Eg = sum(f["E"][:, i + 10 * (j + 10 * 7)] for i, j in nodes) / 4
    assert np.allclose(a.vel[1][0], E_CH / M_AR * Eg * wl["dt"], rtol=1e-12, atol=0)


def test_unit_field_is_the_grains_mesh_field():
    # linearity: fields(counts) - fields(0) = Q(counts) * U_g on the cube nodes
    wl = W.tiny(nx=10, ny=8, nz=14, grains=[[2.3, 6.6, 7.2], [7.5, 2.5, 6.5]], cutoff=2)
    o = oracle.Oracle(wl)
    rng = np.random.default_rng(1)
    n = 300
    o.set_particles(0, rng.random((n, 3)) * [10, 8, 14], np.zeros((n, 3)), np.arange(n))
    o.set_particles(1, rng.random((n, 3)) * [10, 8, 14], np.zeros((n, 3)), np.arange(n))
    f0 = o.fields()
    o.set_counts(grain_count=[[9, 2], [0, 0]])
    f1 = o.fields()
    U = o.unit_fields()
    w = o.derived()["w"]
    Q = -7 * w * E_CH
    g = 0
    gi, gj, gk = 2, 6, 7
    c = 2
    side = 2 * c + 2
    for cz in range(side):
        for cy in range(side):
            for cx in range(side):
                i, j, k = (gi - c + cx) % 10, (gj - c + cy) % 8, gk - c + cz
                nidx = i + 10 * (j + 8 * k)
                d = f1["E"][:, nidx] - f0["E"][:, nidx]
                assert np.allclose(d, Q * U[g, :, cz, cy, cx], rtol=1e-9,
                                   atol=1e-9 * np.abs(Q * U[g]).max())


def test_md_region_is_the_periodic_cube():
    wl = W.tiny(nx=10, ny=8, nz=14, grains=[[0.5, 7.5, 7.2]], cutoff=2)
    o = oracle.Oracle(wl)
    cnt = 0
    for k in range(14):
        for j in range(8):
            for i in range(10):
                inside = o.md_grains(i, j, k) == [0]
                di = min((i - 0) % 10, (0 - i) % 10)
                dj = min((j - 7) % 8, (7 - j) % 8)
                assert inside == (di <= 2 and dj <= 2 and abs(k - 7) <= 2)
                cnt += inside
    assert cnt == 125


def test_grain_absorbs_and_counts():
    wl = W.tiny(nx=8, ny=8, nz=12, grains=[[4.5, 4.5, 6.5]], cutoff=1)
    dt, dx = wl["dt"], wl["dx"]
    o = _state(wl, oracle.NO_MCC | oracle.NO_MESH | oracle.FROZEN_Q,
               e_pos=[[4.5, 4.5, 5.9], [4.5, 4.5, 5.9]],
               e_vel=[[0, 0, 1.0 * dx / dt], [0, 0, -0.2 * dx / dt]], Q=0.0)
    o.step(1)
    assert o.alive[0].tolist() == [0, 1]
    assert o.grain_count.tolist() == [[1, 0]]


def test_charge_and_particle_conservation_full_run():
    wl = W.small_fp64()
    o = oracle.Oracle(wl)
    o.init_particles()
    n0 = [o.pos[s].shape[0] for s in range(2)]
    o.step(30)
    for s in range(2):
        tot = o.n_alive(s) + o.wall_count[:, s].sum() + o.grain_count[:, s].sum()
        assert tot == n0[s]
    rf = o.deposit_fixed()
    Qp = o.derived()["Qp"]
    # net charge on the mesh (plasma + grains) = -(charge lost to the walls)
    lost = (o.wall_count[:, 1].sum() - o.wall_count[:, 0].sum())
    assert rf.sum() == -lost * Qp


def test_oracle_is_deterministic():
    wl = W.small_fp64()
    a, b = oracle.Oracle(wl), oracle.Oracle(wl)
    a.init_particles()
    b.init_particles()
    a.step(5)
    b.step(5)
    for s in range(2):
        assert np.array_equal(a.pos[s], b.pos[s]) and np.array_equal(a.vel[s], b.vel[s])


def test_collisionless_push_conserves_leapfrog_energy():
    # Energy conservation of a collisionless push: a potential well
    # phi = c (z dx - z0)^2 on the nodes, differenced by the oracle's own E
    # stencil (exact on quadratics) and gathered by CIC (exact on linear
    # fields), gives each particle a linear restoring force k = 2 q c.  The
    # leapfrog of Eq. (1)-(2) then keeps 1/2 m v_{n-1/2}.v_{n+1/2} + q phi(x_n)
    # constant to rounding (the difference of consecutive values cancels
    # term by term), for electrons (c < 0) and, in the mirrored well, ions.
    wl = W.tiny(nx=6, ny=5, nz=40)
    dt, dx, nz = wl["dt"], wl["dx"], wl["nz"]
    z0 = 0.5 * nz * dx
    rng = np.random.default_rng(7)
    for s, q, m, w in ((0, -E_CH, ME, 2.0e9), (1, E_CH, M_AR, 4.0e7)):
        c = m * w * w / (2.0 * q)  # V/m^2, well for the species' charge sign
        o = oracle.Oracle(wl, flags=oracle.NO_MCC)
        k = np.repeat(np.arange(nz + 1), wl["nx"] * wl["ny"])
        phi = c * (k * dx - z0) ** 2
        E = o.efield(phi)
        n = 64
        pos = np.column_stack([rng.uniform(0, 6, n), rng.uniform(0, 5, n),
                               rng.uniform(0.35 * nz, 0.65 * nz, n)])
        vth = np.sqrt(E_CH * (3.0 if s == 0 else 0.03) / m)
        vel = rng.normal(size=(n, 3)) * vth * 0.3
        o.set_particles(s, pos, vel, np.arange(n))
        o.set_particles(1 - s, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0))
        v_prev = o.vel[s].copy()
        x_prev = o.pos[s].copy()
        inv = None
        for step in range(400):
            o.step_in_field(E, 1)
            assert o.n_alive(s) == n  # the well keeps every particle off the electrodes
            v_next = o.vel[s]
            energy = 0.5 * m * np.sum(v_prev * v_next, axis=1) + q * c * (x_prev[:, 2] * dx - z0) ** 2
            if inv is None:
                inv = energy
                scale = np.abs(0.5 * m * np.sum(vel * vel, axis=1)) + np.abs(q * c) * (0.15 * nz * dx) ** 2
            assert np.all(np.abs(energy - inv) <= 1e-10 * scale), (s, step)
            v_prev = v_next.copy()
            x_prev = o.pos[s].copy()
