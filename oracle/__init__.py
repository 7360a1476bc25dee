"""Plain FP64 CPU oracle of the PIC-MCC/PPPM step (arXiv:1801.00972, Sec. III).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  It shares no code with
the HIP library: the arithmetic lives in ``pic_oracle.c`` (plain C, FP64,
OpenMP over independent particles), this module only marshals arguments.

A workload is a plain dict (see ``paper_1801_00972_amd.workloads``); both this
oracle and the HIP library read the same dict, nothing else is shared.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

NO_MESH, NO_MCC, FIXED_POINT, FROZEN_Q, IMMOBILE_IONS, NO_MD = 1, 2, 4, 8, 16, 32


def build(verbose: bool = False, native: bool = False, out: str | None = None) -> str:
    """Compile pic_oracle.c into a shared library (gcc -O3, OpenMP, no
    fast-math, no FMA contraction).  The default is the portable liboracle.so
    the tests load; native=True adds -march=native for the machine it runs on
    (the CPU-baseline timing builds it there, into `out`)."""
    src = os.path.join(_HERE, "pic_oracle.c")
    target = out or _SO
    tmp = target + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-ffp-contract=off"] + (["-march=native"] if native else []) + ["-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


def use_library(path: str) -> None:
    """Load the oracle from another build of pic_oracle.c (the CPU-baseline
    timing uses a -march=native build); call before any oracle function."""
    global _SO, _lib
    if _lib is not None and _SO != path:
        raise RuntimeError("the oracle library is already loaded from " + _SO)
    _SO = path


class _Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ppc_e", C.c_int32), ("ppc_i", C.c_int32), ("n_grains", C.c_int32),
        ("cutoff", C.c_int32), ("md_sub", C.c_int32), ("flags", C.c_int32),
        ("coulomb_interval", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double), ("n0", C.c_double),
        ("Te_eV", C.c_double), ("Ti_eV", C.c_double),
        ("p_gas", C.c_double), ("T_gas", C.c_double),
        ("sigma_e", C.c_double), ("sigma_i", C.c_double),
        ("V_dc", C.c_double), ("V_rf", C.c_double), ("f_rf", C.c_double),
        ("grain_radius", C.c_double), ("E_cap_eV", C.c_double),
        ("Q_frozen_e", C.c_double), ("coulomb_lnL", C.c_double),
        ("xs_n", C.c_int32), ("pad1", C.c_int32),
        ("xs_E", C.POINTER(C.c_double)), ("xs_e_el", C.POINTER(C.c_double)),
        ("xs_e_ex", C.POINTER(C.c_double)), ("xs_i_cx", C.POINTER(C.c_double)),
        ("xs_i_el", C.POINTER(C.c_double)), ("E_ex_eV", C.c_double),
        ("seed", C.c_uint64),
        ("grain_pos", C.POINTER(C.c_double)),
        ("xs_e_iz", C.POINTER(C.c_double)), ("E_iz_eV", C.c_double),
    ]


class _Derived(C.Structure):
    _fields_ = [
        ("w", C.c_double), ("Qp", C.c_int64), ("n_gas", C.c_double),
        ("q", C.c_double * 2), ("m", C.c_double * 2), ("vth", C.c_double * 2),
        ("g_cap", C.c_double * 2), ("P_null", C.c_double * 2),
        ("T_null", C.c_uint64 * 2), ("vth_gas", C.c_double), ("sg_max", C.c_double * 2),
    ]


class _State(C.Structure):
    _fields_ = [
        ("n", C.c_int64 * 2),
        ("pos", C.POINTER(C.c_double) * 2),
        ("vel", C.POINTER(C.c_double) * 2),
        ("id", C.POINTER(C.c_uint32) * 2),
        ("alive", C.POINTER(C.c_uint8) * 2),
        ("margin", C.POINTER(C.c_double) * 2),
        ("grain_count", C.POINTER(C.c_int64)),
        ("wall_count", (C.c_int64 * 2) * 2),
        ("cap_violation", C.c_int64 * 2),
        ("n_collisions", C.c_int64 * 2),
        ("step", C.c_uint32),
        ("pad0", C.c_uint32),
        ("md_margin", C.c_int64 * 2),
        ("cap", C.c_int64 * 2),
        ("next_id", C.c_uint32 * 2),
        ("n_ionizations", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_philox4x32_10.restype = None
        L.orc_derive.argtypes = [C.POINTER(_Config), C.POINTER(_Derived)]
        L.orc_rf_voltage.argtypes = [C.POINTER(_Config), C.c_uint32]
        L.orc_rf_voltage.restype = C.c_double
        L.orc_init_particles.argtypes = [C.POINTER(_Config), C.POINTER(_State)]
        L.orc_deposit.argtypes = [C.POINTER(_Config), C.POINTER(_State), dp]
        L.orc_deposit_fixed.argtypes = [C.POINTER(_Config), C.POINTER(_State),
                                        C.POINTER(C.c_int64)]
        L.orc_moments.argtypes = [C.POINTER(_Config), C.POINTER(_State), dp, dp]
        L.orc_xs_sgmax.argtypes = [C.POINTER(_Config), C.c_int]
        L.orc_xs_sgmax.restype = C.c_double
        L.orc_xs_at.argtypes = [C.POINTER(_Config), dp, C.c_double]
        L.orc_xs_at.restype = C.c_double
        L.orc_unit_potentials.argtypes = [C.POINTER(_Config), dp]
        L.orc_fine_phi.argtypes = [C.POINTER(_Config), C.POINTER(_State), dp, dp, dp, C.c_double,
                                   C.POINTER(C.c_int32), dp]
        L.orc_coulomb.argtypes = [C.POINTER(_Config), C.POINTER(_State)]
        L.orc_coulomb.restype = C.c_int64
        L.orc_coulomb_pair.argtypes = [C.POINTER(_Config), C.c_int, C.c_int, dp, dp, C.c_double,
                                       C.c_double]
        L.orc_coulomb_pair.restype = None
        L.orc_coulomb_var.argtypes = [C.POINTER(_Config), C.c_int, C.c_int, C.c_double, C.c_double,
                                      C.c_double]
        L.orc_coulomb_var.restype = C.c_double
        L.orc_fine_moments.argtypes = [C.POINTER(_Config), C.POINTER(_State), dp, C.c_double,
                                       C.POINTER(C.c_int32), dp, dp]
        L.orc_poisson.argtypes = [C.POINTER(_Config), dp, C.c_double, dp]
        L.orc_efield.argtypes = [C.POINTER(_Config), dp, dp]
        L.orc_fields.argtypes = [C.POINTER(_Config), C.POINTER(_State), dp,
                                 C.POINTER(C.c_int64), dp, dp]
        L.orc_unit_fields.argtypes = [C.POINTER(_Config), dp]
        L.orc_md_grains.argtypes = [C.POINTER(_Config), C.c_int, C.c_int, C.c_int,
                                    C.POINTER(C.c_int), C.c_int]
        L.orc_oml_collect.argtypes = [C.POINTER(_Config), C.c_int, C.c_double, C.c_int64, dp, dp,
                                      C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_oml_collect.restype = C.c_int64
        L.orc_place_grains.argtypes = [C.c_uint64, C.c_int, dp, C.c_double, C.c_double, dp]
        L.orc_step.argtypes = [C.POINTER(_Config), C.POINTER(_State), dp]
        L.orc_step_in_field.argtypes = [C.POINTER(_Config), C.POINTER(_State), dp, dp]
        _lib = L
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


class Oracle:
    """One replica of the method, held in numpy arrays, stepped by pic_oracle.c."""

    def __init__(self, wl: dict, flags: int = 0, Q_frozen_e: float = 0.0):
        self.wl = dict(wl)
        self.flags = flags
        if wl.get("grain_pos") is None and wl.get("cluster"):
            cl = wl["cluster"]  # seeded placement (the oracle's own implementation)
            self.grain_pos = place_grains(int(wl.get("seed", 0)), int(cl["n"]), cl["center"],
                                          float(cl["radius"]), float(cl.get("min_sep", 0.0)))
        else:
            g = wl.get("grain_pos")
            self.grain_pos = np.ascontiguousarray(
                np.asarray(np.zeros((0, 3)) if g is None else g, dtype=np.float64).reshape(-1, 3))
        cfg = _Config()
        cfg.nx, cfg.ny, cfg.nz = int(wl["nx"]), int(wl["ny"]), int(wl["nz"])
        cfg.ppc_e = cfg.ppc_i = int(wl["ppc"])
        cfg.n_grains = self.grain_pos.shape[0]
        cfg.cutoff = int(wl.get("cutoff", 3))
        cfg.md_sub = int(wl.get("md_sub", 40))
        cfg.flags = flags
        for k in ("dx", "dt", "n0", "Te_eV", "Ti_eV", "p_gas", "T_gas", "sigma_e",
                  "sigma_i", "V_dc", "V_rf", "f_rf", "grain_radius", "E_cap_eV"):
            setattr(cfg, k, float(wl[k]))
        cfg.Q_frozen_e = float(Q_frozen_e)
        cfg.coulomb_interval = int(wl.get("coulomb_interval", 0))
        cfg.coulomb_lnL = float(wl.get("coulomb_lnL", 10.0))
        xs = wl.get("xs")
        self._xs = {}
        if xs:
            for k in ("E", "e_el", "e_ex", "i_cx", "i_el", "e_iz"):
                if xs.get(k) is not None:
                    self._xs[k] = np.ascontiguousarray(xs[k], np.float64)
            cfg.xs_n = len(self._xs["E"])
            cfg.xs_E = _ptr(self._xs["E"], C.c_double)
            cfg.xs_e_el = _ptr(self._xs["e_el"], C.c_double)
            cfg.xs_e_ex = _ptr(self._xs.get("e_ex"), C.c_double)
            cfg.xs_i_cx = _ptr(self._xs["i_cx"], C.c_double)
            cfg.xs_i_el = _ptr(self._xs.get("i_el"), C.c_double)
            cfg.E_ex_eV = float(xs.get("E_ex", 0.0))
            cfg.xs_e_iz = _ptr(self._xs.get("e_iz"), C.c_double)
            cfg.E_iz_eV = float(xs.get("E_iz", 0.0))
        cfg.seed = int(wl.get("seed", 0))
        cfg.grain_pos = _ptr(self.grain_pos, C.c_double)
        self.cfg = cfg
        self.nx, self.ny, self.nz = cfg.nx, cfg.ny, cfg.nz
        self.n_nodes = self.nx * self.ny * (self.nz + 1)
        self.n_grains = cfg.n_grains
        self._U = None
        self.grain_count = np.zeros((self.n_grains, 2), dtype=np.int64)
        self.st = _State()
        self.st.grain_count = _ptr(self.grain_count, C.c_int64)
        self.pos = [np.zeros((0, 3)), np.zeros((0, 3))]
        self.vel = [np.zeros((0, 3)), np.zeros((0, 3))]
        self.id = [np.zeros(0, np.uint32), np.zeros(0, np.uint32)]
        self.alive = [np.zeros(0, np.uint8), np.zeros(0, np.uint8)]
        self.margin = [np.zeros(0), np.zeros(0)]
        self._bind()

    # ---- state plumbing ------------------------------------------------
    def _bind(self):
        for s in range(2):
            self.st.n[s] = self.st.cap[s] = self.pos[s].shape[0]
            self.st.pos[s] = _ptr(self.pos[s], C.c_double)
            self.st.vel[s] = _ptr(self.vel[s], C.c_double)
            self.st.id[s] = _ptr(self.id[s], C.c_uint32)
            self.st.alive[s] = _ptr(self.alive[s], C.c_uint8)
            self.st.margin[s] = _ptr(self.margin[s], C.c_double)

    def set_particles(self, species: int, pos, vel, ids):
        """Load one species (positions in cell units: x and y are periodic, z
        must lie between the electrodes, 0 <= z < nz).  The arrays are copied:
        stepping the oracle never changes the caller's."""
        n = len(ids)
        pos = np.array(pos, np.float64, order="C", copy=True).reshape(n, 3)
        if n and not (np.isfinite(pos).all() and (pos[:, 2] >= 0).all() and (pos[:, 2] < self.nz).all()):
            raise ValueError("set_particles: a position is not finite or has z outside [0, nz)")
        self.pos[species] = pos
        self.vel[species] = np.array(vel, np.float64, order="C", copy=True).reshape(n, 3)
        self.id[species] = np.array(ids, np.uint32, order="C", copy=True)
        self.alive[species] = np.ones(n, np.uint8)
        self.margin[species] = np.full(n, np.inf)
        self.st.next_id[species] = int(self.id[species].max()) + 1 if n else 0
        self._bind()

    def set_counts(self, grain_count=None, wall_count=None, step=None):
        if grain_count is not None:
            self.grain_count[...] = np.asarray(grain_count, np.int64).reshape(self.n_grains, 2)
        if wall_count is not None:
            wc = np.asarray(wall_count, np.int64).reshape(2, 2)
            for a in range(2):
                for b in range(2):
                    self.st.wall_count[a][b] = int(wc[a, b])
        if step is not None:
            self.st.step = int(step)

    @property
    def step_index(self) -> int:
        return int(self.st.step)

    @property
    def wall_count(self) -> np.ndarray:
        return np.array([[self.st.wall_count[a][b] for b in range(2)] for a in range(2)])

    @property
    def cap_violation(self):
        return [int(self.st.cap_violation[s]) for s in range(2)]

    @property
    def n_collisions(self):
        return [int(self.st.n_collisions[s]) for s in range(2)]

    @property
    def n_ionizations(self) -> int:
        return int(self.st.n_ionizations)

    @property
    def next_id(self):
        return [int(self.st.next_id[s]) for s in range(2)]

    def _grow(self):
        """Room for the particles that this step's ionisations may create (at
        most one electron and one ion per electron)."""
        if self._xs.get("e_iz") is None or self.flags & NO_MCC:
            return False
        extra = self.pos[0].shape[0]
        used = [self.pos[s].shape[0] for s in range(2)]
        for s in range(2):
            self.pos[s] = np.concatenate([self.pos[s], np.zeros((extra, 3))])
            self.vel[s] = np.concatenate([self.vel[s], np.zeros((extra, 3))])
            self.id[s] = np.concatenate([self.id[s], np.zeros(extra, np.uint32)])
            self.alive[s] = np.concatenate([self.alive[s], np.zeros(extra, np.uint8)])
            self.margin[s] = np.concatenate([self.margin[s], np.full(extra, np.inf)])
        self._bind()
        for s in range(2):
            self.st.n[s] = used[s]
        return True

    def _trim(self):
        for s in range(2):
            n = int(self.st.n[s])
            for name in ("pos", "vel", "id", "alive", "margin"):
                arr = getattr(self, name)
                arr[s] = np.ascontiguousarray(arr[s][:n])
        self._bind()

    @property
    def md_margin(self):
        """Plain pushes per species with |v_{k+1/2}| dt >= cutoff dx (grains present)."""
        return [int(self.st.md_margin[s]) for s in range(2)]

    def compact(self):
        """Drop removed particles, keeping the order of the survivors."""
        for s in range(2):
            keep = self.alive[s] != 0
            self.pos[s] = np.ascontiguousarray(self.pos[s][keep])
            self.vel[s] = np.ascontiguousarray(self.vel[s][keep])
            self.id[s] = np.ascontiguousarray(self.id[s][keep])
            self.margin[s] = np.ascontiguousarray(self.margin[s][keep])
            self.alive[s] = np.ascontiguousarray(self.alive[s][keep])
        self._bind()

    def n_alive(self, s: int) -> int:
        return int(np.count_nonzero(self.alive[s]))

    # ---- method --------------------------------------------------------
    def derived(self) -> dict:
        d = _Derived()
        rc = lib().orc_derive(C.byref(self.cfg), C.byref(d))
        if rc:
            raise ValueError(f"orc_derive failed ({rc})")
        return {"w": d.w, "Qp": d.Qp, "n_gas": d.n_gas, "q": list(d.q), "m": list(d.m),
                "vth": list(d.vth), "g_cap": list(d.g_cap), "P_null": list(d.P_null),
                "T_null": list(d.T_null), "vth_gas": d.vth_gas, "sg_max": list(d.sg_max)}

    def rf_voltage(self, k: int) -> float:
        return lib().orc_rf_voltage(C.byref(self.cfg), k)

    def init_particles(self):
        ncell = self.nx * self.ny * self.nz
        n = ncell * int(self.wl["ppc"])
        for s in range(2):
            self.pos[s] = np.zeros((n, 3))
            self.vel[s] = np.zeros((n, 3))
            self.id[s] = np.zeros(n, np.uint32)
            self.alive[s] = np.zeros(n, np.uint8)
            self.margin[s] = np.full(n, np.inf)
        self._bind()
        rc = lib().orc_init_particles(C.byref(self.cfg), C.byref(self.st))
        if rc:
            raise RuntimeError(f"orc_init_particles failed ({rc})")

    def deposit(self) -> np.ndarray:
        rho = np.zeros(self.n_nodes)
        rc = lib().orc_deposit(C.byref(self.cfg), C.byref(self.st), _ptr(rho, C.c_double))
        if rc:
            raise RuntimeError(f"orc_deposit failed ({rc})")
        return rho

    def deposit_fixed(self) -> np.ndarray:
        rho = np.zeros(self.n_nodes, np.int64)
        rc = lib().orc_deposit_fixed(C.byref(self.cfg), C.byref(self.st), _ptr(rho, C.c_int64))
        if rc:
            raise RuntimeError(f"orc_deposit_fixed failed ({rc})")
        return rho

    def moments(self):
        """Densities n [2][nodes] (m^-3) and fluxes [2][3][nodes] (m^-2 s^-1)
        of electrons and ions at the current state."""
        n = np.zeros(2 * self.n_nodes)
        flux = np.zeros(6 * self.n_nodes)
        rc = lib().orc_moments(C.byref(self.cfg), C.byref(self.st), _ptr(n, C.c_double),
                               _ptr(flux, C.c_double))
        if rc:
            raise RuntimeError(f"orc_moments failed ({rc})")
        return n.reshape(2, self.n_nodes), flux.reshape(2, 3, self.n_nodes)

    def fine_moments(self, origin, h: float, cells):
        """Densities [2][fine nodes] and fluxes [2][3][fine nodes] on the fine
        grid of a sub-box (Sec. IV, the grid over the grains' region): lower
        corner `origin` (grid units), cell edge `h` (grid units), `cells`
        cells per axis, (cells + 1) nodes per axis, x fastest."""
        o = np.ascontiguousarray(origin, np.float64)
        m = np.ascontiguousarray(cells, np.int32)
        fn = int(np.prod(m.astype(np.int64) + 1))
        n = np.zeros(2 * fn)
        flux = np.zeros(6 * fn)
        rc = lib().orc_fine_moments(C.byref(self.cfg), C.byref(self.st), _ptr(o, C.c_double),
                                    float(h), _ptr(m, C.c_int32), _ptr(n, C.c_double),
                                    _ptr(flux, C.c_double))
        if rc:
            raise RuntimeError(f"orc_fine_moments failed ({rc})")
        return n.reshape(2, fn), flux.reshape(2, 3, fn)

    def poisson(self, rho, V: float) -> np.ndarray:
        rho = np.ascontiguousarray(rho, np.float64)
        phi = np.zeros(self.n_nodes)
        rc = lib().orc_poisson(C.byref(self.cfg), _ptr(rho, C.c_double), float(V),
                               _ptr(phi, C.c_double))
        if rc:
            raise RuntimeError(f"orc_poisson failed ({rc})")
        return phi

    def efield(self, phi) -> np.ndarray:
        phi = np.ascontiguousarray(phi, np.float64)
        E = np.zeros(3 * self.n_nodes)
        lib().orc_efield(C.byref(self.cfg), _ptr(phi, C.c_double), _ptr(E, C.c_double))
        return E.reshape(3, self.n_nodes)

    def fields(self, fixed_point: bool = False):
        """rho (C/m^3), phi (V), E (V/m, [3][nodes]) at the current step; plus
        the int64 fixed-point rho when fixed_point is set."""
        rho = np.zeros(self.n_nodes)
        phi = np.zeros(self.n_nodes)
        E = np.zeros(3 * self.n_nodes)
        rf = np.zeros(self.n_nodes, np.int64) if fixed_point else None
        rc = lib().orc_fields(C.byref(self.cfg), C.byref(self.st), _ptr(rho, C.c_double),
                              _ptr(rf, C.c_int64), _ptr(phi, C.c_double), _ptr(E, C.c_double))
        if rc:
            raise RuntimeError(f"orc_fields failed ({rc})")
        out = {"rho": rho, "phi": phi, "E": E.reshape(3, self.n_nodes)}
        if fixed_point:
            out["rho_fixed"] = rf
        return out

    def unit_fields(self, progress=None) -> np.ndarray:
        """The grains' unit-charge fields on their cubes.  With a progress
        callback they are computed one grain at a time (each grain's field
        depends on its own position only) and progress(g) is called after
        grain g."""
        side = 2 * self.cfg.cutoff + 2
        U = np.zeros((self.n_grains, 3, side, side, side))
        if self.n_grains and progress is None:
            rc = lib().orc_unit_fields(C.byref(self.cfg), _ptr(U, C.c_double))
            if rc:
                raise RuntimeError(f"orc_unit_fields failed ({rc})")
        for g in range(self.n_grains if progress is not None else 0):
            one = Oracle(dict(self.wl, grain_pos=self.grain_pos[g:g + 1]), flags=self.flags)
            Ug = np.zeros((1, 3, side, side, side))
            rc = lib().orc_unit_fields(C.byref(one.cfg), _ptr(Ug, C.c_double))
            if rc:
                raise RuntimeError(f"orc_unit_fields failed ({rc})")
            U[g] = Ug[0]
            progress(g)
        return U

    def md_grains(self, i: int, j: int, k: int):
        out = (C.c_int * 64)()
        n = lib().orc_md_grains(C.byref(self.cfg), i, j, k, out, 64)
        return [out[t] for t in range(min(n, 64))]

    def _units(self, progress=None):
        if self.n_grains == 0 or (self.flags & NO_MESH):
            return None
        if self._U is None:
            self._U = np.ascontiguousarray(self.unit_fields(progress))
        return self._U

    def unit_potentials(self):
        """phi of a unit (1 C) charge of each grain on its MD cube's nodes."""
        side = 2 * int(self.cfg.cutoff) + 2
        U = np.zeros(max(self.n_grains, 1) * side ** 3)
        rc = lib().orc_unit_potentials(C.byref(self.cfg), _ptr(U, C.c_double))
        if rc:
            raise RuntimeError(f"orc_unit_potentials failed ({rc})")
        return U

    def fine_phi(self, phi, origin, h: float, cells, Uphi=None):
        """The potential on the fine grid (see fine_moments) from the mesh
        potential phi: interpolated, with the grains' Coulomb potential in
        place of their unit mesh potential inside their MD cubes."""
        phi = np.ascontiguousarray(phi, np.float64).reshape(-1)
        U = self.unit_potentials() if Uphi is None else np.ascontiguousarray(Uphi, np.float64)
        o = np.ascontiguousarray(origin, np.float64)
        m = np.ascontiguousarray(cells, np.int32)
        out = np.zeros(int(np.prod(m.astype(np.int64) + 1)))
        rc = lib().orc_fine_phi(C.byref(self.cfg), C.byref(self.st), _ptr(phi, C.c_double),
                                _ptr(U, C.c_double), _ptr(o, C.c_double), float(h),
                                _ptr(m, C.c_int32), _ptr(out, C.c_double))
        if rc:
            raise RuntimeError(f"orc_fine_phi failed ({rc})")
        return out

    def xs_sgmax(self, sp: int) -> float:
        """max over g <= g_cap of g sigma_total(E(g)) of the tables."""
        return float(lib().orc_xs_sgmax(C.byref(self.cfg), sp))

    def xs_at(self, table: str, E_eV: float) -> float:
        return float(lib().orc_xs_at(C.byref(self.cfg), _ptr(self._xs[table], C.c_double), E_eV))

    def coulomb(self) -> int:
        """One pass of the Coulomb collisions (Table I, binary model of
        Takizuka and Abe) at the current step; returns the collision count."""
        rc = lib().orc_coulomb(C.byref(self.cfg), C.byref(self.st))
        if rc < 0:
            raise RuntimeError(f"orc_coulomb failed ({rc})")
        return int(rc)

    def coulomb_pair(self, sa: int, sb: int, va, vb, delta: float, phi: float):
        """One binary collision with given delta = tan(theta/2) and azimuth."""
        a = np.array(va, np.float64)
        b = np.array(vb, np.float64)
        lib().orc_coulomb_pair(C.byref(self.cfg), sa, sb, _ptr(a, C.c_double), _ptr(b, C.c_double),
                               float(delta), float(phi))
        return a, b

    def coulomb_var(self, sa: int, sb: int, u: float, nL: float, dtc: float) -> float:
        return float(lib().orc_coulomb_var(C.byref(self.cfg), sa, sb, float(u), float(nL),
                                           float(dtc)))

    def oml_collect(self, species: int, R_c: float, pos, vel, max_calls: int):
        """OML test mode (grain charging, Sec. IV.B): test particles moved in
        the field of grain 0 alone (charge Q_frozen_e e, no mesh, no
        collisions) until the grain absorbs them or they leave the sphere of
        R_c cells around it.  Returns (absorbed, left, still inside)."""
        pos = np.ascontiguousarray(pos, np.float64).copy()
        vel = np.ascontiguousarray(vel, np.float64).copy()
        n_out, n_open = C.c_int64(0), C.c_int64(0)
        hits = lib().orc_oml_collect(C.byref(self.cfg), int(species), float(R_c), len(pos),
                                     _ptr(pos, C.c_double), _ptr(vel, C.c_double), int(max_calls),
                                     C.byref(n_out), C.byref(n_open))
        if hits < 0:
            raise RuntimeError(f"orc_oml_collect failed ({hits})")
        return int(hits), int(n_out.value), int(n_open.value)

    def step(self, n: int = 1):
        U = self._units()
        for _ in range(n):
            grown = self._grow()
            rc = lib().orc_step(C.byref(self.cfg), C.byref(self.st), _ptr(U, C.c_double))
            if grown:
                self._trim()
            if rc:
                raise RuntimeError(f"orc_step failed ({rc})")

    def step_in_field(self, E, n: int = 1):
        E = None if E is None else np.ascontiguousarray(E, np.float64).reshape(-1)
        U = self._units()
        for _ in range(n):
            grown = self._grow()
            rc = lib().orc_step_in_field(C.byref(self.cfg), C.byref(self.st),
                                         _ptr(E, C.c_double), _ptr(U, C.c_double))
            if grown:
                self._trim()
            if rc:
                raise RuntimeError(f"orc_step_in_field failed ({rc})")


def place_grains(seed: int, n: int, center, radius: float, min_sep: float) -> np.ndarray:
    """Seeded grain placement: n grains uniform in a sphere (cell units) with
    a minimum separation, by rejection on Philox draws (see pic_oracle.h)."""
    c = np.ascontiguousarray(center, np.float64)
    out = np.zeros((n, 3))
    rc = lib().orc_place_grains(int(seed), int(n), _ptr(c, C.c_double), float(radius),
                                float(min_sep), _ptr(out, C.c_double))
    if rc:
        raise ValueError("grain placement failed: no room at the minimum separation")
    return out


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]
