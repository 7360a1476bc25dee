"""ctypes binding of include/pic.h (argument marshalling only).

Every function named pic_* here calls the C function of the same name in the
in-tree HIP library libpic.so; all arithmetic runs in its kernels.  There is no
fallback: if the library is missing this module raises on first use.
PyTorch supplies the HIP stream and, optionally, device output tensors.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ECONFIG, PIC_ENOMEM, PIC_EDEVICE, PIC_ENUMERIC, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6
PIC_FP64, PIC_FP32R = 0, 1
PIC_PHI, PIC_E, PIC_RHO, PIC_RHO_FIXED, PIC_N, PIC_FLUX = 1, 2, 4, 8, 16, 32
PIC_FINE_N, PIC_FINE_FLUX, PIC_FINE_PHI = 64, 128, 256
PIC_MAX_FINE_NODES = 1 << 26

SYMBOLS = ("pic_init", "pic_step", "pic_grain_charges", "pic_fields", "pic_destroy",
           "pic_last_error", "pic_get_state", "pic_set_state", "pic_get_counters", "pic_derived",
           "pic_profile_enable", "pic_profile_read", "pic_get_tuning", "pic_set_tuning",
           "pic_autotune", "pic_average", "pic_average_read", "pic_set_fine_grid",
           "pic_fields_static", "pic_save", "pic_load", "pic_grain_positions",
           "pic_energy")
PIC_MAX_PHASE_BINS = 64
PIC_PROF_PUSH, PIC_PROF_FIELD, PIC_PROF_SORT, PIC_PROF_LISTS, PIC_PROF_COULOMB = 0, 1, 2, 3, 4


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class pic_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ppc", C.c_int32), ("n_grains", C.c_int32), ("pp_cutoff_cells", C.c_int32),
        ("md_subcycles", C.c_int32), ("precision", C.c_int32), ("max_refine", C.c_int32),
        ("sort_interval", C.c_int32),
        ("dx", C.c_double), ("dt", C.c_double), ("n0", C.c_double),
        ("Te_eV", C.c_double), ("Ti_eV", C.c_double),
        ("p_gas_Pa", C.c_double), ("T_gas_K", C.c_double),
        ("sigma_e_el", C.c_double), ("sigma_i_cx", C.c_double),
        ("V_dc", C.c_double), ("V_rf", C.c_double), ("f_rf", C.c_double),
        ("grain_radius", C.c_double), ("E_cap_eV", C.c_double), ("refine_tol", C.c_double),
        ("seed", C.c_uint64),
        ("grain_pos", C.POINTER(C.c_double)),
        ("coulomb_interval", C.c_int32), ("reserved0", C.c_int32), ("coulomb_lnL", C.c_double),
        ("xs_n", C.c_int32), ("reserved1", C.c_int32),
        ("xs_E", C.POINTER(C.c_double)), ("xs_e_el", C.POINTER(C.c_double)),
        ("xs_e_ex", C.POINTER(C.c_double)), ("xs_i_cx", C.POINTER(C.c_double)),
        ("xs_i_el", C.POINTER(C.c_double)), ("E_ex_eV", C.c_double),
        ("cluster_center", C.c_double * 3), ("cluster_radius", C.c_double),
        ("grain_min_sep", C.c_double),
        ("xs_e_iz", C.POINTER(C.c_double)), ("E_iz_eV", C.c_double), ("max_particles", C.c_int64),
    ]


class pic_state_view(C.Structure):
    _fields_ = [
        ("capacity", C.c_int64 * 2), ("n", C.c_int64 * 2),
        ("pos", C.POINTER(C.c_double) * 2), ("vel", C.POINTER(C.c_double) * 2),
        ("id", C.POINTER(C.c_uint32) * 2),
        ("grain_count", C.POINTER(C.c_int64)),
        ("wall_count", (C.c_int64 * 2) * 2),
        ("step", C.c_uint32), ("pad0", C.c_uint32),
    ]


class pic_counters(C.Structure):
    _fields_ = [
        ("n_alive", C.c_int64 * 2), ("wall_count", (C.c_int64 * 2) * 2),
        ("cap_violation", C.c_int64 * 2), ("n_collisions", C.c_int64 * 2),
        ("md_particles", C.c_int64 * 2),
        ("step", C.c_uint32), ("refine_sweeps", C.c_int32), ("refine_residual", C.c_double),
        ("numeric_bad", C.c_int64), ("tile_fallback", C.c_int64), ("n_coulomb", C.c_int64),
        ("refine_unconverged", C.c_int64), ("md_margin", C.c_int64 * 2),
        ("n_ionizations", C.c_int64), ("iz_dropped", C.c_int64),
    ]


class pic_fine_grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("h", C.c_double), ("cells", C.c_int32 * 3),
                ("reserved", C.c_int32)]


class pic_tuning(C.Structure):
    _fields_ = [("sort_interval", C.c_int32), ("ion_sort_interval", C.c_int32),
                ("tile_margin", C.c_int32), ("ion_tile_margin", C.c_int32),
                ("batch_push", C.c_int32), ("batch_blocks", C.c_int32), ("use_graphs", C.c_int32)]


TUNING_KEYS = tuple(f[0] for f in pic_tuning._fields_)

_lib = None


def lib():
    """Load libpic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pic_init.argtypes = [C.POINTER(pic_config), C.c_int, P, C.POINTER(P)]
        L.pic_step.argtypes = [P, C.c_int]
        L.pic_grain_charges.argtypes = [P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.pic_fields.argtypes = [P, C.c_int, C.c_uint, C.POINTER(P), C.c_int]
        L.pic_fields_static.argtypes = [P, C.c_int, C.c_uint, C.POINTER(P), C.c_int]
        L.pic_grain_positions.argtypes = [P, C.c_int, C.POINTER(C.c_double)]
        L.pic_energy.argtypes = [P, C.c_int, C.POINTER(C.c_double)]
        L.pic_save.argtypes = [P, C.c_char_p]
        L.pic_load.argtypes = [P, C.c_char_p]
        L.pic_destroy.argtypes = [P]
        L.pic_destroy.restype = None
        L.pic_last_error.argtypes = [P]
        L.pic_last_error.restype = C.c_char_p
        L.pic_get_state.argtypes = [P, C.c_int, C.POINTER(pic_state_view)]
        L.pic_set_state.argtypes = [P, C.c_int, C.POINTER(pic_state_view)]
        L.pic_get_counters.argtypes = [P, C.c_int, C.POINTER(pic_counters)]
        L.pic_derived.argtypes = [P, C.c_int, C.POINTER(C.c_double)]
        L.pic_profile_enable.argtypes = [P, C.c_int]
        L.pic_profile_read.argtypes = [P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.pic_get_tuning.argtypes = [P, C.POINTER(pic_tuning)]
        L.pic_set_tuning.argtypes = [P, C.POINTER(pic_tuning)]
        L.pic_autotune.argtypes = [P, C.c_int, C.POINTER(pic_tuning), C.POINTER(C.c_double), C.c_int,
                                   C.POINTER(C.c_int)]
        L.pic_average.argtypes = [P, C.c_int, C.c_int]
        L.pic_average_read.argtypes = [P, C.c_int, C.c_int, C.c_uint, C.POINTER(P), C.c_int,
                                       C.POINTER(C.c_int64)]
        L.pic_set_fine_grid.argtypes = [P, C.c_int, C.POINTER(pic_fine_grid)]
        for name in ("pic_init", "pic_step", "pic_grain_charges", "pic_fields", "pic_get_state",
                     "pic_set_state", "pic_get_counters", "pic_derived", "pic_profile_enable",
                     "pic_profile_read", "pic_get_tuning", "pic_set_tuning", "pic_autotune",
                     "pic_average", "pic_average_read", "pic_set_fine_grid", "pic_fields_static",
                     "pic_save", "pic_load", "pic_grain_positions",
           "pic_energy"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != PIC_OK:
        msg = lib().pic_last_error(ctx)
        raise PicError(rc, msg.decode() if msg else "error")


def make_config(wl: dict, sort_interval: int = 8, max_refine: int = 2):
    """pic_config from a workload dict; returns (config, keep-alive arrays)."""
    cluster = wl.get("cluster") if wl.get("grain_pos") is None else None
    g = np.ascontiguousarray(np.asarray(np.zeros((0, 3)) if wl.get("grain_pos") is None
                                        else wl["grain_pos"], np.float64).reshape(-1, 3))
    c = pic_config()
    c.nx, c.ny, c.nz = int(wl["nx"]), int(wl["ny"]), int(wl["nz"])
    c.ppc = int(wl["ppc"])
    c.n_grains = int(cluster["n"]) if cluster else g.shape[0]
    if cluster:
        # the library places the grains (seeded; pic_grain_positions reads them)
        for a in range(3):
            c.cluster_center[a] = float(cluster["center"][a])
        c.cluster_radius = float(cluster["radius"])
        c.grain_min_sep = float(cluster.get("min_sep", 0.0))
    c.pp_cutoff_cells = int(wl.get("cutoff", 3))
    c.md_subcycles = int(wl.get("md_sub", 40))
    prec = wl.get("precision", "fp64")
    c.precision = PIC_FP32R if prec == "fp32r" else PIC_FP64
    c.max_refine = int(wl.get("max_refine", max_refine))
    c.sort_interval = int(wl.get("sort_interval", sort_interval))
    c.dx, c.dt, c.n0 = float(wl["dx"]), float(wl["dt"]), float(wl["n0"])
    c.Te_eV, c.Ti_eV = float(wl["Te_eV"]), float(wl["Ti_eV"])
    c.p_gas_Pa, c.T_gas_K = float(wl["p_gas"]), float(wl["T_gas"])
    c.sigma_e_el, c.sigma_i_cx = float(wl["sigma_e"]), float(wl["sigma_i"])
    c.V_dc, c.V_rf, c.f_rf = float(wl["V_dc"]), float(wl["V_rf"]), float(wl["f_rf"])
    c.grain_radius = float(wl["grain_radius"])
    c.E_cap_eV = float(wl["E_cap_eV"])
    c.refine_tol = float(wl.get("refine_tol", 1e-10))
    c.seed = int(wl.get("seed", 0))
    c.grain_pos = g.ctypes.data_as(C.POINTER(C.c_double)) if not cluster else None
    c.coulomb_interval = int(wl.get("coulomb_interval", 0))
    c.coulomb_lnL = float(wl.get("coulomb_lnL", 10.0))
    keep = [g]
    xs = wl.get("xs")
    if xs:
        # cross-section tables: a dict of E (eV) and e_el, e_ex, i_cx, i_el (m^2), E_ex (eV)
        arrays = {k: np.ascontiguousarray(xs[k], np.float64)
                  for k in ("E", "e_el", "e_ex", "i_cx", "i_el", "e_iz") if xs.get(k) is not None}
        keep.append(arrays)
        c.xs_n = len(arrays["E"])
        for k, field in (("E", "xs_E"), ("e_el", "xs_e_el"), ("e_ex", "xs_e_ex"), ("i_cx", "xs_i_cx"),
                         ("i_el", "xs_i_el"), ("e_iz", "xs_e_iz")):
            if k in arrays:
                setattr(c, field, arrays[k].ctypes.data_as(C.POINTER(C.c_double)))
        c.E_ex_eV = float(xs.get("E_ex", 0.0))
        c.E_iz_eV = float(xs.get("E_iz", 0.0))
    c.max_particles = int(wl.get("max_particles", 0))
    return c, keep


def current_stream():
    """The torch current HIP stream handle (None without a GPU)."""
    import torch
    if torch.cuda.is_available():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return None


# ---------------------------------------------------------------- C names
def pic_init(cfgs, n_replicas, hip_stream=None):
    arr = (pic_config * n_replicas)(*cfgs)
    out = C.c_void_p()
    rc = lib().pic_init(arr, n_replicas, hip_stream, C.byref(out))
    _check(rc, None)
    return out


def pic_step(ctx, n_steps):
    _check(lib().pic_step(ctx, int(n_steps)), ctx)


def pic_grain_charges(ctx, replica, n_grains):
    counts = np.zeros((n_grains, 2), np.int64)
    Q = np.zeros(n_grains)
    _check(lib().pic_grain_charges(ctx, replica, counts.ctypes.data_as(C.POINTER(C.c_int64)),
                                   Q.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return counts, Q


def pic_fields(ctx, replica, what, outs, out_on_device=False):
    """outs: list of buffers (numpy arrays or torch tensors) in PHI, E, RHO, RHO_FIXED order."""
    ptrs = (C.c_void_p * len(outs))()
    for i, o in enumerate(outs):
        ptrs[i] = o.data_ptr() if hasattr(o, "data_ptr") else o.ctypes.data
    _check(lib().pic_fields(ctx, replica, what, ptrs, 1 if out_on_device else 0), ctx)


def pic_fields_static(ctx, replica, what, outs, out_on_device=False):
    """pic_fields staged in the library's fixed device array (allocates nothing)."""
    ptrs = (C.c_void_p * len(outs))()
    for i, o in enumerate(outs):
        ptrs[i] = o.data_ptr() if hasattr(o, "data_ptr") else o.ctypes.data
    _check(lib().pic_fields_static(ctx, replica, what, ptrs, 1 if out_on_device else 0), ctx)


def pic_grain_positions(ctx, replica, n_grains):
    out = np.zeros((max(n_grains, 1), 3))
    _check(lib().pic_grain_positions(ctx, replica, out.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return out[:n_grains].copy()


def pic_energy(ctx, replica):
    out = (C.c_double * 4)()
    _check(lib().pic_energy(ctx, replica, out), ctx)
    return dict(kinetic_e=out[0], kinetic_i=out[1], field=out[2], total=out[3])


def pic_save(ctx, path):
    _check(lib().pic_save(ctx, os.fsencode(path)), ctx)


def pic_load(ctx, path):
    _check(lib().pic_load(ctx, os.fsencode(path)), ctx)


def pic_average(ctx, interval, phase_bins=1):
    _check(lib().pic_average(ctx, int(interval), int(phase_bins)), ctx)


def pic_average_read(ctx, replica, bin, what, outs, out_on_device=False):
    """outs: buffers in PHI, N, FLUX order; returns the number of samples."""
    ptrs = (C.c_void_p * max(len(outs), 1))()
    for i, o in enumerate(outs):
        ptrs[i] = o.data_ptr() if hasattr(o, "data_ptr") else o.ctypes.data
    n = C.c_int64(0)
    _check(lib().pic_average_read(ctx, replica, bin, what, ptrs, 1 if out_on_device else 0,
                                  C.byref(n)), ctx)
    return int(n.value)


def pic_set_fine_grid(ctx, replica, origin=None, h=None, cells=None):
    """Sets the fine diagnostic grid of a replica (origin None removes it)."""
    if origin is None:
        _check(lib().pic_set_fine_grid(ctx, replica, None), ctx)
        return
    g = pic_fine_grid()
    for a in range(3):
        g.origin[a] = float(origin[a])
        g.cells[a] = int(cells[a])
    g.h = float(h)
    _check(lib().pic_set_fine_grid(ctx, replica, C.byref(g)), ctx)


def pic_destroy(ctx):
    lib().pic_destroy(ctx)


def pic_last_error(ctx=None):
    m = lib().pic_last_error(ctx)
    return m.decode() if m else ""


def pic_get_state(ctx, replica, capacity, n_grains):
    st = {}
    v = pic_state_view()
    bufs = []
    for s in range(2):
        pos = np.zeros((capacity[s], 3))
        vel = np.zeros((capacity[s], 3))
        ids = np.zeros(capacity[s], np.uint32)
        bufs.append((pos, vel, ids))
        v.capacity[s] = capacity[s]
        v.pos[s] = pos.ctypes.data_as(C.POINTER(C.c_double))
        v.vel[s] = vel.ctypes.data_as(C.POINTER(C.c_double))
        v.id[s] = ids.ctypes.data_as(C.POINTER(C.c_uint32))
    gc = np.zeros((max(n_grains, 1), 2), np.int64)
    v.grain_count = gc.ctypes.data_as(C.POINTER(C.c_int64))
    _check(lib().pic_get_state(ctx, replica, C.byref(v)), ctx)
    for s in range(2):
        n = v.n[s]
        st[s] = dict(pos=bufs[s][0][:n].copy(), vel=bufs[s][1][:n].copy(), id=bufs[s][2][:n].copy())
    st["grain_count"] = gc[:n_grains].copy()
    st["wall_count"] = np.array([[v.wall_count[a][b] for b in range(2)] for a in range(2)])
    st["step"] = int(v.step)
    return st


def pic_set_state(ctx, replica, state, n_grains):
    v = pic_state_view()
    keep = []
    for s in range(2):
        pos = np.ascontiguousarray(state[s]["pos"], np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(state[s]["vel"], np.float64).reshape(-1, 3)
        ids = np.ascontiguousarray(state[s]["id"], np.uint32)
        keep += [pos, vel, ids]
        v.n[s] = v.capacity[s] = len(ids)
        v.pos[s] = pos.ctypes.data_as(C.POINTER(C.c_double))
        v.vel[s] = vel.ctypes.data_as(C.POINTER(C.c_double))
        v.id[s] = ids.ctypes.data_as(C.POINTER(C.c_uint32))
    gc = np.ascontiguousarray(state.get("grain_count", np.zeros((n_grains, 2))), np.int64).reshape(-1)
    if n_grains:
        v.grain_count = gc.ctypes.data_as(C.POINTER(C.c_int64))
    wc = np.asarray(state.get("wall_count", np.zeros((2, 2))), np.int64)
    for a in range(2):
        for b in range(2):
            v.wall_count[a][b] = int(wc[a, b])
    v.step = int(state.get("step", 0))
    _check(lib().pic_set_state(ctx, replica, C.byref(v)), ctx)


def pic_get_counters(ctx, replica):
    c = pic_counters()
    _check(lib().pic_get_counters(ctx, replica, C.byref(c)), ctx)
    return dict(n_alive=list(c.n_alive), wall_count=[[c.wall_count[a][b] for b in range(2)] for a in range(2)],
                cap_violation=list(c.cap_violation), n_collisions=list(c.n_collisions),
                md_particles=list(c.md_particles), step=int(c.step),
                refine_sweeps=int(c.refine_sweeps), refine_residual=float(c.refine_residual),
                numeric_bad=int(c.numeric_bad), tile_fallback=int(c.tile_fallback),
                n_coulomb=int(c.n_coulomb), refine_unconverged=int(c.refine_unconverged),
                md_margin=list(c.md_margin), n_ionizations=int(c.n_ionizations),
                iz_dropped=int(c.iz_dropped))


def pic_derived(ctx, replica):
    out = (C.c_double * 7)()
    _check(lib().pic_derived(ctx, replica, out), ctx)
    return dict(w=out[0], Qp=int(out[1]), n_gas=out[2], g_cap=[out[3], out[4]],
                T_null=[int(out[5]), int(out[6])])


def pic_profile_enable(ctx, on=True):
    _check(lib().pic_profile_enable(ctx, 1 if on else 0), ctx)


def pic_profile_read(ctx, kernel_class):
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().pic_profile_read(ctx, kernel_class, C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def pic_get_tuning(ctx):
    t = pic_tuning()
    _check(lib().pic_get_tuning(ctx, C.byref(t)), ctx)
    return {k: int(getattr(t, k)) for k in TUNING_KEYS}


def pic_set_tuning(ctx, tuning: dict):
    t = pic_tuning()
    cur = pic_get_tuning(ctx)
    unknown = set(tuning) - set(TUNING_KEYS)
    if unknown:
        raise ValueError(f"unknown tuning keys {sorted(unknown)}")
    for k in TUNING_KEYS:
        setattr(t, k, int(tuning.get(k, cur[k])))
    _check(lib().pic_set_tuning(ctx, C.byref(t)), ctx)


def pic_autotune(ctx, trial_steps=48, capacity=64):
    """Runs the search; returns the list of (settings, ms per step) tried."""
    tried = (pic_tuning * capacity)()
    ms = (C.c_double * capacity)()
    n = C.c_int()
    _check(lib().pic_autotune(ctx, int(trial_steps), tried, ms, capacity, C.byref(n)), ctx)
    return [({k: int(getattr(tried[i], k)) for k in TUNING_KEYS}, float(ms[i]))
            for i in range(min(n.value, capacity))]


# ---------------------------------------------------------------- convenience
class Simulation:
    """One context over one or more replicas (workload dicts)."""

    def __init__(self, workloads, stream=None, sort_interval=8, max_refine=2):
        if isinstance(workloads, dict):
            workloads = [workloads]
        self.wls = list(workloads)
        made = [make_config(w, sort_interval=sort_interval, max_refine=max_refine) for w in self.wls]
        self._keep = [m[1] for m in made]
        self.ctx = pic_init([m[0] for m in made], len(made),
                            stream if stream is not None else current_stream())
        self.n_nodes = [w["nx"] * w["ny"] * (w["nz"] + 1) for w in self.wls]
        self.n_grains = [int(m[0].n_grains) for m in made]
        self.capacity = [self._slots(w) for w in self.wls]
        self.fine_nodes = [0] * len(self.wls)

    @staticmethod
    def _slots(w):
        """Host room per species for pic_get_state: at most the library's
        particles per species (the loaded count, max_particles, or a quarter
        more with ionisation)."""
        n = w["nx"] * w["ny"] * w["nz"] * w["ppc"]
        if int(w.get("max_particles", 0)) > 0:
            return max(n, int(w["max_particles"]))
        if (w.get("xs") or {}).get("e_iz") is not None:
            return n + n // 4
        return n

    def step(self, n=1):
        pic_step(self.ctx, n)

    def fields(self, replica=0, what=PIC_PHI | PIC_E | PIC_RHO):
        nn = self.n_nodes[replica]
        fn = self.fine_nodes[replica]
        outs, names = [], []
        for bit, name, shape, dt in ((PIC_PHI, "phi", (nn,), np.float64), (PIC_E, "E", (3, nn), np.float64),
                                     (PIC_RHO, "rho", (nn,), np.float64),
                                     (PIC_RHO_FIXED, "rho_fixed", (nn,), np.int64),
                                     (PIC_N, "n", (2, nn), np.float64),
                                     (PIC_FLUX, "flux", (2, 3, nn), np.float64),
                                     (PIC_FINE_N, "fine_n", (2, fn), np.float64),
                                     (PIC_FINE_FLUX, "fine_flux", (2, 3, fn), np.float64),
                                     (PIC_FINE_PHI, "fine_phi", (fn,), np.float64)):
            if what & bit:
                outs.append(np.zeros(shape, dt))
                names.append(name)
        pic_fields(self.ctx, replica, what, outs, False)
        return dict(zip(names, outs))

    def average(self, interval, phase_bins=1):
        """Start (interval > 0) or stop (0) sampling the time averages."""
        pic_average(self.ctx, interval, phase_bins)

    def set_fine_grid(self, origin=None, h=None, cells=None, replica=0):
        """Sets (or, with origin None, removes) the replica's fine diagnostic
        grid: lower corner and cell edge in grid units, cells per axis."""
        pic_set_fine_grid(self.ctx, replica, origin, h, cells)
        self.fine_nodes[replica] = 0 if origin is None else int(np.prod([int(c) + 1 for c in cells]))

    def averages(self, replica=0, bin=-1, what=PIC_PHI | PIC_N | PIC_FLUX):
        nn = self.n_nodes[replica]
        fn = self.fine_nodes[replica]
        outs, names = [], []
        for bit, name, shape in ((PIC_PHI, "phi", (nn,)), (PIC_N, "n", (2, nn)),
                                 (PIC_FLUX, "flux", (2, 3, nn)), (PIC_FINE_N, "fine_n", (2, fn)),
                                 (PIC_FINE_FLUX, "fine_flux", (2, 3, fn)),
                                 (PIC_FINE_PHI, "fine_phi", (fn,))):
            if what & bit:
                outs.append(np.zeros(shape))
                names.append(name)
        n = pic_average_read(self.ctx, replica, bin, what, outs, False)
        out = dict(zip(names, outs))
        out["samples"] = n
        return out

    def get_state(self, replica=0):
        cap = [self.capacity[replica]] * 2
        return pic_get_state(self.ctx, replica, cap, self.n_grains[replica])

    def set_state(self, state, replica=0):
        pic_set_state(self.ctx, replica, state, self.n_grains[replica])

    def grain_positions(self, replica=0):
        """The replica's grains [n][3] in cell units (given or placed by the library)."""
        return pic_grain_positions(self.ctx, replica, self.n_grains[replica])

    def energy(self, replica=0):
        """FP64 kinetic (per species), field and total energy (J) at this step."""
        return pic_energy(self.ctx, replica)

    def save(self, path):
        """Checkpoint every replica (pic_save)."""
        pic_save(self.ctx, path)

    def load(self, path):
        """Resume from a checkpoint written by a context of the same workloads."""
        pic_load(self.ctx, path)

    def counters(self, replica=0):
        return pic_get_counters(self.ctx, replica)

    def grain_charges(self, replica=0):
        return pic_grain_charges(self.ctx, replica, self.n_grains[replica])

    def derived(self, replica=0):
        return pic_derived(self.ctx, replica)

    def tuning(self):
        return pic_get_tuning(self.ctx)

    def set_tuning(self, **kw):
        pic_set_tuning(self.ctx, kw)

    def tuning_key(self):
        """What the best settings depend on: the shapes of the replicas, the
        arithmetic form and the device."""
        import torch
        dev = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "none"
        shapes = [(w["nx"], w["ny"], w["nz"], w["ppc"], len(w.get("grain_pos", [])), w.get("cutoff", 3),
                   w.get("precision", "fp64")) for w in self.wls]
        return json.dumps([dev, shapes])

    def autotune(self, trial_steps=48, cache=None):
        """Chooses the launch settings by timing live steps (pic_autotune) and
        applies them.  With `cache` (a JSON file path) a previous result for
        the same key is applied without searching, and a new one is stored.
        Returns (settings, trials); trials is empty for a cache hit."""
        key = self.tuning_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_tuning(**table[key])
                return self.tuning(), []
        trials = pic_autotune(self.ctx, trial_steps)
        best = self.tuning()
        if cache:
            table[key] = best
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return best, trials

    def close(self):
        if self.ctx:
            pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
