"""Helpers for comparing the HIP library with the oracle on the same state.

Particles are matched by (species, id).  A discrete decision (collision
acceptance, electrode crossing, grain hit) may differ between the two only
where the oracle's recorded margin for that particle is below `flip_margin`;
such particles are reported and left out of the continuous comparisons.
"""
import numpy as np

import oracle


def oracle_from_state(wl, state, flags=0):
    o = oracle.Oracle(wl, flags=flags)
    for s in range(2):
        o.set_particles(s, state[s]["pos"], state[s]["vel"], state[s]["id"])
    o.set_counts(grain_count=state.get("grain_count"), wall_count=state.get("wall_count"),
                 step=state.get("step", 0))
    return o


def min_image(d, n):
    return d - n * np.round(d / n)


def compare_step(wl, gpu_after, orc, tol_pos, tol_vel, flip_margin):
    """Compare one species-resolved particle state after a step.  Returns a
    report dict; raises AssertionError on a mismatch outside the margins."""
    rep = {"flips": 0, "max_dpos": 0.0, "max_dvel": 0.0, "n": 0}
    vth = [np.sqrt(wl["Te_eV"] * 1.602176634e-19 / 9.1093837015e-31),
           np.sqrt(max(wl["Ti_eV"], 1e-6) * 1.602176634e-19 / (39.948 * 1.66053906660e-27))]
    for s in range(2):
        oid = orc.id[s]
        alive = orc.alive[s] != 0
        margin = orc.margin[s]
        gid = gpu_after[s]["id"]
        assert len(np.unique(gid)) == len(gid), "duplicate ids on the GPU"
        o_alive_ids = set(oid[alive].tolist())
        g_ids = set(gid.tolist())
        diff = o_alive_ids.symmetric_difference(g_ids)
        if diff:
            idx = {int(i): k for k, i in enumerate(oid)}
            for i in diff:
                k = idx.get(int(i))
                assert k is not None, f"species {s}: id {i} unknown to the oracle"
                assert margin[k] <= flip_margin, (
                    f"species {s} id {i}: survival differs with margin {margin[k]:.3e}")
            rep["flips"] += len(diff)
        common = np.array(sorted(o_alive_ids & g_ids), dtype=np.int64)
        if len(common) == 0:
            continue
        o_order = np.argsort(oid)
        o_k = o_order[np.searchsorted(oid[o_order], common)]
        g_order = np.argsort(gid)
        g_k = g_order[np.searchsorted(gid[g_order], common)]
        keep = margin[o_k] > flip_margin
        rep["flips"] += int(np.count_nonzero(~keep))
        o_k, g_k = o_k[keep], g_k[keep]
        op, gp = orc.pos[s][o_k], gpu_after[s]["pos"][g_k]
        d = op - gp
        d[:, 0] = min_image(d[:, 0], wl["nx"])
        d[:, 1] = min_image(d[:, 1], wl["ny"])
        dpos = np.max(np.abs(d)) if len(d) else 0.0
        ov, gv = orc.vel[s][o_k], gpu_after[s]["vel"][g_k]
        scale = np.maximum(np.max(np.abs(ov), axis=1), vth[s])
        dvel = np.max(np.abs(ov - gv).max(axis=1) / scale) if len(ov) else 0.0
        rep["max_dpos"] = max(rep["max_dpos"], float(dpos))
        rep["max_dvel"] = max(rep["max_dvel"], float(dvel))
        rep["n"] += len(o_k)
        assert dpos <= tol_pos, f"species {s}: position differs by {dpos:.3e} cells"
        assert dvel <= tol_vel, f"species {s}: velocity differs by {dvel:.3e} (relative)"
    return rep


def rel_inf(a, b, floor=0.0):
    den = max(np.max(np.abs(b)), floor)
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))


def compare_step_all(wl, gpu_after, orc, tol_pos, tol_vel, flip_margin):
    """compare_step for very large states (tens of millions of particles):
    the same checks with sorted id arrays instead of Python sets."""
    rep = {"flips": 0, "max_dpos": 0.0, "max_dvel": 0.0, "n": 0}
    vth = [np.sqrt(wl["Te_eV"] * 1.602176634e-19 / 9.1093837015e-31),
           np.sqrt(max(wl["Ti_eV"], 1e-6) * 1.602176634e-19 / (39.948 * 1.66053906660e-27))]
    for s in range(2):
        oid, margin = orc.id[s], orc.margin[s]
        alive = orc.alive[s] != 0
        gid = gpu_after[s]["id"]
        g_order = np.argsort(gid, kind="stable")
        gs = gid[g_order]
        assert not np.any(gs[1:] == gs[:-1]), "duplicate ids on the GPU"
        o_order = np.argsort(oid, kind="stable")
        os_ = oid[o_order]
        # particles alive on one side only: allowed where the decision's margin is small
        o_alive_sorted = np.sort(oid[alive])
        diff = np.setxor1d(o_alive_sorted, gs, assume_unique=True)
        if len(diff):
            k = np.searchsorted(os_, diff)
            assert np.all(k < len(os_)) and np.all(os_[np.minimum(k, len(os_) - 1)] == diff), \
                f"species {s}: ids unknown to the oracle"
            bad = margin[o_order[k]] > flip_margin
            assert not np.any(bad), (f"species {s}: survival differs for {int(bad.sum())} "
                                     f"particles with margins up to {margin[o_order[k]].max():.3e}")
            rep["flips"] += len(diff)
        common = np.intersect1d(o_alive_sorted, gs, assume_unique=True)
        if len(common) == 0:
            continue
        o_k = o_order[np.searchsorted(os_, common)]
        g_k = g_order[np.searchsorted(gs, common)]
        keep = margin[o_k] > flip_margin
        rep["flips"] += int(np.count_nonzero(~keep))
        o_k, g_k = o_k[keep], g_k[keep]
        d = orc.pos[s][o_k] - gpu_after[s]["pos"][g_k]
        d[:, 0] = min_image(d[:, 0], wl["nx"])
        d[:, 1] = min_image(d[:, 1], wl["ny"])
        dpos = float(np.max(np.abs(d))) if len(d) else 0.0
        del d
        ov, gv = orc.vel[s][o_k], gpu_after[s]["vel"][g_k]
        scale = np.maximum(np.max(np.abs(ov), axis=1), vth[s])
        dvel = float(np.max(np.abs(ov - gv).max(axis=1) / scale)) if len(ov) else 0.0
        rep["max_dpos"] = max(rep["max_dpos"], dpos)
        rep["max_dvel"] = max(rep["max_dvel"], dvel)
        rep["n"] += len(o_k)
        assert dpos <= tol_pos, f"species {s}: position differs by {dpos:.3e} cells"
        assert dvel <= tol_vel, f"species {s}: velocity differs by {dvel:.3e} (relative)"
    return rep
