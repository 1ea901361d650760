"""Glue between the HIP path (through the C ABI binding) and the FP64 oracle."""
import math

import numpy as np

from oracle import sim as osim

# Bound on the FP32 error of one overlap in the HIP sweep, as a multiple of
# the box length (block-relative FP32 coordinates).
E_DELTA_REL = 2.0 ** -18


def gpu_params(abm, **kw):
    base = dict(dt=0.01, k=2.0, gamma=1.0, adherence=1.8, mass=0.1, max_disp=3.0, box_len=15.0)
    base.update(kw)
    return abm.params(**base)


def oracle_params(**kw):
    base = dict(dt=0.01, k=2.0, gamma=1.0, adherence=1.8, mass=0.1, max_disp=3.0, box_len=15.0)
    base.update(kw)
    kw2 = {k: v for k, v in base.items() if k not in ("resort_every", "diag")}
    return osim.make_params(**kw2)


def gpu_state(abm, b, sim=0):
    """Full state of one simulation in the library's storage order."""
    return dict(pos=b.query(abm.POS, sim), diam=b.query(abm.DIAM, sim), vol=b.query(abm.VOL, sim),
                growth=b.query(abm.GROWTH, sim), uid=b.query(abm.UID, sim), static=b.query(abm.STATIC, sim),
                nz=b.query(abm.NZ, sim))


def oracle_from_state(st, params, cap=None, next_uid=None, iteration=0):
    n = st["pos"].shape[0]
    return osim.OracleSim(st["pos"], st["diam"], params, vol=st["vol"], growth=st["growth"], uid=st["uid"],
                          cap=cap or max(n, 1), next_uid=next_uid, is_static=st["static"], nz=st["nz"],
                          iteration=iteration)


def force_tolerance(o, L):
    """Per-agent bound: 1e-5 relative to sum |F_N|, plus the FP32 error bound
    e of the centre distance times the conditioning of the force vector
    F_N (x_i - x_j) / d: through the overlap, |dF_N/d delta| (Eq 4.1), and
    through the direction, |F_N| / d (the centre line's error over d)."""
    n = o.n
    return 1e-5 * o.sum_abs_fn[:n] + E_DELTA_REL * L * (o.sum_dfn[:n] + o.sum_fn_d[:n]) + 1e-12


def compare_single_step(abm, b, o, sim=0, L=15.0, check_static=True):
    """GPU state after one DIAG step vs the oracle stepped once from the same
    state (both already stepped).  Returns a dict of measured errors."""
    n = o.n
    g_uid = b.query(abm.UID, sim)
    # match by uid
    order_g = np.argsort(g_uid, kind="stable")
    order_o = np.argsort(o.uid[:n], kind="stable")
    assert np.array_equal(g_uid[order_g], o.uid[:n][order_o]), "agent sets differ"
    out = {}
    g_nbr = b.query(abm.NBR_COUNT, sim)
    g_con = b.query(abm.CONTACT_COUNT, sim)
    g_nz = b.query(abm.NZ, sim)
    g_box = b.query(abm.BOX, sim)
    g_f = b.query(abm.FORCE, sim)
    g_d = b.query(abm.DISP, sim)
    g_pos = b.query(abm.POS, sim)
    # only agents that existed at the start of the step carry diagnostics
    old_o = order_o[o.is_new[:n][order_o] == 0]
    old_g = order_g[o.is_new[:n][order_o] == 0]
    assert np.array_equal(g_box[old_g], o.box[:n][old_o]), "box ids differ"
    assert np.array_equal(g_nbr[old_g], o.nbr[:n][old_o]), "neighbour counts differ"
    assert np.array_equal(g_con[old_g], o.contacts[:n][old_o]), "contact counts differ"
    assert np.array_equal(np.minimum(g_nz[old_g], 255), np.minimum(o.nz[:n][old_o], 255)), "nz counts differ"
    fo = o.force()[old_o]
    fg = g_f[old_g]
    tol = force_tolerance(o, L)[old_o]
    err = np.linalg.norm(fg - fo, axis=1)
    out["force_normwise_rel"] = float(np.linalg.norm(fg - fo) / max(np.linalg.norm(fo), 1e-300))
    out["force_max_err_over_tol"] = float((err / tol).max()) if err.size else 0.0
    assert out["force_normwise_rel"] <= 1e-5, out
    assert np.all(err <= tol), out
    do = o.disp()[old_o]
    dg = g_d[old_g]
    assert np.array_equal(np.any(dg != 0, axis=1), np.any(do != 0, axis=1)), "move decisions differ"
    scale = o.params.dt / o.params.mass
    derr = np.linalg.norm(dg - do, axis=1)
    assert np.all(derr <= scale * tol + 1e-12), "displacements differ"
    perr = np.abs(g_pos[order_g] - o.pos()[order_o]).max(axis=1)
    out["pos_max_abs_err"] = float(perr.max()) if perr.size else 0.0
    assert out["pos_max_abs_err"] <= 1e-4, out
    if check_static:
        g_st = b.query(abm.STATIC, sim)[order_g]
        o_st = o.is_static[:n][order_o]
        out["static_gpu"] = int(g_st.sum())
        out["static_oracle"] = int(o_st.sum())
        # the rule is radius-exact on both sides; a flag can only differ where a
        # distance to a changed agent sits within the position error of L
        out["static_mismatch"] = int(np.count_nonzero(g_st != o_st))
        assert out["static_mismatch"] == 0, out
    return out


def compare_positions_single_step(abm, b, o, start_pos, sim=0, L=15.0):
    """Production (non-diagnostic) step against the oracle stepped once from
    the same state: the same agents move, and every new position is within
    dt/m times the force tolerance of the oracle's."""
    n = o.n
    g_uid = b.query(abm.UID, sim)
    order_g = np.argsort(g_uid, kind="stable")
    order_o = np.argsort(o.uid[:n], kind="stable")
    assert np.array_equal(g_uid[order_g], o.uid[:n][order_o]), "agent sets differ"
    pg = b.query(abm.POS, sim)[order_g]
    po = o.pos()[order_o]
    p0 = np.full((n, 3), np.nan)  # daughters of this step have no start position
    p0[: start_pos.shape[0]] = start_pos
    p0 = p0[order_o]
    old = o.is_new[:n][order_o] == 0
    moved_g = np.any(pg[old] != p0[old], axis=1)
    moved_o = np.any(po[old] != p0[old], axis=1)
    assert np.array_equal(moved_g, moved_o), "move decisions differ"
    tol = (o.params.dt / o.params.mass) * force_tolerance(o, L)[order_o][old] + 1e-12
    err = np.linalg.norm(pg[old] - po[old], axis=1)
    assert np.all(err <= tol + 1e-13 * np.abs(po[old]).max(axis=1)), float((err / tol).max())
    return {"pos_max_abs_err": float(err.max()) if err.size else 0.0, "moved": int(moved_o.sum())}
