"""Glue between the HIP path (through the C ABI binding) and the FP64 oracle."""
import numpy as np

from oracle import sim as osim


def gpu_params(abm, **kw):
    base = dict(dt=0.01, k=2.0, gamma=1.0, adherence=1.8, mass=0.1, max_disp=3.0, box_len=15.0)
    base.update(kw)
    return abm.params(**base)


def oracle_params(**kw):
    base = dict(dt=0.01, k=2.0, gamma=1.0, adherence=1.8, mass=0.1, max_disp=3.0, box_len=15.0)
    base.update(kw)
    kw2 = {k: v for k, v in base.items() if k not in ("resort_every", "diag", "record")}
    return osim.make_params(**kw2)


def gpu_state(abm, b, sim=0):
    """Full state of one simulation in the library's storage order."""
    return dict(pos=b.query(abm.POS, sim), diam=b.query(abm.DIAM, sim), vol=b.query(abm.VOL, sim),
                growth=b.query(abm.GROWTH, sim), uid=b.query(abm.UID, sim), static=b.query(abm.STATIC, sim),
                nz=b.query(abm.NZ, sim), age=b.query(abm.AGE, sim))


def oracle_from_state(st, params, cap=None, next_uid=None, iteration=0):
    n = st["pos"].shape[0]
    return osim.OracleSim(st["pos"], st["diam"], params, vol=st["vol"], growth=st["growth"], uid=st["uid"],
                          cap=cap or max(n, 1), next_uid=next_uid, is_static=st["static"], nz=st["nz"],
                          iteration=iteration, age=st.get("age"))


def force_tolerance(o):
    """Per-agent force tolerance of the parity tests: 1e-5 relative to the sum
    of |F_N| over the agent's contacts (cancellation-safe, Eq 4.1-4.2), plus
    1e-12 absolute for agents without contacts."""
    return 1e-5 * o.sum_abs_fn[: o.n] + 1e-12


def threshold_ties(o):
    """Agents whose oracle force norm lies within 1e-6 of the sum of |F_N| of
    the adherence threshold: the move decision is a tie that the two sides'
    summation orders may decide differently (reported, not a failure)."""
    fn = np.linalg.norm(o.force(), axis=1)
    return np.abs(fn - o.params.adherence) <= 1e-6 * o.sum_abs_fn[: o.n]


def compare_single_step(abm, b, o, sim=0, check_static=True, check_nbr=True):
    """GPU state after one step with recorded fields (ABM_DIAG, or ABM_RECORD
    with check_nbr=False) against the oracle stepped once from the same state
    (both already stepped), agent by agent:
      - box ids, contact and non-zero-force counts (and with check_nbr the
        neighbour counts) bit-exact;
      - force per agent within 1e-5 sum |F_N| and normwise within 1e-5;
      - the same move decisions (threshold ties excepted), displacements
        within dt/m times the force tolerance (twice that where the cap
        engages), positions within the displacement tolerance;
      - the same static flags.
    Returns a dict of measured errors."""
    n = o.n
    g_uid = b.query(abm.UID, sim)
    order_g = np.argsort(g_uid, kind="stable")
    order_o = np.argsort(o.uid[:n], kind="stable")
    assert np.array_equal(g_uid[order_g], o.uid[:n][order_o]), "agent sets differ"
    out = {}
    g_con = b.query(abm.CONTACT_COUNT, sim)
    g_nz = b.query(abm.NZ, sim)
    g_box = b.query(abm.BOX, sim)
    g_f = b.query(abm.FORCE, sim)
    g_d = b.query(abm.DISP, sim)
    g_pos = b.query(abm.POS, sim)
    # only agents that existed at the start of the step carry recorded fields
    keep = o.is_new[:n][order_o] == 0
    old_o = order_o[keep]
    old_g = order_g[keep]
    # Agents skipped as static: the oracle records -1 contacts and no force.
    # The production sweep does not visit units whose agents are all static,
    # so their recorded fields keep older values; only the skipped agents of
    # visited units record -1.  Recorded fields are compared for the others.
    skip = o.contacts[:n][old_o] < 0
    assert np.all(skip[g_con[old_g] < 0]), "an agent recorded as skipped is not static"
    old_o, old_g = old_o[~skip], old_g[~skip]
    out["static_skipped"] = int(skip.sum())
    assert np.array_equal(g_box[old_g], o.box[:n][old_o]), "box ids differ"
    if check_nbr:
        g_nbr = b.query(abm.NBR_COUNT, sim)
        assert np.array_equal(g_nbr[old_g], o.nbr[:n][old_o]), "neighbour counts differ"
    assert np.array_equal(g_con[old_g], o.contacts[:n][old_o]), "contact counts differ"
    assert np.array_equal(np.minimum(g_nz[old_g], 255), np.minimum(o.nz[:n][old_o], 255)), "nz counts differ"
    fo = o.force()[old_o]
    fg = g_f[old_g]
    tol = force_tolerance(o)[old_o]
    err = np.linalg.norm(fg - fo, axis=1)
    out["agents"] = int(old_o.size)
    out["force_normwise_rel"] = float(np.linalg.norm(fg - fo) / max(np.linalg.norm(fo), 1e-300))
    out["force_max_err_over_tol"] = float((err / tol).max()) if err.size else 0.0
    assert out["force_normwise_rel"] <= 1e-5, out
    assert np.all(err <= tol), out
    ties = threshold_ties(o)[old_o]
    out["ties"] = int(ties.sum())
    do = o.disp()[old_o]
    dg = g_d[old_g]
    mo, mg = np.any(do != 0, axis=1), np.any(dg != 0, axis=1)
    assert np.array_equal(mg[~ties], mo[~ties]), "move decisions differ"
    scale = o.params.dt / o.params.mass
    capped = np.linalg.norm(do, axis=1) >= o.params.max_disp * (1 - 1e-12)
    dtol = scale * tol * np.where(capped, 2.0, 1.0) + 1e-15
    derr = np.linalg.norm(dg - do, axis=1)
    ok = derr <= dtol
    assert np.all(ok[~ties]), ("displacements differ", float((derr / dtol)[~ties].max()))
    perr = np.linalg.norm(g_pos[old_g] - o.pos()[old_o], axis=1)
    ptol = dtol + 1e-13 * np.abs(o.pos()[old_o]).max(axis=1)
    out["pos_max_abs_err"] = float(perr.max()) if perr.size else 0.0
    assert np.all((perr <= ptol)[~ties]), out
    all_o = order_o[keep]
    all_g = order_g[keep]
    sk = skip
    assert np.array_equal(g_pos[all_g][sk], o.pos()[all_o][sk]), "a static agent moved"
    if check_static:
        g_st = b.query(abm.STATIC, sim)[order_g]
        o_st = o.is_static[:n][order_o]
        out["static_gpu"] = int(g_st.sum())
        out["static_oracle"] = int(o_st.sum())
        out["static_mismatch"] = int(np.count_nonzero(g_st != o_st))
        assert out["static_mismatch"] == 0, out
    fp64 = b.fp64_agents() if hasattr(b, "fp64_agents") else None
    if fp64 is not None:
        out["fp64_agents"] = int(fp64)
    return out


def compare_positions_single_step(abm, b, o, st, sim=0):
    """Production step against the oracle stepped once from the same state
    (st: the start state from gpu_state): the same agents move, and every new
    position is within dt/m times the force tolerance of the oracle's.
    Agents are matched by uid (removals reorder the oracle's rows)."""
    n = o.n
    g_uid = b.query(abm.UID, sim)
    order_g = np.argsort(g_uid, kind="stable")
    order_o = np.argsort(o.uid[:n], kind="stable")
    assert np.array_equal(g_uid[order_g], o.uid[:n][order_o]), "agent sets differ"
    pg = b.query(abm.POS, sim)[order_g]
    po = o.pos()[order_o]
    su = np.asarray(st["uid"])
    so = np.argsort(su, kind="stable")
    ou = o.uid[:n][order_o]
    k = np.searchsorted(su[so], ou)
    k = np.minimum(k, su.size - 1)
    present = su[so][k] == ou  # daughters of this step have no start position
    p0 = np.full((n, 3), np.nan)
    p0[present] = np.asarray(st["pos"])[so][k[present]]
    old = (o.is_new[:n][order_o] == 0) & present
    moved_g = np.any(pg[old] != p0[old], axis=1)
    moved_o = np.any(po[old] != p0[old], axis=1)
    assert np.array_equal(moved_g, moved_o), "move decisions differ"
    tol = 2.0 * (o.params.dt / o.params.mass) * force_tolerance(o)[order_o][old] + 1e-12
    err = np.linalg.norm(pg[old] - po[old], axis=1)
    assert np.all(err <= tol + 1e-13 * np.abs(po[old]).max(axis=1)), float((err / tol).max())
    return {"pos_max_abs_err": float(err.max()) if err.size else 0.0, "moved": int(moved_o.sum())}
