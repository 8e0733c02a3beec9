"""GPU-vs-oracle comparison helpers.

Teacher forcing: the oracle is fed the GPU's binary32 state, upcast, before every
comparison.  The oracle takes every decision in FP64 (the plain definition); a decision
whose FP64 quantity lies within 1e-4 m of its threshold is in the ambiguous band (the
oracle marks it per agent) and may legitimately come out either way on the GPU, whose
keys are binary32.  Outside the band, index sets, masks and flags must be bit-exact.

What is compared, per agent:
  * collision / goal / done flags and the reward: exact, unless the oracle marks the agent
    in the collision or goal band (then excluded and counted);
  * world_done and t: exact, unless the world holds an agent in the band (counted); the
    world's state is compared whenever the world outcome agrees;
  * partner masks: exact, unless the observer has a partner within 1e-4 m of the radius;
  * road index lists: the set of selected points exact unless the K-th cut or the radius
    has a point within 1e-4 m of it; the order exact except that two points whose FP64
    distances differ by less than 1e-4 m may swap (several orders are then correct); for
    in-band agents the list must still be valid (no duplicates, distances in order within
    1e-4 m, slot by slot within 1e-4 m of the oracle's);
  * features (states, rewards, ego, partner and road rows): within TOL relative, the road
    rows matched by point index.
Every exclusion is counted in `stats` and bounded by the caller.
"""
import numpy as np

TOL = 1e-5  # |gpu - oracle| <= TOL * max(|oracle|, 1) per component (m, m/s, rad)
BAND = 1e-4  # m
BAND_COLL, BAND_GOAL, BAND_PARTNER_R, BAND_KTH, BAND_LIDAR, BAND_ROAD_R = 1, 2, 4, 8, 16, 32


def wrapd(a):
    return (np.asarray(a, np.float64) + np.pi) % (2 * np.pi) - np.pi


def assert_close(g, o, what, tol=TOL, floor=1.0, angle=False):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    d = wrapd(g - o) if angle else g - o
    lim = tol * np.maximum(np.abs(o), floor)
    bad = np.abs(d) > lim
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError("%s: %d mismatches, first at %s gpu=%r oracle=%r" %
                             (what, int(bad.sum()), tuple(i), g[tuple(i)], o[tuple(i)]))


def new_stats():
    return dict(agents=0, steps=0, flag_band_agents=0, world_band=0, partner_band_agents=0,
                road_band_agents=0, order_tie_agents=0, order_tie_slots=0,
                lidar_band_agents=0, lidar_band_rays=0, lidar_rays=0, max_state_rel=0.0,
                collisions=0, worlds_done=0)


def _slot_owner(agent_off, P, S):
    ao = np.asarray(agent_off, np.int64)
    if P >= 0:
        return np.arange(S, dtype=np.int64) // max(P, 1)
    n = np.diff(ao)
    return np.repeat(np.arange(int(ao[-1])), np.repeat(np.maximum(n - 1, 0), n))


def _agent_dist(o, i, idx):
    """FP64 distances from agent i (the oracle's state) to its world's road points idx."""
    ao, ro = o["geom"]["agent_off"], o["geom"]["road_off"]
    w = int(np.searchsorted(ao, i, side="right") - 1)
    r0 = int(ro[w])
    qx = o["geom"]["road_x"][r0 + idx]
    qy = o["geom"]["road_y"][r0 + idx]
    return np.hypot(qx - o["state"][0, i], qy - o["state"][1, i])


def _road_row(g, o, i, K, stats):
    """One agent's road index list and rows (see the module docstring)."""
    gi, oi = g["road_idx"][i], o["road_idx"][i]
    ng, no = int((gi >= 0).sum()), int((oi >= 0).sum())
    band = int(o["band"][i])
    assert np.all(gi[ng:] == -1) and np.all(gi[:ng] >= 0), ("padding", i, gi)
    assert len(set(gi[:ng].tolist())) == ng, ("duplicate road index", i)
    in_band = bool(band & (BAND_KTH | BAND_ROAD_R))
    dg = _agent_dist(o, i, gi[:ng])
    do = _agent_dist(o, i, oi[:no])
    if in_band:
        stats["road_band_agents"] += 1
        if not band & BAND_ROAD_R:
            assert ng == no, ("road count", i, ng, no)
        m = min(ng, no)
        assert np.all(np.abs(dg[:m] - do[:m]) < BAND), ("in-band slot distances", i)
        assert np.all(np.diff(dg) > -BAND), ("in-band order", i)
    else:
        assert ng == no, ("road count", i, ng, no)
        assert set(gi[:ng].tolist()) == set(oi[:no].tolist()), \
            ("road set", i, sorted(set(gi[:ng].tolist()) ^ set(oi[:no].tolist())))
        swap = gi[:ng] != oi[:no]
        if swap.any():
            # only points at (near) equal distance may change places
            assert np.all(np.abs(dg[swap] - do[swap]) < BAND), ("road order", i, np.nonzero(swap)[0])
            stats["order_tie_agents"] += 1
            stats["order_tie_slots"] += int(swap.sum())
    # rows, matched by point index
    pos = {int(q): s for s, q in enumerate(oi[:no])}
    for s in range(ng):
        t = pos.get(int(gi[s]))
        if t is None:
            continue  # an in-band point the oracle did not select
        for c in (0, 1, 3):
            assert_close(g["road"][i, s, c], o["road"][i, t, c], "road[%d] agent %d slot %d" % (c, i, s))
        assert_close(g["road"][i, s, 2], o["road"][i, t, 2], "road dir agent %d slot %d" % (i, s), angle=True)
    assert np.all(g["road"][i, ng:] == 0.0)


def compare_obs(g, o, K, N=0, stats=None):
    """Observation of the same binary32 state (o: the FP64 oracle's, with band bits)."""
    stats = stats if stats is not None else new_stats()
    A = g["ego"].shape[0]
    assert_close(g["ego"], o["ego"], "ego")
    # partners
    S = g["pmask"].shape[0]
    if S:
        owner = _slot_owner(o["geom"]["agent_off"], o["geom"]["partners"], S)
        diff = g["pmask"] != o["pmask"]
        if diff.any():
            bad_owner = np.unique(owner[diff])
            assert np.all(o["band"][bad_owner] & BAND_PARTNER_R), \
                _first_diff(g["pmask"], o["pmask"], "pmask")
            stats["partner_band_agents"] += len(bad_owner)
        same = ~diff
        for c in (0, 1, 3, 4, 5):
            assert_close(g["partner"][same, c], o["partner"][same, c], "partner[%d]" % c)
        assert_close(g["partner"][same, 2], o["partner"][same, 2], "partner heading", angle=True)
    # road
    if K:
        rows_equal = np.all(g["road_idx"] == o["road_idx"], axis=1)
        eq = np.nonzero(rows_equal)[0]
        for c in (0, 1, 3):
            assert_close(g["road"][eq, :, c], o["road"][eq, :, c], "road[%d]" % c)
        assert_close(g["road"][eq, :, 2], o["road"][eq, :, 2], "road dir", angle=True)
        for i in np.nonzero(~rows_equal)[0]:
            _road_row(g, o, int(i), K, stats)
        stats["road_band_agents"] += int(((o["band"][eq] & (BAND_KTH | BAND_ROAD_R)) != 0).sum())
    if N:
        compare_lidar(g, o, stats)
    stats["agents"] += A
    return stats


def compare_lidar(g, o, stats=None):
    """Hit types exact and distances within the tolerance on every ray outside the band
    (the oracle marks each ray whose nearest hit lies within 1e-4 m of a threshold)."""
    band = o["lidar_band"] != 0
    if stats is not None:
        stats["lidar_band_agents"] += int(band.any(axis=1).sum())
        stats["lidar_band_rays"] += int(band.sum())
        stats["lidar_rays"] += int(band.size)
    ok = ~band
    assert np.array_equal(g["lidar_hit"][ok], o["lidar_hit"][ok]), \
        _first_diff(np.where(ok, g["lidar_hit"], 0), np.where(ok, o["lidar_hit"], 0), "lidar hit types")
    assert_close(g["lidar"][ok], o["lidar"][ok], "lidar")


def compare_step(g, o, agent_off, stats, what=""):
    """Outcome of one step from the same pre-step state: flags and rewards per agent
    (agents in the collision or goal band excluded), world outcome per world (worlds
    holding such an agent may differ), and the state of every world whose outcome agrees."""
    ao = np.asarray(agent_off, np.int64)
    W = len(ao) - 1
    agent_w = np.repeat(np.arange(W), np.diff(ao))
    band_a = (o["band"] & (BAND_COLL | BAND_GOAL)) != 0
    band_w = np.zeros(W, bool)
    np.logical_or.at(band_w, agent_w, band_a)
    same_w = (g["world_done"] == o["world_done"]) & (g["t"] == o["t"])
    assert np.all(same_w | band_w), "world outcome %s: worlds %s" % (what, np.nonzero(~(same_w | band_w))[0][:8])
    stats["world_band"] += int((~same_w).sum())
    keep = same_w[agent_w] & ~band_a
    stats["flag_band_agents"] += int(band_a.sum())
    assert np.array_equal(g["flags"][keep], o["flags"][keep]), \
        "flags %s: " % what + _first_diff(g["flags"][keep], o["flags"][keep], "flags")
    assert_close(g["reward"][keep], o["reward"][keep], "reward %s" % what)
    st = same_w[agent_w]
    st_g, st_o = g["state"][:, st], o["state"][:, st]
    assert_close(st_g, st_o, "state %s" % what)
    if st_o.size:
        rel = np.abs(st_g - st_o) / np.maximum(np.abs(st_o), 1.0)
        stats["max_state_rel"] = max(stats["max_state_rel"], float(rel.max()))
    stats["collisions"] += int(((g["flags"] & 3) != 0).sum())
    stats["worlds_done"] += int(g["world_done"].sum())
    stats["steps"] += 1


def _first_diff(a, b, name):
    d = np.argwhere(a != b)
    if len(d) == 0:
        return name + ": equal"
    i = tuple(d[0])
    return "%s: %d differ, first at %s gpu=%r oracle=%r" % (name, len(d), i, a[i], b[i])


def oracle_for(scene, state, flags, t, O, params=None):
    orc = O.OracleSim(scene, params)
    orc.set_state(state[0], state[1], state[2], state[3], flags=flags, t=t)
    return orc


def check_bounds(stats, max_frac=0.01, road_frac=0.03, ray_frac=0.002):
    """Exclusions stay rare: at most max_frac of the compared agents in the collision,
    goal or partner-radius band, road_frac in the band of the K-th cut or the radius
    (higher: at a reset agents sit on lane points, where the points ahead and behind are
    equidistant, so a few per cent of reset observations have a near tie at the cut), and
    ray_frac of the compared LIDAR rays in their band."""
    n = max(stats["agents"], 1)
    for k in ("flag_band_agents", "partner_band_agents"):
        assert stats[k] <= max_frac * n, (k, stats[k], n)
    assert stats["road_band_agents"] <= road_frac * n, ("road_band_agents", stats["road_band_agents"], n)
    assert stats["lidar_band_rays"] <= ray_frac * max(stats["lidar_rays"], 1), \
        ("lidar_band_rays", stats["lidar_band_rays"], stats["lidar_rays"])


def teacher_forced_run(scene, sim, O, actions, steps, stats=None, max_band_frac=0.01):
    """Step the GPU `steps` times; before each step hand its state to the oracle, step the
    oracle in FP64 (with the GPU simulator's parameters) and compare; then compare the
    observation of the GPU's new state.  Returns the exclusion counts."""
    K, N = scene.params.top_k, scene.params.lidar_rays
    stats = stats if stats is not None else new_stats()
    g = sim.host_outputs()
    orc = oracle_for(scene, g["state"], g["flags"], g["t"], O, sim.params)
    compare_obs(g, orc.obs(), K, N, stats)
    import torch
    for k in range(steps):
        pre = g
        act = torch.as_tensor(np.ascontiguousarray(actions[k]), device=sim.device)
        sim.step(act)
        g = sim.host_outputs()
        orc = oracle_for(scene, pre["state"], pre["flags"], pre["t"], O, sim.params)
        o = orc.step(actions[k].astype(np.float64))
        compare_step(g, o, scene.agent_off, stats, "step %d" % k)
        # observation of the GPU's new state, teacher-forced
        orc2 = oracle_for(scene, g["state"], g["flags"], g["t"], O, sim.params)
        compare_obs(g, orc2.obs(), K, N, stats)
    check_bounds(stats, max_band_frac)
    return stats
