"""GPU-vs-oracle comparison helpers (teacher forcing: the oracle is fed the GPU's binary32
state, upcast, before every comparison, so that decisions computed from identical inputs
can be compared bit for bit)."""
import numpy as np

TOL = 1e-5  # |gpu - oracle| <= TOL * max(|oracle|, 1) per component (m, m/s, rad)
BAND_COLL, BAND_GOAL = 1, 2


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


def compare_obs(g, o, K, N=0):
    """Observation of the same binary32 state: index sets and masks bit-exact, features
    within TOL."""
    assert np.array_equal(g["road_idx"], o["road_idx"]), _first_diff(g["road_idx"], o["road_idx"], "road_idx")
    assert np.array_equal(g["pmask"], o["pmask"]), _first_diff(g["pmask"], o["pmask"], "pmask")
    assert_close(g["ego"], o["ego"], "ego")
    for c in (0, 1, 3, 4, 5):
        assert_close(g["partner"][:, c], o["partner"][:, c], "partner[%d]" % c)
    assert_close(g["partner"][:, 2], o["partner"][:, 2], "partner heading", angle=True)
    if K:
        for c in (0, 1, 3):
            assert_close(g["road"][:, :, c], o["road"][:, :, c], "road[%d]" % c)
        assert_close(g["road"][:, :, 2], o["road"][:, :, 2], "road dir", angle=True)
    if N:
        compare_lidar(g, o)


def compare_lidar(g, o):
    band = (o["band"] & 16) != 0
    ok = ~band
    assert np.array_equal(g["lidar_hit"][ok], o["lidar_hit"][ok]), "lidar hit types differ"
    assert_close(g["lidar"][ok], o["lidar"][ok], "lidar")


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


def teacher_forced_run(scene, sim, O, actions, steps, stats=None):
    """Step the GPU `steps` times; before each step hand its state to the oracle, step the
    oracle in FP64 (with the GPU simulator's parameters) and compare; then compare the
    observation of the GPU's new state."""
    K, N = scene.params.top_k, scene.params.lidar_rays
    stats = stats if stats is not None else {}
    stats.setdefault("band_worlds", 0)
    stats.setdefault("max_state_rel", 0.0)
    g = sim.host_outputs()
    orc = oracle_for(scene, g["state"], g["flags"], g["t"], O, sim.params)
    compare_obs(g, orc.obs(), K, N)
    import torch
    for k in range(steps):
        pre = g
        act = torch.as_tensor(np.ascontiguousarray(actions[k]), device=sim.device)
        sim.step(act)
        g = sim.host_outputs()
        orc = oracle_for(scene, pre["state"], pre["flags"], pre["t"], O, sim.params)
        o = orc.step(actions[k].astype(np.float64))
        # worlds whose discrete outcome sits within 1e-4 m of a threshold are not compared
        skip_w = np.zeros(scene.num_worlds, bool)
        for w in range(scene.num_worlds):
            a0, a1 = scene.agent_off[w], scene.agent_off[w + 1]
            if (o["band"][a0:a1] & (BAND_COLL | BAND_GOAL)).any():
                skip_w[w] = True
        stats["band_worlds"] += int(skip_w.sum())
        agent_w = np.repeat(np.arange(scene.num_worlds), np.diff(scene.agent_off))
        keep_a = ~skip_w[agent_w]
        assert np.array_equal(g["world_done"][~skip_w], o["world_done"][~skip_w]), "world_done, step %d" % k
        assert np.array_equal(g["t"][~skip_w], o["t"][~skip_w]), "t, step %d" % k
        assert np.array_equal(g["flags"][keep_a], o["flags"][keep_a]), \
            "flags, step %d: " % k + _first_diff(g["flags"][keep_a], o["flags"][keep_a], "flags")
        assert_close(g["reward"][keep_a], o["reward"][keep_a], "reward step %d" % k)
        st_g, st_o = g["state"][:, keep_a], o["state"][:, keep_a]
        assert_close(st_g, st_o, "state step %d" % k)
        rel = np.abs(st_g - st_o) / np.maximum(np.abs(st_o), 1.0)
        stats["max_state_rel"] = max(stats["max_state_rel"], float(rel.max()) if rel.size else 0.0)
        # observation of the GPU's new state, teacher-forced
        orc2 = oracle_for(scene, g["state"], g["flags"], g["t"], O, sim.params)
        compare_obs(g, orc2.obs(), K, N)
    return stats
