"""The precision of the distance decisions.

The paper fixes no precision.  The oracle takes the radius filters, the goal and parking
tests and the road ranking key in FP64 (the plain definition); the GPU kernels take them
in binary32 with a fixed operation order, which the oracle reproduces in its secondary
mode (decide32).  These tests run the two modes from the same states on samples of every
workload and check, with the comparison the GPU parity tests use, that the binary32
decisions give the definition's index sets, masks and flags for every agent outside the
1e-4 m band, and only a few agents inside it (counts printed).  A mistake in either mode
(a strict radius, a dropped tie-break) fails here.
"""
import numpy as np
import pytest

from tests._parity import check_bounds, compare_obs, compare_step, new_stats


def _run(oracle_mod, sc, acts, steps):
    K, N = sc.params.top_k, sc.params.lidar_rays
    b32 = oracle_mod.OracleSim(sc, decide32=True)
    g = b32.obs()
    stats = new_stats()
    o = oracle_mod.OracleSim(sc).obs()
    compare_obs(g, o, K, N, stats)
    for k in range(steps):
        pre = g
        g = b32.step(acts[k])
        ref = oracle_mod.OracleSim(sc)
        ref.set_state(*pre["state"], flags=pre["flags"], t=pre["t"])
        o = ref.step(acts[k])
        compare_step(g, o, sc.agent_off, stats, "step %d" % k)
        ref2 = oracle_mod.OracleSim(sc)
        ref2.set_state(*g["state"], flags=g["flags"], t=g["t"])
        compare_obs(g, ref2.obs(), K, N, stats)
    check_bounds(stats, 0.01)
    return stats


@pytest.mark.parametrize("cfg,worlds,steps", [(0, None, 91), (1, [0, 9, 77, 200], 6),
                                               (2, [0, 1, 2, 3, 4, 5], 6), (3, [0, 3, 100, 511], 6),
                                               (4, [0, 4095], 2)])
def test_binary32_decisions_match_fp64_outside_band(oracle_mod, cfg, worlds, steps):
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(cfg, worlds=worlds)
    acts = S.make_actions(cfg, steps, sc.num_agents).astype(np.float64)
    st = _run(oracle_mod, sc, acts, steps)
    print("config %d: %s" % (cfg, st))
    assert st["agents"] > 0


def test_partner_exactly_at_radius_is_observed(oracle_mod):
    """A partner at exactly the observation radius (FP64 and binary32 squared distance
    both equal R^2) is observed: the radius filter is inclusive (Fig. 1)."""
    from tests._util import tiny_world
    from paper_2408_01584_amd import scenes as S
    p = S.SimParams(top_k=4, partners=2, obs_radius=50.0)
    sc = tiny_world([(0.0, 0.0, 0.0, 4.5, 2.0), (30.0, 40.0, 0.0, 4.5, 2.0), (50.0, 0.0, 0.0, 4.5, 2.0),
                     ], params=p)
    for d32 in (False, True):
        r = oracle_mod.OracleSim(sc, decide32=d32).reset()
        # agent 0: slot 0 = agent 1 at (30, 40), slot 1 = agent 2 at (50, 0): both at 50 m
        assert list(r["pmask"][:2]) == [1, 1], d32
        # agent 1 sees agent 0 (50 m) but not agent 2 (sqrt(20^2 + 40^2) = 44.7 m: seen too)
        assert list(r["pmask"][2:4]) == [1, 1], d32
        assert r["band"][0] & 4  # and it is marked as a near-threshold decision


def test_partner_just_beyond_radius_is_not_observed(oracle_mod):
    from tests._util import tiny_world
    from paper_2408_01584_amd import scenes as S
    p = S.SimParams(top_k=4, partners=1, obs_radius=50.0)
    sc = tiny_world([(0.0, 0.0, 0.0, 4.5, 2.0), (50.001, 0.0, 0.0, 4.5, 2.0)], params=p)
    for d32 in (False, True):
        r = oracle_mod.OracleSim(sc, decide32=d32).reset()
        assert list(r["pmask"]) == [0, 0], d32


@pytest.mark.parametrize("cfg,worlds,steps", [(0, None, 91), (1, [0, 1, 2, 3, 4, 5, 6, 7], 12),
                                               (2, [0, 1, 2, 3, 4, 5, 6, 7], 10)])
def test_binary32_decisions_with_penalty_and_termination(oracle_mod, cfg, worlds, steps):
    """The same with a collision penalty and termination on collision (the settings of the
    GPU test of those rules): collisions end agents' episodes and finished worlds reset."""
    import dataclasses
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(cfg, worlds=worlds)
    sc.params = dataclasses.replace(sc.params, collision_penalty=0.5, terminate_on_collision=True)
    acts = S.make_actions(cfg, steps, sc.num_agents).astype(np.float64)
    st = _run(oracle_mod, sc, acts, steps)
    print("config %d with penalty and termination: %s" % (cfg, st))
    assert st["collisions"] > 0
    assert st["worlds_done"] > 0 or cfg != 0
