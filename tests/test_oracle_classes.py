"""Pins of the oracle's agent classes and "all nontrivial" initialisation (Sec. 3.2: cars
and cyclists collide with road edges, pedestrians may cross them; only agents that start
more than a set distance -- 2 m in the paper -- from their goal are controlled, the others
stay in the scene as parked obstacles).  Hand scenarios."""
import dataclasses

import numpy as np

from tests._util import tiny_world


def _sim(oracle_mod, sc, classes=None, **kw):
    if classes is not None:
        sc.agent_class = np.asarray(classes, np.uint8)
    p = dataclasses.replace(sc.params, **kw) if kw else sc.params
    return oracle_mod.OracleSim(sc, p)


def test_pedestrians_cross_road_edges(oracle_mod):
    """Three boxes straddling an edge line (far apart from each other): the vehicle and the
    cyclist collide with the edge, the pedestrian does not; a pedestrian still collides
    with another agent."""
    O = oracle_mod
    agents = [(0.0, 0.0, 0.0, 4.5, 2.0), (30.0, 0.0, 0.0, 4.5, 2.0), (60.0, 0.3, 0.0, 0.8, 0.8),
              (61.0, 0.3, 0.0, 4.5, 2.0)]
    sc = tiny_world(agents, edges=[[(-50.0, 0.5), (100.0, 0.5)]])
    orc = _sim(O, sc, classes=[O.VEHICLE, O.CYCLIST, O.PEDESTRIAN, O.VEHICLE])
    r = orc.step(np.zeros((4, 2)))
    f = r["flags"]
    assert f[0] & O.COLL_EDGE and f[1] & O.COLL_EDGE
    assert not f[2] & O.COLL_EDGE and f[2] & O.COLL_AGENT
    assert f[3] & O.COLL_AGENT and f[3] & O.COLL_EDGE
    # without classes every agent is a vehicle
    r0 = _sim(O, tiny_world(agents, edges=[[(-50.0, 0.5), (100.0, 0.5)]])).step(np.zeros((4, 2)))
    assert r0["flags"][2] & O.COLL_EDGE


def test_parked_agents(oracle_mod):
    """Agent 1 starts 1.5 m from its goal (min_goal_dist 2 m): it is parked (VISIBLE |
    STATIC), never moves, earns no reward although inside the goal radius, observes
    nothing, is seen by agent 0 as a partner and by its LIDAR, and blocks it; the world ends
    when agent 0 is done, and the auto-reset parks agent 1 again."""
    O = oracle_mod
    from paper_2408_01584_amd import scenes as S
    p = S.SimParams(top_k=4, partners=1, lidar_rays=8, episode_len=3)
    agents = [(6.0, 0.0, 0.0, 4.5, 2.0), (12.0, 0.0, 0.0, 4.5, 2.0)]
    sc = tiny_world(agents, goals=[(200.0, 0.0), (13.5, 0.0)], speeds=[10.0, 0.0], params=p)
    orc = _sim(O, sc, min_goal_dist=2.0)
    r = orc.reset()
    assert r["flags"].tolist() == [O.ALIVE | O.VISIBLE, O.VISIBLE | O.STATIC]
    assert np.all(r["ego"][1] == 0.0) and r["ego"][0, 7] == 1.0
    assert r["pmask"][0] == 1 and r["pmask"][1] == 0  # 0 sees 1; 1 observes nothing
    np.testing.assert_allclose(r["lidar"][0, 0], 12.0 - 2.25 - 6.0, atol=1e-9)  # forward ray
    assert r["lidar_hit"][0, 0] == 2 and np.all(r["lidar_hit"][1] == 0)
    # agent 0 (10 m/s, 1.5 m behind) accelerates into the parked car, touching it in the
    # second step; agent 1's action is ignored
    act = np.array([[40.0, 0.0], [5.0, 0.3]])
    r = orc.step(act)
    assert r["state"][0, 1] == 12.0 and r["state"][3, 1] == 0.0
    assert r["reward"][1] == 0.0 and r["flags"][1] == O.VISIBLE | O.STATIC
    r = orc.step(act)
    assert r["flags"][0] & O.COLL_AGENT and r["flags"][1] == O.VISIBLE | O.STATIC
    # episode length 3: the third step ends the world (agent 0 still driving) and resets
    r = orc.step(act)
    assert r["world_done"][0] == 1 and r["t"][0] == 0
    assert r["flags"][1] & (O.VISIBLE | O.STATIC) == O.VISIBLE | O.STATIC
    assert r["flags"][0] & O.ALIVE


def test_world_with_only_parked_agents_ends_at_once(oracle_mod):
    O = oracle_mod
    sc = tiny_world([(0.0, 0.0, 0.0, 4.5, 2.0)], goals=[(1.0, 0.0)])
    orc = _sim(O, sc, min_goal_dist=2.0, auto_reset=False)
    r = orc.step(np.zeros((1, 2)))
    assert r["world_done"][0] == 1 and r["flags"][0] == O.VISIBLE | O.STATIC


def test_threshold_is_inclusive_and_off_by_default(oracle_mod):
    """Exactly 2 m from the goal is parked (only agents farther away are controlled);
    2.01 m is controlled; min_goal_dist 0 controls everybody."""
    O = oracle_mod
    sc = tiny_world([(0.0, 0.0, 0.0, 4.5, 2.0), (50.0, 0.0, 0.0, 4.5, 2.0), (90.0, 0.0, 0.0, 4.5, 2.0)],
                    goals=[(2.0, 0.0), (52.01, 0.0), (90.0, 0.0)])
    r = _sim(O, sc, min_goal_dist=2.0).reset()
    assert r["flags"].tolist() == [O.VISIBLE | O.STATIC, O.ALIVE | O.VISIBLE, O.VISIBLE | O.STATIC]
    r0 = _sim(O, sc).reset()
    assert r0["flags"].tolist() == [O.ALIVE | O.VISIBLE] * 3
