"""Agent classes and parked agents on the GPU against the oracle (teacher-forced): a
batch with pedestrians and cyclists and with the "all nontrivial" initialisation parking
the agents that start near their goal, and the oracle's hand scenarios run on the GPU."""
import dataclasses

import numpy as np
import pytest
import torch

from tests._parity import compare_obs, teacher_forced_run
from tests._util import tiny_world

pytestmark = pytest.mark.gpu


def _sim(sc, params):
    from paper_2408_01584_amd.sim import Sim
    return Sim(sc, params=params)


@pytest.mark.parametrize("cfg,worlds,steps", [(1, 12, 4), (2, 24, 3), (0, None, 91)])
def test_classes_and_parked_agents_match_oracle(gpu, oracle_mod, cfg, worlds, steps):
    """20 % pedestrians, 10 % cyclists; agents starting within 45 m of their goal parked
    (goals lie 30-80 m ahead, so about 30 % are); auto-reset on."""
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(cfg, worlds=worlds) if worlds else S.make_scene(cfg)
    rng = np.random.default_rng(cfg)
    sc.agent_class = rng.choice(np.array([0, 1, 2], np.uint8), sc.num_agents, p=[0.7, 0.1, 0.2])
    p = dataclasses.replace(sc.params, min_goal_dist=45.0)
    sim = _sim(sc, p)
    g = sim.host_outputs()
    parked = (g["flags"] & oracle_mod.STATIC) != 0
    assert 0 < parked.sum() < sc.num_agents
    acts = S.make_actions(cfg, steps, sc.num_agents)
    st = teacher_forced_run(sc, sim, oracle_mod, acts, steps)
    g = sim.host_outputs()
    # parked agents never move, across auto-resets too
    assert np.array_equal(g["state"][:, parked], np.stack([sc.x, sc.y, sc.yaw, sc.speed])[:, parked])
    print("classes cfg %d: %d parked of %d," % (cfg, parked.sum(), sc.num_agents), st)


def test_parked_agent_scenario(gpu, oracle_mod):
    O = oracle_mod
    from paper_2408_01584_amd import scenes as S
    p = S.SimParams(top_k=4, partners=1, lidar_rays=8, episode_len=3, min_goal_dist=2.0)
    sc = tiny_world([(6.0, 0.0, 0.0, 4.5, 2.0), (12.0, 0.0, 0.0, 4.5, 2.0)],
                    goals=[(200.0, 0.0), (13.5, 0.0)], speeds=[10.0, 0.0], params=p)
    sim = _sim(sc, p)
    orc = O.OracleSim(sc, p)
    o = orc.reset()
    g = sim.host_outputs()
    assert g["flags"].tolist() == [O.ALIVE | O.VISIBLE, O.VISIBLE | O.STATIC]
    compare_obs(g, o, 4, 8)
    act = np.array([[40.0, 0.0], [5.0, 0.3]], np.float32)
    for k in range(3):
        sim.step(torch.as_tensor(act, device="cuda"))
        o = orc.step(act.astype(np.float64))
        g = sim.host_outputs()
        assert np.array_equal(g["flags"], o["flags"]), (k, g["flags"], o["flags"])
        assert np.array_equal(g["world_done"], o["world_done"])
        compare_obs(g, o, 4, 8)
    assert g["world_done"][0] == 1 and g["flags"][1] & O.STATIC


def test_pedestrian_crosses_edge(gpu, oracle_mod):
    O = oracle_mod
    agents = [(0.0, 0.0, 0.0, 4.5, 2.0), (30.0, 0.0, 0.0, 4.5, 2.0), (60.0, 0.3, 0.0, 0.8, 0.8),
              (61.0, 0.3, 0.0, 4.5, 2.0)]
    sc = tiny_world(agents, edges=[[(-50.0, 0.5), (100.0, 0.5)]])
    sc.agent_class = np.array([O.VEHICLE, O.CYCLIST, O.PEDESTRIAN, O.VEHICLE], np.uint8)
    sim = _sim(sc, sc.params)
    sim.step(torch.zeros((4, 2), device="cuda"))
    g = sim.host_outputs()
    o = O.OracleSim(sc).step(np.zeros((4, 2)))
    assert np.array_equal(g["flags"], o["flags"])
    assert not g["flags"][2] & O.COLL_EDGE and g["flags"][2] & O.COLL_AGENT and g["flags"][0] & O.COLL_EDGE


def test_graph_mode_with_every_option(gpu):
    """The HIP-graph step with the simplified model, a view cone turned every step, agent
    classes and parked agents gives the same bits as direct launches."""
    import math
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    sc = S.make_scene(4, worlds=[1, 2, 3])
    rng = np.random.default_rng(4)
    sc.agent_class = rng.choice(np.array([0, 1, 2], np.uint8), sc.num_agents)
    p = dataclasses.replace(sc.params, dynamics=1, lidar_fov=math.radians(100.0), min_goal_dist=40.0)
    acts = torch.as_tensor(S.make_delta_actions(4, 5, sc.num_agents), device="cuda")
    heads = torch.as_tensor(rng.uniform(-2, 2, (5, sc.num_agents)).astype(np.float32), device="cuda")
    ref = Sim(sc, params=p)
    gr = Sim(sc, params=p, graph=True)
    for k in range(5):
        for s in (ref, gr):
            s.buf["lidar_head"][:sc.num_agents].copy_(heads[k])
            s.step(acts[k])
        a, b = ref.host_outputs(), gr.host_outputs()
        for n in a:
            assert np.array_equal(a[n], b[n]), (k, n)
    assert (a["flags"] & 64).any() and (a["lidar_hit"] == 2).any()
