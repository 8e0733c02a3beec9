"""Planar LIDAR on the GPU against the oracle (teacher-forced) and against closed forms:
a wall seen at 10 / cos(a), a box 20 m ahead hit at 17.75 m (L = 4.5)."""
import math

import numpy as np
import pytest
import torch

from tests._parity import compare_obs, oracle_for, teacher_forced_run
from tests._util import tiny_world

pytestmark = pytest.mark.gpu


def _sim(scene, **kw):
    from paper_2408_01584_amd.sim import Sim
    return Sim(scene, **kw)


def test_lidar_cfg4_subset(gpu, oracle_mod):
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(4, worlds=[0, 9])
    acts = S.make_actions(4, 4, sc.num_agents)
    sim = _sim(sc)
    stats = teacher_forced_run(sc, sim, oracle_mod, acts, 4)
    g = sim.host_outputs()
    assert (g["lidar_hit"] == 1).any() and (g["lidar_hit"] == 2).any() and (g["lidar_hit"] == 0).any()
    print("lidar cfg4 subset:", stats)


def test_lidar_closed_forms(gpu, oracle_mod):
    from paper_2408_01584_amd import scenes as S
    p = S.SimParams(top_k=4, partners=1, lidar_rays=30, lidar_range=50.0)
    sc = tiny_world([(0.0, 0.0, 0.0, 4.5, 2.0)], edges=[[(10.0, -200.0), (10.0, 200.0)]], params=p)
    g = _sim(sc).host_outputs()
    ang = 2 * np.pi * np.arange(30) / 30
    want = np.where(np.cos(ang) >= 0.2, 10.0 / np.maximum(np.cos(ang), 1e-9), 50.0)
    np.testing.assert_allclose(g["lidar"][0], want, rtol=1e-5)
    np.testing.assert_array_equal(g["lidar_hit"][0], np.where(np.cos(ang) >= 0.2, 1, 0))
    sc2 = tiny_world([(0.0, 0.0, 0.5, 4.5, 2.0), (20.0 * math.cos(0.5), 20.0 * math.sin(0.5), 0.5, 4.5, 2.0)],
                     params=p)
    g2 = _sim(sc2).host_outputs()
    np.testing.assert_allclose(g2["lidar"][0, 0], 17.75, rtol=1e-5)
    assert g2["lidar_hit"][0, 0] == 2 and g2["lidar_hit"][0, 15] == 0 and g2["lidar"][0, 15] == 50.0
    np.testing.assert_allclose(g2["lidar"][1, 15], 17.75, rtol=1e-5)


def test_lidar_many_rays(gpu, oracle_mod):
    """N = 200 rays (several per lane) on a config-1 world."""
    from paper_2408_01584_amd import scenes as S
    import dataclasses
    sc = S.make_scene(1, worlds=[3])
    sc.params = dataclasses.replace(sc.params, lidar_rays=200, top_k=32, partners=63)
    sim = _sim(sc)
    g = sim.host_outputs()
    o = oracle_for(sc, g["state"], g["flags"], g["t"], oracle_mod).obs()
    compare_obs(g, o, 32, 200)


def _cone_run(sc, oracle_mod, fov, N, steps, seed, head_range=math.pi):
    """Step the GPU with a fresh random head angle per agent before every step (the
    head-rotation action) and compare each observation with the oracle's, teacher-forced."""
    import dataclasses
    from paper_2408_01584_amd import scenes as S
    sc.params = dataclasses.replace(sc.params, lidar_rays=N, lidar_fov=float(np.float32(fov)))
    sim = _sim(sc)
    acts = S.make_actions(4, steps, sc.num_agents)
    rng = np.random.default_rng(seed)
    hits = np.zeros(3, np.int64)
    for k in range(steps):
        head = rng.uniform(-head_range, head_range, sc.num_agents).astype(np.float32)
        sim.buf["lidar_head"][:sc.num_agents].copy_(torch.as_tensor(head))
        sim.step(torch.as_tensor(acts[k], device="cuda"))
        g = sim.host_outputs()
        orc = oracle_for(sc, g["state"], g["flags"], g["t"], oracle_mod, sim.params)
        orc.set_state(head=head)
        compare_obs(g, orc.obs(), sc.params.top_k, N)
        hits += np.bincount(g["lidar_hit"].ravel(), minlength=3)[:3]
    return hits


@pytest.mark.parametrize("fov_deg,N", [(120.0, 61), (360.0, 64), (0.6, 16), (90.0, 1)])
def test_view_cone_matches_oracle(gpu, oracle_mod, fov_deg, N):
    """View cones of 120 degrees (the paper's human view), the full turn, and a cone far
    narrower than the angle widening, on two worlds of the LIDAR workload, with the head
    turned at random before every step."""
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(4, worlds=[0, 9])
    hits = _cone_run(sc, oracle_mod, math.radians(fov_deg), N, 3, seed=int(fov_deg * 10))
    assert hits[1] > 0 and (hits[2] > 0 or N == 1), hits
    print("cone %.1f deg x %d rays: hit counts %s" % (fov_deg, N, hits.tolist()))


def test_view_cone_closed_form(gpu):
    """A wall x = 10 ahead, head turned by 0.3 rad: ray k of a 31-ray 120-degree cone hits
    at 10 / cos(0.3 + fov((k + 1/2)/31 - 1/2)) while in range."""
    from paper_2408_01584_amd import scenes as S
    fov = float(np.float32(math.radians(120.0)))
    p = S.SimParams(top_k=4, partners=1, lidar_rays=31, lidar_range=50.0, lidar_fov=fov)
    sc = tiny_world([(0.0, 0.0, 0.0, 4.5, 2.0)], edges=[[(10.0, -300.0), (10.0, 300.0)]], params=p)
    sim = _sim(sc)
    sim.buf["lidar_head"][0] = 0.3
    sim.obs()
    g = sim.host_outputs()
    ang = 0.3 + fov * ((np.arange(31) + 0.5) / 31 - 0.5)
    want = np.where(np.cos(ang) >= 0.2, 10.0 / np.maximum(np.cos(ang), 1e-9), 50.0)
    np.testing.assert_allclose(g["lidar"][0], want, rtol=1e-5)
    np.testing.assert_array_equal(g["lidar_hit"][0], np.where(np.cos(ang) >= 0.2, 1, 0))
