"""Edge cases of the GPU step against the oracle: masked reset, padding when fewer than K
road points are in range, the largest K, the exact slow path of the top-K selection
(a distance bin too large to stage), exact ties, empty worlds and worlds without road,
agents far from every road point, determinism, and the non-finite-action check."""
import math

import numpy as np
import pytest
import torch

from tests._parity import compare_obs, oracle_for, teacher_forced_run

pytestmark = pytest.mark.gpu


def _sim(scene, **kw):
    from paper_2408_01584_amd.sim import Sim
    return Sim(scene, **kw)


def _params(**kw):
    from paper_2408_01584_amd import scenes as S
    base = dict(top_k=16, partners=3)
    base.update(kw)
    return S.SimParams(**base)


def test_masked_reset(gpu, oracle_mod):
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(1, worlds=3)
    acts = S.make_actions(1, 5, sc.num_agents)
    sim = _sim(sc)
    for k in range(5):
        sim.step(torch.as_tensor(acts[k], device="cuda"))
    pre = sim.host_outputs()
    mask = torch.tensor([0, 1, 0], dtype=torch.uint8, device="cuda")
    sim.reset(mask)
    g = sim.host_outputs()
    orc = oracle_for(sc, pre["state"], pre["flags"], pre["t"], oracle_mod)
    o = orc.reset(mask=np.array([0, 1, 0], np.uint8))
    assert list(g["t"]) == list(o["t"]) == [5, 0, 5]
    np.testing.assert_array_equal(g["state"], o["state"].astype(np.float32))
    np.testing.assert_array_equal(g["flags"], o["flags"])
    compare_obs(g, o, sc.params.top_k)


def test_pruned_radius_redo_after_external_move(gpu, oracle_mod):
    """The road top-K searches a radius derived from each agent's previous K-th key and how
    far it moved in the step.  Agents moved outside the step (the caller writing the state
    buffers) can have fewer than K points within that radius, which must send them back to
    the full radius: gd_obs after such a move, and the steps after it, match the oracle."""
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(1, worlds=2)
    acts = S.make_actions(1, 6, sc.num_agents)
    sim = _sim(sc)
    for k in range(3):
        sim.step(torch.as_tensor(acts[k], device="cuda"))
    b = sim.buf
    b["x"][0::3] += 30.0   # into other parts of the map
    b["y"][1::3] -= 60.0
    b["x"][2::7] += 1000.0  # far from every road point: fewer than K in the full radius
    sim.obs()
    g = sim.host_outputs()
    orc = oracle_for(sc, g["state"], g["flags"], g["t"], oracle_mod)
    compare_obs(g, orc.obs(), sc.params.top_k)
    assert (g["road_idx"][2::7] == -1).all()
    st = teacher_forced_run(sc, sim, oracle_mod, acts[3:], 3)
    print("after external move:", st)


def test_padding_and_max_k(gpu, oracle_mod):
    """K = 960 (the maximum): every agent of the 500-point scene has fewer candidates."""
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(0)
    sc.params = _params(top_k=960, partners=7)
    acts = S.make_actions(0, 4, sc.num_agents)
    sim = _sim(sc)
    teacher_forced_run(sc, sim, oracle_mod, acts, 4)
    g = sim.host_outputs()
    assert (g["road_idx"] == -1).any() and (g["road_idx"] >= 0).sum(1).max() <= 500


def _ring_world(n_ring=3000, radius=10.0, dup=40, extra=200, seed=0):
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0, 2 * np.pi, n_ring)
    pts = [(radius * math.cos(a), radius * math.sin(a)) for a in ang]
    pts += [(3.0, 4.0)] * dup                                   # exact duplicates (ties)
    pts += [tuple(v) for v in rng.uniform(-40, 40, (extra, 2))]
    return pts


@pytest.mark.parametrize("K,n_ring", [(100, 3000), (960, 800)])
def test_topk_slow_path_and_ties(gpu, oracle_mod, K, n_ring):
    """3000 points at one distance fall into a single distance bin much larger than the
    staging buffer (K = 100), so the cut bin is taken element by element; 40 duplicates
    test the index tie-break.  K = 960 with an 800-point ring stages the whole ring."""
    from tests._util import tiny_world
    pts = _ring_world(n_ring=n_ring)
    road = [(x, y, 0.1, 0 | 256) for (x, y) in pts]
    sc = tiny_world([(0.0, 0.0, 0.3, 4.5, 2.0), (1.0, 1.0, -0.2, 4.5, 2.0)], extra_road=road,
                    params=_params(top_k=K, partners=1))
    sim = _sim(sc)
    g = sim.host_outputs()
    o = oracle_for(sc, g["state"], g["flags"], g["t"], oracle_mod).obs()
    compare_obs(g, o, K)
    assert (g["road_idx"][0] >= 0).sum() == min(K, len(pts))


def test_empty_worlds_and_no_road(gpu, oracle_mod):
    """A batch with a world without agents, a world without road points, and an agent
    1 km away from every road point."""
    from paper_2408_01584_amd import scenes as S
    w0 = S.make_world(1, 0, 256)
    empty = {k: (np.zeros(0) if k != "road_meta" else np.zeros(0, np.int32)) for k in w0}
    empty.update(road_x=w0["road_x"][:50], road_y=w0["road_y"][:50], road_dir=w0["road_dir"][:50],
                 road_meta=w0["road_meta"][:50].copy())
    empty["road_meta"][-1] |= S.META_LAST
    noroad = {k: v for k, v in S.make_world(1, 1, 256).items()}
    for k in ("road_x", "road_y", "road_dir"):
        noroad[k] = np.zeros(0)
    noroad["road_meta"] = np.zeros(0, np.int32)
    far = {k: np.array(v, copy=True) for k, v in S.make_world(1, 2, 256).items()}
    far["x"][0] += 1000.0
    sc = S.assemble(1, [w0, empty, noroad, far], _params(top_k=200, partners=63))
    acts = S.make_actions(1, 3, sc.num_agents)
    sim = _sim(sc)
    teacher_forced_run(sc, sim, oracle_mod, acts, 3)
    g = sim.host_outputs()
    a2 = sc.agent_off[2]
    assert np.all(g["road_idx"][a2:sc.agent_off[3]] == -1)


def test_determinism(gpu):
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(2, worlds=[7, 8, 9, 10])
    acts = torch.as_tensor(S.make_actions(2, 6, sc.num_agents), device="cuda")
    a, b = _sim(sc), _sim(sc)
    for k in range(6):
        a.step(acts[k])
        b.step(acts[k])
    x, y = a.host_outputs(), b.host_outputs()
    for key in x:
        assert np.array_equal(x[key], y[key]), key


def test_nonfinite_action_reported(gpu):
    """A NaN action (forced from the host) is flagged by gd_check when GD_CHECK_FINITE is
    set; every kernel still runs to completion on the NaN state."""
    from paper_2408_01584_amd import gd as G
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(0)
    sim = _sim(sc, check_finite=True)
    act = torch.zeros((sc.num_agents, 2), device="cuda")
    sim.step(act)
    sim.check()
    act[3, 1] = float("nan")  # NaN steering propagates into the pose
    sim.step(act)
    with pytest.raises(G.GDError) as e:
        sim.check()
    assert e.value.status == G.GD_E_NONFINITE
    sim.check()  # cleared
    g = sim.host_outputs()
    assert np.isnan(g["state"][0, 3]) and (g["road_idx"][3] == -1).all()


def test_large_world_32bit_point_indices(gpu, oracle_mod):
    """A world of 70 000 road points (more than 16-bit point indices hold) takes the kernel
    variant with 32-bit indices and the road read through the caches; the agents sit in the
    last of 140 copies of the 500-point scene, so their top-K indices exceed 65535."""
    from paper_2408_01584_amd import scenes as S
    base = S.make_scene(0)
    tiles = 140
    offs = [(1000.0 * (k % 12), 1000.0 * (k // 12)) for k in range(tiles)]
    sc = base.copy()
    sc.road_x = np.concatenate([base.road_x + ox for ox, _ in offs]).astype(base.road_x.dtype)
    sc.road_y = np.concatenate([base.road_y + oy for _, oy in offs]).astype(base.road_y.dtype)
    sc.road_dir = np.tile(base.road_dir, tiles)
    sc.road_meta = np.tile(base.road_meta, tiles)
    sc.road_off = np.array([0, base.num_road * tiles], np.int32)
    ox, oy = offs[-1]
    for name, o in (("x", ox), ("goal_x", ox), ("y", oy), ("goal_y", oy)):
        setattr(sc, name, (getattr(base, name) + o).astype(getattr(base, name).dtype))
    acts = S.make_actions(0, 3, sc.num_agents)
    sim = _sim(sc)
    st = teacher_forced_run(sc, sim, oracle_mod, acts, 3)
    g = sim.host_outputs()
    assert g["road_idx"].max() >= 65536
    print("70 000-point world:", st)
