"""Pins of the oracle's differentiable rollout: the hand-derived vector-Jacobian
product against FP64 central finite differences (h = 1e-6) and a one-step closed form.

The smooth reward is r = -|goal - p| - softplus(s), with s the signed distance to the
nearest road edge (positive off-road), an instance of the configurable agent-road
distance rewards of Sec. 3.2 "Rewards"; the dynamics are App. B.
"""
import math

import numpy as np
import pytest

H = 1e-6


@pytest.fixture(scope="module")
def cfg3():
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(3, worlds=4)
    acts = S.make_actions(3, 20, sc.num_agents)
    return sc, acts.astype(np.float64)


def test_vjp_matches_central_differences(oracle_mod, cfg3):
    """Agents' objectives are independent (no interaction terms in the reward), so one
    pair of perturbed rollouts per (step, action channel), moving every agent at once,
    gives every agent's partial derivative."""
    sc, acts = cfg3
    sim = oracle_mod.OracleSim(sc)
    T, A = acts.shape[0], sc.num_agents
    rng = np.random.default_rng(7)
    gr = rng.uniform(0.5, 1.5, (T, A))
    ref = sim.rollout(acts, tol=1e-5)
    ga, g0 = sim.rollout_vjp(acts, gr)
    stable = ref["unstable"] == 0
    assert stable.sum() > 0.7 * A, stable.sum()
    fd = np.zeros_like(ga)
    for t in range(T):
        for ch in range(2):
            p, m = acts.copy(), acts.copy()
            p[t, :, ch] += H
            m[t, :, ch] -= H
            jp = (sim.rollout(p)["rewards"] * gr).sum(0)
            jm = (sim.rollout(m)["rewards"] * gr).sum(0)
            fd[t, :, ch] = (jp - jm) / (2 * H)
    err = np.abs(ga - fd)[:, stable]
    scale = np.maximum(np.abs(fd[:, stable]), 1e-1)
    assert np.max(err / scale) < 1e-5, np.max(err / scale)
    # the off-road term is active for some agents (gradients differ from goal-only)
    assert np.any(ref["seg"] >= 0)


def test_vjp_initial_state_matches_central_differences(oracle_mod, cfg3):
    sc, acts = cfg3
    sim = oracle_mod.OracleSim(sc)
    T, A = acts.shape[0], sc.num_agents
    gr = np.ones((T, A))
    ref = sim.rollout(acts, tol=1e-5)
    _, g0 = sim.rollout_vjp(acts, gr)
    stable = ref["unstable"] == 0
    base = [sim.x.copy(), sim.y.copy(), sim.yaw.copy(), sim.v.copy()]
    for q, arr in enumerate((sim.x, sim.y, sim.yaw, sim.v)):
        arr[:] = base[q] + H
        jp = sim.rollout(acts)["rewards"].sum(0)
        arr[:] = base[q] - H
        jm = sim.rollout(acts)["rewards"].sum(0)
        arr[:] = base[q]
        fd = (jp - jm) / (2 * H)
        err = np.abs(g0[q] - fd)[stable] / np.maximum(np.abs(fd[stable]), 1e-1)
        assert np.max(err) < 1e-5, (q, np.max(err))


def test_one_step_goal_gradient_closed_form(oracle_mod):
    """No road edge within the radius (s = -R, constant): r_0 = -|g - p_1| and
    dr/da = (g - p_1)/|g - p_1| . (dt^2/2) (cos(yaw + beta), sin(yaw + beta)) while the
    midpoint speed is unclipped."""
    from tests._util import tiny_world
    sc = tiny_world([(0.0, 0.0, 0.4, 4.5, 2.0)], goals=[(30.0, 20.0)], speeds=[6.0],
                    edges=[[(500.0, 0.0), (501.0, 0.0)]])
    sim = oracle_mod.OracleSim(sc)
    a, d = 1.2, 0.15
    acts = np.array([[[a, d]]])
    ga, _ = sim.rollout_vjp(acts, np.ones((1, 1)))
    out = sim.rollout(acts)
    x1, y1 = out["states"][1, 0, 0], out["states"][1, 1, 0]
    beta = math.atan(0.5 * math.tan(d))
    u = np.array([30.0 - x1, 20.0 - y1]) / math.hypot(30.0 - x1, 20.0 - y1)
    want = u @ (0.5 * 0.01 * np.array([math.cos(float(np.float32(0.4)) + beta), math.sin(float(np.float32(0.4)) + beta)]))
    np.testing.assert_allclose(ga[0, 0, 0], want, rtol=1e-12)
    np.testing.assert_allclose(out["rewards"][0, 0], -math.hypot(30.0 - x1, 20.0 - y1) - math.log1p(math.exp(-50.0)),
                               rtol=1e-14)


def test_offroad_sign_convention(oracle_mod):
    """An edge polyline has the drivable area on its left: a point on its right is
    off-road (positive signed distance, lower reward)."""
    from tests._util import tiny_world
    edge = [[(-100.0, 0.0), (100.0, 0.0)]]  # runs +x: left (+y) is drivable
    on = tiny_world([(0.0, 3.0, 0.0, 4.5, 2.0)], goals=[(0.0, 3.0)], edges=edge)
    off = tiny_world([(0.0, -3.0, 0.0, 4.5, 2.0)], goals=[(0.0, -3.0)], edges=edge)
    z = np.zeros((1, 1, 2))
    r_on = oracle_mod.OracleSim(on).rollout(z)["rewards"][0, 0]
    r_off = oracle_mod.OracleSim(off).rollout(z)["rewards"][0, 0]
    np.testing.assert_allclose(r_on, -math.log1p(math.exp(-3.0)), rtol=1e-12)
    np.testing.assert_allclose(r_off, -(3.0 + math.log1p(math.exp(-3.0))), rtol=1e-12)


def test_smooth_reward_ignores_edges_beyond_the_radius(oracle_mod):
    """With the only road edge just outside the observation radius the off-road term is
    the constant softplus(-R).  A small radius (3 m) makes the difference visible: the
    agent sits 3.5 m on the off-road side of the edge, where an edge inside the radius
    would give softplus(+3.5)."""
    from tests._util import tiny_world
    from paper_2408_01584_amd import scenes as S
    p = S.SimParams(top_k=4, partners=0, obs_radius=3.0)
    edge = [[(-100.0, 0.0), (100.0, 0.0)]]  # runs +x: the drivable side is +y
    goal = (0.0, -3.5)
    out = tiny_world([(0.0, -3.5, 0.0, 4.5, 2.0)], goals=[goal], edges=edge, params=p)
    r = oracle_mod.OracleSim(out).rollout(np.zeros((1, 1, 2)))
    assert r["seg"][0, 0] == -1
    np.testing.assert_allclose(r["rewards"][0, 0], -math.log1p(math.exp(-3.0)), rtol=1e-12)
    # 2.5 m away the edge is inside the radius and the agent is off-road: s = +2.5
    inside = tiny_world([(0.0, -2.5, 0.0, 4.5, 2.0)], goals=[(0.0, -2.5)], edges=edge, params=p)
    r = oracle_mod.OracleSim(inside).rollout(np.zeros((1, 1, 2)))
    assert r["seg"][0, 0] == 0
    np.testing.assert_allclose(r["rewards"][0, 0], -(2.5 + math.log1p(math.exp(-2.5))), rtol=1e-12)


def test_nearest_edge_ties_take_the_lowest_index(oracle_mod):
    """Two edge segments at exactly the same distance, one with the agent on its off-road
    side and one with it on its drivable side: the lower road index decides the sign of
    the off-road distance (r = -softplus(+1) or -softplus(-1))."""
    from tests._util import tiny_world
    above = [(-10.0, 1.0), (10.0, 1.0)]    # agent on its right: off-road, s = +1
    below = [(-10.0, -1.0), (10.0, -1.0)]  # agent on its left: on-road, s = -1
    for edges, want_seg, s in (([above, below], 0, 1.0), ([below, above], 0, -1.0)):
        sc = tiny_world([(0.0, 0.0, 0.0, 4.5, 2.0)], goals=[(0.0, 0.0)], edges=edges)
        r = oracle_mod.OracleSim(sc).rollout(np.zeros((1, 1, 2)))
        assert r["seg"][0, 0] == want_seg
        softplus = max(s, 0.0) + math.log1p(math.exp(-abs(s)))
        np.testing.assert_allclose(r["rewards"][0, 0], -softplus, rtol=1e-12)
