"""Pins of the oracle's rollout observation (the continuous features of the relative-frame
observation, Fig. 1 and Sec. 3.2 "Sensor modalities": own speed, goal in the own frame,
and per partner slot the partner's position in the own frame, heading difference and
speed) and of its vector-Jacobian product.

The observation couples the agents of a world (an agent's state enters its partners'
observations), so the central differences perturb one action of one agent at a time."""
import math

import numpy as np
import pytest

from tests._util import tiny_world

# The objective sums T x A x (3 + 4P) observation terms of size up to tens of metres, so
# the rounding noise of a difference quotient is about 1e-16 |J| / h: h = 1e-5 keeps it
# near 1e-7 while the truncation error stays far below the tolerance.
H = 1e-5


def _states(sc, x, y, yaw, v):
    st = np.zeros((2, 4, sc.num_agents))
    st[1] = np.array([x, y, yaw, v], dtype=np.float64)
    return st


def test_obs_closed_form(oracle_mod):
    """Hand-placed agents: rotations by 0 and pi/2, a partner exactly at the radius
    (inclusive), one beyond it, a heading difference across the wrap, slot order."""
    from paper_2408_01584_amd import scenes as S
    agents = [(0.0, 0.0, 0.0, 4.5, 2.0), (10.0, 5.0, math.pi / 2, 4.5, 2.0), (50.0, 0.0, 0.0, 4.5, 2.0),
              (0.0, -60.0, 3.0, 4.5, 2.0)]
    goals = [(20.0, 0.0), (10.0, 15.0), (50.0, 0.0), (0.0, -50.0)]
    sc = tiny_world(agents, edges=[[(-5, 20), (5, 20)]], goals=goals,
                    params=S.SimParams(top_k=8, partners=3, obs_radius=50.0))
    orc = oracle_mod.OracleSim(sc)
    x, y, yaw = [a[0] for a in agents], [a[1] for a in agents], [a[2] for a in agents]
    v = [2.0, 3.0, 4.0, 5.0]
    obs, band = orc.rollout_obs(_states(sc, x, y, yaw, v))
    o = obs[0]
    # agent 0: speed 2, goal 20 m ahead; partners 1 (10, 5, pi/2, 3), 2 at exactly 50 m
    # (50, 0, 0, 4), 3 beyond the radius (60 m)
    np.testing.assert_allclose(o[0, :3], [2.0, 20.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(o[0, 3:7], [10.0, 5.0, math.pi / 2, 3.0], atol=1e-12)
    np.testing.assert_allclose(o[0, 7:11], [50.0, 0.0, 0.0, 4.0], atol=1e-12)
    np.testing.assert_array_equal(o[0, 11:15], 0.0)
    # agent 1 heads along +y: the goal 10 m north is 10 m ahead; agent 0 at (-10, -5)
    # relative lies 5 m to the right... in its frame (-5, 10); agent 2 at (40, -5) -> (-5, -40)
    np.testing.assert_allclose(o[1, :3], [3.0, 10.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(o[1, 3:7], [-5.0, 10.0, -math.pi / 2, 2.0], atol=1e-12)
    np.testing.assert_allclose(o[1, 7:11], [-5.0, -40.0, -math.pi / 2, 4.0], atol=1e-12)
    # agent 3 (yaw 3.0) sees agent 0 (yaw 0) 60 m away: masked; slots skip itself
    np.testing.assert_array_equal(o[3, 3:7], 0.0)
    # agent 2 sees agent 0 at exactly 50 m behind it: (-50, 0), heading difference 0
    np.testing.assert_allclose(o[2, 3:7], [-50.0, 0.0, 0.0, 2.0], atol=1e-12)
    # the partner exactly at the radius is a decision at its threshold: marked
    assert band[0, 0] == 1 and band[0, 2] == 1 and band[0, 1] == 0


def test_obs_heading_difference_wraps(oracle_mod):
    from paper_2408_01584_amd import scenes as S
    agents = [(0.0, 0.0, 3.0, 4.5, 2.0), (10.0, 0.0, -3.0, 4.5, 2.0)]
    sc = tiny_world(agents, params=S.SimParams(top_k=8, partners=1))
    obs, _ = oracle_mod.OracleSim(sc).rollout_obs(_states(sc, [0, 10], [0, 0], [3.0, -3.0], [1, 1]))
    assert obs[0, 0, 5] == pytest.approx(-6.0 + 2 * math.pi, abs=1e-12)
    assert obs[0, 1, 5] == pytest.approx(6.0 - 2 * math.pi, abs=1e-12)


def test_obs_equals_step_observation(oracle_mod):
    """The rollout observation of a state holds the same numbers as the step's ego and
    partner observations of that state (speed, goal x', goal y'; x', y', heading
    difference, speed per slot), which the observation pins cover on their own."""
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(3, worlds=2)
    acts = S.make_actions(3, 3, sc.num_agents).astype(np.float64)
    orc = oracle_mod.OracleSim(sc)
    ro = orc.rollout(acts, obs=True)
    P = sc.params.partners
    for t in range(3):
        st = ro["states"][t + 1]
        o2 = oracle_mod.OracleSim(sc)
        o2.set_state(st[0], st[1], st[2], st[3])
        ob = o2.obs()
        o = ro["obs"][t]
        np.testing.assert_allclose(o[:, 0], ob["ego"][:, 0], rtol=0, atol=1e-12)
        np.testing.assert_allclose(o[:, 1:3], ob["ego"][:, 3:5], rtol=0, atol=1e-12)
        part = ob["partner"].reshape(sc.num_agents, P, 6)[:, :, :4]
        np.testing.assert_allclose(o[:, 3:].reshape(sc.num_agents, P, 4), part, rtol=0, atol=1e-12)


@pytest.fixture(scope="module")
def world32():
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(3, worlds=1)  # 32 agents, 31 partner slots
    acts = S.make_actions(3, 6, sc.num_agents).astype(np.float64)
    return sc, acts


def _objective(orc, acts, gr, go):
    r = orc.rollout(acts, obs=True)
    return float((r["rewards"] * gr).sum() + (r["obs"] * go).sum())


def test_vjp_with_obs_matches_central_differences(oracle_mod, world32):
    sc, acts = world32
    orc = oracle_mod.OracleSim(sc)
    T, A = acts.shape[0], sc.num_agents
    rng = np.random.default_rng(11)
    gr = rng.uniform(0.5, 1.5, (T, A))
    go = rng.normal(0.0, 1.0, (T, A, orc.obs_features()))
    ref = orc.rollout(acts, tol=1e-5, obs=True)
    # no decision of this rollout sits at its threshold, so every partial is compared
    assert ref["unstable"].sum() == 0 and ref["obs_band"].sum() == 0
    # partners within the radius (about two per agent on this map): the coupling is exercised
    active = (np.abs(ref["obs"][:, :, 3:]).reshape(T, A, -1, 4).sum(-1) > 0).sum()
    assert active > 5 * T, active
    ga, _ = orc.rollout_vjp(acts, gr, go)
    fd = np.zeros_like(ga)
    for t in range(T):
        for i in range(A):
            for ch in range(2):
                p, m = acts.copy(), acts.copy()
                p[t, i, ch] += H
                m[t, i, ch] -= H
                fd[t, i, ch] = (_objective(orc, p, gr, go) - _objective(orc, m, gr, go)) / (2 * H)
    err = np.abs(ga - fd) / np.maximum(np.abs(fd), 1e-1)
    assert err.max() < 1e-5, err.max()
    # the observation terms change the gradient (they are not a no-op)
    ga0, _ = orc.rollout_vjp(acts, gr)
    assert np.abs(ga - ga0).max() > 1e-2


def test_vjp_with_zero_obs_gradient_equals_reward_vjp(oracle_mod, world32):
    sc, acts = world32
    orc = oracle_mod.OracleSim(sc)
    T, A = acts.shape[0], sc.num_agents
    gr = np.random.default_rng(2).uniform(0.5, 1.5, (T, A))
    a1, s1 = orc.rollout_vjp(acts, gr)
    a2, s2 = orc.rollout_vjp(acts, gr, np.zeros((T, A, orc.obs_features())))
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(s1, s2)
