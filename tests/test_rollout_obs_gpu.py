"""The rollout's observation on the GPU against the FP64 oracle: the observation formed
from the GPU's own state log (teacher-forced: the oracle reads the same states), and the
backward kernel with an observation gradient against the oracle's vector-Jacobian
product (pinned on the CPU by central differences that perturb one agent at a time).

The observation couples the agents of a world through the partner slots, so a world in
which some partner distance comes within 1e-3 m of the radius on the FP64 trajectory (the
binary32 rollout may then mask it differently) is excluded from the gradient comparison
as a whole, with the reward-threshold exclusions of the rollout tests; both are counted."""
import numpy as np
import pytest
import torch

from tests._parity import assert_close

pytestmark = pytest.mark.gpu

REL = 1e-3


def _setup(worlds=4, T=20):
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    sc = S.make_scene(3, worlds=worlds)
    acts = S.make_actions(3, T, sc.num_agents)
    return sc, acts, Sim(sc)


def test_rollout_obs_matches_oracle(gpu, oracle_mod):
    sc, acts, sim = _setup()
    T, A = acts.shape[0], sc.num_agents
    rew, ck, st, obs = sim.rollout_fwd(torch.as_tensor(acts, device="cuda"), 10, obs=True)
    st, obs = st.cpu().numpy(), obs.cpu().numpy()
    F = 3 + 4 * sc.params.partners
    assert obs.shape == (T, A, F) and st.shape == (T, 4, A)
    # the log holds the states after each step: the checkpoint of step 10 is the state
    # after step 9
    np.testing.assert_array_equal(ck.cpu().numpy()[1], st[9])
    orc = oracle_mod.OracleSim(sc)
    full = np.concatenate([np.stack([sc.x, sc.y, sc.yaw, sc.speed])[None], st], 0).astype(np.float64)
    o, band = orc.rollout_obs(full)
    P = sc.params.partners
    m_g = np.abs(obs[:, :, 3:]).reshape(T, A, P, 4).sum(-1) > 0
    m_o = np.abs(o[:, :, 3:]).reshape(T, A, P, 4).sum(-1) > 0
    ok = band == 0
    assert band.mean() < 0.01, band.mean()
    assert np.array_equal(m_g[ok], m_o[ok]), "partner masks differ"
    assert_close(obs[ok][:, :3], o[ok][:, :3], "ego features")
    pg = obs[:, :, 3:].reshape(T, A, P, 4)[ok]
    po = o[:, :, 3:].reshape(T, A, P, 4)[ok]
    assert_close(pg[..., :2], po[..., :2], "partner position")
    assert_close(pg[..., 2], po[..., 2], "heading difference", angle=True)
    assert_close(pg[..., 3], po[..., 3], "partner speed")
    print("rollout obs: %d agent-steps compared, %d in the band, %d partner slots within the radius"
          % (ok.sum(), (~ok).sum(), m_g.sum()))


def _near_radius_worlds(sc, states, R, margin=1e-3):
    ao = np.asarray(sc.agent_off)
    bad = np.zeros(len(ao) - 1, bool)
    for w in range(len(ao) - 1):
        x, y = states[1:, 0, ao[w]:ao[w + 1]], states[1:, 1, ao[w]:ao[w + 1]]
        d = np.hypot(x[:, :, None] - x[:, None, :], y[:, :, None] - y[:, None, :])
        bad[w] = bool((np.abs(d - R) < margin).any())
    return bad


def test_rollout_obs_gradient_matches_oracle_vjp(gpu, oracle_mod):
    sc, acts, sim = _setup()
    T, A = acts.shape[0], sc.num_agents
    rng = np.random.default_rng(4)
    gr = rng.uniform(0.5, 1.5, (T, A)).astype(np.float32)
    go = rng.normal(0.0, 1.0, (T, A, 3 + 4 * sc.params.partners)).astype(np.float32)
    a_t = torch.as_tensor(acts, device="cuda")
    _, ck, st, _ = sim.rollout_fwd(a_t, 10, obs=True)
    ga, g0 = sim.rollout_bwd(a_t, ck, torch.as_tensor(gr, device="cuda"), 10, want_state0=True,
                             grad_obs=torch.as_tensor(go, device="cuda"), states=st)
    ga, g0 = ga.cpu().numpy(), g0.cpu().numpy()
    orc = oracle_mod.OracleSim(sc)
    ref = orc.rollout(acts.astype(np.float64), tol=1e-3)
    oga, og0 = orc.rollout_vjp(acts.astype(np.float64), gr.astype(np.float64), go.astype(np.float64))
    ao = np.asarray(sc.agent_off)
    world_of = np.repeat(np.arange(len(ao) - 1), np.diff(ao))
    bad_w = _near_radius_worlds(sc, ref["states"], sc.params.obs_radius)
    np.logical_or.at(bad_w, world_of, ref["unstable"] != 0)
    ok = ~bad_w[world_of]
    assert bad_w.sum() <= 1, bad_w
    num = np.linalg.norm((ga - oga)[:, ok].transpose(1, 0, 2).reshape(ok.sum(), -1), axis=1)
    den = np.linalg.norm(oga[:, ok].transpose(1, 0, 2).reshape(ok.sum(), -1), axis=1)
    rel = num / np.maximum(den, 1e-6)
    assert rel.max() < REL, rel.max()
    rel0 = np.linalg.norm(g0[:, ok] - og0[:, ok], axis=0) / np.maximum(np.linalg.norm(og0[:, ok], axis=0), 1e-6)
    assert rel0.max() < REL, rel0.max()
    # the observation terms change the gradient
    ga_r, _ = sim.rollout_bwd(a_t, ck, torch.as_tensor(gr, device="cuda"), 10)
    assert np.abs(ga_r.cpu().numpy() - ga).max() > 1e-2
    print("rollout bwd with grad_obs: %d/%d agents (%d worlds excluded), max per-agent rel err %.2e "
          "(state0 %.2e)" % (ok.sum(), ok.size, bad_w.sum(), rel.max(), rel0.max()))


def test_rollout_obs_gradient_checkpoint_invariant(gpu):
    sc, acts, sim = _setup(worlds=2)
    T, A = acts.shape[0], sc.num_agents
    a_t = torch.as_tensor(acts, device="cuda")
    go = torch.as_tensor(np.random.default_rng(6).normal(0, 1, (T, A, 3 + 4 * sc.params.partners)),
                         dtype=torch.float32, device="cuda")
    gr = torch.ones((T, A), device="cuda")
    outs = []
    for C in (1, 7, 20):
        _, ck, st, obs = sim.rollout_fwd(a_t, C, obs=True)
        ga, _ = sim.rollout_bwd(a_t, ck, gr, C, grad_obs=go, states=st)
        outs.append((obs.cpu().numpy(), ga.cpu().numpy()))
    for o, g in outs[1:]:
        assert np.array_equal(o, outs[0][0]) and np.array_equal(g, outs[0][1])


def test_autograd_function_with_obs(gpu):
    from paper_2408_01584_amd.sim import DiffRollout
    sc, acts, sim = _setup(worlds=2)
    a_t = torch.as_tensor(acts, device="cuda").requires_grad_(True)
    rew, obs = DiffRollout.apply(a_t, sim, 10, True)
    w1 = torch.linspace(0.5, 1.5, rew.numel(), device="cuda").reshape(rew.shape)
    w2 = torch.sin(torch.arange(obs.numel(), device="cuda", dtype=torch.float32)).reshape(obs.shape)
    ((rew * w1).sum() + (obs * w2).sum()).backward()
    _, ck, st, _ = sim.rollout_fwd(a_t.detach(), 10, obs=True)
    ga, _ = sim.rollout_bwd(a_t.detach(), ck, w1, 10, grad_obs=w2, states=st)
    assert torch.equal(a_t.grad, ga)


def test_rollout_obs_refused_for_ragged_partners(gpu):
    from paper_2408_01584_amd import gd as G
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    sc = S.make_scene(2, worlds=2)  # ragged partner slots
    sim = Sim(sc)
    with pytest.raises(G.GDError) as e:
        sim.rollout_fwd(torch.zeros((3, sc.num_agents, 2), device="cuda"), 10, obs=True)
    assert e.value.status == G.GD_E_UNSUPPORTED
