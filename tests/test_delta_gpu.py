"""The simplified bicycle model (Sec. 3.2 "Agent dynamics") on the GPU against the FP64 oracle:
the full step teacher-forced, the differentiable rollout and its backward kernel, and the
expert-action inversion element by element, plus a round trip of the inversion through
the GPU's own rollout."""
import dataclasses

import numpy as np
import pytest
import torch

from tests._parity import TOL, assert_close, teacher_forced_run

pytestmark = pytest.mark.gpu


def _delta_sim(sc, **launch):
    from paper_2408_01584_amd.sim import Sim
    p = dataclasses.replace(sc.params, dynamics=1)
    return Sim(sc, params=p, **launch), p


@pytest.mark.parametrize("cfg,worlds,steps", [(0, None, 6), (1, 24, 4), (2, 40, 3)])
def test_delta_step_teacher_forced(gpu, oracle_mod, cfg, worlds, steps):
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(cfg, worlds=worlds) if worlds else S.make_scene(cfg)
    acts = S.make_delta_actions(cfg, steps, sc.num_agents)
    sim, _ = _delta_sim(sc)
    st = teacher_forced_run(sc, sim, oracle_mod, acts, steps)
    print("delta step cfg %d:" % cfg, st)


def test_delta_rollout_and_gradient_match_oracle(gpu, oracle_mod):
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(3, worlds=4)
    T, A = 20, sc.num_agents
    acts = S.make_delta_actions(3, T, A)
    sim, p = _delta_sim(sc)
    a_t = torch.as_tensor(acts, device="cuda")
    rew, ckpt = sim.rollout_fwd(a_t, 10)
    gr = np.random.default_rng(3).uniform(0.5, 1.5, (T, A)).astype(np.float32)
    ga, g0 = sim.rollout_bwd(a_t, ckpt, torch.as_tensor(gr, device="cuda"), 10, want_state0=True)
    orc = oracle_mod.OracleSim(sc, p)
    o = orc.rollout(acts.astype(np.float64), tol=1e-3)
    oga, og0 = orc.rollout_vjp(acts.astype(np.float64), gr.astype(np.float64))
    ok = o["unstable"] == 0
    assert ok.mean() > 0.8, ok.mean()
    g = rew.cpu().numpy()
    err = np.abs(g[:, ok] - o["rewards"][:, ok]) / np.maximum(np.abs(o["rewards"][:, ok]), 1.0)
    assert err.max() < 1e-4, err.max()
    np.testing.assert_allclose(ckpt.cpu().numpy()[1], o["states"][10], rtol=1e-5, atol=1e-4)
    ga, g0 = ga.cpu().numpy(), g0.cpu().numpy()
    num = np.linalg.norm((ga - oga)[:, ok].transpose(1, 0, 2).reshape(ok.sum(), -1), axis=1)
    den = np.linalg.norm(oga[:, ok].transpose(1, 0, 2).reshape(ok.sum(), -1), axis=1)
    rel = num / np.maximum(den, 1e-6)
    assert rel.max() < 1e-3, rel.max()
    rel0 = np.linalg.norm(g0[:, ok] - og0[:, ok], axis=0) / np.maximum(np.linalg.norm(og0[:, ok], axis=0), 1e-6)
    assert rel0.max() < 1e-3, rel0.max()
    print("delta rollout: %d/%d agents, reward err %.2e, grad err %.2e, state0 %.2e" %
          (ok.sum(), ok.size, err.max(), rel.max(), rel0.max()))


def _log(oracle_mod, A, T, seed, wrap=False):
    """A binary32 log [T+1, 4, A] written by the oracle's simplified model from random
    commands, with some agents standing still and some reversing."""
    rng = np.random.default_rng(seed)
    x, y = rng.uniform(-200, 200, A), rng.uniform(-200, 200, A)
    yaw, v = rng.uniform(-np.pi, np.pi, A), rng.uniform(-4, 15, A)
    acc = rng.uniform(-1.5, 1.5, (T, A))
    curv = rng.uniform(-0.3, 0.3, (T, A))
    still = rng.random(A) < 0.05
    still[0] = True
    v[still] = 0.0
    acc[:, still] = 0.0
    out = [np.stack([x, y, yaw, v])]
    for t in range(T):
        x, y, yaw, v = oracle_mod.delta_dynamics(x, y, yaw, v, np.stack([acc[t], curv[t]], -1))
        out.append(np.stack([x, y, yaw, v]))
    st = np.stack(out)
    if wrap:
        st[:, 2] = (st[:, 2] + np.pi) % (2 * np.pi) - np.pi
    # standing agents whose logged heading still changes (sensor noise)
    st[1:, 2, still] += rng.uniform(-0.01, 0.01, (T, still.sum()))
    return np.ascontiguousarray(st.astype(np.float32))


def _check_inversion(g, o, band):
    # no step of these logs sits at a decision threshold of the inversion, so nothing is
    # excluded (a change that put steps there would show here first)
    ok = band == 0
    assert ok.all(), int((~ok).sum())
    assert_close(g[..., 0][ok], o[..., 0][ok], "accel")
    assert_close(g[..., 1][ok], o[..., 1][ok], "curvature")


@pytest.mark.parametrize("cfg,worlds,T,wrap", [(3, None, 20, False), (2, 64, 37, True),
                                               (0, None, 91, True), (3, 3, 1, False)])
def test_inversion_matches_oracle(gpu, oracle_mod, cfg, worlds, T, wrap):
    """Element by element at the tolerance of the step (1e-5 relative, floor 1), on the
    full rollout workload, on a ragged uneven batch (agents not a multiple of the
    workgroup, T not a multiple of the step chunk, wrapped headings), on one small world
    over a whole episode and for a single step."""
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(cfg, worlds=worlds) if worlds else S.make_scene(cfg)
    sim, _ = _delta_sim(sc)
    st = _log(oracle_mod, sc.num_agents, T, seed=10 + cfg, wrap=wrap)
    g = sim.invert_actions(torch.as_tensor(st, device="cuda")).cpu().numpy()
    o, band = oracle_mod.invert_actions(st.astype(np.float64), float(np.float32(sc.params.dt)))
    _check_inversion(g, o, band)
    # standing agents get a zero command on both sides
    d = 0.5 * (st[:-1, 3] + st[1:, 3]) * sc.params.dt
    z = np.abs(d) < 1e-4
    assert z.any() and np.all(g[..., 1][z] == 0.0)


def test_inversion_round_trip_through_gpu_rollout(gpu):
    """Log a GPU rollout (checkpoint every step), invert it on the GPU and replay the
    inverted commands: every logged state comes back within the step tolerance."""
    from paper_2408_01584_amd import scenes as S
    sc = S.make_scene(3, worlds=16)
    T, A = 30, sc.num_agents
    acts = torch.as_tensor(S.make_delta_actions(3, T + 1, A), device="cuda")
    sim, _ = _delta_sim(sc)
    _, log = sim.rollout_fwd(acts, 1)  # [T+1, 4, A]: the states before steps 0..T
    inv = sim.invert_actions(log.contiguous())
    _, replay = sim.rollout_fwd(torch.cat([inv, acts[T:]]).contiguous(), 1)
    rl, lg = replay.cpu().numpy(), log.cpu().numpy()
    # agents with a step shorter than 2 mm (speed crossing zero) cannot replay that
    # step's turn (the inversion leaves the command at zero there): not compared
    d = 0.5 * (lg[:-1, 3] + lg[1:, 3]) * sc.params.dt
    ok = (np.abs(d) >= 2e-3).all(0)
    assert ok.mean() > 0.9, ok.mean()
    np.testing.assert_allclose(inv.cpu().numpy()[:, ok], acts[:T].cpu().numpy()[:, ok], rtol=0, atol=1e-3)
    assert_close(rl[:, :, ok], lg[:, :, ok], "replayed states", tol=TOL)
    print("round trip: %d/%d agents" % (ok.sum(), ok.size))


def test_inversion_edge_cases(gpu):
    """T = 0 writes nothing; the bicycle model refuses inversion; overlapping buffers are
    refused; more steps than the limit are refused."""
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd import gd as G
    from paper_2408_01584_amd.sim import Sim
    sc = S.make_scene(0)
    sim, _ = _delta_sim(sc)
    assert sim.invert_actions(torch.zeros((1, 4, sc.num_agents), device="cuda")).shape == (0, sc.num_agents, 2)
    bic = Sim(sc)
    with pytest.raises(G.GDError) as e:
        bic.invert_actions(torch.zeros((3, 4, sc.num_agents), device="cuda"))
    assert e.value.status == G.GD_E_ARG
    buf = torch.zeros(64 * sc.num_agents, device="cuda")
    with pytest.raises(G.GDError) as e:
        G.gd_invert_actions(sim.handle, buf.data_ptr(), 3, buf.data_ptr() + 16, 0)
    assert e.value.status == G.GD_E_ARG
    with pytest.raises(G.GDError) as e:
        G.gd_invert_actions(sim.handle, buf.data_ptr(), (1 << 20) + 1, buf.data_ptr(), 0)
    assert e.value.status == G.GD_E_SIZE
