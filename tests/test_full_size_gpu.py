"""The uneven batch (1024 worlds, 1-128 agents, lognormal road sizes) and the LIDAR
workload (4096 worlds x 64 agents, 6000 points, 30 rays) at full size, in the launch
configuration the benchmark times, checked on a sample of worlds that the oracle
recomputes one by one (teacher-forced: from the GPU's state before the step, and the
observation of the GPU's state after it).

The LIDAR batch holds 64 generated worlds, each repeated 64 times: the same sizes and
launch shape as the benchmark's 4096 distinct worlds at 1/64 of the generation time."""
import numpy as np
import pytest
import torch

from tests._parity import check_bounds, compare_obs, compare_step, new_stats, oracle_for

pytestmark = pytest.mark.gpu


def _world(sc, out, w, P):
    ao = np.asarray(sc.agent_off, np.int64)
    a0, a1 = int(ao[w]), int(ao[w + 1])
    n = a1 - a0
    if P >= 0:
        s0, s1 = a0 * P, a1 * P
    else:
        m = np.diff(ao)
        s0 = int((m[:w] * (m[:w] - 1)).sum())
        s1 = s0 + n * (n - 1)
    r = {k: out[k][a0:a1] for k in ("ego", "road", "road_idx", "lidar", "lidar_hit", "reward", "flags")}
    r.update(partner=out["partner"][s0:s1], pmask=out["pmask"][s0:s1], world_done=out["world_done"][w:w + 1],
             t=out["t"][w:w + 1], state=out["state"][:, a0:a1])
    return r, a0, a1


def _check(sc, sim, oracle_mod, acts, sample, source):
    """one step of the full batch, then each sampled world against the oracle"""
    from paper_2408_01584_amd import scenes as S
    p = sim.params
    K, N, P = p.top_k, p.lidar_rays, p.partners
    pre = sim.host_outputs()
    sim.step(torch.as_tensor(acts, device="cuda"))
    post = sim.host_outputs()
    stats = new_stats()
    for w in sample:
        sub = S.make_scene(sc.cfg, worlds=[source(w)])
        gp, a0, a1 = _world(sc, pre, w, P)
        gq, _, _ = _world(sc, post, w, P)
        orc = oracle_for(sub, gp["state"], gp["flags"], gp["t"], oracle_mod, p)
        o = orc.step(acts[a0:a1].astype(np.float64))
        compare_step(gq, o, sub.agent_off, stats, "world %d" % w)
        orc2 = oracle_for(sub, gq["state"], gq["flags"], gq["t"], oracle_mod, p)
        compare_obs(gq, orc2.obs(), K, N, stats)
    check_bounds(stats)
    return stats


def test_uneven_batch_full_size_sampled(gpu, oracle_mod):
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    sc = S.make_scene(2)
    sim = Sim(sc)
    acts = S.make_actions(2, 4, sc.num_agents)
    for k in range(3):
        sim.step(torch.as_tensor(acts[k], device="cuda"))
    W = sc.num_worlds
    na, nr = np.diff(sc.agent_off), np.diff(sc.road_off)
    rng = np.random.default_rng(11)
    sample = sorted({0, W - 1, W // 2, int(na.argmax()), int(na.argmin()), int(nr.argmax()),
                     *rng.choice(W, 6, replace=False).tolist()})
    st = _check(sc, sim, oracle_mod, acts[3], sample, lambda w: w)
    print("uneven batch, %d worlds, %d sampled:" % (W, len(sample)), st)


def test_lidar_workload_full_size_sampled(gpu, oracle_mod):
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    spec = S.CONFIGS[4]
    base = [S.make_world(4, w, spec.worlds) for w in range(64)]
    sc = S.assemble(4, [base[i % 64] for i in range(spec.worlds)], spec.params,
                    world_ids=[i % 64 for i in range(spec.worlds)])
    assert sc.num_agents == 262144 and sc.num_road == 24576000
    sim = Sim(sc)
    acts = S.make_actions(4, 3, sc.num_agents)
    for k in range(2):
        sim.step(torch.as_tensor(acts[k], device="cuda"))
    sample = [0, 63, 64 * 17 + 5, 2048 + 40, spec.worlds - 1]
    st = _check(sc, sim, oracle_mod, acts[2], sample, lambda w: w % 64)
    print("LIDAR workload, 4096 worlds, %d sampled:" % len(sample), st)
