"""The collision penalty and termination on collision (Sec. 3.2 "Rewards", "Termination")
on the GPU against the FP64 oracle, teacher-forced with auto-reset on: a collided agent's
reward carries the penalty, it is done and removed, and worlds whose agents have all
finished reset in the same step."""
import dataclasses

import numpy as np
import pytest

from tests._parity import teacher_forced_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,worlds,steps", [(0, None, 91), (1, [0, 1, 2, 3, 4, 5, 6, 7], 12),
                                               (2, [0, 1, 2, 3, 4, 5, 6, 7], 10)])
def test_penalty_and_termination_match_oracle(gpu, oracle_mod, cfg, worlds, steps):
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    sc = S.make_scene(cfg, worlds=worlds) if worlds else S.make_scene(cfg)
    p = dataclasses.replace(sc.params, collision_penalty=0.5, terminate_on_collision=True,
                            auto_reset=True)
    sc.params = p
    sim = Sim(sc, params=p)
    acts = S.make_actions(cfg, steps, sc.num_agents)
    st = teacher_forced_run(sc, sim, oracle_mod, acts, steps)
    print("penalty + termination, config %d:" % cfg, st)
    # the paths under test ran: agents collided (and were removed), worlds finished
    assert st["collisions"] > 0
    assert st["worlds_done"] > 0 or cfg != 0


def test_penalty_without_termination_keeps_agents(gpu, oracle_mod):
    """Without termination a collided agent keeps driving and keeps its penalty while it
    overlaps."""
    from paper_2408_01584_amd import scenes as S
    from paper_2408_01584_amd.sim import Sim
    sc = S.make_scene(1, worlds=[3, 4, 5, 6])
    p = dataclasses.replace(sc.params, collision_penalty=0.25, terminate_on_collision=False)
    sc.params = p
    sim = Sim(sc, params=p)
    acts = S.make_actions(1, 10, sc.num_agents)
    st = teacher_forced_run(sc, sim, oracle_mod, acts, 10)
    print("penalty only:", st)
    assert st["collisions"] > 0
    g = sim.host_outputs()
    hit = (g["flags"] & 3) != 0
    np.testing.assert_array_equal(g["reward"][hit & ((g["flags"] & 4) == 0)], -0.25)
