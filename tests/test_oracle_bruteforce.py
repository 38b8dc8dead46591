"""Brute-force enumeration on 4x4 grids: the oracle against the declarative
checker of tests/bruteforce_spec.py (one step from every enumerated state)."""
import numpy as np
import pytest

from oracle import oracle as o
from tests import bruteforce_spec as bf


def run_oracle(spec, st, acts):
    B = st["pos_x"].shape[0]
    table = np.tile(o.spec_table([spec]), (B, 1))
    b = o.OracleBatch(table)
    b.set_state(bf.flat_state(st))
    obs, rew, done = b.step(1, actions=acts.reshape(1, -1))
    return obs[0], rew[0], done[0], b.get_state()


FAMILIES = {
    "one_agent_all_walls_r1": lambda: bf.case_one_agent(r=1, C=4),
    "one_agent_r2_sample": lambda: bf.case_one_agent(r=2, C=3, subsample=200_000, seed=3),
    "one_agent_r4_sample": lambda: bf.case_one_agent(r=4, C=4, subsample=100_000, seed=4),
    "one_agent_truncate": lambda: bf.case_one_agent(r=1, C=3, L=1, subsample=50_000, seed=5),
    "seeker_hider_capture_off": lambda: bf.case_seeker_hider(n_patterns=256, flags=1),
    "seeker_hider_capture_on": lambda: bf.case_seeker_hider(n_patterns=64, flags=3, seed=2),
    "seeker_hider_r3_no_collide": lambda: bf.case_seeker_hider(n_patterns=32, r=3, C=4,
                                                               flags=0, seed=6),
    "three_agents_open": lambda: bf.case_three_agents(r=2, C=3, flags=1),
    "three_agents_capture": lambda: bf.case_three_agents(r=1, C=4, flags=3, S=1),
    "one_agent_occluded_r3": lambda: bf.case_one_agent(r=3, C=4, flags=8 | 3,
                                                       subsample=100_000, seed=7),
    "seeker_hider_occluded_r3": lambda: bf.case_seeker_hider(n_patterns=96, r=3, C=4,
                                                             flags=8 | 1, seed=8),
    "seeker_hider_occluded_capture": lambda: bf.case_seeker_hider(n_patterns=64, r=2, C=3,
                                                                  flags=8 | 3, seed=9),
}


@pytest.mark.parametrize("family", list(FAMILIES))
def test_oracle_bruteforce(family):
    spec, st, acts = FAMILIES[family]()
    obs, rew, done, new = run_oracle(spec, st, acts)
    bf.check_step(spec, st, acts, obs, rew, done, new)
    if spec["flags"] & 2 and spec["n"] > spec["S"]:
        assert (done & 1).any()  # the capture rule fired somewhere
