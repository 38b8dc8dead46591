"""The oracle against hand-worked single steps (tests/golden/hand_worked.json)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as o

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_worked.json")
CASES = json.load(open(GOLDEN))["cases"]


def load_case(case):
    """(spec dict, state dict) of a golden case; one env, seed 0, env id 0."""
    sp = dict(case["spec"])
    sp.setdefault("wall_pct", 0)
    H, W, n = sp["H"], sp["W"], sp["n"]
    walls = np.zeros(H * W, np.uint8)
    for x, y in case["walls"]:
        walls[y * W + x] = 1
    st = dict(walls=walls,
              pos_x=np.array([p[0] for p in case["pos"]], np.uint8),
              pos_y=np.array([p[1] for p in case["pos"]], np.uint8),
              found=np.array([case["found"]], np.uint32),
              t=np.array([case["t"]], np.uint32),
              episode=np.zeros(1, np.uint32), steps=np.zeros(1, np.uint32),
              seed=np.zeros(1, np.uint64), env_id=np.zeros(1, np.uint32))
    assert len(case["actions"]) == n
    return sp, st


def check_case(case, obs, rew, done, state):
    n, C = case["spec"]["n"], case["spec"]["C"]
    if "expect_pos" in case:
        assert [[int(a), int(b)] for a, b in zip(state["pos_x"], state["pos_y"])] == case["expect_pos"]
    if "expect_rew" in case:
        assert rew.tolist() == case["expect_rew"]
        assert not np.any(np.signbit(rew[rew == 0]))
    if "expect_done" in case:
        assert int(done[0]) == case["expect_done"]
    if "expect_found" in case:
        assert int(state["found"][0]) == case["expect_found"]
    if "expect_t" in case:
        assert int(state["t"][0]) == case["expect_t"]
    if "expect_episode" in case:
        assert int(state["episode"][0]) == case["expect_episode"]
    if "expect_obs" in case:
        got = obs.reshape(n, C)
        want = np.array([[int(h, 16) for h in row] for row in case["expect_obs"]], np.uint32)
        assert np.array_equal(got, want), (got, want)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_oracle_hand_worked(case):
    sp, st = load_case(case)
    b = o.OracleBatch([sp])
    b.set_state(st)
    obs, rew, done = b.step(1, actions=np.array([case["actions"]], np.int8))
    check_case(case, obs[0], rew[0], done[0], b.get_state())
    assert int(b.steps[0]) == 1
