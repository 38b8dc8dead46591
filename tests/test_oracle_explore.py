"""Pins of the oracle's exploration rule (flag 16, reading R27): a
hand-worked episode (tests/golden/explore_hand_worked.json) and a numpy
restatement of the discovery map and of the exploration rewards, checked
step by step on real multi-step trajectories with and without occlusion."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as o
from paper_2604_27162_amd import workloads as wl
from tests import bruteforce_spec as bf

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "explore_hand_worked.json")))
EXPLORE = 16


def check_hand_worked(libpath=None):
    sp = GOLD["spec"]
    b = o.OracleBatch([sp], libpath=libpath)
    st = b.get_state()
    st["walls"][:] = 0
    st["pos_x"][:] = GOLD["start"]["pos_x"]
    st["pos_y"][:] = GOLD["start"]["pos_y"]
    b.set_state(st)
    for a, want in zip(GOLD["actions"], GOLD["expected"]):
        _, rew, done, mp = b.step(1, actions=np.array([a], np.int8), maps=True)
        st = b.get_state()
        assert [int(st["pos_x"][0]), int(st["pos_y"][0])] == want["pos"], want["notes"]
        assert list(rew[0]) == want["rew"], want["notes"]
        assert list(mp[0]) == want["map"], want["notes"]
        assert done[0, 0] == 0


def test_hand_worked_episode():
    check_hand_worked()


def restated_step(spec, walls, xs, ys, old_map):
    """Numpy restatement for one env: the seekers' window cells (inside the
    map, visible when occluding) after the moves, each seeker's count of
    cells absent from old_map, and the new map."""
    H, W, S, r = spec["H"], spec["W"], spec["S"], spec["r"]
    D = 2 * r + 1
    seen = np.zeros((H, W), bool)
    fresh = np.zeros(spec["n"], np.int64)
    for i in range(min(S, spec["n"])):
        win = np.zeros((H, W), bool)
        vis = None
        if spec["flags"] & 8:
            vis = bf.visible_window(spec, walls[None], np.array([xs[i]]), np.array([ys[i]]))[0]
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                cx, cy = xs[i] + dx, ys[i] + dy
                if 0 <= cx < W and 0 <= cy < H and (vis is None or vis[dy + r, dx + r]):
                    win[cy, cx] = True
        fresh[i] = int((win & ~old_map).sum())
        seen |= win
    return fresh, old_map | seen


def map_words(spec, m):
    H, W = spec["H"], spec["W"]
    rw = (W + 31) // 32
    out = np.zeros(H * rw, np.uint32)
    for y in range(H):
        for x in range(W):
            if m[y, x]:
                out[y * rw + (x >> 5)] |= np.uint32(1 << (x & 31))
    return out


def check_restated(occlude, libpath=None, n_envs=24, steps=110):
    specs = wl.workload_specs("uneven8k", n_envs)
    specs += [wl.spec(9, 11, 3, 2, 3, 20, S=2), wl.spec(6, 40, 4, 3, 4, 15)]
    for s in specs:
        s["flags"] |= EXPLORE | (8 if occlude else 0)
    b = o.OracleBatch(specs, libpath=libpath)
    b.reset(17)
    maps = [np.zeros((s["H"], s["W"]), bool) for s in specs]
    grow = 0
    for k in range(steps):
        before = b.get_state()
        _, rew, done, mp = b.step(1, maps=True)
        st = b.get_state()
        for e, s in enumerate(specs):
            a0 = int(b.agent_off[e])
            n = s["n"]
            walls = st["walls"][b.grid_off[e]:b.grid_off[e] + s["H"] * s["W"]]
            # post-move positions: the new state unless the episode ended
            if done[0, e]:
                xs = ys = None
            else:
                xs = st["pos_x"][a0:a0 + n].astype(int)
                ys = st["pos_y"][a0:a0 + n].astype(int)
            if xs is not None:
                fresh, new_map = restated_step(s, walls, xs, ys, maps[e])
                grow += int((new_map & ~maps[e]).sum())
                maps[e] = new_map
                got = np.round(rew[0, a0:a0 + n] * 128).astype(np.int64)
                frac = np.where(np.arange(n) < s["S"], got - 128 * np.floor(rew[0, a0:a0 + n]).astype(np.int64), 0)
                assert (frac[:s["S"]] == fresh[:s["S"]]).all(), (k, e)
                assert (rew[0, a0 + s["S"]:a0 + n] == np.round(rew[0, a0 + s["S"]:a0 + n])).all()
            else:
                maps[e] = np.zeros_like(maps[e])
            off = int(b.disc_off[e])
            np.testing.assert_array_equal(mp[0, off:off + len(map_words(s, maps[e]))],
                                          map_words(s, maps[e]), err_msg=f"step {k} env {e}")
        del before
    assert grow > 0


@pytest.mark.parametrize("occlude", [False, True])
def test_restated_maps_and_rewards(occlude):
    check_restated(occlude)
