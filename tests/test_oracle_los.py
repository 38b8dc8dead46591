"""Pins of the oracle's line-of-sight rule (occlusion flag 8): hand-worked
boards (tests/golden/los_hand_worked.json), the symmetry of the rule, its
special cases, the segment-sampling restatement of tests/bruteforce_spec.py on
random boards, and trajectory-level consequences (occlusion only removes
observation bits and detections)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as o
from paper_2604_27162_amd import workloads as wl
from tests import bruteforce_spec as bf

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "los_hand_worked.json")))["cases"]
OCC = 8


def board(case):
    w = np.zeros(case["H"] * case["W"], np.uint8)
    for x, y in case["walls"]:
        w[y * case["W"] + x] = 1
    return w


def spec_of(case, n=1, flags=OCC):
    return wl.spec(case["H"], case["W"], n, case["r"], 4, 0, S=1, flags=flags)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_worked_hidden_sets(case):
    sp, w = spec_of(case), board(case)
    ax, ay = case["agent"]
    r = case["r"]
    got = {(dx, dy) for dy in range(-r, r + 1) for dx in range(-r, r + 1)
           if not o.los(sp, w, ax, ay, ax + dx, ay + dy)}
    assert got == {tuple(h) for h in case["hidden"]}


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_worked_through_the_step(case):
    """A hider in a hidden cell is neither observed nor detected; in a visible
    cell of the same distance it is both. The seeker stays put (actions 0)."""
    r = case["r"]
    ax, ay = case["agent"]
    hidden = [tuple(h) for h in case["hidden"]]
    hx, hy = hidden[-1]
    vis = [(dx, dy) for dy in range(-r, r + 1) for dx in range(-r, r + 1)
           if (dx, dy) not in hidden and (dx, dy) != (0, 0)
           and [ax + dx, ay + dy] not in case["walls"]]
    for (dx, dy), seen in (((hx, hy), False), (vis[0], True)):
        sp = spec_of(case, n=2, flags=OCC | 1)
        b = o.OracleBatch([sp])
        st = b.get_state()
        st["walls"][:] = board(case)
        st["pos_x"][:] = [ax, ax + dx]
        st["pos_y"][:] = [ay, ay + dy]
        st["t"][:] = 0
        b.set_state(st)
        obs, rew, done = b.step(1, actions=np.zeros((1, 2), np.int8))
        D = 2 * r + 1
        w = (D * D + 31) // 32
        k = (dy + r) * D + (dx + r)
        opp = obs[0][2 * w:3 * w]  # seeker's opponent channel
        assert bool((opp[k >> 5] >> (k & 31)) & 1) == seen
        assert list(rew[0]) == ([1.0, -1.0] if seen else [0.0, 0.0])


def random_boards(n, H, W, pct, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return (g.random((n, H * W)) < pct).astype(np.uint8)


def test_symmetric_on_random_boards():
    sp = wl.spec(9, 9, 1, 4, 4, 30, flags=OCC)
    g = np.random.Generator(np.random.PCG64(11))
    for w in random_boards(40, 9, 9, 0.3, 12):
        for _ in range(40):
            ax, ay, cx, cy = (int(v) for v in g.integers(0, 9, 4))
            assert o.los(sp, w, ax, ay, cx, cy) == o.los(sp, w, cx, cy, ax, ay)


def test_special_cases():
    sp = wl.spec(9, 9, 1, 4, 4, 0, flags=OCC)
    empty = np.zeros(81, np.uint8)
    full = np.ones(81, np.uint8)
    for dy in range(-4, 5):
        for dx in range(-4, 5):
            assert o.los(sp, empty, 4, 4, 4 + dx, 4 + dy)  # nothing blocks inside the map
            near = max(abs(dx), abs(dy)) <= 1
            assert o.los(sp, full, 4, 4, 4 + dx, 4 + dy) == near  # only neighbours
    # a straight line is cut by one wall between the ends
    w = empty.copy()
    w[4 * 9 + 6] = 1
    assert not o.los(sp, w, 4, 4, 8, 4) and o.los(sp, w, 4, 4, 6, 4)
    # cells past the map edge hide what lies behind them
    assert not o.los(sp, empty, 0, 4, -2, 4) and o.los(sp, empty, 0, 4, -1, 4)


def test_matches_segment_sampling_on_random_boards():
    """The oracle's exact interval test against the sampled segments of the
    brute-force checker, every window offset up to r = 4, walls and outside."""
    H = W = 7
    sp = wl.spec(H, W, 1, 4, 4, 30, flags=OCC)
    g = np.random.Generator(np.random.PCG64(13))
    for w in random_boards(60, H, W, 0.3, 14):
        ax, ay = (int(v) for v in g.integers(0, 7, 2))
        for dy in range(-4, 5):
            for dx in range(-4, 5):
                blocked = False
                for ex, ey in bf.crossed_cells(dx, dy):
                    bx, by = ax + ex, ay + ey
                    inside = 0 <= bx < W and 0 <= by < H
                    blocked |= (not inside) or bool(w[by * W + bx])
                assert o.los(sp, w, ax, ay, ax + dx, ay + dy) == (not blocked)


def test_occlusion_only_removes_bits_and_detections():
    """Capture off: moves do not depend on detection, so the trajectories with
    and without occlusion coincide; every occluded observation word is a
    subset of the plain one, every |reward| is no larger, and occlusion
    actually hides something."""
    plain = wl.workload_specs("uneven8k", 60)
    for s in plain:
        s["flags"] = 1 | 4  # collisions, desync; no capture
    occl = [dict(s, flags=s["flags"] | OCC) for s in plain]
    a, b = o.OracleBatch(plain), o.OracleBatch(occl)
    a.reset(31)
    b.reset(31)
    oa, ra, da = a.step(120)
    ob, rb, db = b.step(120)
    assert np.array_equal(da, db)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa["pos_x"], sb["pos_x"]) and np.array_equal(sa["pos_y"], sb["pos_y"])
    assert ((ob & ~oa) == 0).all()
    assert (np.abs(rb) <= np.abs(ra)).all()
    assert (ob != oa).any() and (rb != ra).any()
