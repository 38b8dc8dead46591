"""Pins of the oracle's terrain rules (flag 32, reading R28): a hand-worked
episode (tests/golden/terrain_hand_worked.json), the cases that reduce to the
plain rules (walkers on a map without water or mud, flyers anywhere but
walls), the tile generation against rocRAND's independent Philox, the move
and stuck chances against their stated rates, and invariants of the stuck /
rescue rule and of the classes along random trajectories."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as o
from paper_2604_27162_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "terrain_hand_worked.json")))
GROUND, WALL, WATER, MUD = 0, 1, 2, 3
ENTER = {wl.WALKER: {GROUND, MUD}, wl.SWIMMER: {WATER}, wl.FLYER: {GROUND, WATER, MUD}}
DX = (0, 0, 0, 1, -1)
DY = (0, -1, 1, 0, 0)


def check_hand_worked(libpath=None):
    for case in GOLD["cases"]:
        b = o.OracleBatch([case["spec"]], libpath=libpath)
        st = b.get_state()
        st["walls"][:] = case["tiles"]
        st["pos_x"][:] = case["start"]["pos_x"]
        st["pos_y"][:] = case["start"]["pos_y"]
        st["t"][:] = 0
        st["stuck"][:] = 0
        b.set_state(st)
        for a, want in zip(case["actions"], case["expected"]):
            obs, rew, done = b.step(1, actions=np.array([a], np.int8))
            s = b.get_state()
            what = f'{case["name"]}: {want["notes"]}'
            assert [[int(x), int(y)] for x, y in zip(s["pos_x"], s["pos_y"])] == want["pos"], what
            assert int(s["stuck"][0]) == want["stuck"], what
            assert list(rew[0]) == want["rew"], what
            assert obs[0].reshape(3, 3).tolist() == want["obs"], what
            assert done[0, 0] == 0


def test_hand_worked_episode():
    check_hand_worked()


def classes_of(spec):
    w = int(spec.get("classes", 0))
    return [(w >> (2 * i)) & 3 for i in range(spec["n"])]


def random_terrain_specs(n_envs, seed, base="uneven8k"):
    """Terrain versions of a workload's specs with seeded percentages, chances
    and classes."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in wl.workload_specs(base, n_envs):
        water, mud = int(g.integers(10, 30)), int(g.integers(0, 25))
        if s["wall_pct"] + water + mud > 99:
            water = mud = 0
        speed = [int(v) for v in g.choice([0, 35, 70, 100], 9)]
        cls = [int(c) for c in g.integers(0, 3, s["n"])]
        out.append(wl.with_terrain(s, water, mud, int(g.integers(0, 101)), speed, cls))
    return out


def compare_runs(a_specs, b_specs, seed, steps, libpath=None):
    a = o.OracleBatch(a_specs, libpath=libpath)
    b = o.OracleBatch(b_specs, libpath=libpath)
    np.testing.assert_array_equal(a.reset(seed), b.reset(seed))
    for x, y in zip(a.step(steps), b.step(steps)):
        np.testing.assert_array_equal(x, y)
    sa, sb = a.get_state(), b.get_state()
    for k in ("pos_x", "pos_y", "found", "t", "episode", "steps"):
        np.testing.assert_array_equal(sa[k], sb[k], err_msg=k)
    return sa, sb


def check_reduces_to_plain(libpath=None, n_envs=40, steps=150):
    """Walkers with no water or mud and certain moves are the plain game;
    flyers with certain moves are too, whatever the water and mud (the walls
    are the same cells: the same draw decides wall or not)."""
    plain = wl.workload_specs("uneven8k", n_envs)
    walkers = [wl.with_terrain(s, 0, 0, 77, (100,) * 9, [wl.WALKER] * s["n"]) for s in plain]
    compare_runs(plain, walkers, 13, steps, libpath)
    flyers = [wl.with_terrain(s, 20, 15, 90, (100,) * 9, [wl.FLYER] * s["n"]) for s in plain]
    sa, sb = compare_runs(plain, flyers, 14, steps, libpath)
    assert not sb["stuck"].any()  # flyers never get stuck
    # the terrain map has water and mud where the plain map is open ground
    assert np.array_equal(sa["walls"] == WALL, sb["walls"] == WALL)
    assert (sb["walls"] == WATER).any() and (sb["walls"] == MUD).any()
    # with line of sight too: water and mud do not block sight
    occ = [dict(s, flags=s["flags"] | 8) for s in plain]
    occ_flyers = [dict(s, flags=s["flags"] | 8) for s in flyers]
    compare_runs(occ, occ_flyers, 15, steps, libpath)


def test_reduces_to_plain():
    check_reduces_to_plain()


def check_generation(rocrand_philox, libpath=None):
    """Tile types from the wall stream words (rocRAND) and the cumulative
    thresholds floor(p 2^32 / 100)."""
    specs = [wl.with_terrain(wl.spec(9, 13, 2, 2, 3, 12), 23, 17),
             wl.with_terrain(wl.spec(16, 5, 1, 1, 3, 0), 40, 30)]
    b = o.OracleBatch(specs, libpath=libpath)
    seed = 0x1234567876543210
    b.reset(seed)
    walls = b.get_state()["walls"]
    off = 0
    for e, s in enumerate(specs):
        cells = s["H"] * s["W"]
        rows = [[seed & 0xffffffff, seed >> 32, e, (2 << 24) | g, 0, 0] for g in range((cells + 3) // 4)]
        words = rocrand_philox(rows).reshape(-1)[:cells]
        thr = [int((p << 32) // 100) for p in (s["wall_pct"], s["wall_pct"] + s["water_pct"],
                                                s["wall_pct"] + s["water_pct"] + s["mud_pct"])]
        want = np.where(words < thr[0], WALL, np.where(words < thr[1], WATER,
                                                       np.where(words < thr[2], MUD, GROUND)))
        np.testing.assert_array_equal(walls[off:off + cells], want, err_msg=f"env {e}")
        off += cells


def test_generation_against_rocrand(rocrand_philox):
    check_generation(rocrand_philox)


def one_step_east(spec, n_envs, seed, libpath=None):
    """Every agent of n_envs copies of spec tries to move east once from the
    reset state; returns (moved, stuck_after, attempted) per agent."""
    b = o.OracleBatch([spec] * n_envs, libpath=libpath)
    b.reset(seed)
    st = b.get_state()
    acts = np.full((1, b.agents_total), 3, np.int8)
    b.step(1, actions=acts)
    new = b.get_state()
    n, W = spec["n"], spec["W"]
    walls = st["walls"].reshape(n_envs, spec["H"], W)
    x0 = st["pos_x"].reshape(n_envs, n).astype(int)
    y0 = st["pos_y"].reshape(n_envs, n).astype(int)
    ok = np.zeros((n_envs, n), bool)
    tile = np.full((n_envs, n), -1)
    for e in range(n_envs):
        for i in range(n):
            tx = x0[e, i] + 1
            if tx < W:
                tile[e, i] = walls[e, y0[e, i], tx]
                ok[e, i] = tile[e, i] in ENTER[classes_of(spec)[i]]
    moved = new["pos_x"].reshape(n_envs, n).astype(int) != x0
    stuck = ((new["stuck"][:, None] >> np.arange(n)) & 1).astype(bool)
    return moved, stuck, ok, tile


def binomial_ok(k, m, p, z=5.0):
    return abs(k - m * p) <= z * np.sqrt(m * p * (1 - p)) + 1


def check_chances(libpath=None):
    """Move chance: one walker per env on an open map, ground speed 35%.
    Stuck chance: all-mud map (99% mud), mud speed 50% and stuck 50%, drawn
    from separate words: P(stuck | moved) = 1/2."""
    # no desynchronised start: no env may end its episode in this one step
    sp = wl.with_terrain(wl.spec(8, 8, 1, 1, 3, 0, S=1, flags=wl.COLLIDE), 0, 0, 0,
                         (35, 0, 100, 0, 0, 0, 0, 0, 0), [wl.WALKER])
    moved, _, ok, _ = one_step_east(sp, 3000, 21, libpath)
    assert not (moved & ~ok).any()
    k, m = int(moved[ok].sum()), int(ok.sum())
    assert m > 2000 and binomial_ok(k, m, 0.35), (k, m)
    sp = wl.with_terrain(wl.spec(8, 8, 1, 1, 3, 0, S=1, flags=wl.COLLIDE), 0, 99, 50,
                         (100, 0, 50, 0, 0, 0, 0, 0, 0), [wl.WALKER])
    moved, stuck, ok, tile = one_step_east(sp, 3000, 22, libpath)
    assert not (stuck & ~(moved & (tile == MUD))).any()  # only entering mud sticks
    mud = ok & (tile == MUD)
    k, m = int(moved[mud].sum()), int(mud.sum())
    assert m > 2000 and binomial_ok(k, m, 0.5), (k, m)
    k2 = int(stuck[moved & mud].sum())
    assert binomial_ok(k2, k, 0.5), (k2, k)


def test_move_and_stuck_chances():
    check_chances()


def check_trajectory_invariants(libpath=None, n_envs=60, steps=150):
    """Along random terrain trajectories: every agent stands on a tile its
    class may enter; an agent stuck before a step does not move (unless the
    env reset); an agent stuck after a step was stuck before or entered mud
    as a walker, and each of its adjacent teammates was stuck before or
    entered mud as a walker; a freed agent has an adjacent teammate."""
    specs = random_terrain_specs(n_envs, 5)
    b = o.OracleBatch(specs, libpath=libpath)
    b.reset(8)
    prev = b.get_state()
    seen_stuck = seen_free = 0
    for _ in range(steps):
        _, _, done = b.step(1)
        new = b.get_state()
        for e, s in enumerate(specs):
            if done[0, e]:
                assert new["stuck"][e] == 0
                continue
            n, W = s["n"], s["W"]
            a0, g0 = int(b.agent_off[e]), int(b.grid_off[e])
            walls = new["walls"][g0:g0 + s["H"] * W]
            cls = classes_of(s)
            x0, y0 = prev["pos_x"][a0:a0 + n].astype(int), prev["pos_y"][a0:a0 + n].astype(int)
            x1, y1 = new["pos_x"][a0:a0 + n].astype(int), new["pos_y"][a0:a0 + n].astype(int)
            sb, sa = int(prev["stuck"][e]), int(new["stuck"][e])
            into_mud = [(x1[i], y1[i]) != (x0[i], y0[i]) and cls[i] == wl.WALKER and
                        walls[y1[i] * W + x1[i]] == MUD for i in range(n)]
            for i in range(n):
                assert walls[y1[i] * W + x1[i]] in ENTER[cls[i]], (e, i)
                was, now = (sb >> i) & 1, (sa >> i) & 1
                if was:
                    assert (x1[i], y1[i]) == (x0[i], y0[i]), (e, i)
                mates = [j for j in range(n) if j != i and (j < s["S"]) == (i < s["S"]) and
                         abs(x1[j] - x1[i]) <= 1 and abs(y1[j] - y1[i]) <= 1]
                if now:
                    seen_stuck += 1
                    assert was or into_mud[i], (e, i)
                    for j in mates:
                        assert (sb >> j) & 1 or into_mud[j], (e, i, j)
                if was and not now:
                    seen_free += 1
                    assert mates, (e, i)
        prev = new
    assert seen_stuck > 0 and seen_free > 0


def test_trajectory_invariants():
    check_trajectory_invariants()


def test_terrain_state_round_trip():
    specs = random_terrain_specs(30, 6)
    a = o.OracleBatch(specs)
    a.reset(3)
    a.step(40)
    b = o.OracleBatch(specs)
    b.set_state(a.get_state())
    for x, y in zip(a.step(60), b.step(60)):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("water,mud", [(99, 0), (0, 99)])
def test_reset_rejects_maps_without_room(water, mud):
    """Every class present needs n cells it may stand on."""
    sp = wl.with_terrain(wl.spec(4, 4, 3, 1, 3, 0), water, mud, 0, (100,) * 9,
                         [wl.WALKER, wl.SWIMMER, wl.FLYER])
    with pytest.raises(ValueError):
        o.OracleBatch([sp]).reset(1)
