"""Each plausible mistake planted in a copy of the oracle (on the CPU) must be
caught by at least one pin: the hand-worked grids, the brute-force checker,
or the rocRAND-based generator checks."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as o
from tests import bruteforce_spec as bf
from tests import test_oracle_explore as explore
from tests import test_oracle_golden as golden
from tests import test_oracle_radio as radio
from tests import test_oracle_rng as rng
from tests import test_oracle_terrain as terrain

SRC = open(o.SRC).read()

MUTATIONS = {
    "north_south_swapped": ("OR_DY[5] = { 0, -1, 1, 0, 0 }", "OR_DY[5] = { 0, 1, -1, 0, 0 }"),
    "manhattan_not_chebyshev": ("int cheb = ddx > ddy ? ddx : ddy;", "int cheb = ddx + ddy;"),
    "collisions_ignored": ("if (j != i && px[j] == tx && py[j] == ty) blocked = 1;",
                           "if (0) blocked = 1;"),
    "window_bit_transposed": ("int k = (dy + r) * d + (dx + r);", "int k = (dx + r) * d + (dy + r);"),
    "hider_reward_sign": ("int v = or_is_seeker(i, S) ? count[i] : -count[i];", "int v = count[i];"),
    "truncation_off_by_one": ("int truncated = b->t[e] >= L;", "int truncated = b->t[e] > L;"),
    "wall_index_transposed": ("int type = walls[ty * W + tx], cls = or_class(sp, i);",
                              "int type = walls[tx * H + ty], cls = or_class(sp, i);"),
    "philox_weyl_constant": ("k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;"),
    "philox_key_word": ("uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi1 ^ c1 ^ k1;"),
    "wall_channel_drops_outside": (
        "if (!inb || !or_enterable(walls[cy * W + cx], cls)) oi[0 * w + word] |= bit;",
        "if (inb && !or_enterable(walls[cy * W + cx], cls)) oi[0 * w + word] |= bit;"),
    "found_not_latched": ("b->found[e] |= 1u << h;", "b->found[e] = 1u << h;"),
    "respawn_old_episode": ("or_spawn(sp, walls, px, py, seed, env, b->ep[e]);",
                            "or_spawn(sp, walls, px, py, seed, env, b->ep[e] - 1);"),
    "action_keyed_by_t": ("b->steps[e], 0, i & 3), 5u);", "b->t[e], 0, i & 3), 5u);"),
    "obs_before_reset": ("    /* 5 auto-reset (the new episode's discovery map is empty) */\n    if (d) {",
                         "    or_observe(sp, walls, px, py, bel, obs);\n    if (0) {"),
    "opponent_as_teammate": ("if (or_is_seeker(j, S) == or_is_seeker(i, S))", "if (1)"),
    "los_corner_touch_blocks": ("return a.num * b.den < b.num * a.den;",
                                "return a.num * b.den <= b.num * a.den;"),
    "los_target_blocks_itself": ("if ((ex == 0 && ey == 0) || (ex == dx && ey == dy)) continue;",
                                 "if (ex == 0 && ey == 0) continue;"),
    "los_negative_direction_interval": ("lo->num = -(2 * e + 1); lo->den = -2 * d;",
                                        "lo->num = -(2 * e - 1); lo->den = -2 * d;"),
    "los_outside_not_blocking": (
        "int blocking = !or_in_bounds(bx, by, W, H) || walls[by * W + bx] == OR_WALL;",
        "int blocking = or_in_bounds(bx, by, W, H) && walls[by * W + bx] == OR_WALL;"),
    "explore_counted_after_update": ("if (pass == 0) {", "if (pass == 1) {"),
    "hiders_explore": ("for (int i = 0; i < S && i < n; ++i) {", "for (int i = 0; i < n; ++i) {"),
    "explore_map_kept_at_auto_reset": (
        " bel[i] = 0;\n        if (flags & OR_EXPLORE)\n            memset(",
        " bel[i] = 0;\n        if (0)\n            memset("),
    "explore_ignores_occlusion": (
        "if ((flags & OR_OCCLUDE) && !or_visible(sp, walls, px[i], py[i], cx, cy))\n                            continue;",
        "if (0)\n                            continue;"),
    "explore_reward_scale": ("0.0078125f", "0.00390625f"),
    "detection_ignores_los": (
        "int vis = !(flags & OR_OCCLUDE) || or_visible(sp, walls, px[i], py[i], px[h], py[h]);",
        "int vis = 1;"),
    "terrain_stuck_agent_moves": ("if (terrain && (b->stuck[e] >> i) & 1u) continue;", "if (0) continue;"),
    "terrain_speed_ignored": ("if (!or_chance(u, sp[SP_SPEED + 3 * cls + tile])) continue;",
                              "if (0) continue;"),
    "terrain_speed_tile_swapped": ("int tile = type == OR_GROUND ? 0 : (type == OR_WATER ? 1 : 2);",
                                   "int tile = type == OR_GROUND ? 0 : (type == OR_WATER ? 2 : 1);"),
    "terrain_swimmer_on_ground": ("case OR_GROUND: return cls == OR_WALKER || cls == OR_FLYER;",
                                  "case OR_GROUND: return 1;"),
    "terrain_flyer_gets_stuck": ("if (cls == OR_WALKER && type == OR_MUD) {", "if (type == OR_MUD) {"),
    "terrain_stuck_same_word": ("                                     2 * (i & 1) + 1);",
                                "                                     2 * (i & 1));"),
    "terrain_rescue_by_opponent": ("if (or_is_seeker(j, S) != or_is_seeker(i, S)) continue;",
                                   "if (0) continue;"),
    "terrain_rescue_by_stuck": ("if (j == i || ((before >> j) & 1u)) continue;",
                                "if (j == i) continue;"),
    "terrain_never_rescued": (
        "if (ddx >= -1 && ddx <= 1 && ddy >= -1 && ddy <= 1) b->stuck[e] &= ~(1u << i);",
        "if (0) b->stuck[e] &= ~(1u << i);"),
    "terrain_water_mud_swapped": (
        "type = x < Tw ? OR_WATER : (x < Tm ? OR_MUD : OR_GROUND);",
        "type = x < Tw ? OR_MUD : (x < Tm ? OR_WATER : OR_GROUND);"),
    "terrain_obs_ignores_class": (
        "if (!inb || !or_enterable(walls[cy * W + cx], cls)) oi[0 * w + word] |= bit;",
        "if (!inb || walls[cy * W + cx] == OR_WALL) oi[0 * w + word] |= bit;"),
    "terrain_water_blocks_sight": (
        "int blocking = !or_in_bounds(bx, by, W, H) || walls[by * W + bx] == OR_WALL;",
        "int blocking = !or_in_bounds(bx, by, W, H) || walls[by * W + bx] != OR_GROUND;"),
    "terrain_stuck_kept_at_auto_reset": (
        "        b->found[e] = 0;\n        b->stuck[e] = 0;\n        for (int i = 0;",
        "        b->found[e] = 0;\n        for (int i = 0;"),
    "radio_sequential_delivery": ("if (target[i] != i) bel[target[i]] |= sent[i];",
                                  "if (target[i] != i) bel[target[i]] |= bel[i];"),
    "radio_message_overwrites": ("if (target[i] != i) bel[target[i]] |= sent[i];",
                                 "if (target[i] != i) bel[target[i]] = sent[i];"),
    "radio_target_off_by_one": ("if (v / 5 >= 1 && v / 5 <= n) target[i] = v / 5 - 1;",
                                "if (v / 5 >= 1 && v / 5 < n) target[i] = v / 5;"),
    "radio_move_ignored_with_target": ("a[i] = v % 5;", "a[i] = v <= 4 ? v : 0;"),
    "radio_draw_misses_last_agent": ("b->steps[e], 0, i & 3), (uint32_t)n);",
                                     "b->steps[e], 0, i & 3), (uint32_t)n - 1u);"),
    "radio_draw_stream": ("OR_STREAM_RADIO, (uint32_t)(i >> 2)", "OR_STREAM_ACTION, (uint32_t)(i >> 2)"),
    "radio_sight_not_recorded": ("if (radio) bel[i] |= 1u << h;", "if (0) bel[i] |= 1u << h;"),
    "radio_beliefs_kept_at_reset": ("        for (int i = 0; i < n; ++i) bel[i] = 0;\n",
                                    "        for (int i = 0; i < n && 0; ++i) bel[i] = 0;\n"),
    "radio_belief_word_missing": ("oi[aw - 1] = belief[i];", "oi[aw - 1] = 0;"),
    "spawn_agent_key_zero": ("OR_STREAM_SPAWN, (uint32_t)i, e, (uint32_t)j, 0), cells)",
                             "OR_STREAM_SPAWN, 0u, e, (uint32_t)j, 0), cells)"),
    "spawn_attempt_episode_swapped": ("OR_STREAM_SPAWN, (uint32_t)i, e, (uint32_t)j, 0), cells)",
                                      "OR_STREAM_SPAWN, (uint32_t)i, (uint32_t)j, e, 0), cells)"),
    "spawn_word_1": ("OR_STREAM_SPAWN, (uint32_t)i, e, (uint32_t)j, 0), cells)",
                     "OR_STREAM_SPAWN, (uint32_t)i, e, (uint32_t)j, 1), cells)"),
    "spawn_cap_63": ("for (int j = 0; j < OR_SPAWN_ATTEMPTS && !placed; ++j)",
                     "for (int j = 0; j < OR_SPAWN_ATTEMPTS - 1 && !placed; ++j)"),
    "spawn_cap_65": ("for (int j = 0; j < OR_SPAWN_ATTEMPTS && !placed; ++j)",
                     "for (int j = 0; j <= OR_SPAWN_ATTEMPTS && !placed; ++j)"),
    "spawn_scan_from_cell_0": ("uint32_t cc = (c + d) % cells;", "uint32_t cc = (d - 1) % cells;"),
}


def build_mutant(old, new, d):
    assert SRC.count(old) == 1, old
    path = os.path.join(d, "mut.c")
    open(path, "w").write(SRC.replace(old, new))
    lib = os.path.join(d, "libmut.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", lib, path])
    return lib


def run_pins(libpath, rocrand_philox):
    """Return the name of the first pin that fails, or None."""
    def golden_pin():
        for case in golden.CASES:
            sp, st = golden.load_case(case)
            b = o.OracleBatch([sp], libpath=libpath)
            b.set_state(st)
            obs, rew, done = b.step(1, actions=np.array([case["actions"]], np.int8))
            golden.check_case(case, obs[0], rew[0], done[0], b.get_state())

    def brute_pin():
        fams = [bf.case_one_agent(r=1, C=4, subsample=30_000, seed=1),
                bf.case_seeker_hider(n_patterns=12, flags=1),
                bf.case_seeker_hider(n_patterns=12, flags=3, seed=2),
                bf.case_three_agents(r=1, C=4, flags=3, S=1),
                bf.case_one_agent(r=3, C=4, flags=8 | 3, subsample=20_000, seed=7),
                bf.case_seeker_hider(n_patterns=12, r=3, C=4, flags=8 | 1, seed=8)]
        for spec, st, acts in fams:
            B = st["pos_x"].shape[0]
            table = np.tile(o.spec_table([spec]), (B, 1))
            b = o.OracleBatch(table, libpath=libpath)
            b.set_state(bf.flat_state(st))
            obs, rew, done = b.step(1, actions=acts.reshape(1, -1))
            bf.check_step(spec, st, acts, obs[0], rew[0], done[0], b.get_state())

    def philox_pin():
        L = o.lib(libpath)
        g = np.random.Generator(np.random.PCG64(5))
        rows = g.integers(0, 2**30, size=(64, 6), dtype=np.uint64)
        ref = rocrand_philox(rows)
        for r, want in zip(rows, ref):
            out = np.zeros(4, np.uint32)
            L.or_philox_block(*[int(v) for v in r[2:]], *[int(v) for v in r[:2]],
                              out.ctypes.data)
            assert np.array_equal(out, want)

    pins = [("golden", golden_pin), ("bruteforce", brute_pin), ("philox", philox_pin),
            ("streams", lambda: rng.check_stream_layout(rocrand_philox, libpath)),
            ("respawn", lambda: rng.check_respawn_keyed_by_episode(rocrand_philox, libpath)),
            ("spawn", lambda: rng.check_spawn_rule(rocrand_philox, libpath)),
            ("explore_golden", lambda: explore.check_hand_worked(libpath)),
            ("explore_restated", lambda: explore.check_restated(False, libpath, n_envs=6, steps=60)),
            ("explore_restated_occluded",
             lambda: explore.check_restated(True, libpath, n_envs=6, steps=60)),
            ("terrain_golden", lambda: terrain.check_hand_worked(libpath)),
            ("terrain_plain", lambda: terrain.check_reduces_to_plain(libpath, n_envs=12, steps=60)),
            ("terrain_generation", lambda: terrain.check_generation(rocrand_philox, libpath)),
            ("terrain_chances", lambda: terrain.check_chances(libpath)),
            ("terrain_invariants",
             lambda: terrain.check_trajectory_invariants(libpath, n_envs=40, steps=100)),
            ("radio_golden", lambda: radio.check_hand_worked(libpath)),
            ("radio_plain", lambda: radio.check_reduces_to_plain(libpath, n_envs=12, steps=60)),
            ("radio_draws", lambda: radio.check_radio_draws(rocrand_philox, libpath)),
            ("radio_invariants",
             lambda: radio.check_trajectory_invariants(libpath, n_envs=20, steps=60))]
    for name, fn in pins:
        try:
            fn()
        except AssertionError:
            return name
    return None


def test_unmutated_oracle_passes_pins(rocrand_philox):
    with tempfile.TemporaryDirectory() as d:
        lib = build_mutant("OR_DY[5]", "OR_DY[5]", d)
        assert run_pins(lib, rocrand_philox) is None


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_mutation_is_caught(name, rocrand_philox):
    old, new = MUTATIONS[name]
    with tempfile.TemporaryDirectory() as d:
        lib = build_mutant(old, new, d)
        assert run_pins(lib, rocrand_philox) is not None, name
