"""Exploration (flag 16) on the GPU against the oracle, bit-exact through the
C ABI: rewards, the per-step discovery maps (centralised observation) and the
maps kept in the state, in both launch modes, with and without line of
sight, in batches mixing exploring and plain envs under every tiling, across
state round trips, and in a multi-batch call."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, workloads as wl  # noqa: E402
from tests.test_gpu_parity import DEV, assert_outputs, assert_state, u32  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def exploring(specs, extra=0):
    return [dict(s, flags=s["flags"] | wl.EXPLORE | extra) for s in specs]


def assert_maps(g_maps, o_maps, what=""):
    np.testing.assert_array_equal(u32(g_maps).reshape(o_maps.shape), o_maps, err_msg=f"maps {what}")


def run_maps(specs, seed, steps, mode=hase.PERSISTENT, lanes=None, actions=None, env_id_base=0):
    print(f"case: explore {len(specs)} envs, {steps} steps, seed {seed}, mode {mode}, "
          f"lanes {lanes}", flush=True)
    g = hase.HaseBatch(specs, env_id_base=env_id_base, device=DEV, lanes=lanes)
    ob = o.OracleBatch(specs, env_id_base=env_id_base)
    np.testing.assert_array_equal(u32(g.reset(seed)), ob.reset(seed), err_msg="obs0")
    assert_state(g, ob)
    go, gr, gd, gm = g.step(steps, actions=actions, mode=mode, maps=True)
    torch.cuda.synchronize()
    oo, orr, od, om = ob.step(steps, actions=actions, maps=True)
    assert_outputs((go, gr, gd), (oo, orr, od))
    assert_maps(gm, om)
    assert_state(g, ob)
    g.close()
    return orr, od, om


@pytest.mark.parametrize("name,ne,steps", [("small", 500, 270), ("single1k", 333, 300),
                                           ("multi10", 123, 280), ("uneven8k", 611, 260)])
@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_exploring_workloads(name, ne, steps, mode):
    rew, done, maps = run_maps(exploring(wl.workload_specs(name, ne)), seed=300 + len(name),
                               steps=steps, mode=mode, env_id_base=5)
    assert (done == 2).any()
    assert (rew != np.round(rew)).any()  # exploration rewards were paid
    assert maps.any()


@pytest.mark.parametrize("name,ne,steps", [("single1k", 257, 280), ("uneven8k", 401, 260)])
def test_exploring_with_line_of_sight(name, ne, steps):
    run_maps(exploring(wl.workload_specs(name, ne), wl.OCCLUDE), seed=77, steps=steps)


def test_exploring_collisions_off_and_external_actions():
    specs = exploring(wl.workload_specs("uneven8k", 233))
    for s in specs:
        s["flags"] &= ~wl.COLLIDE
    agents = sum(s["n"] for s in specs)
    acts = wl.random_actions(150, agents, seed=12, draw_frac=0.3, invalid_frac=0.05)
    run_maps(specs, seed=43, steps=150, actions=acts)


@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
def test_mixed_exploring_occluding_and_plain_envs(lanes):
    """Exploring, occluding, both and plain envs interleaved in one batch."""
    base = wl.workload_specs("uneven8k", 280)
    extra = [0, wl.EXPLORE, wl.OCCLUDE, wl.EXPLORE | wl.OCCLUDE]
    specs = [dict(s, flags=s["flags"] | extra[i % 4]) for i, s in enumerate(base)]
    run_maps(specs, seed=58, steps=130, lanes=[lanes, lanes, max(lanes, 4), max(lanes, 8)])


def test_one_lane_per_env_fits_small_boards_only():
    """lanes 1 keeps 64 boards and 64 maps in one wave's LDS (64 KiB): boards
    of up to 31 rows fit, 64 rows are refused by the tiler (no launch)."""
    small = exploring([wl.spec(24, 30, 2, 3, 3, 15)] * 70)
    run_maps(small, seed=3, steps=90, lanes=[1, 1, 4, 8])
    big = hase.HaseBatch(exploring([wl.spec(64, 64, 2, 3, 3, 15)] * 3), device=DEV)
    with pytest.raises(hase.HaseError) as ei:
        big.set_tiling([1, 4, 16, 16])
    assert ei.value.code == hase.EINVAL
    assert big.get_tiling()[0] == 4
    big.close()


def test_hand_worked_episode_on_the_gpu():
    gold = json.load(open(os.path.join(HERE, "golden", "explore_hand_worked.json")))
    sp = gold["spec"]
    g = hase.HaseBatch([sp], device=DEV)
    g.reset(1)
    st = g.get_state()
    st["walls"][:] = 0
    st["pos_x"][:] = gold["start"]["pos_x"]
    st["pos_y"][:] = gold["start"]["pos_y"]
    st["t"][:] = 0
    g.set_state(st)
    for a, want in zip(gold["actions"], gold["expected"]):
        _, rew, done, mp = g.step(1, actions=np.array([a], np.int8), maps=True)
        torch.cuda.synchronize()
        st = g.get_state()
        assert [int(st["pos_x"][0]), int(st["pos_y"][0])] == want["pos"], want["notes"]
        assert list(rew.cpu().numpy()[0]) == want["rew"], want["notes"]
        assert list(u32(mp)[0]) == want["map"], want["notes"]
        assert list(st["discovered"]) == want["map"]
    g.close()


def test_state_round_trip_carries_the_maps():
    """Maps read back mid-episode and loaded into a fresh batch continue the
    same trajectory; a state without maps starts them empty (the oracle is
    given empty maps to match)."""
    specs = exploring(wl.workload_specs("uneven8k", 97))
    g = hase.HaseBatch(specs, device=DEV)
    ob = o.OracleBatch(specs)
    g.reset(21)
    ob.reset(21)
    for k in (1, 29, 64):
        gout = g.step(k, maps=True)
        torch.cuda.synchronize()
        oout = ob.step(k, maps=True)
        assert_outputs(gout[:3], oout[:3], f"{k} steps")
        assert_maps(gout[3], oout[3], f"{k} steps")
        assert_state(g, ob)
    st = g.get_state()
    assert st["discovered"].any()
    g2 = hase.HaseBatch(specs, device=DEV, lanes=[2, 8, 16, 16])
    g2.set_state(st)
    gout = g2.step(40, maps=True)
    torch.cuda.synchronize()
    oout = ob.step(40, maps=True)
    assert_outputs(gout[:3], oout[:3], "after round trip")
    assert_maps(gout[3], oout[3], "after round trip")
    # no maps in the state: cleared
    st = ob.get_state()
    nomaps = {k: v for k, v in st.items() if k != "discovered"}
    g2.set_state(nomaps)
    st["discovered"][:] = 0
    ob.set_state(st)
    assert not g2.get_state()["discovered"].any()
    gout = g2.step(25, maps=True)
    torch.cuda.synchronize()
    oout = ob.step(25, maps=True)
    assert_outputs(gout[:3], oout[:3], "after clearing")
    assert_maps(gout[3], oout[3], "after clearing")
    g.close()
    g2.close()


def test_set_state_rejects_map_bits_past_the_width():
    specs = exploring([wl.spec(8, 20, 2, 2, 3, 10)] * 3)
    g = hase.HaseBatch(specs, device=DEV)
    g.reset(4)
    st = g.get_state()
    st["discovered"][5] |= np.uint32(1 << 20)
    with pytest.raises(hase.HaseError) as ei:
        g.set_state(st)
    assert ei.value.code == hase.ESTATE
    g.close()


def test_maps_output_is_optional_and_changes_nothing_else():
    specs = exploring(wl.workload_specs("multi10", 77), wl.OCCLUDE)
    a, b = hase.HaseBatch(specs, device=DEV), hase.HaseBatch(specs, device=DEV)
    a.reset(8)
    b.reset(8)
    oa = a.step(120)
    ob_ = b.step(120, maps=True)
    torch.cuda.synchronize()
    for x, y in zip(oa, ob_[:3]):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    np.testing.assert_array_equal(a.get_state()["discovered"], b.get_state()["discovered"])
    a.close()
    b.close()


def test_step_multi_with_exploring_requests():
    specs = [wl.spec(32, 32, 2, 3, 3, 15, flags=wl.DEFAULT_FLAGS | wl.EXPLORE),
             wl.spec(16, 16, 6, 2, 4, 20, flags=wl.DEFAULT_FLAGS | wl.EXPLORE | wl.OCCLUDE),
             wl.spec(24, 40, 3, 2, 3, 10)]
    n_envs, steps, seeds = [90, 41, 33], [50, 35, 44], [71, 72, 73]
    bs = []
    for sp, ne, sd in zip(specs, n_envs, seeds):
        b = hase.HaseBatch([sp] * ne, device=DEV)
        b.reset(sd)
        bs.append(b)
    outs = [b.alloc_outputs(k, maps=True) for b, k in zip(bs, steps)]
    ws = torch.empty(hase.multi_workspace_bytes(bs), dtype=torch.uint8, device=DEV)
    items = [(b, k, 0, None, *out) for b, k, out in zip(bs, steps, outs)]
    hase.step_multi(items, max(steps), ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for sp, ne, sd, k, b, out in zip(specs, n_envs, seeds, steps, bs, outs):
        ob = o.OracleBatch([sp] * ne)
        ob.reset(sd)
        oo = ob.step(k, maps=True)
        assert_outputs(out[:3], oo[:3])
        if b.map_words:
            assert_maps(out[3][:, :b.map_words], oo[3])
        assert_state(b, ob)


def test_full_size_explore16k_sampled():
    """The benchmark's exploring workload at full size (16384 envs, persistent
    launch with map output, default tiling), sampled envs against one-env
    oracle runs (an env's trajectory depends only on its seed, id and spec)."""
    from tests.test_gpu_parity import fbits, offsets

    w = wl.WORKLOADS["explore16k"]
    specs = wl.workload_specs("explore16k")
    steps = 2000
    print(f"case: full size explore16k, {len(specs)} envs x {steps} steps", flush=True)
    g = hase.HaseBatch(specs, device=DEV)
    g.reset(w["seed"])
    go, gr, gd, gm = g.step(steps, maps=True)
    torch.cuda.synchronize()
    obs_off, agent_off = offsets(specs)
    map_off = g.map_offsets()
    rng = np.random.Generator(np.random.PCG64(2))
    sample = sorted(set([0, len(specs) - 1] + list(rng.choice(len(specs), 24, replace=False))))
    for e in sample:
        s = specs[e]
        nw = s["n"] * s["C"] * (((2 * s["r"] + 1) ** 2 + 31) // 32)
        mw = s["H"] * ((s["W"] + 31) // 32)
        one = o.OracleBatch([s], env_ids=[e])
        one.reset(w["seed"])
        oo, orr, od, om = one.step(steps, maps=True)
        np.testing.assert_array_equal(u32(go[:, obs_off[e]:obs_off[e] + nw]), oo,
                                      err_msg=f"obs env {e}")
        np.testing.assert_array_equal(fbits(gr[:, agent_off[e]:agent_off[e] + s["n"]]),
                                      orr.view(np.uint32), err_msg=f"rew env {e}")
        np.testing.assert_array_equal(gd[:, e].cpu().numpy(), od[:, 0], err_msg=f"done env {e}")
        np.testing.assert_array_equal(u32(gm[:, int(map_off[e]):int(map_off[e]) + mw]), om,
                                      err_msg=f"maps env {e}")
    g.close()
    del go, gr, gd, gm
    torch.cuda.empty_cache()


def test_odd_map_shapes():
    """Map outputs whose word count is not a multiple of 4 (ragged 16-byte
    chunks) and rows of two words whose second word is nearly empty."""
    shapes = [(7, 45, 2, 2), (9, 33, 3, 3), (5, 2, 1, 1), (11, 64, 4, 4), (3, 31, 2, 1)]
    specs = []
    for i in range(60):
        H, W, n, r = shapes[i % len(shapes)]
        specs.append(dict(wl.spec(H, W, n, r, 3 + (i % 2), 5, L=40), flags=wl.DEFAULT_FLAGS |
                          wl.EXPLORE | (wl.OCCLUDE if i % 3 == 0 else 0)))
    run_maps(specs, seed=37, steps=120, lanes=[2, 4, 8, 16])
