"""Terrain (flag 32) on the GPU against the oracle, bit-exact through the C
ABI: random terrain batches in both launch modes, the terrain workload, with
exploration, batches mixing every env kind under every tiling, the
hand-worked episodes, state round trips with stuck agents, external actions,
a multi-batch call, and the full-size workload sampled."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, workloads as wl  # noqa: E402
from tests.test_gpu_explore import assert_maps, run_maps  # noqa: E402
from tests.test_gpu_parity import DEV, assert_outputs, assert_state, run_pair, u32  # noqa: E402
from tests.test_oracle_terrain import random_terrain_specs  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_random_terrain(mode):
    specs = random_terrain_specs(311, 7)
    _, _, done = run_pair(specs, seed=91, steps=220, mode=mode, env_id_base=4)
    assert (done == 2).any()


@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_terrain_workload(mode):
    run_pair(wl.workload_specs("terrain4k", 157), seed=5, steps=240, mode=mode)


def test_terrain_with_exploration():
    specs = [dict(s, flags=s["flags"] | wl.EXPLORE) for s in random_terrain_specs(203, 8)]
    run_maps(specs, seed=17, steps=200)


@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_terrain_with_line_of_sight(mode):
    """Only walls and outside block sight; water and mud do not."""
    specs = [dict(s, flags=s["flags"] | wl.OCCLUDE) for s in random_terrain_specs(257, 13)]
    run_pair(specs, seed=19, steps=200, mode=mode)


def test_terrain_with_line_of_sight_and_exploration():
    specs = [dict(s, flags=s["flags"] | wl.OCCLUDE | wl.EXPLORE)
             for s in random_terrain_specs(199, 14)]
    run_maps(specs, seed=21, steps=180)


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_every_kind_in_one_batch(lanes):
    """All eight env kinds interleaved: plain, exploring, occluding, both,
    and the same four with terrain (fewer than 4 lanes per env would not fit
    two 64-row tile planes and a discovery map per env in one wave's LDS)."""
    ter = random_terrain_specs(320, 9)
    extra = [0, wl.EXPLORE, wl.OCCLUDE, wl.EXPLORE | wl.OCCLUDE, None, wl.EXPLORE, wl.OCCLUDE,
             wl.OCCLUDE | wl.EXPLORE]
    specs = []
    for i, s in enumerate(ter):
        k = i % 8
        if k < 4:
            base = {f: s[f] for f in ("H", "W", "n", "S", "r", "C", "wall_pct", "flags", "L")}
            base["flags"] &= ~wl.TERRAIN
            specs.append(dict(base, flags=base["flags"] | extra[k]))
        else:
            specs.append(dict(s, flags=s["flags"] | (extra[k] or 0)))
    run_maps(specs, seed=61, steps=150, lanes=[lanes, lanes, max(lanes, 4), max(lanes, 8)])


def test_collisions_off_and_external_actions():
    specs = random_terrain_specs(229, 10)
    for s in specs:
        s["flags"] &= ~wl.COLLIDE
    agents = sum(s["n"] for s in specs)
    acts = wl.random_actions(160, agents, seed=14, draw_frac=0.3, invalid_frac=0.05)
    run_pair(specs, seed=44, steps=160, actions=acts)


def test_hand_worked_episodes_on_the_gpu():
    gold = json.load(open(os.path.join(HERE, "golden", "terrain_hand_worked.json")))
    for case in gold["cases"]:
        g = hase.HaseBatch([case["spec"]], device=DEV)
        # the state is loaded, not reset (the tiny maps have no room for
        # every class, which a reset refuses)
        z = np.zeros(1, np.uint32)
        g.set_state(dict(walls=np.array(case["tiles"], np.uint8),
                         pos_x=np.array(case["start"]["pos_x"], np.uint8),
                         pos_y=np.array(case["start"]["pos_y"], np.uint8),
                         found=z, t=z, episode=z, steps=z, seed=np.ones(1, np.uint64), stuck=z))
        for a, want in zip(case["actions"], case["expected"]):
            obs, rew, done = g.step(1, actions=np.array([a], np.int8))
            torch.cuda.synchronize()
            s = g.get_state()
            what = f'{case["name"]}: {want["notes"]}'
            assert [[int(x), int(y)] for x, y in zip(s["pos_x"], s["pos_y"])] == want["pos"], what
            assert int(s["stuck"][0]) == want["stuck"], what
            assert list(rew.cpu().numpy()[0]) == want["rew"], what
            assert u32(obs)[0].reshape(3, 3).tolist() == want["obs"], what
        g.close()


def test_state_round_trip_with_stuck_agents():
    specs = random_terrain_specs(120, 11)
    g = hase.HaseBatch(specs, device=DEV)
    ob = o.OracleBatch(specs)
    g.reset(23)
    ob.reset(23)
    for k in (1, 37, 70):
        gout = g.step(k)
        torch.cuda.synchronize()
        assert_outputs(gout, ob.step(k), f"{k} steps")
        assert_state(g, ob)
    st = g.get_state()
    assert st["stuck"].any()
    g2 = hase.HaseBatch(specs, device=DEV, lanes=[2, 8, 16, 16])
    g2.set_state(st)
    gout = g2.step(50)
    torch.cuda.synchronize()
    assert_outputs(gout, ob.step(50), "after round trip")
    assert_state(g2, ob)
    g.close()
    g2.close()


def test_set_state_rejects_bad_tiles_and_stuck_bits():
    ter = wl.with_terrain(wl.spec(8, 8, 3, 2, 3, 10), 20, 10)
    plain = wl.spec(8, 8, 3, 2, 3, 10)
    g = hase.HaseBatch([ter, plain], device=DEV)
    g.reset(2)
    for field, idx, value in (("walls", 3, 4), ("walls", 64 + 3, 2), ("stuck", 0, 8),
                              ("stuck", 1, 1)):
        st = g.get_state()
        st[field][idx] = value
        with pytest.raises(hase.HaseError) as ei:
            g.set_state(st)
        assert ei.value.code == hase.ESTATE, (field, idx, value)
    g.close()


def test_step_multi_with_terrain_requests():
    specs = [wl.with_terrain(wl.spec(32, 32, 4, 3, 4, 10)),
             dict(wl.with_terrain(wl.spec(16, 24, 6, 2, 3, 15)), flags=wl.DEFAULT_FLAGS |
                  wl.TERRAIN | wl.EXPLORE),
             wl.spec(24, 40, 3, 2, 3, 10)]
    n_envs, steps, seeds = [70, 41, 33], [60, 45, 52], [81, 82, 83]
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


def test_full_size_terrain4k_sampled():
    from tests.test_gpu_parity import sampled_check

    w = wl.WORKLOADS["terrain4k"]
    specs = wl.workload_specs("terrain4k")
    steps = 2000
    print(f"case: full size terrain4k, {len(specs)} envs x {steps} steps", flush=True)
    g = hase.HaseBatch(specs, device=DEV)
    g.reset(w["seed"])
    out = g.step(steps)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(3))
    sample = sorted(set([0, len(specs) - 1] + list(rng.choice(len(specs), 16, replace=False))))
    sampled_check(specs, w["seed"], steps, out, sample)
    g.close()
    del out
    torch.cuda.empty_cache()


EDGE = {
    "max_agents_64x64": wl.with_terrain(wl.spec(64, 64, 20, 4, 4, 10), 20, 15, 40,
                                        (100, 0, 50, 0, 90, 0, 70, 70, 70),
                                        [i % 3 for i in range(20)]),
    "tiny_3x3_flyers": wl.with_terrain(wl.spec(3, 3, 2, 1, 4, 0, L=9), 40, 40, 100, (100,) * 9,
                                       [wl.FLYER, wl.FLYER]),
    "nobody_moves": wl.with_terrain(wl.spec(16, 16, 4, 2, 3, 10), 20, 20, 50, (0,) * 9,
                                    [0, 1, 2, 0]),
    "always_stuck_walkers": wl.with_terrain(wl.spec(16, 16, 6, 3, 3, 5), 10, 60, 100, (100,) * 9,
                                            [wl.WALKER] * 6),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_terrain_edge_specs(name):
    run_pair([EDGE[name]] * 67, seed=12, steps=180)


def test_one_lane_per_env_terrain():
    """Two tile planes per env at one lane per env fit small boards."""
    specs = random_terrain_specs(140, 12, base="small")
    run_pair(specs, seed=29, steps=150, lanes=[1, 1, 4, 8])


def test_reset_refuses_a_class_without_room():
    sp = wl.with_terrain(wl.spec(8, 8, 3, 1, 3, 0), 0, 30, 0, (100,) * 9,
                         [wl.WALKER, wl.SWIMMER, wl.FLYER])
    g = hase.HaseBatch([wl.spec(8, 8, 2, 1, 3, 0), sp], device=DEV)
    with pytest.raises(hase.HaseError) as ei:
        g.reset(3)
    assert ei.value.code == hase.EGRID
    with pytest.raises(ValueError):
        o.OracleBatch([wl.spec(8, 8, 2, 1, 3, 0), sp]).reset(3)
    g.close()
