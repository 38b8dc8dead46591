"""Radio belief sharing (flag 64) on the GPU against the oracle, bit-exact
through the C ABI: radio batches with every other feature in both launch
modes, external actions carrying radio targets, the hand-worked steps, every
radio kind in one batch under several tilings, state round trips with
beliefs, a multi-batch call, and the full-size radio workload sampled."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, workloads as wl  # noqa: E402
from tests.test_gpu_explore import run_maps  # noqa: E402
from tests.test_gpu_parity import DEV, assert_outputs, assert_state, run_pair, u32  # noqa: E402
from tests.test_oracle_radio import radio_specs  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def plain_radio(specs):
    """Radio on the given specs without exploration (those go through run_maps)."""
    return [dict(s, flags=(s["flags"] | wl.RADIO) & ~wl.EXPLORE) for s in specs]


@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_radio_uneven_batch(mode):
    specs = plain_radio(radio_specs(300, 21))
    _, _, done = run_pair(specs, seed=31, steps=200, mode=mode, env_id_base=3)
    assert (done == 2).any()


@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_radio_workload(mode):
    run_pair(wl.workload_specs("radio4k", 150), seed=6, steps=220, mode=mode)


def test_radio_with_exploration():
    run_maps(radio_specs(260, 22), seed=41, steps=180)


def test_external_radio_actions():
    specs = plain_radio(radio_specs(200, 23))
    acts = wl.radio_actions(150, specs, 9, draw_frac=0.25)
    run_pair(specs, seed=43, steps=150, actions=acts)


def test_external_radio_actions_with_exploration():
    specs = radio_specs(150, 24)
    acts = wl.radio_actions(120, specs, 10, draw_frac=0.1)
    run_maps(specs, seed=44, steps=120, actions=acts)


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_every_radio_kind_in_one_batch(lanes):
    """Radio alone and with exploration, line of sight and terrain in every
    combination, beside envs without radio (4 lanes or more: terrain and
    exploration together need it at 2 lanes)."""
    base = wl.workload_specs("uneven8k", 256)
    specs = []
    for i, s in enumerate(base):
        k = i % 16
        sp = dict(s, flags=s["flags"] | (wl.EXPLORE if k & 1 else 0) | (wl.OCCLUDE if k & 2 else 0) |
                  (wl.RADIO if k & 8 else 0))
        if k & 4:
            sp = wl.with_terrain(sp, 15, 10, 40, None, [i % 3 for i in range(sp["n"])])
        specs.append(sp)
    run_maps(specs, seed=51, steps=150, lanes=[lanes, lanes, max(lanes, 4), max(lanes, 8)])


def test_one_and_two_lanes_per_env():
    specs = plain_radio(radio_specs(120, 25))
    # one lane per env holds 64 boards in a wave's LDS: terrain (two planes)
    # only on 16-cell sides
    small = [s for s in specs if s["H"] <= (16 if s["flags"] & wl.TERRAIN else 32)][:100]
    run_pair(small, seed=53, steps=150, lanes=[1, 2, 4, 8])
    run_pair(small, seed=54, steps=150, lanes=[2, 1, 4, 8])


def test_hand_worked_steps_on_the_gpu():
    gold = json.load(open(os.path.join(HERE, "golden", "radio_hand_worked.json")))
    for case in gold["cases"]:
        sp = case["spec"]
        n = sp["n"]
        g = hase.HaseBatch([sp], device=DEV)
        z = np.zeros(1, np.uint32)
        g.set_state(dict(walls=np.zeros(sp["H"] * sp["W"], np.uint8),
                         pos_x=np.array(case["start"]["pos_x"], np.uint8),
                         pos_y=np.array(case["start"]["pos_y"], np.uint8),
                         found=z, t=z, episode=z, steps=z, seed=np.ones(1, np.uint64),
                         belief=np.zeros(n, np.uint32)))
        for a, want in zip(case["actions"], case["expected"]):
            obs, rew, done = g.step(1, actions=np.array([a], np.int8))
            torch.cuda.synchronize()
            s = g.get_state()
            what = f'{case["name"]}: {want["notes"]}'
            assert s["belief"].tolist() == want["belief"], what
            assert int(s["found"][0]) == want["found"], what
            assert list(rew.cpu().numpy()[0]) == want["rew"], what
            assert int(done.cpu().numpy()[0, 0]) == want["done"], what
            per = u32(obs)[0].reshape(n, -1)
            if "obs" in want:
                assert per.tolist() == want["obs"], what
                assert [[int(x), int(y)] for x, y in zip(s["pos_x"], s["pos_y"])] == want["pos"], what
            else:
                assert per[:, -1].tolist() == want["belief_words"], what
        g.close()


def test_state_round_trip_with_beliefs():
    specs = plain_radio(radio_specs(90, 26))
    g = hase.HaseBatch(specs, device=DEV)
    ob = o.OracleBatch(specs)
    g.reset(27)
    ob.reset(27)
    for k in (1, 29, 60):
        gout = g.step(k)
        torch.cuda.synchronize()
        assert_outputs(gout, ob.step(k), f"{k} steps")
        assert_state(g, ob)
    st = g.get_state()
    assert st["belief"].any()
    g2 = hase.HaseBatch(specs, device=DEV, lanes=[2, 8, 16, 16])
    g2.set_state(st)
    np.testing.assert_array_equal(u32(g2.observe()), ob.observe(), err_msg="observe")
    gout = g2.step(40)
    torch.cuda.synchronize()
    assert_outputs(gout, ob.step(40), "after round trip")
    assert_state(g2, ob)
    g.close()
    g2.close()


def test_set_state_rejects_bad_beliefs():
    radio = wl.spec(8, 8, 4, 2, 3, 10, S=2, flags=wl.DEFAULT_FLAGS | wl.RADIO)
    plain = wl.spec(8, 8, 4, 2, 3, 10, S=2)
    g = hase.HaseBatch([radio, plain], device=DEV)
    g.reset(2)
    for idx, value in ((0, 1), (1, 2), (2, 1 << 4), (4, 1 << 2)):
        st = g.get_state()
        st["belief"][idx] = value
        with pytest.raises(hase.HaseError) as ei:
            g.set_state(st)
        assert ei.value.code == hase.ESTATE, (idx, value)
    st = g.get_state()
    st["belief"][1] = 0b1100  # both hiders of the radio env: accepted
    g.set_state(st)
    assert g.get_state()["belief"][1] == 0b1100
    g.close()


def test_step_multi_with_radio_requests():
    specs = [wl.spec(32, 32, 10, 4, 4, 10, flags=wl.DEFAULT_FLAGS | wl.RADIO),
             dict(wl.with_terrain(wl.spec(16, 24, 6, 2, 3, 15)), flags=wl.DEFAULT_FLAGS |
                  wl.TERRAIN | wl.EXPLORE | wl.RADIO),
             wl.spec(24, 40, 3, 2, 3, 10)]
    n_envs, steps, seeds = [70, 41, 33], [60, 45, 52], [91, 92, 93]
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
        assert_state(b, ob)


def test_full_size_radio4k_sampled():
    from tests.test_gpu_parity import sampled_check

    w = wl.WORKLOADS["radio4k"]
    specs = wl.workload_specs("radio4k")
    steps = 2000
    print(f"case: full size radio4k, {len(specs)} envs x {steps} steps", flush=True)
    g = hase.HaseBatch(specs, device=DEV)
    g.reset(w["seed"])
    out = g.step(steps)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(4))
    sample = sorted(set([0, len(specs) - 1] + list(rng.choice(len(specs), 16, replace=False))))
    sampled_check(specs, w["seed"], steps, out, sample)
    g.close()
    del out
    torch.cuda.empty_cache()


R = wl.DEFAULT_FLAGS | wl.RADIO
EDGE = {
    "max_agents_64x64_one_seeker": wl.spec(64, 64, 20, 4, 4, 10, S=1, flags=R),
    "max_agents_64x64_one_hider": wl.spec(64, 64, 20, 4, 4, 10, S=19, flags=R | wl.OCCLUDE),
    "no_seekers": wl.spec(16, 16, 6, 2, 3, 10, S=0, flags=R),
    "no_hiders": wl.spec(16, 16, 6, 2, 3, 10, S=6, flags=R),
    "alone": wl.spec(8, 8, 1, 1, 3, 10, S=1, flags=R),
    "collisions_off": wl.spec(12, 12, 10, 2, 3, 5, flags=R & ~wl.COLLIDE),
    "capture_ends_tiny": wl.spec(6, 6, 8, 3, 4, 0, S=4, flags=R, L=30),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_radio_edge_specs(name):
    run_pair([EDGE[name]] * 67, seed=12, steps=160)


@pytest.mark.parametrize("lanes", [[1, 2, 4, 8], [2, 4, 8, 16], [16, 16, 16, 16]])
def test_radio_edge_specs_every_tiling(lanes):
    specs = [s for s in EDGE.values() if s["H"] <= 16 or lanes[3] >= 8]
    acts = wl.radio_actions(120, specs * 9, 15, draw_frac=0.3)
    run_pair(specs * 9, seed=13, steps=120, actions=acts, lanes=lanes)
