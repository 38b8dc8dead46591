"""HIP library vs the CPU oracle, bit-exact, through the C ABI (python binding).

Sizes: the oracle finishes each case in seconds; env counts are not multiples
of any tile size (ragged last tiles) and runs cross episode boundaries. The
full-size cases run the workloads' real shapes in the benchmark's launch
configuration and check sampled envs against one-env oracle runs (an env's
trajectory depends only on its seed, id and spec).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, workloads as wl  # noqa: E402
from tests import bruteforce_spec as bf  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def fbits(t):
    return t.detach().cpu().numpy().view(np.uint32)


def assert_outputs(g_out, o_out, what=""):
    go, gr, gd = g_out
    oo, orr, od = o_out
    np.testing.assert_array_equal(u32(go).reshape(oo.shape), oo, err_msg=f"obs {what}")
    np.testing.assert_array_equal(fbits(gr).reshape(orr.shape), orr.view(np.uint32),
                                  err_msg=f"rew {what}")
    np.testing.assert_array_equal(gd.cpu().numpy().reshape(od.shape), od, err_msg=f"done {what}")


def assert_state(g, ob):
    st = g.get_state()
    for k, v in ob.get_state().items():
        if k != "env_id":
            np.testing.assert_array_equal(st[k], v, err_msg=f"state {k}")


def run_pair(specs, seed, steps, env_id_base=0, actions=None, mode=hase.PERSISTENT, lanes=None):
    print(f"case: {len(specs)} envs, {steps} steps, seed {seed}, mode {mode}, lanes {lanes}",
          flush=True)
    g = hase.HaseBatch(specs, env_id_base=env_id_base, device=DEV, lanes=lanes)
    ob = o.OracleBatch(specs, env_id_base=env_id_base)
    np.testing.assert_array_equal(u32(g.reset(seed)), ob.reset(seed), err_msg="obs0")
    assert_state(g, ob)
    gout = g.step(steps, actions=actions, mode=mode)
    torch.cuda.synchronize()
    oout = ob.step(steps, actions=actions)
    assert_outputs(gout, oout)
    assert_state(g, ob)
    g.close()
    return oout


WORKLOADS = [("small", 1000, 300), ("single1k", 333, 600), ("multi10", 123, 320),
             ("uneven8k", 611, 300)]


@pytest.mark.parametrize("name,ne,steps", WORKLOADS)
@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_workload_trajectories(name, ne, steps, mode):
    specs = wl.workload_specs(name, ne)
    _, _, done = run_pair(specs, seed=100 + len(name), steps=steps, mode=mode, env_id_base=7)
    assert (done == 2).any()  # truncations happened
    if name in ("small", "multi10"):
        assert (done & 1).any()  # captures happened


@pytest.mark.parametrize("name", ["small", "multi10", "uneven8k"])
def test_external_actions_with_draws_and_invalid(name):
    specs = wl.workload_specs(name, 157)
    agents = sum(s["n"] for s in specs)
    acts = wl.random_actions(150, agents, seed=3, draw_frac=0.25, invalid_frac=0.1)
    run_pair(specs, seed=31, steps=150, actions=acts)


BF_FAMILIES = {
    "one_agent_all_walls_r1": lambda: bf.case_one_agent(r=1, C=4),
    "one_agent_r4_sample": lambda: bf.case_one_agent(r=4, C=4, subsample=100_000, seed=4),
    "one_agent_truncate": lambda: bf.case_one_agent(r=1, C=3, L=1, subsample=50_000, seed=5),
    "seeker_hider_capture_off": lambda: bf.case_seeker_hider(n_patterns=256, flags=1),
    "seeker_hider_capture_on": lambda: bf.case_seeker_hider(n_patterns=64, flags=3, seed=2),
    "seeker_hider_r3_no_collide": lambda: bf.case_seeker_hider(n_patterns=32, r=3, C=4, flags=0,
                                                               seed=6),
    "three_agents_open": lambda: bf.case_three_agents(r=2, C=3, flags=1),
    "three_agents_capture": lambda: bf.case_three_agents(r=1, C=4, flags=3, S=1),
}


@pytest.mark.parametrize("family", list(BF_FAMILIES))
def test_bruteforce_cases(family):
    spec, st, acts = BF_FAMILIES[family]()
    B = st["pos_x"].shape[0]
    print(f"case: brute force {family}, {B} envs", flush=True)
    specs = [spec] * B
    flat = bf.flat_state(st)
    g = hase.HaseBatch(specs, device=DEV)
    g.set_state(flat)
    ob = o.OracleBatch(np.tile(o.spec_table([spec]), (B, 1)))
    ob.set_state(flat)
    np.testing.assert_array_equal(u32(g.observe()), ob.observe(), err_msg="observe")
    gout = g.step(1, actions=acts.reshape(1, -1))
    torch.cuda.synchronize()
    oout = ob.step(1, actions=acts.reshape(1, -1))
    assert_outputs(gout, oout, family)
    assert_state(g, ob)
    g.close()


EDGE_SPECS = {
    "tiny_2x2_r4": wl.spec(2, 2, 2, 4, 4, 0, L=7),
    "max_agents_64x64": wl.spec(64, 64, 20, 4, 4, 25),
    "max_agents_small_grid": wl.spec(5, 5, 20, 2, 3, 0),
    "no_hiders": wl.spec(16, 16, 3, 2, 4, 10, S=3),
    "no_seekers": wl.spec(16, 16, 3, 2, 4, 10, S=0),
    "single_agent": wl.spec(12, 7, 1, 1, 3, 20),
    "episode_len_1": wl.spec(8, 8, 4, 3, 4, 10, L=1),
    "no_flags": wl.spec(20, 30, 6, 3, 3, 15, flags=0),
    "dense_walls": wl.spec(10, 10, 4, 2, 4, 90),
    "open_wide": wl.spec(3, 64, 8, 4, 3, 0),
    "tall": wl.spec(64, 3, 8, 4, 4, 5),
    "odd_sizes": wl.spec(37, 45, 11, 3, 4, 17),
}


@pytest.mark.parametrize("name", list(EDGE_SPECS))
def test_edge_specs(name):
    specs = [EDGE_SPECS[name]] * 70
    run_pair(specs, seed=9, steps=90)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
def test_every_tiling_matches(lanes):
    """Variants exist for at most 4 agents per lane."""
    specs = wl.workload_specs("uneven8k", 301) + [EDGE_SPECS["max_agents_64x64"]] * 5
    run_pair(specs, seed=55, steps=120, lanes=[lanes, lanes, max(lanes, 4), max(lanes, 8)])


@pytest.mark.parametrize("lanes", [[4, 4, 16, 16], [16, 4, 16, 8], [4, 16, 16, 16]])
def test_two_width_launch_matches(lanes):
    """Plain envs at 4 and 16 lanes per env in one combined launch (the
    default tiling of uneven plain batches), beside a 20-agent bucket."""
    specs = wl.workload_specs("uneven8k", 411) + [EDGE_SPECS["max_agents_64x64"]] * 7
    run_pair(specs, seed=57, steps=150, lanes=lanes)
    run_pair(specs, seed=58, steps=40, lanes=lanes, mode=hase.PER_LAUNCH)


@pytest.mark.parametrize("agents", [(1, 10), (5, 10), (1, 8), (5, 8)])
def test_three_width_launch_matches(agents):
    """The combined launch with envs of the 10-agent bucket that have at most
    8 agents at 8 lanes per env: all three widths, only 8 and 16, only 4 and
    8, only 8. Counts are ragged for every width and radius; 16x16 grids with
    many agents end episodes often, so respawns run in every tile."""
    lo, hi = agents
    specs = [s for s in wl.workload_specs("uneven8k", 1400) if lo <= s["n"] <= hi][:333]
    specs += [wl.spec(16, 16, n, r, 4, 20, L=40) for n in range(max(lo, 5), min(hi, 8) + 1)
              for r in (1, 2, 3, 4)] * 3
    run_pair(specs, seed=61, steps=150)
    run_pair(specs, seed=62, steps=40, mode=hase.PER_LAUNCH)


def test_unsupported_tiling_rejected():
    g = hase.HaseBatch(wl.workload_specs("multi10", 16), device=DEV)
    with pytest.raises(hase.HaseError) as ei:
        g.set_tiling([4, 4, 2, 16])  # 10 agents on 2 lanes: 5 agents per lane
    assert ei.value.code == hase.EINVAL
    assert g.get_tiling() == [4, 4, 16, 16]


def test_mixed_edge_specs_one_batch():
    specs = [EDGE_SPECS[k] for k in EDGE_SPECS] * 9
    run_pair(specs, seed=10, steps=80, lanes=[2, 8, 4, 16])


def test_too_few_free_cells_is_reported():
    """Same first failing env as the oracle (5x5 grids, 20 agents, 10% walls)."""
    specs = [wl.spec(8, 8, 2, 2, 3, 10)] * 10 + [wl.spec(5, 5, 20, 1, 3, 10)] * 60
    g = hase.HaseBatch(specs, device=DEV)
    with pytest.raises(hase.HaseError) as ei:
        g.reset(9)
    assert ei.value.code == hase.EGRID
    with pytest.raises(ValueError) as eo:
        o.OracleBatch(specs).reset(9)
    bad = int(str(eo.value).split()[1])
    assert f"env {bad} " in str(ei.value)
    with pytest.raises(hase.HaseError) as ei:
        g.step(1)
    assert ei.value.code == hase.ENOTREADY


def crowded_state(specs, seed):
    """Host state of 8x8 envs with n + 1 or n + 2 open cells (agents on the
    first n of them): every respawn rejects most draws and often scans."""
    g = np.random.Generator(np.random.PCG64(seed))
    walls, px, py = [], [], []
    for s in specs:
        free = g.choice(64, size=s["n"] + int(g.integers(1, 3)), replace=False)
        w = np.ones(64, np.uint8)
        w[free] = 0
        walls.append(w)
        px += [int(c) % 8 for c in free[:s["n"]]]
        py += [int(c) // 8 for c in free[:s["n"]]]
    ne = len(specs)
    return dict(walls=np.concatenate(walls), pos_x=np.array(px, np.uint8),
                pos_y=np.array(py, np.uint8), found=np.zeros(ne, np.uint32),
                t=np.zeros(ne, np.uint32), episode=g.integers(0, 1000, ne).astype(np.uint32),
                steps=g.integers(0, 1000, ne).astype(np.uint32),
                seed=g.integers(0, 2**63, ne).astype(np.uint64))


@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_crowded_respawns(lanes):
    """Episodes of one step on crowded 8x8 grids: every step respawns agents
    that reject most draws, exhaust their 64 attempts and scan (the spawn
    rule beyond agent 0's first draw), in every bucket."""
    specs = [wl.spec(8, 8, n, 2, 4, 0, L=1) for n in (2, 3, 4, 6, 9, 10, 13, 20) for _ in range(23)]
    st = crowded_state(specs, seed=lanes)
    print(f"case: crowded respawns, lanes {lanes}", flush=True)
    g = hase.HaseBatch(specs, env_id_base=3, device=DEV,
                       lanes=[lanes, lanes, max(lanes, 4), max(lanes, 8)])
    g.set_state(st)
    ob = o.OracleBatch(specs, env_id_base=3)
    ob.set_state(dict(st, env_id=np.arange(3, 3 + len(specs), dtype=np.uint32)))
    gout = g.step(60)
    torch.cuda.synchronize()
    oout = ob.step(60)
    assert_outputs(gout, oout, f"crowded lanes {lanes}")
    assert_state(g, ob)
    g.close()


def test_set_state_without_room_is_rejected():
    """A loaded grid with fewer open cells than agents is refused before any
    step (an auto-reset could not place every agent)."""
    specs = [wl.spec(8, 8, 4, 2, 4, 0, L=5)] * 6
    st = crowded_state(specs, seed=1)
    good = {k: v.copy() for k, v in st.items()}
    w = st["walls"].reshape(6, 64)
    # env 4: only 3 open cells for 4 agents (one agent's cell becomes a wall)
    bad = np.flatnonzero(w[4] == 0)
    w[4][bad[3:]] = 1
    w[4][bad[:3]] = 0
    st["pos_x"][4 * 4 + 3], st["pos_y"][4 * 4 + 3] = st["pos_x"][4 * 4], st["pos_y"][4 * 4]
    g = hase.HaseBatch(specs, device=DEV)
    with pytest.raises(hase.HaseError) as ei:
        g.set_state(st)
    assert ei.value.code == hase.EGRID and "env 4 " in str(ei.value)
    with pytest.raises(hase.HaseError) as ei:
        g.step(1)
    assert ei.value.code == hase.ENOTREADY
    g.set_state(good)
    g.step(3)
    g.close()


def test_checkpoint_resume():
    specs = wl.workload_specs("uneven8k", 200)
    a = hase.HaseBatch(specs, device=DEV)
    a.reset(77)
    a.step(150)
    st = a.get_state()
    full = a.step(150)
    b = hase.HaseBatch(specs, device=DEV)
    b.set_state(st)
    resumed = b.step(150)
    torch.cuda.synchronize()
    for x, y in zip(full, resumed):
        assert torch.equal(x, y)


def test_shards_reproduce_one_batch():
    """Two handles over env-id ranges [0,N/2) and [N/2,N) equal one handle."""
    specs = wl.workload_specs("uneven8k", 240)
    whole = hase.HaseBatch(specs, device=DEV)
    h1 = hase.HaseBatch(specs[:120], env_id_base=0, device=DEV)
    h2 = hase.HaseBatch(specs[120:], env_id_base=120, device=DEV)
    w0, a0, b0 = whole.reset(5), h1.reset(5), h2.reset(5)
    assert torch.equal(w0, torch.cat([a0, b0]))
    wo, wr, wd = whole.step(100)
    ao, ar, ad = h1.step(100)
    bo, br, bd = h2.step(100)
    assert torch.equal(wo, torch.cat([ao, bo], 1))
    assert torch.equal(wr, torch.cat([ar, br], 1))
    assert torch.equal(wd, torch.cat([ad, bd], 1))


def test_graph_replay_continues_trajectory():
    """Repeated persistent calls into the same buffers replay one captured
    graph; every call continues the trajectory."""
    specs = wl.workload_specs("multi10", 90)
    g = hase.HaseBatch(specs, device=DEV)
    ob = o.OracleBatch(specs)
    g.reset(8)
    ob.reset(8)
    bufs = g.alloc_outputs(40)
    for call in range(4):
        g.step_into(*bufs, 40)
        torch.cuda.synchronize()
        assert_outputs(bufs, ob.step(40), f"call {call}")
    # a different step count in between captures another graph
    assert_outputs(g.step(7), ob.step(7), "7 steps")
    g.step_into(*bufs, 40)
    torch.cuda.synchronize()
    assert_outputs(bufs, ob.step(40), "after")


# ---------------------------------------------------------------- full size

def sampled_check(specs, seed, steps, g_out, sample, env_id_base=0):
    obs_off, agent_off = offsets(specs)
    go, gr, gd = g_out
    for e in sample:
        s = specs[e]
        nw = obs_words(s)
        one = o.OracleBatch([s], env_ids=[env_id_base + e])
        one.reset(seed)
        oo, orr, od = one.step(steps)
        np.testing.assert_array_equal(u32(go[:, obs_off[e]:obs_off[e] + nw]), oo,
                                      err_msg=f"obs env {e}")
        np.testing.assert_array_equal(fbits(gr[:, agent_off[e]:agent_off[e] + s["n"]]),
                                      orr.view(np.uint32), err_msg=f"rew env {e}")
        np.testing.assert_array_equal(gd[:, e].cpu().numpy(), od[:, 0], err_msg=f"done env {e}")


def obs_words(s):
    """Observation words of one env per step (radio envs: plus one belief
    word per agent)."""
    d = 2 * s["r"] + 1
    return s["n"] * (s["C"] * ((d * d + 31) // 32) + (1 if s["flags"] & wl.RADIO else 0))


def offsets(specs):
    ow = [obs_words(s) for s in specs]
    na = [s["n"] for s in specs]
    return np.concatenate([[0], np.cumsum(ow)[:-1]]), np.concatenate([[0], np.cumsum(na)[:-1]])


FULL = [("small", 256, 48), ("single16k", 10000, 24), ("single1k", 10000, 24),
        ("multi10", 2000, 24), ("uneven8k", 2000, 40), ("los16k", 4000, 24)]


@pytest.mark.parametrize("name,steps,n_sample", FULL)
def test_full_size_sampled(name, steps, n_sample):
    w = wl.WORKLOADS[name]
    specs = wl.workload_specs(name)
    print(f"case: full size {name}, {len(specs)} envs x {steps} steps", flush=True)
    g = hase.HaseBatch(specs, device=DEV)
    g.reset(w["seed"])
    out = g.step(steps)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(1))
    sample = sorted(set([0, len(specs) - 1] + list(rng.choice(len(specs), n_sample, replace=False))))
    sampled_check(specs, w["seed"], steps, out, sample)
    del out
    g.close()
    torch.cuda.empty_cache()


def test_full_size_per_launch_equals_persistent():
    specs = wl.workload_specs("single16k")
    a = hase.HaseBatch(specs, device=DEV)
    b = hase.HaseBatch(specs, device=DEV)
    a.reset(2)
    b.reset(2)
    x = a.step(300, mode=hase.PERSISTENT)
    y = b.step(300, mode=hase.PER_LAUNCH)
    torch.cuda.synchronize()
    for p, q in zip(x, y):
        assert torch.equal(p, q)
