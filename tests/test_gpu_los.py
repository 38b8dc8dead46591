"""Line of sight (flag 8) on the GPU against the oracle, bit-exact through the
C ABI: occluded workloads in both launch modes, collisions off, the
brute-force 4x4 families with occlusion, batches mixing occluding and plain
envs under every tiling, and a multi-batch call mixing both kinds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, workloads as wl  # noqa: E402
from tests import bruteforce_spec as bf  # noqa: E402
from tests.test_gpu_parity import DEV, assert_outputs, assert_state, run_pair, u32  # noqa: E402

pytestmark = pytest.mark.gpu


def occluded(specs, flags=None):
    return [dict(s, flags=(s["flags"] if flags is None else flags) | wl.OCCLUDE) for s in specs]


@pytest.mark.parametrize("name,ne,steps", [("small", 700, 260), ("single1k", 333, 300),
                                           ("multi10", 123, 300), ("uneven8k", 611, 280)])
@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_occluded_workloads(name, ne, steps, mode):
    specs = occluded(wl.workload_specs(name, ne))
    _, _, done = run_pair(specs, seed=200 + len(name), steps=steps, mode=mode, env_id_base=3)
    assert (done == 2).any()


def test_occluded_collisions_off_and_external_actions():
    specs = occluded(wl.workload_specs("uneven8k", 301), flags=wl.CAPTURE_ENDS | wl.DESYNC)
    agents = sum(s["n"] for s in specs)
    acts = wl.random_actions(140, agents, seed=9, draw_frac=0.3, invalid_frac=0.05)
    run_pair(specs, seed=41, steps=140, actions=acts)


BF_OCC = {
    "one_agent_occluded_r3": lambda: bf.case_one_agent(r=3, C=4, flags=8 | 3, subsample=100_000,
                                                       seed=7),
    "one_agent_occluded_r4": lambda: bf.case_one_agent(r=4, C=3, flags=8 | 1, subsample=60_000,
                                                       seed=10),
    "seeker_hider_occluded_r3": lambda: bf.case_seeker_hider(n_patterns=96, r=3, C=4, flags=8 | 1,
                                                             seed=8),
    "seeker_hider_occluded_capture": lambda: bf.case_seeker_hider(n_patterns=64, r=2, C=3,
                                                                  flags=8 | 3, seed=9),
    "seeker_hider_occluded_no_collide": lambda: bf.case_seeker_hider(n_patterns=48, r=4, C=4,
                                                                     flags=8, seed=11),
}


@pytest.mark.parametrize("family", list(BF_OCC))
def test_occluded_bruteforce(family):
    spec, st, acts = BF_OCC[family]()
    B = st["pos_x"].shape[0]
    print(f"case: brute force {family}, {B} envs", flush=True)
    flat = bf.flat_state(st)
    g = hase.HaseBatch([spec] * B, device=DEV)
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


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
def test_mixed_occluding_and_plain_envs(lanes):
    """Occluding and plain envs interleaved in one batch (same variants)."""
    base = wl.workload_specs("uneven8k", 260)
    specs = [dict(s, flags=s["flags"] | (wl.OCCLUDE if i % 3 else 0)) for i, s in enumerate(base)]
    run_pair(specs, seed=57, steps=120,
             lanes=[lanes, lanes, max(lanes, 4), max(lanes, 8)])


def test_uniform_occluded_batch_state_roundtrip():
    """An occluded uniform batch (one variant, routed to the mixed kernel) is
    checked step by step across three calls, with the state read back."""
    specs = occluded(wl.workload_specs("single1k", 129))
    g = hase.HaseBatch(specs, device=DEV)
    ob = o.OracleBatch(specs)
    np.testing.assert_array_equal(u32(g.reset(5)), ob.reset(5))
    for k in (1, 37, 90):
        gout = g.step(k)
        torch.cuda.synchronize()
        assert_outputs(gout, ob.step(k), f"{k} steps")
        assert_state(g, ob)
    g.close()


def test_step_multi_with_occluded_request():
    specs = [wl.spec(32, 32, 2, 3, 3, 15, flags=wl.DEFAULT_FLAGS | wl.OCCLUDE),
             wl.spec(16, 16, 6, 2, 4, 20)]
    n_envs, steps, seeds = [90, 41], [50, 35], [71, 72]
    bs = []
    for sp, ne, sd in zip(specs, n_envs, seeds):
        b = hase.HaseBatch([sp] * ne, device=DEV)
        b.reset(sd)
        bs.append(b)
    outs = [b.alloc_outputs(k) for b, k in zip(bs, steps)]
    ws = torch.empty(hase.multi_workspace_bytes(bs), dtype=torch.uint8, device=DEV)
    items = [(b, k, 0, None, *out) for b, k, out in zip(bs, steps, outs)]
    hase.step_multi(items, max(steps), ws, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for sp, ne, sd, k, out in zip(specs, n_envs, seeds, steps, outs):
        ob = o.OracleBatch([sp] * ne)
        ob.reset(sd)
        assert_outputs(out, ob.step(k))
