"""The per-step true-state output (observability modes with the true state,
Sec. 3.3) against the oracle's state after every step, element by element,
in both launch modes and for every env kind in one batch; and for an arena
range."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def kinds_specs(per_kind=9):
    base = [wl.spec(16, 16, 2, 2, 3, 10), wl.spec(24, 20, 7, 3, 4, 15, L=40),
            wl.spec(40, 33, 12, 4, 4, 12, L=60), wl.spec(9, 9, 4, 1, 3, 20, L=13)]
    feats = [0, wl.OCCLUDE, wl.EXPLORE, wl.OCCLUDE | wl.EXPLORE, wl.RADIO, wl.RADIO | wl.EXPLORE]
    out = []
    for i, f in enumerate(feats):
        for j in range(per_kind):
            out.append(dict(base[(i + j) % 4], flags=base[(i + j) % 4]["flags"] | f))
    for j in range(per_kind):
        out.append(wl.with_terrain(base[j % 4]))
        out.append(wl.with_terrain(dict(base[(j + 1) % 4], flags=base[(j + 1) % 4]["flags"] | wl.OCCLUDE | wl.RADIO)))
    return out


def oracle_states(ob, steps, actions=None):
    """The oracle's state after each of `steps` single steps."""
    pos, env = [], []
    for k in range(steps):
        ob.step(1, actions=None if actions is None else actions[k:k + 1])
        st = ob.get_state()
        pos.append(st["pos_x"].astype(np.uint16) | (st["pos_y"].astype(np.uint16) << 8))
        env.append(np.stack([st["found"], st["t"], st["episode"], st["stuck"]], axis=1))
    return np.array(pos), np.array(env).astype(np.uint32)


@pytest.mark.parametrize("mode", [hase.PERSISTENT, hase.PER_LAUNCH])
def test_true_state_every_kind(mode):
    specs = kinds_specs()
    steps = 70
    print(f"case: true state, {len(specs)} envs, mode {mode}", flush=True)
    g = hase.HaseBatch(specs, env_id_base=4, device=DEV)
    ob = o.OracleBatch(specs, env_id_base=4)
    g.reset(77)
    ob.reset(77)
    obs, rew, done, mp, pos, env = g.step(steps, mode=mode, maps=True, state=True)
    torch.cuda.synchronize()
    want_pos, want_env = oracle_states(ob, steps)
    assert np.array_equal(pos.cpu().numpy().view(np.uint16), want_pos)
    assert np.array_equal(env.cpu().numpy().view(np.uint32), want_env)
    # and the last row is the state hase_get_state returns
    st = g.get_state()
    assert np.array_equal(st["found"], want_env[-1, :, 0]) and np.array_equal(st["t"], want_env[-1, :, 1])
    # episodes ended, hiders found and agents stuck along the way
    assert (want_env[:, :, 2] > 0).any() and (want_env[:, :, 0] != 0).any()
    assert (want_env[:, :, 3] != 0).any()
    g.close()


def test_true_state_with_external_actions():
    specs = wl.workload_specs("uneven8k", 97)
    agents = sum(s["n"] for s in specs)
    acts = wl.random_actions(50, agents, seed=5, draw_frac=0.2, invalid_frac=0.05)
    g = hase.HaseBatch(specs, device=DEV)
    ob = o.OracleBatch(specs)
    g.reset(8)
    ob.reset(8)
    _, _, _, pos, env = g.step(50, actions=acts, state=True)
    torch.cuda.synchronize()
    want_pos, want_env = oracle_states(ob, 50, acts)
    assert np.array_equal(pos.cpu().numpy().view(np.uint16), want_pos)
    assert np.array_equal(env.cpu().numpy().view(np.uint32), want_env)
    g.close()


def test_true_state_of_an_arena_range():
    spec = wl.with_terrain(wl.spec(20, 24, 6, 3, 4, 10, L=30))
    ar = hase.HaseArena(300, max_height=32, max_width=32, max_agents=10, max_ranges=4, device=DEV)
    out = ar.alloc_outputs(spec, 45, 60, state=True)
    ar.reset_range(100, 45, spec, 12, 60, out, env_id_base=3)
    ar.step(25)
    ar.step(50)
    torch.cuda.synchronize()
    ob = o.OracleBatch([spec] * 45, env_id_base=3)
    ob.reset(12)
    want_pos, want_env = oracle_states(ob, 60)
    assert np.array_equal(out["pos"].cpu().numpy().view(np.uint16), want_pos)
    assert np.array_equal(out["env_state"].cpu().numpy().view(np.uint32), want_env)
    ar.close()
