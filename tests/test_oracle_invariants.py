"""Multi-step invariants and closed forms of the oracle."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2604_27162_amd import workloads as wl
from tests.invariants import check_invariants


def run_checked(specs, seed, steps, actions=None):
    b = o.OracleBatch(specs)
    b.reset(seed)
    n_done = 0
    for k in range(steps):
        prev = b.get_state()
        act = None if actions is None else actions[k:k + 1]
        obs, rew, done = b.step(1, actions=act)
        check_invariants(b.spec, prev, b.get_state(), obs[0], rew[0], done[0])
        n_done += int((done[0] != 0).sum())
    return n_done


@pytest.mark.parametrize("name,ne,steps", [("small", 24, 300), ("single1k", 8, 300),
                                           ("multi10", 6, 200), ("uneven8k", 24, 120)])
def test_invariants_workloads(name, ne, steps):
    specs = wl.workload_specs(name, ne)
    assert run_checked(specs, seed=11, steps=steps) > 0


def test_invariants_external_actions_with_draws_and_invalid():
    specs = wl.workload_specs("multi10", 4)
    acts = wl.random_actions(120, 40, seed=9, draw_frac=0.3, invalid_frac=0.1)
    run_checked(specs, seed=12, steps=120, actions=acts)


def test_truncation_count_closed_form():
    """Capture off: env with initial elapsed time t0 truncates floor((t0+T)/L)
    times in T steps."""
    L, T = 37, 500
    specs = [wl.spec(8, 8, 2, 2, 3, 10, flags=wl.COLLIDE | wl.DESYNC, L=L)] * 64
    b = o.OracleBatch(specs)
    b.reset(5)
    t0 = b.t.astype(np.int64).copy()
    _, _, done = b.step(T)
    assert np.array_equal((done == 2).sum(0), (t0 + T) // L)
    assert not (done & 1).any()


def test_desync_uniform():
    L = 16
    specs = [wl.spec(4, 4, 1, 1, 3, 0, flags=wl.DESYNC, L=L)] * 8000
    b = o.OracleBatch(specs)
    b.reset(3)
    cnt = np.bincount(b.t.astype(np.int64), minlength=L)
    exp = len(specs) / L
    assert ((cnt - exp) ** 2 / exp).sum() < 37.7  # 0.999 quantile, 15 dof
    b2 = o.OracleBatch([wl.spec(4, 4, 1, 1, 3, 0, flags=0, L=L)] * 10)
    b2.reset(3)
    assert (b2.t == 0).all()


def test_random_walk_uniform_stationary():
    """One agent on an open 5x5 grid: the lazy walk with rejected moves at the
    border is symmetric, so its stationary law is uniform over the 25 cells."""
    specs = [wl.spec(5, 5, 1, 1, 3, 0, flags=0, L=65535)] * 6000
    b = o.OracleBatch(specs)
    b.reset(21)
    b.step(200)
    cell = b.py.astype(np.int64) * 5 + b.px
    cnt = np.bincount(cell, minlength=25)
    exp = len(specs) / 25
    assert ((cnt - exp) ** 2 / exp).sum() < 51.2  # 0.999 quantile, 24 dof


def test_spawn_uniform_and_distinct():
    """Open 6x6 grid: agent 0's first draw is always accepted, so it is uniform
    over the 36 cells; agents never share a cell."""
    sp = wl.spec(6, 6, 3, 2, 1, 0, flags=0)
    walls = np.zeros(36, np.uint8)
    cnt = np.zeros(36, np.int64)
    for env in range(7200):
        px, py = o.spawn(sp, walls, seed=8, env=env, episode=env % 5)
        cells = py.astype(int) * 6 + px
        assert len(set(cells.tolist())) == 3
        cnt[cells[0]] += 1
    exp = 7200 / 36
    assert ((cnt - exp) ** 2 / exp).sum() < 66.6  # 0.999 quantile, 35 dof


def test_spawn_fallback_exact_free_cells():
    """Exactly n free cells: whatever the draws, the n agents take all of them."""
    g = np.random.Generator(np.random.PCG64(4))
    for trial in range(40):
        n = int(g.integers(1, 8))
        free = g.choice(64, size=n, replace=False)
        walls = np.ones(64, np.uint8)
        walls[free] = 0
        sp = wl.spec(8, 8, n, 1, 1, 0, flags=0)
        px, py = o.spawn(sp, walls, seed=trial, env=trial, episode=trial)
        assert sorted((py.astype(int) * 8 + px).tolist()) == sorted(free.tolist())


def test_reset_rejects_too_few_free_cells():
    sp = wl.spec(2, 2, 4, 2, 1, 99, flags=0)
    b = o.OracleBatch([sp] * 3)
    with pytest.raises(ValueError):
        b.reset(1)


def test_wall_density_binomial():
    sp = wl.spec(64, 64, 1, 1, 1, 25, flags=0)
    b = o.OracleBatch([sp] * 40)
    b.reset(17)
    frac = b.walls.mean()
    sd = np.sqrt(0.25 * 0.75 / b.walls.size)
    assert abs(frac - 0.25) < 5 * sd


def test_full_view_reproduces_grid():
    """r >= max(H, W): the in-map bits of the wall channel are the wall grid."""
    sp = wl.spec(4, 4, 1, 4, 3, 30, flags=0)  # n=1, r=4, C=3 -> 3 words/channel
    b = o.OracleBatch([sp] * 50)
    obs0 = b.reset(2)
    d = 9
    for e in range(50):
        walls = b.walls[e * 16:(e + 1) * 16].reshape(4, 4)
        ch0 = obs0[e * 9:e * 9 + 3]
        x, y = int(b.px[e]), int(b.py[e])
        for cy in range(4):
            for cx in range(4):
                k = (cy - y + 4) * d + (cx - x + 4)
                assert bool((int(ch0[k >> 5]) >> (k & 31)) & 1) == bool(walls[cy, cx])


def test_deterministic_and_env_id_keyed():
    """Same seed and env ids -> same trajectory; results depend on the env's id,
    not on its index in the batch."""
    specs = wl.workload_specs("small", 6)
    a = o.OracleBatch(specs, env_ids=[10, 11, 12, 13, 14, 15])
    b = o.OracleBatch(specs[::-1], env_ids=[15, 14, 13, 12, 11, 10])
    oa0, ob0 = a.reset(7), b.reset(7)
    oa, ra, da = a.step(100)
    ob, rb, db = b.step(100)
    wpe = 6  # words per env: n=2, C=3, w=1
    for i in range(6):
        j = 5 - i
        assert np.array_equal(oa[:, i * wpe:(i + 1) * wpe], ob[:, j * wpe:(j + 1) * wpe])
        assert np.array_equal(ra[:, 2 * i:2 * i + 2], rb[:, 2 * j:2 * j + 2])
        assert np.array_equal(da[:, i], db[:, j])
