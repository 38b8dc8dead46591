"""Pins of the oracle's counter-based generator and integer range maps.

- Philox4x32-10 against rocRAND's independent engine (host build of its
  open-source header) on random keys/counters.
- A width-generic Philox written here, checked against numpy's Philox4x64-10,
  then instantiated at 4x32 and compared with the oracle.
- The counter layout of every stream (action, spawn, wall, desync) against
  rocRAND words at counters built here from the documented layout.
- The multiply-shift range map at its closed-form boundaries, and a chi-square
  check of the action distribution.
"""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2604_27162_amd import workloads as wl

def test_philox_matches_rocrand(rocrand_philox):
    g = np.random.Generator(np.random.PCG64(123))
    rows = g.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    rows[:8] = 0
    rows[1, 0] = 1
    rows[2, 2] = 2**32 - 1
    rows[3, :] = 2**32 - 1
    # the engine's offset is 4*(c1:c0) in 64 bits, so c1 < 2^30 (the step's
    # counters use c1 = stream << 24 | sub < 2^26)
    rows[:, 3] &= (1 << 30) - 1
    ref = rocrand_philox(rows)
    got = np.array([o.philox(r[2:], r[:2]) for r in rows], dtype=np.uint64)
    assert np.array_equal(ref, got)


# ---- width-generic Philox, pinned to numpy's 4x64 --------------------------

def philox_generic(ctr, key, width, m0, m1, w0, w1, rounds=10):
    mask = (1 << width) - 1
    c0, c1, c2, c3 = (int(v) for v in ctr)
    k0, k1 = (int(v) for v in key)
    for rnd in range(rounds):
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if rnd < rounds - 1:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
    return [c0, c1, c2, c3]


P64 = dict(width=64, m0=0xD2E7470EE14C6C93, m1=0xCA5A826395121157,
           w0=0x9E3779B97F4A7C15, w1=0xBB67AE8584CAA73B)
P32 = dict(width=32, m0=0xD2511F53, m1=0xCD9E8D57, w0=0x9E3779B9, w1=0xBB67AE85)


def test_generic_philox_matches_numpy_4x64():
    g = np.random.Generator(np.random.PCG64(7))
    for _ in range(50):
        key = [int(v) for v in g.integers(0, 2**63, size=2, dtype=np.uint64)]
        ctr = [int(v) for v in g.integers(0, 2**63, size=4, dtype=np.uint64)]
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
        raw = [int(v) for v in bg.random_raw(4)]
        # numpy advances the counter by one before producing its first block
        ctr1 = list(ctr)
        ctr1[0] = (ctr1[0] + 1) & (2**64 - 1)
        assert raw == philox_generic(ctr1, key, **P64)


def test_generic_philox_4x32_matches_oracle():
    g = np.random.Generator(np.random.PCG64(8))
    for _ in range(300):
        key = g.integers(0, 2**32, size=2, dtype=np.uint64)
        ctr = g.integers(0, 2**32, size=4, dtype=np.uint64)
        assert list(o.philox(ctr, key)) == philox_generic(ctr, key, **P32)


# ---- stream layout -----------------------------------------------------------

def _key(seed):
    return [seed & 0xFFFFFFFF, seed >> 32]


def test_stream_layout_against_rocrand(rocrand_philox):
    check_stream_layout(rocrand_philox)


def check_stream_layout(rocrand_philox, libpath=None):
    """Walls, desync time, first-attempt spawn and actions of a tiny env,
    rebuilt from rocRAND words at the documented counters
    (env, stream << 24 | sub, a, b)."""
    seed = 0x0123456789ABCDEF
    sp = wl.spec(5, 7, 3, 1, 3, 40, flags=wl.DESYNC, L=97)
    b = o.OracleBatch([sp], env_id_base=11, libpath=libpath)
    b.reset(seed)
    H, W = 5, 7
    rows = [_key(seed) + [11, (2 << 24) | (c >> 2), 0, 0] for c in range(H * W)]
    words = rocrand_philox(rows)
    T = (40 << 32) // 100
    walls = np.array([int(words[c][c & 3]) < T for c in range(H * W)], np.uint8)
    assert np.array_equal(walls, b.walls)
    d = rocrand_philox([_key(seed) + [11, 3 << 24, 0, 0]])[0][0]
    assert int(b.t[0]) == (int(d) * 97) >> 32
    # actions of 3 agents over 5 steps, replayed by hand on a wall-free copy
    acts = []
    for s in range(5):
        w = rocrand_philox([_key(seed) + [11, 0, s, 0]])[0]
        acts.append([(int(w[i]) * 5) >> 32 for i in range(3)])
    b2 = o.OracleBatch([sp], env_id_base=11, libpath=libpath)
    b2.reset(seed)
    b3 = o.OracleBatch([sp], env_id_base=11, libpath=libpath)
    b3.reset(seed)
    o2, r2, d2 = b2.step(5)
    o3, r3, d3 = b3.step(5, actions=np.array(acts, np.int8))
    assert np.array_equal(o2, o3) and np.array_equal(r2, r3) and np.array_equal(d2, d3)
    assert np.array_equal(b2.px, b3.px) and np.array_equal(b2.py, b3.py)
    # a different step index or agent group gives different actions somewhere
    assert len({tuple(a) for a in acts}) > 1
    # spawn: agent 0's first draw is taken whenever that cell is free
    s0 = rocrand_philox([_key(seed) + [11, (1 << 24) | 0, 0, 0]])[0][0]
    c = (int(s0) * H * W) >> 32
    if not walls[c]:
        b4 = o.OracleBatch([sp], env_id_base=11, libpath=libpath)
        b4.reset(seed)
        assert (int(b4.px[0]), int(b4.py[0])) == (c % W, c // W)


def test_respawn_keyed_by_episode(rocrand_philox):
    check_respawn_keyed_by_episode(rocrand_philox)


def check_respawn_keyed_by_episode(rocrand_philox, libpath=None):
    """Open grid, L = 1: every step truncates, so after step k agent 0 stands
    on its first SPAWN draw of episode k+1."""
    seed, env, H, W = 0xABCDEF12345, 3, 6, 5
    sp = wl.spec(H, W, 2, 1, 3, 0, flags=wl.COLLIDE, L=1)
    b = o.OracleBatch([sp], env_id_base=env, libpath=libpath)
    b.reset(seed)
    rows = [_key(seed) + [env, 1 << 24, e, 0] for e in range(1, 41)]
    words = rocrand_philox(rows)
    for k in range(40):
        _, _, done = b.step(1)
        assert done[0, 0] == 2 and b.ep[0] == k + 1
        c = (int(words[k][0]) * H * W) >> 32
        assert (int(b.px[0]), int(b.py[0])) == (c % W, c // W)


# ---- range maps ---------------------------------------------------------------

def test_range_map_boundaries():
    """floor(x*m/2^32) changes value exactly at x = ceil(v*2^32/m)."""
    for m in list(range(1, 65)) + [100, 256, 1024, 4096, 65535]:
        for v in range(min(m, 40)):
            x0 = -(-(v << 32) // m)  # first x with value v
            assert o.range_map(x0, m) == v
            if x0 > 0:
                assert o.range_map(x0 - 1, m) == v - 1
        assert o.range_map(0, m) == 0
        assert o.range_map(2**32 - 1, m) == m - 1


def test_wall_threshold_closed_form():
    for pct in range(100):
        T = o.wall_threshold(pct)
        # T/2^32 is pct/100 rounded down to a multiple of 2^-32
        assert T * 100 <= pct << 32 < (T + 1) * 100
    assert o.wall_threshold(0) == 0


def test_action_distribution_chi_square():
    """Actions drawn for 1 agent on an open grid are uniform on 0..4."""
    sp = wl.spec(8, 8, 4, 1, 3, 0, flags=0, L=10**4)
    counts = np.zeros(5, np.int64)
    seed = 99
    for s in range(2000):
        w = o.philox([3, 0, s, 0], _key(seed))
        for x in w:
            counts[o.range_map(int(x), 5)] += 1
    exp = counts.sum() / 5
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 18.47  # 0.999 quantile, 4 dof
    del sp


# ---- the spawn rule beyond agent 0's first draw -------------------------------

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_WEYL = (0x9E3779B9, 0xBB67AE85)


def philox_np(ctr, key):
    """Philox4x32-10 blocks for many counters at once (numpy, vectorised over
    rows of ctr [N, 4]; key = (k0, k1)). A third implementation, written
    here for bulk draws and checked against rocRAND before every use."""
    c = [np.asarray(ctr[:, i], np.uint64) for i in range(4)]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    m32 = np.uint64(0xFFFFFFFF)
    for rnd in range(10):
        p0 = np.uint64(PHILOX_M[0]) * c[0]
        p1 = np.uint64(PHILOX_M[1]) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & m32, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & m32]
        k0 = (k0 + np.uint64(PHILOX_WEYL[0])) & m32
        k1 = (k1 + np.uint64(PHILOX_WEYL[1])) & m32
    return np.stack(c, axis=1)


def spawn_restated(free, n, word):
    """The spawn rule (reading R11) written out again: agent i tries the cells
    floor(word(i, j) * cells / 2^32) for attempts j = 0..63 and takes the
    first that is free and not held by an agent < i; when all 64 fail, it
    takes the first such cell scanning row-major from the cell after its
    last draw, wrapping. Returns the cells and, per agent, how it was placed:
    the attempt index, or -1 for the scan."""
    cells = len(free)
    held, how = [], []
    for i in range(n):
        ok = lambda c: free[c] and c not in held  # noqa: E731
        pick = None
        for j in range(64):
            c = (int(word(i, j)) * cells) >> 32
            if ok(c):
                pick = c
                how.append(j)
                break
        if pick is None:
            pick = next((c + d) % cells for d in range(1, cells + 1) if ok((c + d) % cells))
            how.append(-1)
        held.append(pick)
    return held, how


def test_spawn_rule_against_rocrand(rocrand_philox):
    check_spawn_rule(rocrand_philox)


def check_spawn_rule(rocrand_philox, libpath=None, n_envs=3000):
    """Crowded 8x8 grids (n agents, n + 1 or n + 2 free cells, so later agents
    reject most draws and often exhaust their 64 attempts): the oracle's
    positions equal the restated rule fed with SPAWN words (counter
    (env, 1 << 24 | agent, episode, attempt), word 0) for every agent, and the
    cases that tell a wrong agent key, attempt cap or scan start apart from
    the rule all occur."""
    seed = 0x5EED0000ABCD1234
    key = _key(seed)
    g = np.random.Generator(np.random.PCG64(31))
    # the bulk generator against rocRAND first
    probe = g.integers(0, 2**30, size=(256, 4), dtype=np.uint64)
    ref = rocrand_philox([key + [int(v) for v in r] for r in probe])
    assert np.array_equal(philox_np(probe, key), ref)

    H = W = 8
    cells = H * W
    cases = []
    for _ in range(n_envs):
        n = int(g.integers(2, 6))
        free = np.zeros(cells, bool)
        free[g.choice(cells, size=n + int(g.integers(1, 3)), replace=False)] = True
        cases.append((n, free, int(g.integers(0, 2**31)), int(g.integers(0, 5000))))
    # 65 attempts per agent: the 65th tells a cap of 65 apart
    ctr = np.array([[env, (1 << 24) | i, ep, j] for n, _, env, ep in cases
                    for i in range(n) for j in range(65)], np.uint64)
    words = philox_np(ctr, key)[:, 0]
    # spot check of the bulk words against rocRAND itself
    pick = g.choice(len(ctr), size=200, replace=False)
    assert np.array_equal(words[pick],
                          rocrand_philox([key + [int(v) for v in ctr[k]] for k in pick])[:, 0])

    seen = dict(later_agent_after_rejections=0, scan=0, scan_not_from_cell_0=0,
                last_attempt=0, last_attempt_differs_from_scan=0, draw_65_differs_from_scan=0)
    at = 0
    for n, free, env, ep in cases:
        wd = words[at:at + 65 * n].reshape(n, 65)
        at += 65 * n
        want, how = spawn_restated(free, n, lambda i, j: wd[i, j])
        sp = wl.spec(H, W, n, 1, 3, 0, flags=0)
        px, py = o.spawn(sp, (~free).astype(np.uint8), seed=seed, env=env, episode=ep,
                         libpath=libpath)
        got = (py.astype(int) * W + px).tolist()
        assert got == want, (n, np.flatnonzero(free).tolist(), env, ep, got, want, how)
        for i in range(n):
            held = want[:i]
            acceptable = [c for c in range(cells) if free[c] and c not in held]
            last = (int(wd[i, 63]) * cells) >> 32
            if i > 0 and how[i] > 0:
                seen["later_agent_after_rejections"] += 1
            if how[i] == -1:
                seen["scan"] += 1
                if acceptable[0] != want[i]:
                    seen["scan_not_from_cell_0"] += 1
                c65 = (int(wd[i, 64]) * cells) >> 32
                if c65 in acceptable and c65 != want[i]:
                    seen["draw_65_differs_from_scan"] += 1
            if how[i] == 63:
                seen["last_attempt"] += 1
                prev = (int(wd[i, 62]) * cells) >> 32
                scan62 = next((prev + d) % cells for d in range(1, cells + 1)
                              if (prev + d) % cells in acceptable)
                if scan62 != want[i]:
                    seen["last_attempt_differs_from_scan"] += 1
    assert all(v >= 2 for v in seen.values()), seen
