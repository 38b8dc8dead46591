"""Enumerated single-step cases on 4x4 grids and a declarative checker.

The checker restates the step rules with whole-array numpy operations (padded
maps, window slicing, per-role occupancy maps), independently of the oracle's
per-cell loops; it is used to pin the oracle (tests/test_oracle_bruteforce.py)
and the same enumerated states are loaded into the HIP library for parity.

Rules restated (see the step rules documented with the library):
  moves, agent-index order: a move to target T is taken iff T is inside the
    map, not a blocking tile, and (collisions on) no other agent stands on T at
    that moment; out-of-range action codes are stay;
  detection: Chebyshev distance <= r between seeker and hider (and, with the
    occlusion flag 8, the hider's cell visible from the seeker's);
  done: terminated (capture rule, >= 1 hider, all hiders found) | truncated << 1;
  observation: window rows dy = -r..r, columns dx = -r..r, bit (dy+r)(2r+1)+(dx+r);
    with the occlusion flag, invisible window cells read 0 in every channel.
  visibility: a window cell is hidden iff the open segment between the two
    cell centres passes through the inside of a blocking cell (wall or outside
    the map) other than the two end cells. Here found by sampling the segment
    (crossed_cells), not by the interval test of the oracle.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np

DX = np.array([0, 0, 0, 1, -1])
DY = np.array([0, -1, 1, 0, 0])
OCCLUDE = 8


@functools.lru_cache(maxsize=None)
def crossed_cells(dx, dy, N=48):
    """Cells (ex, ey), other than (0, 0) and (dx, dy), whose open unit square
    holds a point of the open segment from (0, 0) to (dx, dy), found by
    sampling t = (2k+1)/(2N), k < N, in exact integer arithmetic (the point is
    ((2k+1) dx, (2k+1) dy) / 2N). Exactness: whether the segment is inside a
    cell's open square is decided by open t-intervals whose ends are 0, 1 or
    (2e +- 1)/(2|d|) for d = dx or dy; for |d| <= 4 every end is a multiple of
    1/24, so a non-empty intersection contains an odd multiple of 1/48, i.e.
    a sample when N is a multiple of 24."""
    out = set()
    for k in range(N):
        X, Y = (2 * k + 1) * dx, (2 * k + 1) * dy
        for ey in range(min(0, dy), max(0, dy) + 1):
            for ex in range(min(0, dx), max(0, dx) + 1):
                if (ex, ey) in ((0, 0), (dx, dy)):
                    continue
                if abs(X - 2 * N * ex) < N and abs(Y - 2 * N * ey) < N:
                    out.add((ex, ey))
    return sorted(out)


def visible_window(spec, walls, x, y):
    """[B][D][D] bool: window cell (dy, dx) of the agent at (x, y) visible."""
    H, W, r = spec["H"], spec["W"], spec["r"]
    D = 2 * r + 1
    B = x.shape[0]
    P = r
    blocking = np.ones((B, H + 2 * P, W + 2 * P), bool)
    blocking[:, P:P + H, P:P + W] = walls.reshape(B, H, W) == 1
    rows = np.arange(B)
    vis = np.ones((B, D, D), bool)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            for ex, ey in crossed_cells(dx, dy):
                vis[:, dy + r, dx + r] &= ~blocking[rows, y + ey + P, x + ex + P]
    return vis


def _state(B, H, W, n):
    return dict(walls=np.zeros((B, H * W), np.uint8), pos_x=np.zeros((B, n), np.uint8),
                pos_y=np.zeros((B, n), np.uint8), found=np.zeros(B, np.uint32),
                t=np.zeros(B, np.uint32), episode=np.zeros(B, np.uint32),
                steps=np.zeros(B, np.uint32), seed=np.full(B, 77, np.uint64),
                env_id=np.arange(B, dtype=np.uint32))


def flat_state(st):
    """Per-env arrays -> the flat host arrays the batch APIs take."""
    out = dict(st)
    out["walls"] = np.ascontiguousarray(st["walls"]).reshape(-1)
    out["pos_x"] = np.ascontiguousarray(st["pos_x"]).reshape(-1)
    out["pos_y"] = np.ascontiguousarray(st["pos_y"]).reshape(-1)
    return out


def case_one_agent(r=1, C=4, flags=3, L=100, subsample=None, seed=0):
    """All 2^16 wall patterns x agent on every free cell x 5 actions."""
    pats = np.arange(1 << 16, dtype=np.int64)
    bits = ((pats[:, None] >> np.arange(16)) & 1).astype(np.uint8)  # [P, 16]
    pi, cell = np.nonzero(bits == 0)  # free cells
    pi = np.repeat(pi, 5)
    cell = np.repeat(cell, 5)
    act = np.tile(np.arange(5), len(pi) // 5)
    if subsample is not None:
        g = np.random.Generator(np.random.PCG64(seed))
        sel = g.choice(len(pi), size=subsample, replace=False)
        pi, cell, act = pi[sel], cell[sel], act[sel]
    B = len(pi)
    st = _state(B, 4, 4, 1)
    st["walls"][:] = bits[pi]
    st["pos_x"][:, 0] = cell % 4
    st["pos_y"][:, 0] = cell // 4
    spec = dict(H=4, W=4, n=1, S=1, r=r, C=C, wall_pct=0, flags=flags, L=L)
    return spec, st, act.reshape(B, 1).astype(np.int8)


def case_seeker_hider(n_patterns=256, r=1, C=4, flags=1, L=100, seed=1):
    """Seeded wall patterns x all ordered placements on free cells x 25 joint actions."""
    g = np.random.Generator(np.random.PCG64(seed))
    walls_l, px, py, acts = [], [], [], []
    for _ in range(n_patterns):
        w = (g.random(16) < 0.25).astype(np.uint8)
        free = np.nonzero(w == 0)[0]
        for c0, c1 in itertools.permutations(free, 2):
            for a0 in range(5):
                for a1 in range(5):
                    walls_l.append(w)
                    px.append((c0 % 4, c1 % 4))
                    py.append((c0 // 4, c1 // 4))
                    acts.append((a0, a1))
    B = len(acts)
    st = _state(B, 4, 4, 2)
    st["walls"][:] = np.array(walls_l)
    st["pos_x"][:] = np.array(px)
    st["pos_y"][:] = np.array(py)
    spec = dict(H=4, W=4, n=2, S=1, r=r, C=C, wall_pct=0, flags=flags, L=L)
    return spec, st, np.array(acts, np.int8)


def case_three_agents(r=2, C=3, flags=1, L=100, S=2):
    """Open grid, all ordered placements of 3 agents x 125 joint actions."""
    pl = np.array(list(itertools.permutations(range(16), 3)))  # [3360, 3]
    ac = np.array(list(itertools.product(range(5), repeat=3)))  # [125, 3]
    P, A = len(pl), len(ac)
    cells = np.repeat(pl, A, axis=0)
    acts = np.tile(ac, (P, 1))
    B = P * A
    st = _state(B, 4, 4, 3)
    st["pos_x"][:] = cells % 4
    st["pos_y"][:] = cells // 4
    spec = dict(H=4, W=4, n=3, S=S, r=r, C=C, wall_pct=0, flags=flags, L=L)
    return spec, st, acts.astype(np.int8)


# --------------------------------------------------------------------- checker

def expected_moves(spec, st, acts):
    """New (x, y) per agent, by the sequential rule."""
    H, W, n = spec["H"], spec["W"], spec["n"]
    collide = bool(spec["flags"] & 1)
    x = st["pos_x"].astype(np.int64).copy()
    y = st["pos_y"].astype(np.int64).copy()
    walls = st["walls"].reshape(-1, H, W)
    a = acts.astype(np.int64)
    a = np.where((a >= 0) & (a <= 4), a, 0)
    B = x.shape[0]
    rows = np.arange(B)
    for i in range(n):
        tx = x[:, i] + DX[a[:, i]]
        ty = y[:, i] + DY[a[:, i]]
        inside = (tx >= 0) & (tx < W) & (ty >= 0) & (ty < H)
        wall = np.zeros(B, bool)
        wall[inside] = walls[rows[inside], ty[inside], tx[inside]] == 1
        occ = np.zeros(B, bool)
        if collide:
            for j in range(n):
                if j != i:
                    occ |= (x[:, j] == tx) & (y[:, j] == ty)
        move = (a[:, i] != 0) & inside & ~wall & ~occ
        x[:, i] = np.where(move, tx, x[:, i])
        y[:, i] = np.where(move, ty, y[:, i])
    return x, y


def expected_detection(spec, x, y, walls=None):
    n, S, r = spec["n"], spec["S"], spec["r"]
    B = x.shape[0]
    cnt = np.zeros((B, n), np.int64)
    found = np.zeros(B, np.uint32)
    occl = bool(spec["flags"] & OCCLUDE)
    for i in range(S):
        vis = visible_window(spec, walls, x[:, i], y[:, i]) if occl else None
        for h in range(S, n):
            seen = np.maximum(np.abs(x[:, i] - x[:, h]), np.abs(y[:, i] - y[:, h])) <= r
            if occl:
                ddy = np.clip(y[:, h] - y[:, i] + r, 0, 2 * r)
                ddx = np.clip(x[:, h] - x[:, i] + r, 0, 2 * r)
                seen &= vis[np.arange(B), ddy, ddx]
            cnt[:, i] += seen
            cnt[:, h] += seen
            found |= (seen.astype(np.uint32) << np.uint32(h))
    sign = np.where(np.arange(n) < S, 1, -1)
    return (cnt * sign).astype(np.float32), found


def expected_obs(spec, walls, x, y):
    """[B][n][C][w] words from padded maps and window slices."""
    H, W, n, S, r, C = (spec[k] for k in ("H", "W", "n", "S", "r", "C"))
    D = 2 * r + 1
    w = (D * D + 31) // 32
    B = x.shape[0]
    P = r  # padding
    inside = np.zeros((H + 2 * P, W + 2 * P), bool)
    inside[P:P + H, P:P + W] = True
    wallmap = np.ones((B, H + 2 * P, W + 2 * P), bool)
    wallmap[:, P:P + H, P:P + W] = walls.reshape(B, H, W) == 1
    role = np.arange(n) < S
    occ_role = np.zeros((2, B, H + 2 * P, W + 2 * P), np.int64)
    rows = np.arange(B)
    for j in range(n):
        np.add.at(occ_role[int(role[j])], (rows, y[:, j] + P, x[:, j] + P), 1)
    dy = np.arange(D)[None, :, None]
    dx = np.arange(D)[None, None, :]
    out = np.zeros((B, n, C, w), np.uint32)
    for i in range(n):
        wy = y[:, i][:, None, None] + dy  # padded coordinates of the window
        wx = x[:, i][:, None, None] + dx
        bb = rows[:, None, None]
        inb = inside[wy, wx]
        ch0 = wallmap[bb, wy, wx]
        same = occ_role[int(role[i])][bb, wy, wx].copy()
        same[:, r, r] -= 1  # the agent itself
        ch1 = (same > 0) & inb
        ch2 = (occ_role[1 - int(role[i])][bb, wy, wx] > 0) & inb
        chans = [ch0, ch1, ch2] + ([~inb] if C == 4 else [])
        if spec["flags"] & OCCLUDE:
            vis = visible_window(spec, walls, x[:, i], y[:, i])
            chans = [m & vis for m in chans]
        for c, m in enumerate(chans):
            flat = m.reshape(B, D * D).astype(np.uint64)
            for k in range(D * D):
                out[:, i, c, k >> 5] |= (flat[:, k] << np.uint64(k & 31)).astype(np.uint32)
    return out


def check_step(spec, st, acts, obs, rew, done, new_state):
    """Assert one step's outputs and new state against the rules. Envs whose
    step ended the episode are checked for done/reward/counters and for a
    valid respawn (positions are drawn)."""
    H, W, n, S, L = (spec[k] for k in ("H", "W", "n", "S", "L"))
    B = st["pos_x"].shape[0]
    x, y = expected_moves(spec, st, acts)
    ex_rew, seen = expected_detection(spec, x, y, st["walls"])
    np.testing.assert_array_equal(rew.reshape(B, n), ex_rew)
    assert not np.signbit(rew[rew == 0]).any()
    found = st["found"] | seen
    hmask = np.uint32(((1 << n) - 1) & ~((1 << S) - 1))
    term = bool(spec["flags"] & 2) and n - S > 0
    term = term & ((found & hmask) == hmask) if term else np.zeros(B, bool)
    t1 = st["t"].astype(np.int64) + 1
    trunc = t1 >= L
    ex_done = term.astype(np.uint8) | (trunc.astype(np.uint8) << 1)
    np.testing.assert_array_equal(done.reshape(B), ex_done)
    nd = ex_done == 0
    nx = new_state["pos_x"].reshape(B, n)
    ny = new_state["pos_y"].reshape(B, n)
    np.testing.assert_array_equal(nx[nd], x[nd])
    np.testing.assert_array_equal(ny[nd], y[nd])
    np.testing.assert_array_equal(new_state["found"][nd], found[nd])
    np.testing.assert_array_equal(new_state["t"][nd], t1[nd])
    np.testing.assert_array_equal(new_state["episode"][nd], st["episode"][nd])
    d = ~nd
    np.testing.assert_array_equal(new_state["t"][d], 0)
    np.testing.assert_array_equal(new_state["found"][d], 0)
    np.testing.assert_array_equal(new_state["episode"][d], st["episode"][d] + 1)
    np.testing.assert_array_equal(new_state["steps"], st["steps"] + 1)
    # every env: positions inside, off walls, distinct (collisions on)
    walls = st["walls"].reshape(B, H, W)
    assert (nx < W).all() and (ny < H).all()
    assert (walls[np.arange(B)[:, None], ny, nx] == 0).all() or not _all_started_free(st, spec)
    if spec["flags"] & 1:
        cell = ny.astype(np.int64) * W + nx
        srt = np.sort(cell, axis=1)
        assert (np.diff(srt, axis=1) != 0).all()
    ex_obs = expected_obs(spec, st["walls"], nx.astype(np.int64), ny.astype(np.int64))
    np.testing.assert_array_equal(obs.reshape(ex_obs.shape), ex_obs)


def _all_started_free(st, spec):
    H, W = spec["H"], spec["W"]
    B = st["pos_x"].shape[0]
    walls = st["walls"].reshape(B, H, W)
    return bool((walls[np.arange(B)[:, None], st["pos_y"], st["pos_x"]] == 0).all())
