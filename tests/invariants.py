"""Properties every step must satisfy, at any batch size.

Given the spec table, the state before and after a step and the step's
outputs, check (per env):
  - agents inside the map and off blocking tiles; distinct cells with collisions on;
  - obs: wall channel popcount = blocked-or-outside cells of the window; centre
    bit clear; outside channel is a subset of the wall channel; teammate and
    opponent channels disjoint from each other and from the wall channel; their
    popcounts add up to the other agents within Chebyshev distance r; padding 0;
  - rewards sum to zero; on steps that did not end the episode a seeker's reward
    is the popcount of its opponent channel and a hider's is minus it;
  - done => t = 0 and episode + 1; not done => t + 1, same episode; step count + 1.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("H", "W", "n", "S", "r", "C", "wall_pct", "flags", "L")


def popcount32(a):
    a = a.astype(np.uint64)
    c = np.zeros(a.shape, np.int64)
    for s in range(32):
        c += ((a >> np.uint64(s)) & np.uint64(1)).astype(np.int64)
    return c


def offsets(table):
    H, W, n, r, C = (table[:, i].astype(np.int64) for i in (0, 1, 2, 4, 5))
    d = 2 * r + 1
    w = (d * d + 31) // 32
    def excl(v):
        o = np.zeros(len(v), np.int64)
        o[1:] = np.cumsum(v)[:-1]
        return o
    return excl(H * W), excl(n), excl(n * C * w), w


def check_invariants(table, prev, new, obs, rew, done, envs=None):
    """Check the listed properties on envs (default: all)."""
    table = np.asarray(table)
    goff, aoff, ooff, wv = offsets(table)
    ne = table.shape[0]
    envs = range(ne) if envs is None else envs
    for e in envs:
        H, W, n, S, r, C, _, flags, L = (int(v) for v in table[e][:9])
        d = 2 * r + 1
        w = int(wv[e])
        walls = new["walls"][goff[e]:goff[e] + H * W].reshape(H, W)
        x = new["pos_x"][aoff[e]:aoff[e] + n].astype(np.int64)
        y = new["pos_y"][aoff[e]:aoff[e] + n].astype(np.int64)
        assert (x < W).all() and (y < H).all(), e
        assert (walls[y, x] == 0).all(), e
        if flags & 1:
            assert len(set(zip(x.tolist(), y.tolist()))) == n, e
        o = obs[ooff[e]:ooff[e] + n * C * w].reshape(n, C, w)
        pad = np.zeros(w, np.uint64)
        for k in range(d * d, 32 * w):
            pad[k >> 5] |= np.uint64(1) << np.uint64(k & 31)
        centre_word, centre_bit = (r * d + r) >> 5, np.uint32(1 << ((r * d + r) & 31))
        rr = rew[aoff[e]:aoff[e] + n]
        assert float(rr.sum()) == 0.0, e
        for i in range(n):
            oi = o[i].astype(np.uint64)
            assert not (oi & pad[None, :]).any(), (e, i)
            for c in range(C):
                assert not (o[i, c, centre_word] & centre_bit), (e, i, c)
            blocked = 0
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    cx, cy = x[i] + dx, y[i] + dy
                    if not (0 <= cx < W and 0 <= cy < H) or walls[cy, cx]:
                        blocked += 1
            assert popcount32(oi[0]).sum() == blocked, (e, i)
            assert not (oi[1] & oi[0]).any() and not (oi[2] & oi[0]).any(), (e, i)
            if flags & 1:
                assert not (oi[1] & oi[2]).any(), (e, i)
            if C == 4:
                assert not (oi[3] & ~oi[0]).any(), (e, i)
            near = int(((np.maximum(np.abs(x - x[i]), np.abs(y - y[i])) <= r).sum()) - 1)
            if flags & 1:
                assert popcount32(oi[1]).sum() + popcount32(oi[2]).sum() == near, (e, i)
            if done[e] == 0 and (flags & 1):
                opp = int(popcount32(oi[2]).sum())
                assert rr[i] == (opp if i < S else -opp), (e, i)
        if done[e]:
            assert new["t"][e] == 0 and new["episode"][e] == prev["episode"][e] + 1, e
            assert new["found"][e] == 0, e
        else:
            assert new["t"][e] == prev["t"][e] + 1 and new["episode"][e] == prev["episode"][e], e
        assert new["steps"][e] == prev["steps"][e] + 1, e
