"""Seeded synthetic workloads for the hide-and-seek step.

This module only describes inputs (environment specs, external action arrays,
serving request traces). It holds none of the step's arithmetic, so both the
HIP library's tests/benchmarks and the CPU oracle may import it.

The paper's scenario maps (PNG + JSON, Sec. 3.2) are not available; synthetic
iid-wall grids stand in for them. Named workloads:
  small        1024 envs, 16x16, 10% walls, 1 seeker + 1 hider, r=2, C=3, 256 steps
  single1k     1024 envs, 32x32, 15% walls, 1 + 1, r=3 (7x7), C=3, 10k steps
  single16k    16384 envs, same as single1k
  los16k       single16k with line-of-sight occlusion in the windows (flag 8)
  explore16k   single16k with exploration rewards and discovery maps (flag 16)
  terrain4k    4096 envs, 32x32, 10% walls, 15% water, 10% mud, 5 + 5 agents of
               cycling classes (walker, swimmer, flyer), r=4, C=4, 2000 steps
               (flag 32)
  multi10      4096 envs, 32x32, 15% walls, 5 + 5, r=4 (9x9), C=4, 2000 steps
  uneven8k     8192 per-env specs: side {16,32,64} w.p. (.5,.3,.2), n ~ U{1..10},
               walls ~ U{5..25}%, r ~ U{2,3,4}, C=4, 2000 steps
  serving      Poisson request trace, each request 256..4096 envs of one spec drawn
               from the uneven8k ranges, 128..1024 steps
Every env: episode length 256, flags = collide | capture-ends | desync.
"""
from __future__ import annotations

import numpy as np

COLLIDE = 1
CAPTURE_ENDS = 2
DESYNC = 4
OCCLUDE = 8  # line-of-sight occlusion in the windows
EXPLORE = 16  # exploration rewards and per-env discovery maps
TERRAIN = 32  # tile types, agent classes, move chances, stuck and rescue
RADIO = 64  # per-agent hider beliefs shared by radio messages
WALKER, SWIMMER, FLYER = 0, 1, 2
DEFAULT_FLAGS = COLLIDE | CAPTURE_ENDS | DESYNC
EPISODE_LEN = 256


def spec(H, W, n, r, C, wall_pct, S=None, flags=DEFAULT_FLAGS, L=EPISODE_LEN) -> dict:
    """One environment's configuration. S (seekers, agents [0,S)) defaults
    to ceil(n/2); agents [S,n) are hiders."""
    if S is None:
        S = (n + 1) // 2
    return dict(H=int(H), W=int(W), n=int(n), S=int(S), r=int(r), C=int(C),
                wall_pct=int(wall_pct), flags=int(flags), L=int(L))


def classes_word(classes) -> int:
    """Pack per-agent classes (WALKER, SWIMMER, FLYER) 2 bits per agent."""
    w = 0
    for i, c in enumerate(classes):
        w |= int(c) << (2 * i)
    return w


def with_terrain(s: dict, water_pct=15, mud_pct=10, stuck_pct=25, speed=None, classes=None) -> dict:
    """A copy of spec s with terrain on: tile percentages, the stuck chance,
    move chances (percent, walker / swimmer / flyer x ground / water / mud)
    and agent classes (default: cycling walker, swimmer, flyer)."""
    if speed is None:
        speed = (100, 0, 60, 0, 100, 0, 80, 80, 80)
    if classes is None:
        classes = [i % 3 for i in range(s["n"])]
    return dict(s, flags=s["flags"] | TERRAIN, water_pct=int(water_pct), mud_pct=int(mud_pct),
                stuck_pct=int(stuck_pct), speed=tuple(int(v) for v in speed),
                classes=classes_word(classes))


WORKLOADS = {
    "small": dict(n_envs=1024, spec=spec(16, 16, 2, 2, 3, 10), steps=256, seed=1),
    "single1k": dict(n_envs=1024, spec=spec(32, 32, 2, 3, 3, 15), steps=10000, seed=2),
    "single16k": dict(n_envs=16384, spec=spec(32, 32, 2, 3, 3, 15), steps=10000, seed=2),
    "los16k": dict(n_envs=16384, spec=spec(32, 32, 2, 3, 3, 15, flags=DEFAULT_FLAGS | OCCLUDE),
                   steps=10000, seed=2),
    "explore16k": dict(n_envs=16384, spec=spec(32, 32, 2, 3, 3, 15, flags=DEFAULT_FLAGS | EXPLORE),
                       steps=10000, seed=2),
    "multi10": dict(n_envs=4096, spec=spec(32, 32, 10, 4, 4, 15), steps=2000, seed=3),
    "uneven8k": dict(n_envs=8192, spec=None, steps=2000, seed=4, spec_seed=4),
    "terrain4k": dict(n_envs=4096, spec=with_terrain(spec(32, 32, 10, 4, 4, 10)), steps=2000,
                      seed=5),
    "radio4k": dict(n_envs=4096, spec=spec(32, 32, 10, 4, 4, 10, flags=DEFAULT_FLAGS | RADIO),
                    steps=2000, seed=6),
}


def uneven_specs(n_envs: int = 8192, spec_seed: int = 4) -> list:
    """Per-env specs of the uneven batch, drawn once from PCG64(spec_seed) in
    this order per env: side, n, wall percent, r."""
    g = np.random.Generator(np.random.PCG64(spec_seed))
    out = []
    for _ in range(n_envs):
        side = int(g.choice([16, 32, 64], p=[0.5, 0.3, 0.2]))
        n = int(g.integers(1, 11))
        wall = int(g.integers(5, 26))
        r = int(g.integers(2, 5))
        out.append(spec(side, side, n, r, 4, wall))
    return out


def workload_specs(name: str, n_envs: int | None = None) -> list:
    w = WORKLOADS[name]
    ne = w["n_envs"] if n_envs is None else n_envs
    if w["spec"] is None:
        return uneven_specs(w["n_envs"], w["spec_seed"])[:ne]
    return [dict(w["spec"]) for _ in range(ne)]


def random_actions(n_steps: int, agents_total: int, seed: int, draw_frac: float = 0.0,
                   invalid_frac: float = 0.0) -> np.ndarray:
    """External int8 actions [n_steps][agents_total]: uniform in 0..4, with a
    fraction replaced by -1 (draw from the counter generator) and a fraction
    by out-of-range values (treated as stay)."""
    g = np.random.Generator(np.random.PCG64(seed))
    a = g.integers(0, 5, size=(n_steps, agents_total)).astype(np.int8)
    if draw_frac > 0:
        a[g.random(a.shape) < draw_frac] = -1
    if invalid_frac > 0:
        bad = g.random(a.shape) < invalid_frac
        a[bad] = g.choice(np.array([5, 7, 100, -2, -128], np.int8), size=int(bad.sum()))
    return a


def radio_actions(n_steps: int, specs, seed: int, draw_frac: float = 0.0,
                  msg_frac: float = 0.5) -> np.ndarray:
    """External int8 actions [n_steps][agents_total] for radio envs: move m
    in 0..4 plus 5 * (target + 1) for a fraction of agents (target uniform
    over the env's agents, itself included), some codes past the last agent
    (no message), and a fraction of -1 (move and target drawn)."""
    g = np.random.Generator(np.random.PCG64(seed))
    cols = []
    for s in specs:
        n = int(s["n"])
        m = g.integers(0, 5, size=(n_steps, n))
        code = np.where(g.random((n_steps, n)) < msg_frac, g.integers(1, n + 1, size=(n_steps, n)), 0)
        over = g.random((n_steps, n)) < 0.03
        code = np.where(over, g.integers(n + 1, 25, size=(n_steps, n)), code)
        cols.append(m + 5 * code)
    a = np.concatenate(cols, axis=1).astype(np.int16)
    if draw_frac > 0:
        a[g.random(a.shape) < draw_frac] = -1
    return a.astype(np.int8)


def serving_trace(n_requests: int = 64, rate_per_s: float = 100.0, seed: int = 5) -> list:
    """Poisson request trace: arrival time, env count, one spec from the
    uneven-batch ranges, step budget and a per-request seed."""
    g = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        t += float(g.exponential(1.0 / rate_per_s))
        n_envs = int(g.integers(256, 4097))
        side = int(g.choice([16, 32, 64], p=[0.5, 0.3, 0.2]))
        n = int(g.integers(1, 11))
        wall = int(g.integers(5, 26))
        r = int(g.integers(2, 5))
        steps = int(g.integers(128, 1025))
        reqs.append(dict(rid=rid, arrival_s=t, n_envs=n_envs, spec=spec(side, side, n, r, 4, wall),
                         steps=steps, seed=5 * (1 << 32) + rid))
    return reqs
