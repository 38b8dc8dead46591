"""ctypes wrapper of the CPU oracle (hase_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package. It shares no code
with the HIP path; the only module both sides import is the seeded input
generator module (paper_2604_27162_amd.workloads), which holds no step logic.

Layout of every array (same contract as the C-ABI library, written here
independently):
  obs  one step: concatenation over envs of [n][C*w + radio] uint32,
       w = ceil((2r+1)^2/32), radio = 1 for envs with flag 64 (belief word)
  rew  one step: concatenation over envs of [n] float32
  done one step: [n_envs] uint8, bit 0 terminated, bit 1 truncated
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hase_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

SPEC_FIELDS = ("H", "W", "n", "S", "r", "C", "wall_pct", "flags", "L", "water_pct", "mud_pct",
               "stuck_pct") + tuple(f"speed{k}" for k in range(9)) + ("classes_lo", "classes_hi")
# terrain fields (flag 32) of a spec dict and their values when absent:
# speed = move chances in percent, walker / swimmer / flyer x ground / water /
# mud; classes = 2 bits per agent (0 walker, 1 swimmer, 2 flyer)
TERRAIN_DEFAULTS = dict(water_pct=0, mud_pct=0, stuck_pct=0, speed=(100,) * 9, classes=0)


def spec_row(s: dict) -> list:
    """One int32 row of the spec table from a spec dict."""
    t = {k: s.get(k, v) for k, v in TERRAIN_DEFAULTS.items()}
    speed = [int(v) for v in t["speed"]]
    if len(speed) != 9:
        raise ValueError("speed needs 9 entries (3 classes x 3 tiles)")
    cls = int(t["classes"])
    return ([int(s[f]) for f in SPEC_FIELDS[:9]] +
            [int(t["water_pct"]), int(t["mud_pct"]), int(t["stuck_pct"])] + speed +
            [np.int32(np.uint32(cls & 0xffffffff)), np.int32(np.uint32(cls >> 32))])


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (plain C, single-threaded)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC",
                               "-shared", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class _Batch(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int32),
        ("spec", ctypes.c_void_p),
        ("grid_off", ctypes.c_void_p),
        ("agent_off", ctypes.c_void_p),
        ("obs_off", ctypes.c_void_p),
        ("agents_total", ctypes.c_int64),
        ("obs_total", ctypes.c_int64),
        ("walls", ctypes.c_void_p),
        ("px", ctypes.c_void_p),
        ("py", ctypes.c_void_p),
        ("found", ctypes.c_void_p),
        ("t", ctypes.c_void_p),
        ("ep", ctypes.c_void_p),
        ("steps", ctypes.c_void_p),
        ("seed", ctypes.c_void_p),
        ("env_id", ctypes.c_void_p),
        ("disc_off", ctypes.c_void_p),
        ("disc_total", ctypes.c_int64),
        ("disc", ctypes.c_void_p),
        ("stuck", ctypes.c_void_p),
        ("belief", ctypes.c_void_p),
    ]


_lib = None


def _bind(path: str):
    L = ctypes.CDLL(path)
    L.or_reset.restype = ctypes.c_int
    L.or_reset.argtypes = [ctypes.POINTER(_Batch), ctypes.c_uint64, ctypes.c_void_p]
    L.or_step.restype = None
    L.or_step.argtypes = [ctypes.POINTER(_Batch), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.or_observe_all.restype = None
    L.or_observe_all.argtypes = [ctypes.POINTER(_Batch), ctypes.c_void_p]
    L.or_philox_block.restype = None
    L.or_philox_block.argtypes = [ctypes.c_uint32] * 6 + [ctypes.c_void_p]
    L.or_range.restype = ctypes.c_uint32
    L.or_range.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    L.or_wall_threshold.restype = ctypes.c_uint32
    L.or_wall_threshold.argtypes = [ctypes.c_uint32]
    L.or_spawn_env.restype = None
    L.or_spawn_env.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                               ctypes.c_uint32]
    L.or_los.restype = ctypes.c_int
    L.or_los.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 4
    return L


def lib(path: str | None = None):
    """The oracle library (or, for mutation tests, another build of it)."""
    global _lib
    if path is not None:
        return _bind(path)
    if _lib is None:
        _lib = _bind(build())
    return _lib


def philox(counter, key):
    """Philox4x32-10 block for counter (4 words) and key (2 words)."""
    out = np.zeros(4, np.uint32)
    lib().or_philox_block(*[int(c) for c in counter], *[int(k) for k in key],
                          out.ctypes.data)
    return out


def range_map(x: int, m: int) -> int:
    return int(lib().or_range(int(x), int(m)))


def wall_threshold(pct: int) -> int:
    return int(lib().or_wall_threshold(int(pct)))


def words_per_channel(r: int) -> int:
    d = 2 * r + 1
    return (d * d + 31) // 32


def spec_table(specs) -> np.ndarray:
    """int32 [n_envs][len(SPEC_FIELDS)] from a sequence of dicts, or an int32
    table as is."""
    if isinstance(specs, np.ndarray):
        return np.ascontiguousarray(specs, dtype=np.int32).reshape(-1, len(SPEC_FIELDS))
    rows = [spec_row(s) for s in specs]
    return np.ascontiguousarray(np.array(rows, dtype=np.int32).reshape(-1, len(SPEC_FIELDS)))


class OracleBatch:
    """A batch of independent environments stepped by the oracle.

    specs: sequence of per-env spec dicts with keys H, W, n, S, r, C,
    wall_pct, flags, L. env_ids default to env_id_base + index.
    """

    def __init__(self, specs, env_id_base: int = 0, env_ids=None, libpath=None):
        self._lib = lib(libpath)
        self.spec = spec_table(specs)
        ne = self.spec.shape[0]
        H, W, n, r, C = (self.spec[:, i] for i in (0, 1, 2, 4, 5))
        d = 2 * r.astype(np.int64) + 1
        w = (d * d + 31) // 32
        cells = (H.astype(np.int64) * W)
        radio = (self.spec[:, 7] & 64) != 0
        per_obs = n.astype(np.int64) * (C * w + radio)
        self.n_envs = ne
        self.grid_off = np.zeros(ne, np.int64)
        self.agent_off = np.zeros(ne, np.int64)
        self.obs_off = np.zeros(ne, np.int64)
        if ne > 1:
            self.grid_off[1:] = np.cumsum(cells)[:-1]
            self.agent_off[1:] = np.cumsum(n.astype(np.int64))[:-1]
            self.obs_off[1:] = np.cumsum(per_obs)[:-1]
        self.agents_total = int(n.sum())
        self.obs_total = int(per_obs.sum())
        # discovery maps of exploring envs (flag 16): H rows of ceil(W/32) words
        flags = self.spec[:, 7]
        per_map = np.where(flags & 16, H.astype(np.int64) * ((W.astype(np.int64) + 31) // 32), 0)
        self.disc_off = np.zeros(ne, np.int64)
        if ne > 1:
            self.disc_off[1:] = np.cumsum(per_map)[:-1]
        self.disc_total = int(per_map.sum())
        self.disc = np.zeros(max(self.disc_total, 1), np.uint32)
        self.walls = np.zeros(int(cells.sum()), np.uint8)
        self.px = np.zeros(self.agents_total, np.uint8)
        self.py = np.zeros(self.agents_total, np.uint8)
        self.found = np.zeros(ne, np.uint32)
        self.t = np.zeros(ne, np.uint32)
        self.ep = np.zeros(ne, np.uint32)
        self.steps = np.zeros(ne, np.uint32)
        self.seed = np.zeros(ne, np.uint64)
        self.stuck = np.zeros(ne, np.uint32)
        self.belief = np.zeros(max(self.agents_total, 1), np.uint32)
        if env_ids is None:
            self.env_id = (np.arange(ne, dtype=np.uint64) + env_id_base).astype(np.uint32)
        else:
            self.env_id = np.ascontiguousarray(env_ids, dtype=np.uint32)
        self._c = _Batch(
            ne, self.spec.ctypes.data, self.grid_off.ctypes.data, self.agent_off.ctypes.data,
            self.obs_off.ctypes.data, self.agents_total, self.obs_total,
            self.walls.ctypes.data, self.px.ctypes.data, self.py.ctypes.data,
            self.found.ctypes.data, self.t.ctypes.data, self.ep.ctypes.data,
            self.steps.ctypes.data, self.seed.ctypes.data, self.env_id.ctypes.data,
            self.disc_off.ctypes.data, self.disc_total, self.disc.ctypes.data,
            self.stuck.ctypes.data, self.belief.ctypes.data)

    def reset(self, seed: int) -> np.ndarray:
        obs0 = np.zeros(self.obs_total, np.uint32)
        rc = self._lib.or_reset(ctypes.byref(self._c), ctypes.c_uint64(seed), obs0.ctypes.data)
        if rc != 0:
            raise ValueError(f"env {-rc - 1} has too few free cells for its agents")
        return obs0

    def step(self, n_steps: int = 1, actions=None, maps: bool = False):
        """(obs, rew, done) of n_steps steps, plus the discovery maps
        [n_steps][disc_total] when maps is true."""
        obs = np.zeros((n_steps, self.obs_total), np.uint32)
        rew = np.zeros((n_steps, self.agents_total), np.float32)
        done = np.zeros((n_steps, self.n_envs), np.uint8)
        mp = np.zeros((n_steps, self.disc_total), np.uint32) if maps else None
        aptr = None
        if actions is not None:
            actions = np.ascontiguousarray(actions, dtype=np.int8).reshape(n_steps, self.agents_total)
            aptr = actions.ctypes.data
        self._lib.or_step(ctypes.byref(self._c), int(n_steps), aptr, obs.ctypes.data,
                          rew.ctypes.data, done.ctypes.data,
                          mp.ctypes.data if maps and self.disc_total else None)
        return (obs, rew, done, mp) if maps else (obs, rew, done)

    def observe(self) -> np.ndarray:
        obs = np.zeros(self.obs_total, np.uint32)
        self._lib.or_observe_all(ctypes.byref(self._c), obs.ctypes.data)
        return obs

    # state as plain host arrays (same fields as the library's checkpoint)
    def get_state(self) -> dict:
        return dict(walls=self.walls.copy(), pos_x=self.px.copy(), pos_y=self.py.copy(),
                    found=self.found.copy(), t=self.t.copy(), episode=self.ep.copy(),
                    steps=self.steps.copy(), seed=self.seed.copy(), env_id=self.env_id.copy(),
                    discovered=self.disc[:self.disc_total].copy(), stuck=self.stuck.copy(),
                    belief=self.belief[:self.agents_total].copy())

    def set_state(self, st: dict) -> None:
        self.walls[:] = st["walls"]
        self.px[:] = st["pos_x"]
        self.py[:] = st["pos_y"]
        self.found[:] = st["found"]
        self.t[:] = st["t"]
        self.ep[:] = st["episode"]
        self.steps[:] = st["steps"]
        self.seed[:] = st["seed"]
        self.env_id[:] = st["env_id"]
        if "discovered" in st:  # optional: exploring envs' discovery maps
            self.disc[:self.disc_total] = st["discovered"]
        if "stuck" in st:  # optional: stuck agents of terrain envs
            self.stuck[:] = st["stuck"]
        if "belief" in st:  # optional: per-agent beliefs of radio envs
            self.belief[:self.agents_total] = st["belief"]


def spawn(spec: dict, walls: np.ndarray, seed: int, env: int, episode: int, libpath=None):
    """Positions the spawn rule gives one env (exported for spawn tests;
    libpath: another build of the oracle, e.g. a planted mistake)."""
    sp = spec_table([spec])[0].copy()
    walls = np.ascontiguousarray(walls, dtype=np.uint8)
    px = np.zeros(int(spec["n"]), np.uint8)
    py = np.zeros(int(spec["n"]), np.uint8)
    lib(libpath).or_spawn_env(sp.ctypes.data, walls.ctypes.data, px.ctypes.data, py.ctypes.data,
                       ctypes.c_uint64(seed), int(env), int(episode))
    return px, py


def los(spec: dict, walls: np.ndarray, ax: int, ay: int, cx: int, cy: int) -> bool:
    """Line of sight from cell (ax, ay) to cell (cx, cy) under the oracle's
    rule (cells may lie outside the map; exported for the rule's pins)."""
    sp = spec_table([spec])[0].copy()
    walls = np.ascontiguousarray(walls, dtype=np.uint8)
    return bool(lib().or_los(sp.ctypes.data, walls.ctypes.data, int(ax), int(ay), int(cx),
                             int(cy)))
