"""Python binding of libhase.so (include/hase.h): argument marshalling only.

torch provides device memory (the state buffer and every input/output
tensor) and the stream; every step of the environment runs in the library's
HIP kernels. There is no CPU fallback: if the library is missing or cannot
be loaded, load() raises.

Layouts (per step): obs int32 words (bit-packed windows, see hase.h), rewards
float32 per agent, dones uint8 per env (bit 0 terminated, bit 1 truncated),
and optionally the discovery maps of exploring envs (int32 words).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhase.so")

OK, EINVAL, ENOMEM, EGRID, EHIP, ESTATE, ENOTREADY = 0, -1, -2, -3, -4, -5, -6
COLLIDE, CAPTURE_ENDS, DESYNC, OCCLUDE, EXPLORE, TERRAIN, RADIO = 1, 2, 4, 8, 16, 32, 64
PERSISTENT, PER_LAUNCH = 0, 1
N_BUCKETS = 4


class HaseError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"hase error {code}: {detail}")
        self.code = code


class EnvSpec(ctypes.Structure):
    _fields_ = [("height", ctypes.c_uint16), ("width", ctypes.c_uint16),
                ("n_agents", ctypes.c_uint8), ("n_seekers", ctypes.c_uint8),
                ("view_radius", ctypes.c_uint8), ("n_channels", ctypes.c_uint8),
                ("wall_pct", ctypes.c_uint8), ("flags", ctypes.c_uint8),
                ("episode_len", ctypes.c_uint16), ("water_pct", ctypes.c_uint8),
                ("mud_pct", ctypes.c_uint8), ("stuck_pct", ctypes.c_uint8),
                ("speed_pct", ctypes.c_uint8 * 9), ("agent_classes", ctypes.c_uint64)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_uint32), ("specs", ctypes.POINTER(EnvSpec)),
                ("n_specs", ctypes.c_uint32), ("env_id_base", ctypes.c_uint32)]


class Layout(ctypes.Structure):
    _fields_ = [("state_bytes", ctypes.c_uint64), ("obs_words_per_step", ctypes.c_uint64),
                ("agents_total", ctypes.c_uint64), ("n_envs", ctypes.c_uint64),
                ("cells_total", ctypes.c_uint64), ("map_words_per_step", ctypes.c_uint64)]


class HostState(ctypes.Structure):
    _fields_ = [("walls", ctypes.c_void_p), ("pos_x", ctypes.c_void_p),
                ("pos_y", ctypes.c_void_p), ("found", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("episode", ctypes.c_void_p), ("steps", ctypes.c_void_p),
                ("seed", ctypes.c_void_p), ("discovered", ctypes.c_void_p),
                ("stuck", ctypes.c_void_p), ("belief", ctypes.c_void_p)]


class ArenaDesc(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_uint32), ("max_height", ctypes.c_uint16),
                ("max_width", ctypes.c_uint16), ("max_agents", ctypes.c_uint8),
                ("max_ranges", ctypes.c_uint32)]


class OutPtrs(ctypes.Structure):
    _fields_ = [("obs", ctypes.c_void_p), ("rew", ctypes.c_void_p), ("done", ctypes.c_void_p),
                ("map", ctypes.c_void_p), ("obs0", ctypes.c_void_p), ("err", ctypes.c_void_p),
                ("pos", ctypes.c_void_p), ("env_state", ctypes.c_void_p)]


class Outputs(ctypes.Structure):
    _fields_ = [("obs", ctypes.c_void_p), ("rew", ctypes.c_void_p), ("done", ctypes.c_void_p),
                ("map", ctypes.c_void_p), ("pos", ctypes.c_void_p), ("env_state", ctypes.c_void_p)]


class StepIO(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_void_p), ("n_steps", ctypes.c_uint32),
                ("out_step0", ctypes.c_uint32), ("d_actions", ctypes.c_void_p),
                ("d_obs", ctypes.c_void_p), ("d_rew", ctypes.c_void_p), ("d_done", ctypes.c_void_p),
                ("d_map", ctypes.c_void_p)]


EXPORTS = ("hase_query_layout", "hase_create", "hase_get_offsets", "hase_get_map_offsets",
           "hase_reset", "hase_step", "hase_step_maps", "hase_prepare", "hase_prepare_maps",
           "hase_observe", "hase_get_state", "hase_set_state", "hase_set_tiling",
           "hase_get_tiling", "hase_autotune", "hase_multi_workspace", "hase_step_multi",
           "hase_step_multi_static", "hase_step_outputs", "hase_prepare_outputs",
           "hase_query_arena", "hase_create_arena",
           "hase_reset_range", "hase_step_resident", "hase_release_range", "hase_range_error",
           "hase_destroy", "hase_strerror", "hase_last_error")
STATIC_WORKSPACE_BYTES = 1 << 20

_lib = None


def load(path: str = LIB_PATH):
    """Load libhase.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with python -m paper_2604_27162_amd.build")
    try:
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so both see the same devices, streams and memory
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "hase_query_layout": [ctypes.POINTER(BatchDesc), ctypes.POINTER(Layout)],
        "hase_create": [ctypes.POINTER(BatchDesc), vp, u64, vp, ctypes.POINTER(vp)],
        "hase_get_offsets": [vp, vp, vp],
        "hase_get_map_offsets": [vp, vp],
        "hase_reset": [vp, u64, vp],
        "hase_step": [vp, u32, vp, vp, vp, vp, u32],
        "hase_step_maps": [vp, u32, vp, vp, vp, vp, vp, u32],
        "hase_prepare": [vp, u32, vp, vp, vp, vp],
        "hase_prepare_maps": [vp, u32, vp, vp, vp, vp, vp],
        "hase_observe": [vp, vp],
        "hase_get_state": [vp, ctypes.POINTER(HostState)],
        "hase_set_state": [vp, ctypes.POINTER(HostState)],
        "hase_set_tiling": [vp, ctypes.POINTER(u32 * N_BUCKETS)],
        "hase_get_tiling": [vp, ctypes.POINTER(u32 * N_BUCKETS)],
        "hase_autotune": [vp, u32, vp, vp, vp, ctypes.POINTER(u32 * N_BUCKETS)],
        "hase_multi_workspace": [ctypes.POINTER(vp), u32, ctypes.POINTER(u64)],
        "hase_step_multi": [ctypes.POINTER(StepIO), u32, u32, vp, u64, vp],
        "hase_step_multi_static": [ctypes.POINTER(StepIO), u32, u32, vp],
        "hase_step_outputs": [vp, u32, vp, ctypes.POINTER(Outputs), u32],
        "hase_prepare_outputs": [vp, u32, vp, ctypes.POINTER(Outputs)],
        "hase_query_arena": [ctypes.POINTER(ArenaDesc), ctypes.POINTER(u64)],
        "hase_create_arena": [ctypes.POINTER(ArenaDesc), vp, u64, vp, ctypes.POINTER(vp)],
        "hase_reset_range": [vp, u32, u32, ctypes.POINTER(EnvSpec), u64, u32, u32,
                             ctypes.POINTER(OutPtrs)],
        "hase_step_resident": [vp, u32],
        "hase_release_range": [vp, u32],
        "hase_range_error": [vp, u32, ctypes.POINTER(ctypes.c_int64)],
        "hase_destroy": [vp],
        "hase_strerror": [ctypes.c_int],
        "hase_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.hase_strerror.restype = ctypes.c_char_p
    L.hase_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise HaseError(rc, load().hase_last_error().decode())


def spec_struct(s: dict) -> EnvSpec:
    """EnvSpec from a spec dict (terrain keys water_pct, mud_pct, stuck_pct,
    speed (9 values) and classes default to 0, 0, 0, all 100 and 0)."""
    speed = tuple(int(v) for v in s.get("speed", (100,) * 9))
    return EnvSpec(s["H"], s["W"], s["n"], s["S"], s["r"], s["C"], s["wall_pct"], s["flags"],
                   s["L"], int(s.get("water_pct", 0)), int(s.get("mud_pct", 0)),
                   int(s.get("stuck_pct", 0)), (ctypes.c_uint8 * 9)(*speed),
                   int(s.get("classes", 0)))


def make_desc(specs, env_id_base: int = 0):
    """(BatchDesc, keep-alive array) for a list of spec dicts; a single spec
    repeated over all envs is passed once (uniform batch)."""
    if len(specs) > 1 and all(s == specs[0] for s in specs):
        arr = (EnvSpec * 1)(spec_struct(specs[0]))
        return BatchDesc(len(specs), arr, 1, env_id_base), arr
    arr = (EnvSpec * len(specs))(*[spec_struct(s) for s in specs])
    return BatchDesc(len(specs), arr, len(specs), env_id_base), arr


def query_layout(specs, env_id_base: int = 0) -> Layout:
    desc, keep = make_desc(specs, env_id_base)
    lay = Layout()
    _check(load().hase_query_layout(ctypes.byref(desc), ctypes.byref(lay)))
    del keep
    return lay


class HaseBatch:
    """A batch of environments stepped by the HIP library on one device."""

    def __init__(self, specs, env_id_base: int = 0, device="cuda", stream=None, lanes=None):
        import torch

        self.torch = torch
        L = load()
        self.specs = list(specs)
        self.device = torch.device(device)
        desc, keep = make_desc(self.specs, env_id_base)
        lay = Layout()
        _check(L.hase_query_layout(ctypes.byref(desc), ctypes.byref(lay)))
        self.layout = lay
        self.n_envs = int(lay.n_envs)
        self.obs_words = int(lay.obs_words_per_step)
        self.agents = int(lay.agents_total)
        self.cells = int(lay.cells_total)
        self.map_words = int(lay.map_words_per_step)
        self.state = torch.empty(int(lay.state_bytes), dtype=torch.uint8, device=self.device)
        if self.state.data_ptr() % 256:
            raise RuntimeError("state buffer not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(L.hase_create(ctypes.byref(desc), self.state.data_ptr(), lay.state_bytes,
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        del keep
        self._h = h
        if lanes is not None:
            self.set_tiling(lanes)

    # -- outputs ---------------------------------------------------------
    def alloc_outputs(self, n_steps: int, maps: bool = False):
        """(obs, rew, done) tensors for n_steps, plus the map tensor when maps."""
        t = self.torch
        obs = t.empty((n_steps, self.obs_words), dtype=t.int32, device=self.device)
        rew = t.empty((n_steps, self.agents), dtype=t.float32, device=self.device)
        done = t.empty((n_steps, self.n_envs), dtype=t.uint8, device=self.device)
        if maps:
            mp = t.empty((n_steps, max(1, self.map_words)), dtype=t.int32, device=self.device)
            return obs, rew, done, mp
        return obs, rew, done

    def alloc_state_outputs(self, n_steps: int):
        """(pos, env_state) tensors of the true state after each of n_steps:
        int16 [n_steps][agents] (x | y << 8) and int32 [n_steps][envs][4]
        (found, t, episode, stuck)."""
        t = self.torch
        return (t.empty((n_steps, self.agents), dtype=t.int16, device=self.device),
                t.empty((n_steps, self.n_envs, 4), dtype=t.int32, device=self.device))

    def reset(self, seed: int, obs: bool = True):
        """reset(seed); returns the first observation (None with obs=False:
        then no observation is written)."""
        obs0 = None
        if obs:
            obs0 = self.torch.empty(self.obs_words, dtype=self.torch.int32, device=self.device)
        _check(load().hase_reset(self._h, ctypes.c_uint64(seed),
                                 None if obs0 is None else obs0.data_ptr()))
        return obs0

    def _map_ptr(self, maps, n_steps: int):
        if maps is None:
            return None
        if (maps.device != self.device or not maps.is_contiguous()
                or maps.element_size() != 4 or maps.numel() < n_steps * self.map_words):
            raise ValueError("map tensor has the wrong device, layout or size")
        return maps.data_ptr()

    def _state_ptrs(self, state, n_steps: int):
        if state is None:
            return None, None
        pos, env = state
        if (pos.device != self.device or not pos.is_contiguous() or pos.element_size() != 2
                or pos.numel() < n_steps * self.agents or env.device != self.device
                or not env.is_contiguous() or env.element_size() != 4
                or env.numel() < n_steps * self.n_envs * 4):
            raise ValueError("true-state tensors have the wrong device, layout or size")
        return pos.data_ptr(), env.data_ptr()

    def step_into(self, obs, rew, done, n_steps: int, actions=None, mode: int = PERSISTENT,
                  maps=None, state=None):
        """Enqueue n_steps into preallocated outputs (no synchronisation);
        maps (optional) receives the discovery maps after every step, state
        (optional, alloc_state_outputs) the true state after every step."""
        for tns, shape in ((obs, (n_steps, self.obs_words)), (rew, (n_steps, self.agents)),
                           (done, (n_steps, self.n_envs))):
            if tns.device != self.device or not tns.is_contiguous() or tns.numel() < shape[0] * shape[1]:
                raise ValueError("output tensor has the wrong device, layout or size")
        mptr = self._map_ptr(maps, n_steps)
        aptr = None
        if actions is not None:
            if (actions.dtype != self.torch.int8 or actions.device != self.device
                    or not actions.is_contiguous() or actions.numel() < n_steps * self.agents):
                raise ValueError("actions must be a contiguous int8 device tensor "
                                 "[n_steps][agents_total]")
            aptr = actions.data_ptr()
        pp, ep = self._state_ptrs(state, n_steps)
        outs = Outputs(obs.data_ptr(), rew.data_ptr(), done.data_ptr(), mptr, pp, ep)
        _check(load().hase_step_outputs(self._h, int(n_steps), aptr, ctypes.byref(outs), int(mode)))

    def prepare(self, obs, rew, done, n_steps: int, actions=None, maps=None, state=None) -> None:
        """Capture the persistent-step graph for these buffers without running it."""
        aptr = None if actions is None else actions.data_ptr()
        pp, ep = self._state_ptrs(state, n_steps)
        outs = Outputs(obs.data_ptr(), rew.data_ptr(), done.data_ptr(),
                       self._map_ptr(maps, n_steps), pp, ep)
        _check(load().hase_prepare_outputs(self._h, int(n_steps), aptr, ctypes.byref(outs)))

    def step(self, n_steps: int = 1, actions=None, mode: int = PERSISTENT, maps: bool = False,
             state: bool = False):
        """(obs, rew, done) of n_steps, plus the discovery maps when maps, plus
        the true state (pos, env_state) after every step when state."""
        out = self.alloc_outputs(n_steps, maps)
        st = self.alloc_state_outputs(n_steps) if state else None
        if actions is not None and not self.torch.is_tensor(actions):
            actions = self.torch.as_tensor(np.ascontiguousarray(actions, np.int8)).to(self.device)
        self.step_into(*out[:3], n_steps, actions, mode, out[3] if maps else None, st)
        res = tuple(out[:3])
        if maps:
            res += (out[3][:, :self.map_words],)
        if state:
            res += st
        return res

    def observe(self):
        obs = self.torch.empty(self.obs_words, dtype=self.torch.int32, device=self.device)
        _check(load().hase_observe(self._h, obs.data_ptr()))
        return obs

    # -- state -----------------------------------------------------------
    def get_state(self) -> dict:
        st = dict(walls=np.zeros(self.cells, np.uint8), pos_x=np.zeros(self.agents, np.uint8),
                  pos_y=np.zeros(self.agents, np.uint8), found=np.zeros(self.n_envs, np.uint32),
                  t=np.zeros(self.n_envs, np.uint32), episode=np.zeros(self.n_envs, np.uint32),
                  steps=np.zeros(self.n_envs, np.uint32), seed=np.zeros(self.n_envs, np.uint64),
                  discovered=np.zeros(self.map_words, np.uint32),
                  stuck=np.zeros(self.n_envs, np.uint32),
                  belief=np.zeros(self.agents, np.uint32))
        hs = HostState(*[st[k].ctypes.data for k in
                         ("walls", "pos_x", "pos_y", "found", "t", "episode", "steps", "seed")],
                       st["discovered"].ctypes.data if self.map_words else None,
                       st["stuck"].ctypes.data, st["belief"].ctypes.data)
        _check(load().hase_get_state(self._h, ctypes.byref(hs)))
        return st

    def set_state(self, st: dict) -> None:
        arrs = dict(walls=(np.uint8, self.cells), pos_x=(np.uint8, self.agents),
                    pos_y=(np.uint8, self.agents), found=(np.uint32, self.n_envs),
                    t=(np.uint32, self.n_envs), episode=(np.uint32, self.n_envs),
                    steps=(np.uint32, self.n_envs), seed=(np.uint64, self.n_envs))
        keep = {}
        for k, (dt, n) in arrs.items():
            a = np.ascontiguousarray(st[k], dtype=dt).reshape(-1)
            if a.size != n:
                raise ValueError(f"state field {k} has {a.size} entries, expected {n}")
            keep[k] = a
        disc = None  # absent: every discovery map is cleared
        if st.get("discovered") is not None and self.map_words:
            keep["discovered"] = np.ascontiguousarray(st["discovered"], dtype=np.uint32).reshape(-1)
            if keep["discovered"].size != self.map_words:
                raise ValueError(f"state field discovered has {keep['discovered'].size} entries, "
                                 f"expected {self.map_words}")
            disc = keep["discovered"].ctypes.data
        stuck = None  # absent: nobody is stuck
        if st.get("stuck") is not None:
            keep["stuck"] = np.ascontiguousarray(st["stuck"], dtype=np.uint32).reshape(-1)
            if keep["stuck"].size != self.n_envs:
                raise ValueError("state field stuck must have one entry per env")
            stuck = keep["stuck"].ctypes.data
        belief = None  # absent: every belief is empty
        if st.get("belief") is not None:
            keep["belief"] = np.ascontiguousarray(st["belief"], dtype=np.uint32).reshape(-1)
            if keep["belief"].size != self.agents:
                raise ValueError("state field belief must have one entry per agent")
            belief = keep["belief"].ctypes.data
        hs = HostState(*[keep[k].ctypes.data for k in
                         ("walls", "pos_x", "pos_y", "found", "t", "episode", "steps", "seed")],
                       disc, stuck, belief)
        _check(load().hase_set_state(self._h, ctypes.byref(hs)))

    def offsets(self):
        oo = np.zeros(self.n_envs, np.uint64)
        ao = np.zeros(self.n_envs, np.uint64)
        _check(load().hase_get_offsets(self._h, oo.ctypes.data, ao.ctypes.data))
        return oo, ao

    def map_offsets(self):
        mo = np.zeros(self.n_envs, np.uint64)
        _check(load().hase_get_map_offsets(self._h, mo.ctypes.data))
        return mo

    def set_tiling(self, lanes) -> None:
        arr = (ctypes.c_uint32 * N_BUCKETS)(*[int(x) for x in lanes])
        _check(load().hase_set_tiling(self._h, ctypes.byref(arr)))

    def get_tiling(self):
        arr = (ctypes.c_uint32 * N_BUCKETS)()
        _check(load().hase_get_tiling(self._h, ctypes.byref(arr)))
        return list(arr)

    def autotune(self, n_steps: int = 256):
        """Choose lanes-per-env per agent bucket by timing short persistent runs
        (the state is restored afterwards); returns the chosen tiling."""
        obs, rew, done = self.alloc_outputs(n_steps)
        arr = (ctypes.c_uint32 * N_BUCKETS)()
        _check(load().hase_autotune(self._h, int(n_steps), obs.data_ptr(), rew.data_ptr(),
                                    done.data_ptr(), ctypes.byref(arr)))
        return list(arr)

    @property
    def handle(self):
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hase_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def as_u32(t) -> np.ndarray:
    """Host uint32 view of an int32 obs tensor."""
    return t.detach().cpu().numpy().view(np.uint32)


def multi_workspace_bytes(batches) -> int:
    arr = (ctypes.c_void_p * max(1, len(batches)))(*[b.handle.value for b in batches])
    out = ctypes.c_uint64()
    _check(load().hase_multi_workspace(arr, len(batches), ctypes.byref(out)))
    return int(out.value)


def _step_ios(items):
    ios = (StepIO * max(1, len(items)))()
    for i, it in enumerate(items):
        b, k, s0, act, obs, rew, done = it[:7]
        mp = it[7] if len(it) > 7 else None
        ios[i] = StepIO(b.handle.value, int(k), int(s0), None if act is None else act.data_ptr(),
                        obs.data_ptr(), rew.data_ptr(), done.data_ptr(),
                        None if mp is None else mp.data_ptr())
    return ios


def step_multi(items, n_steps: int, workspace, stream) -> None:
    """Enqueue one multi-batch step: items are (batch, steps, out_step0,
    actions or None, obs, rew, done[, maps]) with per-batch device tensors."""
    _check(load().hase_step_multi(_step_ios(items), len(items), int(n_steps),
                                  workspace.data_ptr(),
                                  workspace.numel() * workspace.element_size(),
                                  ctypes.c_void_p(stream.cuda_stream)))


def step_multi_static(items, n_steps: int, stream) -> None:
    """step_multi with the library's static device workspace (no workspace
    argument; the call allocates nothing; calls on one GPU must not overlap)."""
    _check(load().hase_step_multi_static(_step_ios(items), len(items), int(n_steps),
                                         ctypes.c_void_p(stream.cuda_stream)))


def range_output_sizes(spec: dict, count: int) -> dict:
    """Per-step output sizes (elements) of a range of `count` envs of spec."""
    d = 2 * spec["r"] + 1
    w = (d * d + 31) // 32
    obs_env = spec["n"] * (spec["C"] * w + (1 if spec["flags"] & RADIO else 0))
    map_env = spec["H"] * ((spec["W"] + 31) // 32) if spec["flags"] & EXPLORE else 0
    return dict(obs=count * obs_env, rew=count * spec["n"], done=count, map=count * map_env)


def query_arena(n_slots: int, max_height: int = 64, max_width: int = 64, max_agents: int = 20,
                max_ranges: int = 1024) -> int:
    d = ArenaDesc(n_slots, max_height, max_width, max_agents, max_ranges)
    out = ctypes.c_uint64()
    _check(load().hase_query_arena(ctypes.byref(d), ctypes.byref(out)))
    return int(out.value)


class HaseArena:
    """Resident env slots on one device (include/hase.h, arena): ranges of
    slots are admitted with their own spec, seed, env ids, step budget and
    output tensors, stepped together, and released."""

    def __init__(self, n_slots: int, max_height: int = 64, max_width: int = 64,
                 max_agents: int = 20, max_ranges: int = 1024, device="cuda", stream=None):
        import torch

        self.torch = torch
        L = load()
        self.device = torch.device(device)
        self.desc = ArenaDesc(n_slots, max_height, max_width, max_agents, max_ranges)
        nbytes = ctypes.c_uint64()
        _check(L.hase_query_arena(ctypes.byref(self.desc), ctypes.byref(nbytes)))
        self.state_bytes = int(nbytes.value)
        self.state = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        if self.state.data_ptr() % 256:
            raise RuntimeError("state buffer not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(L.hase_create_arena(ctypes.byref(self.desc), self.state.data_ptr(), nbytes,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n_slots = int(n_slots)

    def alloc_outputs(self, spec: dict, count: int, steps: int, maps: bool = False,
                      state: bool = False):
        """(obs, rew, done[, map][, pos, env_state]) tensors of a range, plus
        obs0 and a pinned host error word, laid out as hase_out_ptrs
        describes."""
        t = self.torch
        sz = range_output_sizes(spec, count)
        out = dict(obs=t.empty((steps, sz["obs"]), dtype=t.int32, device=self.device),
                   rew=t.empty((steps, sz["rew"]), dtype=t.float32, device=self.device),
                   done=t.empty((steps, sz["done"]), dtype=t.uint8, device=self.device),
                   obs0=t.empty(sz["obs"], dtype=t.int32, device=self.device),
                   err=t.full((1,), -2, dtype=t.int32, pin_memory=True))
        if maps and sz["map"]:
            out["map"] = t.empty((steps, sz["map"]), dtype=t.int32, device=self.device)
        if state:
            out["pos"] = t.empty((steps, sz["rew"]), dtype=t.int16, device=self.device)
            out["env_state"] = t.empty((steps, count, 4), dtype=t.int32, device=self.device)
        return out

    def reset_range(self, first_slot: int, count: int, spec: dict, seed: int, steps: int,
                    out: dict, env_id_base: int = 0) -> None:
        """Admit `count` envs of spec at first_slot (enqueued): out holds the
        range's tensors (alloc_outputs; "map" and "obs0" optional)."""
        sz = range_output_sizes(spec, count)
        for k in ("obs", "rew", "done"):
            x = out[k]
            if (x.device != self.device or not x.is_contiguous()
                    or x.numel() < steps * sz[k]):
                raise ValueError(f"output tensor {k} has the wrong device, layout or size")
        mp, o0, er = out.get("map"), out.get("obs0"), out.get("err")
        if mp is not None and (not mp.is_contiguous() or mp.numel() < steps * sz["map"]):
            raise ValueError("map tensor has the wrong layout or size")
        if o0 is not None and (not o0.is_contiguous() or o0.numel() < sz["obs"]):
            raise ValueError("obs0 tensor has the wrong layout or size")
        if er is not None and (er.element_size() * er.numel() < 4
                               or not (er.is_cuda or er.is_pinned())):
            raise ValueError("err must be a device or pinned host tensor of one 32-bit word")
        sp_, se_ = out.get("pos"), out.get("env_state")
        if sp_ is not None and (not sp_.is_contiguous() or sp_.element_size() != 2
                                or sp_.numel() < steps * sz["rew"]):
            raise ValueError("pos tensor has the wrong layout or size")
        if se_ is not None and (not se_.is_contiguous() or se_.element_size() != 4
                                or se_.numel() < steps * 4 * count):
            raise ValueError("env_state tensor has the wrong layout or size")
        ptrs = OutPtrs(out["obs"].data_ptr(), out["rew"].data_ptr(), out["done"].data_ptr(),
                       None if mp is None else mp.data_ptr(), None if o0 is None else o0.data_ptr(),
                       None if er is None else er.data_ptr(),
                       None if sp_ is None else sp_.data_ptr(), None if se_ is None else se_.data_ptr())
        sp = spec_struct(spec)
        _check(load().hase_reset_range(self._h, int(first_slot), int(count), ctypes.byref(sp),
                                       ctypes.c_uint64(seed), int(env_id_base), int(steps),
                                       ctypes.byref(ptrs)))

    def step(self, n_steps: int) -> None:
        _check(load().hase_step_resident(self._h, int(n_steps)))

    def release_range(self, first_slot: int) -> None:
        _check(load().hase_release_range(self._h, int(first_slot)))

    def range_error(self, first_slot: int) -> int:
        """-1, or the first env of the range without room for its agents
        (synchronises)."""
        v = ctypes.c_int64()
        _check(load().hase_range_error(self._h, int(first_slot), ctypes.byref(v)))
        return int(v.value)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hase_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
