"""Continuous-batching serving loop for rollout requests.

A request asks for `n_envs` environments of one spec, stepped `steps` times
from `seed` (env ids 0..n_envs-1 of the request, so its result does not
depend on what else runs). The server keeps every admitted request resident
in one device arena of env slots (include/hase.h, arena): a request is
admitted into a range of free slots as soon as the slots and the device
memory budget allow (footprint = the request's whole output, which stays
resident until the client fetches it, on top of the arena itself), by a
slot-range reset enqueued on the device stream with no host
synchronisation; all admitted requests then advance together, `chunk`
steps per launch, each stopping at its own budget; a finished request's
slots are released (in stream order) and taken by the next admission while
the device works on the chunks already enqueued. At most `depth` chunks are
in flight: the host admits and enqueues ahead while the device steps.

Reported: per-step latency (chunk device time / chunk steps, weighted by the
requests it advanced) as p50/p99, queueing delay (submit to admission),
completion time, device-busy fraction of the wall time and aggregate
agent-steps/s (wall clock and device time).

The scheduling logic talks to an executor (capacity, admit, step, release,
fetch); the HIP executor below is the product path. Tests may plug in
another executor.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    spec: dict
    n_envs: int
    steps: int
    seed: int
    arrival_s: float = 0.0
    # filled by the server
    footprint: int = 0
    state: str = "new"  # queued | active | done | failed | cancelled | rejected
    error: str = ""
    first_slot: int = -1
    outputs: object = None
    left: int = 0          # steps not yet enqueued
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_finish: float = 0.0
    step_latencies_ms: list = field(default_factory=list)
    _event: threading.Event = field(default_factory=threading.Event)

    @property
    def agents(self) -> int:
        return self.n_envs * self.spec["n"]

    def wait(self, timeout=None) -> bool:
        return self._event.wait(timeout)


class SlotAllocator:
    """First-fit allocation of contiguous slot ranges, merged on release."""

    def __init__(self, n_slots: int):
        self.free = [(0, int(n_slots))]  # sorted (start, length)

    def take(self, count: int):
        for i, (s, n) in enumerate(self.free):
            if n >= count:
                if n == count:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + count, n - count)
                return s
        return None

    def give(self, start: int, count: int) -> None:
        self.free.append((start, count))
        self.free.sort()
        merged = []
        for s, n in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + n)
            else:
                merged.append((s, n))
        self.free = merged

    def largest(self) -> int:
        return max((n for _, n in self.free), default=0)


class HipExecutor:
    """Runs requests on the GPU in one arena of resident env slots."""

    def __init__(self, device="cuda:0", n_slots: int = 1 << 18, max_height: int = 64,
                 max_width: int = 64, max_agents: int = 10, max_ranges: int = 4096):
        import torch

        from . import hase

        self.torch = torch
        self.hase = hase
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.arena = hase.HaseArena(n_slots, max_height, max_width, max_agents, max_ranges,
                                    device=self.device, stream=self.stream)
        self.n_slots = n_slots
        self.max_ranges = max_ranges
        self.fixed_bytes = self.arena.state_bytes

    def footprint(self, req: Request) -> int:
        sz = self.hase.range_output_sizes(req.spec, req.n_envs)
        per_step = 4 * sz["obs"] + 4 * sz["rew"] + sz["done"]
        return int(req.steps * per_step + 4 * sz["obs"])

    def admit(self, req: Request) -> None:
        out = self.arena.alloc_outputs(req.spec, req.n_envs, req.steps)
        self.arena.reset_range(req.first_slot, req.n_envs, req.spec, req.seed, req.steps, out)
        req.outputs = out

    def mark(self):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev

    def step(self, n_steps: int) -> None:
        self.arena.step(n_steps)

    def release(self, req: Request) -> None:
        self.arena.release_range(req.first_slot)

    @staticmethod
    def done(ev) -> bool:
        return ev.query()

    @staticmethod
    def wait(ev) -> None:
        ev.synchronize()

    @staticmethod
    def elapsed_ms(a, b) -> float:
        return float(a.elapsed_time(b))

    def check(self, req: Request) -> str:
        """'' when every env of the request had room at its reset (read from
        the request's pinned error word, which the device wrote before the
        request's last chunk ended)."""
        bad = int(req.outputs["err"][0]) & 0xffffffff
        return "" if bad == 0xffffffff else f"env {bad} has too few free cells for its agents"


@dataclass
class Chunk:
    ev_start: object
    ev_step: object
    ev_end: object
    n_steps: int
    items: list          # (request, steps it takes in this chunk)
    finishing: list      # requests whose last step is in this chunk


class Server:
    """Admission by slots and memory footprint, continuous batching in
    chunks of steps, at most `depth` chunks in flight."""

    def __init__(self, executor, budget_bytes: int = 64 << 30, chunk: int = 128, depth: int = 2):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.depth = int(depth)
        self.slots = SlotAllocator(executor.n_slots)
        self.used = int(executor.fixed_bytes)
        self.queue = collections.deque()
        self.active: list[Request] = []
        self.inflight: collections.deque[Chunk] = collections.deque()
        self.finished: list[Request] = []
        self.n_ranges = 0
        self.lock = threading.Lock()
        self.wake = threading.Condition(self.lock)
        self.stop_flag = False
        self.thread = None
        self.agent_steps = 0
        self.step_ms = 0.0
        self.busy_ms = 0.0
        self.chunks = 0

    # ---- client side -------------------------------------------------------
    def submit(self, req: Request) -> Request:
        req.footprint = self.ex.footprint(req)
        req.t_submit = time.perf_counter()
        with self.lock:
            if (req.footprint + self.ex.fixed_bytes > self.budget
                    or req.n_envs > self.ex.n_slots):
                req.state, req.error = "rejected", "larger than the whole budget or arena"
                req._event.set()
                return req
            req.state = "queued"
            self.queue.append(req)
            self.wake.notify()
        return req

    def cancel(self, req: Request) -> bool:
        """Cancel a queued request (admitted ones run to completion)."""
        with self.lock:
            if req.state == "queued":
                self.queue.remove(req)
                req.state = "cancelled"
                req._event.set()
                return True
        return False

    def fetch(self, req: Request, timeout=None):
        """Hand the request's outputs (obs, rew, done) to the client: the
        server keeps no reference to them and their footprint returns to the
        budget."""
        if not req.wait(timeout):
            raise TimeoutError(f"request {req.rid} not finished")
        if req.state != "done":
            raise RuntimeError(f"request {req.rid} {req.state}: {req.error}")
        with self.lock:
            out = req.outputs
            req.outputs = None
            if out is None:
                raise RuntimeError(f"request {req.rid} was already fetched")
            self.used -= req.footprint
            req.footprint = 0
            self.wake.notify()
        return out["obs"], out["rew"], out["done"]

    # ---- scheduler ---------------------------------------------------------
    def _admit(self) -> None:
        """FIFO admission while the head of the queue fits the slots, the
        budget and the arena's range table."""
        while True:
            with self.lock:
                if not self.queue:
                    return
                req = self.queue[0]
                if (self.used + req.footprint > self.budget
                        or self.n_ranges >= self.ex.max_ranges):
                    return
                first = self.slots.take(req.n_envs)
                if first is None:
                    return
                self.queue.popleft()
                self.used += req.footprint
                self.n_ranges += 1
            req.first_slot = first
            try:
                self.ex.admit(req)
            except Exception as err:  # a refused request frees what it took
                with self.lock:
                    self.used -= req.footprint
                    self.n_ranges -= 1
                    self.slots.give(first, req.n_envs)
                req.footprint = 0
                req.state, req.error = "failed", str(err)
                req._event.set()
                continue
            req.state = "active"
            req.left = req.steps
            req.t_admit = time.perf_counter()
            self.active.append(req)

    def _complete(self, ch: Chunk) -> None:
        """Account a chunk the device has finished."""
        ms = self.ex.elapsed_ms(ch.ev_step, ch.ev_end)
        self.step_ms += ms
        self.busy_ms += self.ex.elapsed_ms(ch.ev_start, ch.ev_end)
        self.chunks += 1
        for r, k in ch.items:
            r.step_latencies_ms.append((ms / ch.n_steps, k))
            self.agent_steps += k * r.agents
        for r in ch.finishing:
            err = self.ex.check(r)
            r.t_finish = time.perf_counter()
            if err:
                r.state, r.error = "failed", err
                with self.lock:
                    self.used -= r.footprint
                r.footprint = 0
                r.outputs = None
            else:
                r.state = "done"
            self.finished.append(r)
            r._event.set()

    def step_once(self) -> bool:
        """Admit what fits, enqueue one chunk for every active request, and
        account the chunks the device has finished. Returns False when there
        is nothing to do."""
        self._collect()
        ev_start = self.ex.mark()
        self._admit()
        if not self.active:
            if self.inflight:
                self._complete_oldest()
                return True
            return False
        if len(self.inflight) >= self.depth:
            self._complete_oldest()
        ev_step = self.ex.mark()
        items = [(r, min(self.chunk, r.left)) for r in self.active]
        n = max(k for _, k in items)
        self.ex.step(n)
        finishing, still = [], []
        for r, k in items:
            r.left -= k
            (finishing if r.left == 0 else still).append(r)
        # finished ranges leave now, in stream order after their last steps;
        # their slots are free for the next admission
        for r in finishing:
            self.ex.release(r)
            with self.lock:
                self.slots.give(r.first_slot, r.n_envs)
                self.n_ranges -= 1
        self.active = still
        self.inflight.append(Chunk(ev_start, ev_step, self.ex.mark(), n, items, finishing))
        self._collect()
        return True

    def _collect(self) -> None:
        """Account the chunks the device has finished (no waiting)."""
        while self.inflight and self.ex.done(self.inflight[0].ev_end):
            self._complete(self.inflight.popleft())

    def _complete_oldest(self) -> None:
        ch = self.inflight.popleft()
        self.ex.wait(ch.ev_end)
        self._complete(ch)

    def drain(self) -> None:
        while self.step_once() or self.queue:
            if not self.active and not self.inflight and self.queue:
                # the queue head waits for a client to fetch outputs
                with self.wake:
                    self.wake.wait(0.01)

    # ---- background loop ---------------------------------------------------
    def start(self) -> None:
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def _loop(self) -> None:
        while True:
            with self.lock:
                if self.stop_flag:
                    break
                idle = not self.queue and not self.active and not self.inflight
                if idle:
                    self.wake.wait(0.002)
                    continue
            if not self.step_once():
                with self.wake:
                    self.wake.wait(0.0005)
        while self.inflight:
            self._complete_oldest()

    def stop(self) -> None:
        with self.lock:
            self.stop_flag = True
            self.wake.notify_all()
        if self.thread is not None:
            self.thread.join()

    # ---- metrics -----------------------------------------------------------
    def stats(self, wall_s: float | None = None) -> dict:
        lat = []
        wts = []
        for r in self.finished:
            for v, k in r.step_latencies_ms:
                lat.append(v)
                wts.append(k)
        qd = [r.t_admit - r.t_submit for r in self.finished]
        ct = [r.t_finish - r.t_submit for r in self.finished]

        def wpct(q):
            if not lat:
                return 0.0
            a = np.asarray(lat)
            w = np.asarray(wts, dtype=np.float64)
            o = np.argsort(a)
            cw = np.cumsum(w[o]) / w.sum()
            return float(a[o][min(len(a) - 1, int(np.searchsorted(cw, q / 100.0)))])

        out = {
            "requests_done": sum(r.state == "done" for r in self.finished),
            "chunks": self.chunks,
            "agent_steps": self.agent_steps,
            "step_ms": self.step_ms,
            "busy_ms": self.busy_ms,
            "agent_steps_per_s_device": (self.agent_steps / (self.step_ms / 1e3)
                                         if self.step_ms else 0.0),
            "step_latency_ms_p50": wpct(50),
            "step_latency_ms_p99": wpct(99),
            "queue_delay_s_p50": float(np.percentile(qd, 50)) if qd else 0.0,
            "queue_delay_s_p99": float(np.percentile(qd, 99)) if qd else 0.0,
            "completion_s_p50": float(np.percentile(ct, 50)) if ct else 0.0,
            "completion_s_p99": float(np.percentile(ct, 99)) if ct else 0.0,
        }
        if wall_s:
            out["agent_steps_per_s_wall"] = self.agent_steps / wall_s
            out["device_busy_frac"] = self.busy_ms / 1e3 / wall_s
        return out


def run_trace(server: Server, trace, time_scale: float = 1.0, fetch: bool = True) -> dict:
    """Replay a request trace (workloads.serving_trace) against a started
    server: submit each request at its arrival time (scaled), fetch each
    output as soon as its request is done; returns the server's stats with
    wall-clock throughput. The wall time runs from the first arrival to the
    last completion."""
    reqs = [Request(t["rid"], t["spec"], t["n_envs"], t["steps"], t["seed"], t["arrival_s"])
            for t in trace]
    fetched = []

    def client():
        for r in reqs:
            r.wait()
            if fetch and r.state == "done":
                server.fetch(r)
                fetched.append(r.rid)

    cl = threading.Thread(target=client, daemon=True)
    cl.start()
    t0 = time.perf_counter()
    for r in reqs:
        delay = r.arrival_s * time_scale - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        server.submit(r)
    cl.join()
    wall = max(r.t_finish for r in reqs if r.t_finish) - t0
    st = server.stats(wall)
    st["wall_s"] = wall
    st["requests"] = len(reqs)
    st["failed"] = sum(r.state != "done" for r in reqs)
    return st


def mean_request_agent_steps(n: int = 20000, seed: int = 5) -> float:
    """Mean agent-steps of a request of the serving trace's distribution."""
    from . import workloads as wl

    tr = wl.serving_trace(n, 1.0, seed)
    return float(np.mean([t["n_envs"] * t["spec"]["n"] * t["steps"] for t in tr]))


def main(argv=None):
    """Serve synthetic Poisson traces on the GPU at offered loads rho x the
    measured capacity (agent-steps/s of the uneven batch) and print one JSON
    line per load."""
    import argparse
    import json

    from . import workloads as wl

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--rho", default="0.5,0.9,1.5", help="offered loads, fractions of capacity")
    ap.add_argument("--capacity", type=float, default=0.0,
                    help="agent-steps/s of the uneven 8192-env batch (0: measure it)")
    ap.add_argument("--chunk", type=int, default=128, help="steps per launch")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=1 << 18)
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args(argv)
    import torch

    from . import hase

    cap = args.capacity
    if cap <= 0:
        specs = wl.workload_specs("uneven8k")
        b = hase.HaseBatch(specs, device="cuda:0")
        b.reset(4, obs=False)
        outs = b.alloc_outputs(2000)
        b.step_into(*outs, 2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step_into(*outs, 2000)
        torch.cuda.synchronize()
        cap = sum(s["n"] for s in specs) * 2000 / (time.perf_counter() - t0)
        b.close()
        del outs
        torch.cuda.empty_cache()
    per_req = mean_request_agent_steps()
    ex = HipExecutor("cuda:0", n_slots=args.slots)
    for rho in [float(x) for x in args.rho.split(",")]:
        rate = rho * cap / per_req
        trace = wl.serving_trace(args.requests, rate, args.seed)
        srv = Server(ex, budget_bytes=int(args.budget_gb * (1 << 30)), chunk=args.chunk)
        srv.start()
        try:
            st = run_trace(srv, trace)
        finally:
            srv.stop()
        st.update(rho=rho, capacity_agent_steps_per_s=cap, rate_per_s=rate, chunk=args.chunk,
                  budget_gb=args.budget_gb, slots=args.slots)
        print(json.dumps(st), flush=True)


if __name__ == "__main__":
    main()
