"""Continuous-batching serving loop for rollout requests.

A request asks for `n_envs` environments of one spec, stepped `steps` times
from `seed` (env ids 0..n_envs-1 of the request, so its result does not
depend on what else runs). The server keeps every admitted request's state
resident on the device, admits queued requests as soon as the device-memory
budget allows (footprint = state buffer + the request's whole output, which
stays resident until the client fetches it), and advances all active
requests together, `chunk` steps per launch, through the library's
multi-batch step: requests that arrive while others run join at the next
chunk, finished ones leave and free their budget.

Reported: per-chunk step latency (chunk GPU time / chunk steps, weighted by
the requests it advanced) as p50/p99, queueing delay, completion time and
aggregate agent-steps/s.

The scheduling logic talks to an executor (create / step / release); the
HIP executor below is the product path. Tests may plug in another executor.
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
    batch: object = None
    outputs: tuple = ()
    done_steps: int = 0
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

    def result(self, timeout=None):
        """(obs, rew, done) of every step, after the request finished."""
        if not self._event.wait(timeout):
            raise TimeoutError(f"request {self.rid} not finished")
        if self.state != "done":
            raise RuntimeError(f"request {self.rid} {self.state}: {self.error}")
        return self.outputs


class HipExecutor:
    """Runs requests on the GPU through libhase (one handle per request)."""

    def __init__(self, device="cuda:0", autotune_steps: int = 0):
        import torch

        from . import hase

        self.torch = torch
        self.hase = hase
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.autotune_steps = autotune_steps
        self.workspace = torch.empty(0, dtype=torch.uint8, device=self.device)
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev1 = torch.cuda.Event(enable_timing=True)

    def footprint(self, req: Request) -> int:
        lay = self.hase.query_layout([req.spec] * req.n_envs)
        per_step = 4 * lay.obs_words_per_step + 4 * lay.agents_total + lay.n_envs
        return int(lay.state_bytes + req.steps * per_step)

    def create(self, req: Request):
        b = self.hase.HaseBatch([req.spec] * req.n_envs, env_id_base=0, device=self.device,
                                stream=self.stream)
        b.reset(req.seed)
        if self.autotune_steps:
            b.autotune(self.autotune_steps)
        outs = b.alloc_outputs(req.steps)
        return b, outs

    def step(self, items, n_steps: int) -> float:
        """items: (request, steps) pairs; returns the launch's GPU ms."""
        batches = [r.batch for r, _ in items]
        need = self.hase.multi_workspace_bytes(batches)
        if self.workspace.numel() < need:
            self.workspace = self.torch.empty(max(need, 2 * self.workspace.numel()),
                                              dtype=self.torch.uint8, device=self.device)
        work = [(r.batch, k, r.done_steps, None, *r.outputs) for r, k in items]
        self.ev0.record(self.stream)
        self.hase.step_multi(work, n_steps, self.workspace, self.stream)
        self.ev1.record(self.stream)
        self.ev1.synchronize()
        return float(self.ev0.elapsed_time(self.ev1))

    def release(self, req: Request) -> None:
        if req.batch is not None:
            req.batch.close()
            req.batch.state = None
            req.batch = None


class Server:
    """Admission by memory footprint, continuous batching in chunks of steps."""

    def __init__(self, executor, budget_bytes: int = 64 << 30, chunk: int = 32):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.used = 0
        self.queue = collections.deque()
        self.active: list[Request] = []
        self.finished: list[Request] = []
        self.lock = threading.Lock()
        self.wake = threading.Condition(self.lock)
        self.stop_flag = False
        self.thread = None
        self.agent_steps = 0
        self.gpu_ms = 0.0
        self.chunks = 0

    # ---- client side -------------------------------------------------------
    def submit(self, req: Request) -> Request:
        req.footprint = self.ex.footprint(req)
        req.t_submit = time.perf_counter()
        with self.lock:
            if req.footprint > self.budget:
                req.state, req.error = "rejected", "footprint exceeds the whole budget"
                req._event.set()
                return req
            req.state = "queued"
            self.queue.append(req)
            self.wake.notify()
        return req

    def cancel(self, req: Request) -> bool:
        """Cancel a queued request (active ones run to completion)."""
        with self.lock:
            if req.state == "queued":
                self.queue.remove(req)
                req.state = "cancelled"
                req._event.set()
                return True
        return False

    def fetch(self, req: Request):
        """Hand the outputs to the client and release their budget."""
        out = req.result()
        with self.lock:
            if req.footprint:
                self.used -= req.footprint
                req.footprint = 0
                self.wake.notify()
        return out

    # ---- scheduler ---------------------------------------------------------
    def _admit(self) -> None:
        """FIFO admission while the head of the queue fits the budget."""
        while True:
            with self.lock:
                if not self.queue or self.used + self.queue[0].footprint > self.budget:
                    return
                req = self.queue.popleft()
                self.used += req.footprint
            try:
                req.batch, req.outputs = self.ex.create(req)
            except Exception as err:  # a failed request frees its budget, others go on
                with self.lock:
                    self.used -= req.footprint
                req.footprint = 0
                req.state, req.error = "failed", str(err)
                req._event.set()
                continue
            req.state = "active"
            req.t_admit = time.perf_counter()
            self.active.append(req)

    def step_once(self) -> bool:
        """Admit what fits, advance every active request by up to one chunk.
        Returns False when there is nothing to do."""
        self._admit()
        if not self.active:
            return False
        items = [(r, min(self.chunk, r.steps - r.done_steps)) for r in self.active]
        n = max(k for _, k in items)
        try:
            ms = self.ex.step(items, n)
        except Exception as err:
            for r, _ in items:
                self.ex.release(r)
                r.state, r.error = "failed", str(err)
                with self.lock:
                    self.used -= r.footprint
                r.footprint = 0
                r._event.set()
            self.active = []
            return True
        self.gpu_ms += ms
        self.chunks += 1
        still = []
        for r, k in items:
            r.done_steps += k
            r.step_latencies_ms.append((ms / n, k))
            self.agent_steps += k * r.agents
            if r.done_steps >= r.steps:
                # state memory is released now; the outputs stay until fetched
                self.ex.release(r)
                r.state = "done"
                r.t_finish = time.perf_counter()
                self.finished.append(r)
                r._event.set()
            else:
                still.append(r)
        self.active = still
        return True

    def drain(self) -> None:
        while self.step_once() or self.queue:
            if not self.active and self.queue:
                with self.lock:
                    blocked = bool(self.queue) and self.used + self.queue[0].footprint > self.budget
                if blocked:
                    # waiting for a client to fetch outputs
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
                    return
                idle = not self.queue and not self.active
                if idle:
                    self.wake.wait(0.01)
                    continue
            if not self.step_once():
                with self.wake:
                    self.wake.wait(0.001)

    def stop(self) -> None:
        with self.lock:
            self.stop_flag = True
            self.wake.notify_all()
        if self.thread is not None:
            self.thread.join()

    # ---- metrics -----------------------------------------------------------
    def stats(self, wall_s: float | None = None) -> dict:
        lat = []
        for r in self.finished:
            for v, k in r.step_latencies_ms:
                lat.extend([v] * k)
        lat = np.array(lat) if lat else np.zeros(1)
        qd = [r.t_admit - r.t_submit for r in self.finished]
        ct = [r.t_finish - r.t_submit for r in self.finished]
        out = {
            "requests_done": len(self.finished),
            "chunks": self.chunks,
            "agent_steps": self.agent_steps,
            "gpu_ms": self.gpu_ms,
            "agent_steps_per_s_gpu": self.agent_steps / (self.gpu_ms / 1e3) if self.gpu_ms else 0.0,
            "step_latency_ms_p50": float(np.percentile(lat, 50)),
            "step_latency_ms_p99": float(np.percentile(lat, 99)),
            "queue_delay_s_p50": float(np.percentile(qd, 50)) if qd else 0.0,
            "queue_delay_s_p99": float(np.percentile(qd, 99)) if qd else 0.0,
            "completion_s_p50": float(np.percentile(ct, 50)) if ct else 0.0,
            "completion_s_p99": float(np.percentile(ct, 99)) if ct else 0.0,
        }
        if wall_s:
            out["agent_steps_per_s_wall"] = self.agent_steps / wall_s
        return out


def run_trace(server: Server, trace, time_scale: float = 1.0, fetch: bool = True) -> dict:
    """Replay a request trace (workloads.serving_trace) against a started
    server: submit each request at its arrival time (scaled), wait for all,
    fetch the outputs; returns the server's stats with wall-clock throughput."""
    reqs = [Request(t["rid"], t["spec"], t["n_envs"], t["steps"], t["seed"], t["arrival_s"])
            for t in trace]
    t0 = time.perf_counter()
    for r in reqs:
        delay = r.arrival_s * time_scale - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        server.submit(r)
    for r in reqs:
        r.wait()
        if fetch and r.state == "done":
            server.fetch(r)
    wall = time.perf_counter() - t0
    st = server.stats(wall)
    st["wall_s"] = wall
    st["requests"] = len(reqs)
    st["failed"] = sum(r.state != "done" for r in reqs)
    return st


def main(argv=None):
    """Serve a synthetic Poisson trace on the GPU and print one JSON line of
    latency / throughput statistics."""
    import argparse
    import json

    from . import workloads as wl

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--rate", type=float, default=20.0, help="mean arrivals per second")
    ap.add_argument("--chunk", type=int, default=128, help="steps per multi-batch launch")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--autotune", type=int, default=0, help="autotune steps per request (0: off)")
    args = ap.parse_args(argv)
    trace = wl.serving_trace(args.requests, args.rate, args.seed)
    srv = Server(HipExecutor("cuda:0", autotune_steps=args.autotune),
                 budget_bytes=int(args.budget_gb * (1 << 30)), chunk=args.chunk)
    srv.start()
    try:
        st = run_trace(srv, trace)
    finally:
        srv.stop()
    st.update(rate_per_s=args.rate, chunk=args.chunk, budget_gb=args.budget_gb)
    print(json.dumps(st), flush=True)


if __name__ == "__main__":
    main()
