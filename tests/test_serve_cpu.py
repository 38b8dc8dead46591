"""Serving-loop scheduling on the CPU, with a test-double executor that keeps
each admitted request as an oracle batch (the product executor keeps them in
a device arena). Covers slot and budget admission, chunking with each
request's own budget, release and slot reuse, fetch handing outputs over,
failure isolation and the background loop."""
import threading

import numpy as np
import pytest

from oracle import oracle as o
from paper_2604_27162_amd import serve, workloads as wl


class Ev:
    """Stand-in for a device event: complete at once, no duration."""

    def query(self):
        return True


class OracleArenaExecutor:
    """Executor test double: an arena of n_slots whose admitted ranges are
    oracle batches, stepped synchronously."""

    def __init__(self, n_slots=1000, max_ranges=64, fixed_bytes=1000, bad_rids=()):
        self.n_slots = n_slots
        self.max_ranges = max_ranges
        self.fixed_bytes = fixed_bytes
        self.bad_rids = set(bad_rids)
        self.ranges = {}      # first slot -> request
        self.admitted = []
        self.released = []
        self.steps_taken = {}

    def footprint(self, req):
        s = req.spec
        d = 2 * s["r"] + 1
        obs_words = req.n_envs * s["n"] * s["C"] * ((d * d + 31) // 32)
        per_step = 4 * obs_words + 4 * req.n_envs * s["n"] + req.n_envs
        return req.steps * per_step + 4 * obs_words

    def admit(self, req):
        first, count = req.first_slot, req.n_envs
        assert 0 <= first and first + count <= self.n_slots
        for f, r in self.ranges.items():  # slots are never handed out twice
            assert first + count <= f or f + r.n_envs <= first
        b = o.OracleBatch([req.spec] * count, env_id_base=0)
        b.reset(req.seed)
        req.outputs = dict(obs=np.zeros((req.steps, b.obs_total), np.uint32),
                           rew=np.zeros((req.steps, b.agents_total), np.float32),
                           done=np.zeros((req.steps, b.n_envs), np.uint8))
        req._oracle = b
        self.ranges[first] = req
        self.steps_taken[req.rid] = 0
        self.admitted.append(req.rid)

    def mark(self):
        return Ev()

    def step(self, n):
        for r in self.ranges.values():
            k = min(n, r.steps - self.steps_taken[r.rid])
            if k:
                ob, rw, dn = r._oracle.step(k)
                s0 = self.steps_taken[r.rid]
                r.outputs["obs"][s0:s0 + k] = ob
                r.outputs["rew"][s0:s0 + k] = rw
                r.outputs["done"][s0:s0 + k] = dn
                self.steps_taken[r.rid] += k

    def release(self, req):
        del self.ranges[req.first_slot]
        self.released.append(req.rid)

    @staticmethod
    def done(ev):
        return ev.query()

    @staticmethod
    def wait(ev):
        pass

    @staticmethod
    def elapsed_ms(a, b):
        return 1.0

    def check(self, req):
        return "planted reset failure" if req.rid in self.bad_rids else ""


def make_reqs(n, seed=3, envs=24, steps=70):
    tr = wl.serving_trace(n, rate_per_s=1000.0, seed=seed)
    return [serve.Request(t["rid"], t["spec"], min(t["n_envs"], envs), min(t["steps"], steps),
                          t["seed"]) for t in tr]


def alone(req):
    b = o.OracleBatch([req.spec] * req.n_envs, env_id_base=0)
    b.reset(req.seed)
    return b.step(req.steps)


def test_slot_allocator_first_fit_and_merge():
    a = serve.SlotAllocator(100)
    assert a.take(30) == 0 and a.take(30) == 30 and a.take(50) is None
    a.give(0, 30)
    assert a.take(10) == 0 and a.take(25) == 60 and a.take(20) == 10
    a.give(30, 30)
    a.give(10, 20)
    a.give(0, 10)
    assert a.free == [(0, 60), (85, 15)] and a.largest() == 60
    a.give(60, 25)
    assert a.free == [(0, 100)]


def test_results_same_alone_and_in_mix():
    ex = OracleArenaExecutor()
    srv = serve.Server(ex, budget_bytes=1 << 40, chunk=16)
    reqs = make_reqs(6)
    for r in reqs[:3]:
        srv.submit(r)
    srv.step_once()
    srv.step_once()
    for r in reqs[3:]:  # arrive while others are running
        srv.submit(r)
    srv.drain()
    for r in reqs:
        assert r.state == "done"
        for got, want in zip(srv.fetch(r), alone(r)):
            assert np.array_equal(got, want)
    assert srv.used == ex.fixed_bytes
    assert sorted(ex.released) == sorted(r.rid for r in reqs)


def test_fetch_hands_outputs_over():
    """After fetch the server holds no reference to a request's outputs."""
    ex = OracleArenaExecutor()
    srv = serve.Server(ex, budget_bytes=1 << 40, chunk=32)
    reqs = make_reqs(3, seed=7)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    for r in reqs:
        srv.fetch(r)
    assert all(r.outputs is None for r in srv.finished)
    with pytest.raises(RuntimeError):
        srv.fetch(reqs[0])


def test_admission_waits_for_slots_and_reuses_them():
    ex = OracleArenaExecutor(n_slots=50)
    srv = serve.Server(ex, budget_bytes=1 << 40, chunk=1000)
    reqs = make_reqs(3, seed=4, envs=24)  # two fit at once, the third waits for slots
    for r in reqs:
        srv.submit(r)
    srv.step_once()
    assert [r.state for r in reqs] == ["done", "done", "queued"]
    srv.step_once()
    assert reqs[2].state == "done"
    assert reqs[2].first_slot in (reqs[0].first_slot, reqs[1].first_slot)


def test_admission_waits_for_budget_and_fetch():
    ex = OracleArenaExecutor()
    reqs = make_reqs(3, seed=4)
    fp = [ex.footprint(r) for r in reqs]
    srv = serve.Server(ex, budget_bytes=max(fp) + ex.fixed_bytes, chunk=1000)
    for r in reqs:
        srv.submit(r)
    assert srv.step_once()
    assert [r.state for r in reqs] == ["done", "queued", "queued"]
    # outputs still resident: nothing else fits until the client fetches
    srv.step_once()
    assert reqs[1].state == "queued"
    srv.fetch(reqs[0])
    srv.step_once()
    assert reqs[1].state == "done" and reqs[2].state == "queued"


def test_rejects_request_larger_than_budget():
    ex = OracleArenaExecutor()
    r = make_reqs(1)[0]
    srv = serve.Server(ex, budget_bytes=ex.footprint(r) + ex.fixed_bytes - 1)
    srv.submit(r)
    assert r.state == "rejected"
    with pytest.raises(RuntimeError):
        srv.fetch(r, 0)


def test_cancel_queued_and_failure_isolation():
    reqs = make_reqs(4, seed=6)
    ex = OracleArenaExecutor(bad_rids={reqs[1].rid})
    srv = serve.Server(ex, budget_bytes=1 << 40, chunk=8)
    for r in reqs:
        srv.submit(r)
    assert srv.cancel(reqs[3])
    srv.drain()
    assert reqs[1].state == "failed" and "planted" in reqs[1].error
    assert reqs[3].state == "cancelled"
    for r in (reqs[0], reqs[2]):
        assert r.state == "done"
        for got, want in zip(srv.fetch(r), alone(r)):
            assert np.array_equal(got, want)
    assert srv.used == ex.fixed_bytes


def test_range_table_limit_queues():
    ex = OracleArenaExecutor(max_ranges=2)
    srv = serve.Server(ex, budget_bytes=1 << 40, chunk=1000)
    reqs = make_reqs(3, seed=8)
    for r in reqs:
        srv.submit(r)
    srv.step_once()
    assert [r.state for r in reqs] == ["done", "done", "queued"]
    srv.drain()
    assert reqs[2].state == "done"


def test_background_thread_serves_concurrent_clients():
    ex = OracleArenaExecutor()
    srv = serve.Server(ex, budget_bytes=1 << 40, chunk=16)
    srv.start()
    reqs = make_reqs(5, seed=9)
    res = {}

    def client(r):
        srv.submit(r)
        res[r.rid] = srv.fetch(r, 60)

    th = [threading.Thread(target=client, args=(r,)) for r in reqs]
    for t in th:
        t.start()
    for t in th:
        t.join(60)
    srv.stop()
    for r in reqs:
        for got, want in zip(res[r.rid], alone(r)):
            assert np.array_equal(got, want)
    st = srv.stats(1.0)
    assert st["requests_done"] == 5 and st["step_latency_ms_p99"] >= st["step_latency_ms_p50"]
