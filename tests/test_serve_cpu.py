"""Serving-loop scheduling on the CPU, with a test-double executor that runs
requests on the oracle (the product executor runs them on the GPU)."""
import threading

import numpy as np
import pytest

from oracle import oracle as o
from paper_2604_27162_amd import serve, workloads as wl


class OracleExecutor:
    """Executor test double: every request is an oracle batch."""

    def __init__(self, fail_rids=()):
        self.fail_rids = set(fail_rids)
        self.created = []
        self.released = []

    def footprint(self, req):
        s = req.spec
        d = 2 * s["r"] + 1
        obs_words = req.n_envs * s["n"] * s["C"] * ((d * d + 31) // 32)
        per_step = 4 * obs_words + 4 * req.n_envs * s["n"] + req.n_envs
        return 1000 * req.n_envs + req.steps * per_step

    def create(self, req):
        if req.rid in self.fail_rids:
            raise RuntimeError("planted failure")
        b = o.OracleBatch([req.spec] * req.n_envs, env_id_base=0)
        b.reset(req.seed)
        outs = (np.zeros((req.steps, b.obs_total), np.uint32),
                np.zeros((req.steps, b.agents_total), np.float32),
                np.zeros((req.steps, b.n_envs), np.uint8))
        self.created.append(req.rid)
        return b, outs

    def step(self, items, n_steps):
        assert all(k <= n_steps for _, k in items)
        for r, k in items:
            ob, rw, dn = r.batch.step(k)
            s0 = r.done_steps
            r.outputs[0][s0:s0 + k] = ob
            r.outputs[1][s0:s0 + k] = rw
            r.outputs[2][s0:s0 + k] = dn
        return 1.0

    def release(self, req):
        self.released.append(req.rid)
        req.batch = None


def make_reqs(n, seed=3):
    tr = wl.serving_trace(n, rate_per_s=1000.0, seed=seed)
    out = []
    for t in tr:
        out.append(serve.Request(t["rid"], t["spec"], min(t["n_envs"], 24), min(t["steps"], 70),
                                 t["seed"]))
    return out


def alone(req):
    b = o.OracleBatch([req.spec] * req.n_envs, env_id_base=0)
    b.reset(req.seed)
    return b.step(req.steps)


def test_results_same_alone_and_in_mix():
    ex = OracleExecutor()
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
    assert srv.used == 0


def test_admission_waits_for_budget_and_fetch():
    ex = OracleExecutor()
    reqs = make_reqs(3, seed=4)
    fp = [ex.footprint(r) for r in reqs]
    srv = serve.Server(ex, budget_bytes=max(fp), chunk=1000)
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
    ex = OracleExecutor()
    r = make_reqs(1)[0]
    srv = serve.Server(ex, budget_bytes=ex.footprint(r) - 1)
    srv.submit(r)
    assert r.state == "rejected"
    with pytest.raises(RuntimeError):
        r.result(0)


def test_cancel_queued_and_failure_isolation():
    reqs = make_reqs(4, seed=6)
    ex = OracleExecutor(fail_rids={reqs[1].rid})
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
    assert srv.used == 0
    assert sorted(ex.released) == sorted([reqs[0].rid, reqs[2].rid])


def test_background_thread_serves_concurrent_clients():
    ex = OracleExecutor()
    srv = serve.Server(ex, budget_bytes=1 << 40, chunk=16)
    srv.start()
    reqs = make_reqs(5, seed=9)
    res = {}

    def client(r):
        srv.submit(r)
        res[r.rid] = srv.fetch(r)

    th = [threading.Thread(target=client, args=(r,)) for r in reqs]
    for t in th:
        t.start()
    for t in th:
        t.join(60)
    srv.stop()
    for r in reqs:
        for got, want in zip(res[r.rid], alone(r)):
            assert np.array_equal(got, want)
    st = srv.stats()
    assert st["requests_done"] == 5 and st["step_latency_ms_p99"] >= st["step_latency_ms_p50"]
