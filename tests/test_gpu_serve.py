"""Multi-batch stepping, the serving loop and the autotuner on the GPU.

Every request's result must be bit-identical whether it runs alone or in the
continuous-batching mix (tolerance 0): env ids are request-local and keys
come from the request's own seed."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as o  # noqa: E402
from paper_2604_27162_amd import hase, serve, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def alone(spec, n_envs, seed, steps):
    b = hase.HaseBatch([spec] * n_envs, device=DEV)
    b.reset(seed)
    out = b.step(steps)
    torch.cuda.synchronize()
    b.close()
    return out


def test_step_multi_matches_separate_batches():
    specs = [wl.spec(16, 16, 2, 2, 3, 10), wl.spec(32, 32, 10, 4, 4, 15), wl.spec(64, 64, 5, 3, 4, 20)]
    n_envs = [100, 37, 21]
    steps = [40, 25, 33]
    seeds = [11, 12, 13]
    bs = []
    for sp, ne, sd in zip(specs, n_envs, seeds):
        b = hase.HaseBatch([sp] * ne, device=DEV)
        b.reset(sd)
        bs.append(b)
    outs = [b.alloc_outputs(k) for b, k in zip(bs, steps)]
    ws = torch.empty(hase.multi_workspace_bytes(bs), dtype=torch.uint8, device=DEV)
    stream = torch.cuda.current_stream()
    done = [0, 0, 0]
    # chunks of 16 steps; each request stops at its own budget
    while any(d < k for d, k in zip(done, steps)):
        items = []
        for i, b in enumerate(bs):
            k = min(16, steps[i] - done[i])
            if k > 0:
                items.append((b, k, done[i], None, *outs[i]))
        hase.step_multi(items, 16, ws, stream)
        torch.cuda.synchronize()
        for i in range(3):
            done[i] = min(steps[i], done[i] + 16)
    for i in range(3):
        ref = alone(specs[i], n_envs[i], seeds[i], steps[i])
        for got, want in zip(outs[i], ref):
            assert torch.equal(got, want)


def test_step_multi_uneven_requests_match_oracle():
    """Two uneven plain requests in one multi-batch step: their combined
    launches (4-, 8- and 16-lane tiles of both requests in one grid) give
    each request the oracle's outputs."""
    reqs = [(wl.workload_specs("uneven8k", 1400)[:157], 21, 30),
            ([s for s in wl.workload_specs("uneven8k", 900)[400:] if s["n"] >= 5][:71], 22, 19)]
    bs = []
    for specs, seed, _ in reqs:
        b = hase.HaseBatch(specs, device=DEV)
        b.reset(seed)
        bs.append(b)
    outs = [b.alloc_outputs(k) for b, (_, _, k) in zip(bs, reqs)]
    ws = torch.empty(hase.multi_workspace_bytes(bs), dtype=torch.uint8, device=DEV)
    stream = torch.cuda.current_stream()
    items = [(b, k, 0, None, *out) for b, (_, _, k), out in zip(bs, reqs, outs)]
    hase.step_multi(items, 30, ws, stream)
    torch.cuda.synchronize()
    for (specs, seed, k), (go, gr, gd), b in zip(reqs, outs, bs):
        ob = o.OracleBatch(specs)
        ob.reset(seed)
        oo, orr, od = ob.step(k)
        assert np.array_equal(go.cpu().numpy().view(np.uint32).reshape(oo.shape), oo)
        assert np.array_equal(gr.cpu().numpy().view(np.uint32).reshape(orr.shape), orr.view(np.uint32))
        assert np.array_equal(gd.cpu().numpy().reshape(od.shape), od)
        b.close()


def test_server_alone_vs_mix_bit_exact():
    """Requests served together in the arena, some admitted while others
    run and into slots others left, equal the same requests run alone and
    the oracle (obs, rewards as float32 bits, dones) for every request."""
    trace = wl.serving_trace(10, rate_per_s=1e6, seed=21)
    reqs = [serve.Request(t["rid"], t["spec"], t["n_envs"] // 8, t["steps"] // 4, t["seed"])
            for t in trace]
    ex = serve.HipExecutor(DEV, n_slots=1200, max_ranges=6)
    srv = serve.Server(ex, budget_bytes=64 << 30, chunk=32)
    for r in reqs[:4]:
        srv.submit(r)
    srv.step_once()
    srv.step_once()
    for r in reqs[4:]:
        srv.submit(r)
    srv.drain()
    while srv.inflight:
        srv.step_once()
    st = srv.stats(1.0)
    assert st["requests_done"] == len(reqs)
    slots = [r.first_slot for r in reqs]
    assert len(set(slots)) < len(slots)  # some slots were taken twice
    for r in reqs:
        got = srv.fetch(r)
        assert r.outputs is None
        want = alone(r.spec, r.n_envs, r.seed, r.steps)
        for g, w in zip(got, want):
            assert torch.equal(g, w), r.rid
        ob = o.OracleBatch([r.spec] * r.n_envs)
        ob.reset(r.seed)
        oo, orr, od = ob.step(r.steps)
        go, gr, gd = got
        assert np.array_equal(go.cpu().numpy().view(np.uint32), oo), r.rid
        assert np.array_equal(gr.cpu().numpy().view(np.uint32), orr.view(np.uint32)), r.rid
        assert np.array_equal(gd.cpu().numpy(), od), r.rid
    assert srv.used == ex.fixed_bytes


def test_server_budget_queues_until_fetch():
    trace = wl.serving_trace(3, rate_per_s=1e6, seed=22)
    reqs = [serve.Request(t["rid"], t["spec"], 64, 40, t["seed"]) for t in trace]
    ex = serve.HipExecutor(DEV, n_slots=512, max_ranges=8)
    fp = [ex.footprint(r) for r in reqs]
    srv = serve.Server(ex, budget_bytes=max(fp) + ex.fixed_bytes, chunk=64)
    for r in reqs:
        srv.submit(r)
    srv.step_once()
    while srv.inflight:
        srv.step_once()
    assert reqs[0].state == "done" and reqs[1].state == "queued"
    srv.fetch(reqs[0])
    srv.step_once()
    while srv.inflight:
        srv.step_once()
    assert reqs[1].state == "done"


def test_autotune_restores_state_and_keeps_results():
    specs = wl.workload_specs("uneven8k", 700)
    g = hase.HaseBatch(specs, device=DEV)
    g.reset(4)
    g.step(30)
    before = g.get_state()
    lanes = g.autotune(16)
    after = g.get_state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    assert g.get_tiling() == lanes
    ob = o.OracleBatch(specs)
    ob.reset(4)
    ob.step(30)
    out = g.step(60)
    torch.cuda.synchronize()
    oo, orr, od = ob.step(60)
    assert np.array_equal(out[0].cpu().numpy().view(np.uint32), oo)
    assert np.array_equal(out[2].cpu().numpy(), od)
