#!/usr/bin/env python3
"""Throughput of the vectorised hide-and-seek step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload single16k]

One bench step is one run of the workload's configuration: every env of the
batch advanced by the workload's run length (10,000 env-steps for the
single-agent workloads, 2,000 for the multi-agent and uneven ones, 256 for
the small one) in ONE persistent kernel launch, with actions drawn by the
counter generator, moves, detection and rewards, dones, same-step
auto-reset and observations, and all state resident in HBM. W untimed runs
come first; then exactly K runs are enqueued back to back and timed as one
region bracketed by torch.cuda.synchronize(), with a HIP event on the
kernel's stream between consecutive runs (median and spread per run).

Beside the runs the line reports:
  chunks       calls of 1, 20 and 128 env-steps (each bracketed by a
               synchronize, >= 20 repetitions): the fixed cost per call that
               a trainer stepping in short chunks pays;
  per_launch   the same batch with one kernel launch per env-step;
  int8_actions one run with external int8 actions resident in HBM;
  roofline     algorithmic bytes per run / mean run time against 8 TB/s and
               against a device copy measured on the same GPU;
  cpu_baseline the CPU oracle on the host cores, on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "agent-steps/sec on 1 MI355X (persistent vs per-step launch); % of HBM peak"

DESCR = {
    "single16k": "16384 envs, 32x32 grid, 15% iid walls, 1 seeker + 1 hider, 7x7 window, "
                 "3 bit-packed channels, episode 256, counter-generator actions",
    "single1k": "1024 envs, 32x32 grid, 15% iid walls, 1 seeker + 1 hider, 7x7 window, "
                "3 bit-packed channels, episode 256, counter-generator actions",
    "small": "1024 envs, 16x16 grid, 10% iid walls, 1 seeker + 1 hider, 5x5 window, 3 channels",
    "los16k": "16384 envs, 32x32 grid, 15% iid walls, 1 seeker + 1 hider, 7x7 window with "
              "line-of-sight occlusion, 3 bit-packed channels, episode 256",
    "explore16k": "16384 envs, 32x32 grid, 15% iid walls, 1 seeker + 1 hider, 7x7 window, "
                  "3 bit-packed channels, episode 256, exploration rewards, per-step "
                  "discovery-map output (32 words per env)",
    "multi10": "4096 envs, 32x32 grid, 15% iid walls, 5 seekers + 5 hiders, 9x9 window, "
               "4 channels, collisions in agent order",
    "terrain4k": "4096 envs, 32x32 grid, 10% walls, 15% water, 10% mud, 5 seekers + 5 hiders "
                 "of cycling classes (walker, swimmer, flyer), move chances, stuck 25% and "
                 "rescue, 9x9 window, 4 channels",
    "uneven8k": "8192 envs: sides {16,32,64} (50/30/20%), 1..10 agents, 5..25% walls, "
                "radius 2..4, 4 channels",
    "radio4k": "4096 envs, 32x32 grid, 10% iid walls, 5 seekers + 5 hiders, 9x9 window, "
               "4 channels, radio belief sharing (drawn targets, belief word per agent)",
}


def words(r: int) -> int:
    d = 2 * r + 1
    return (d * d + 31) // 32


EXPLORE = 16
TERRAIN = 32
RADIO = 64


def map_bytes(s) -> int:
    """Bytes of an env's discovery map (0 unless it explores)."""
    return 4 * s["H"] * ((s["W"] + 31) // 32) if s["flags"] & EXPLORE else 0


def out_bytes_per_step(specs, maps: bool = False, actions: bool = False,
                       state: bool = False) -> int:
    """Algorithmic bytes of one step: packed obs words, one float32 reward
    per agent, one uint8 done per env and, with map output, the discovery
    maps of exploring envs; radio envs add a belief word per agent; external
    actions add one int8 read per agent; the true-state output adds a uint16
    position per agent and four uint32 words per env."""
    return sum(4 * s["n"] * (s["C"] * words(s["r"]) + (1 if s["flags"] & RADIO else 0)) +
               4 * s["n"] + 1 + (map_bytes(s) if maps else 0) + (s["n"] if actions else 0) +
               ((2 * s["n"] + 16) if state else 0)
               for s in specs)


def state_bytes_per_launch(specs) -> int:
    """Bytes a launch must read and write once: per-env spec/offset/key words
    and counters (read 56 B, plus the map offset for envs with line of sight
    or exploration; write 16 B), agent positions (2 B each way), the padded
    board planes (read, as stored: rows of 3 words; two tile planes with terrain, plus its 24 B of
    classes and chances and the stuck word both ways) and the discovery map
    of an exploring env (read and write); radio envs read and write a belief
    word per agent."""
    tot = 0
    for s in specs:
        planes = 2 if s["flags"] & TERRAIN else 1
        # rows of 3 words, a slack word, padded to 16 bytes (as staged)
        board = 4 * ((planes * ((s["H"] + 8) * 3 + 1) + 3) // 4 * 4)
        feat = 4 if s["flags"] & (8 | EXPLORE) else 0
        if s["flags"] & TERRAIN:
            # terrain words (24 B), stuck word both ways
            feat += 24 + 8
        if s["flags"] & RADIO:
            feat += 8 * s["n"]
        tot += 56 + feat + 16 + 4 * s["n"] + board + 2 * map_bytes(s)
    return tot


def kernel_source_hash() -> str:
    """Hash of the device sources (counters taken on other sources are stale)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2604_27162_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, steps: int):
    """HBM bytes per launch measured by rocprofv3 counters for this kernel
    source (None if absent or taken on another version of the kernel)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    e = d.get(workload)
    if not e or e.get("kernel_hash") != kernel_source_hash() or e.get("steps") != steps:
        return None
    return e.get("hbm_bytes_per_launch")


def spread(ms) -> dict:
    """Median and spread of a list of per-call times (ms)."""
    import numpy as np

    a = np.asarray(ms, dtype=np.float64)
    return dict(n=int(a.size), median=float(np.median(a)), mean=float(a.mean()),
                min=float(a.min()), max=float(a.max()), p10=float(np.percentile(a, 10)),
                p90=float(np.percentile(a, 90)))


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_run(specs, seed, env_id_base, budget_s, start, out, idx):
    """One thread: step an oracle batch (a contiguous env shard, keyed by its
    global env ids) until the shared deadline; the C oracle releases the GIL."""
    from oracle import oracle

    b = oracle.OracleBatch(specs, env_id_base=env_id_base)
    b.reset(seed)
    start.wait()
    t0 = time.perf_counter()
    steps = 0
    while True:
        b.step(10)
        steps += 10
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    out[idx] = (sum(s["n"] for s in specs) * steps, el)


def cpu_baseline(specs, seed: int, budget_s: float = 10.0, threaded_s: float = 10.0):
    """The oracle on the host: one thread over all envs (the plain oracle)
    for budget_s, then one thread per host core (at most 16) over contiguous
    env shards for threaded_s; value is the all-cores rate."""
    import threading

    single = [None]
    ev = threading.Event()
    ev.set()
    _oracle_run(specs, seed, 0, budget_s, ev, single, 0)
    s_agent_steps, s_el = single[0]
    T = max(1, min(16, os.cpu_count() or 1, len(specs)))
    bounds = [len(specs) * i // T for i in range(T + 1)]
    out = [None] * T
    start = threading.Barrier(T + 1)
    ths = [threading.Thread(target=_oracle_run,
                            args=(specs[bounds[i]:bounds[i + 1]], seed, bounds[i], threaded_s,
                                  start, out, i)) for i in range(T)]
    for t in ths:
        t.start()
    start.wait()
    for t in ths:
        t.join()
    total = sum(a for a, _ in out)
    wall = max(el for _, el in out)
    agents = sum(s["n"] for s in specs)
    return dict(value=total / wall, unit="agent-steps/s", cores=T, kind="oracle",
                sample=f"{T} threads over contiguous shards of the {len(specs)} envs for "
                       f"{wall:.1f} s after reset ({total // agents} env-steps per env in all); "
                       f"single thread over all envs: {s_agent_steps // agents} steps in "
                       f"{s_el:.1f} s",
                single_thread=s_agent_steps / s_el,
                env_steps_per_s=total / wall * len(specs) / agents,
                cpu_model=host_cpu_model(), host_threads_available=os.cpu_count())


def copy_bandwidth(torch, nbytes: int = 4 << 30, reps: int = 5) -> float:
    """GB/s of a plain device-to-device copy of nbytes (read + written)."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (spread(ms)["median"] / 1e3) / 1e9


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed runs of the configuration")
    ap.add_argument("--warmup", type=int, default=2, help="untimed runs before them")
    ap.add_argument("--workload", default="single16k", choices=sorted(DESCR))
    ap.add_argument("--run-steps", type=int, default=0,
                    help="env-steps per run (default: the workload's own run length)")
    ap.add_argument("--lanes", default=None, help="lanes per env per agent bucket, e.g. 4,4,16,16")
    ap.add_argument("--autotune", type=int, default=0, metavar="STEPS",
                    help="choose the tiling with the autotuner (timed runs of STEPS steps)")
    ap.add_argument("--only-runs", action="store_true",
                    help="time the runs only (profiling: no other launch of the step kernel)")
    ap.add_argument("--only-per-launch", action="store_true",
                    help="time only the run with one kernel launch per env-step (profiling)")
    ap.add_argument("--int8-actions", action="store_true",
                    help="the timed runs take external int8 actions resident in HBM (with "
                         "--only-runs: profiling of that leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-maps", action="store_true",
                    help="exploring workloads: skip the per-step discovery-map output")
    ap.add_argument("--true-state", choices=("on", "off", "auto"), default="auto",
                    help="the per-step true-state output (positions, found / t / episode / "
                         "stuck); auto: on for the exploring workload, whose per-step "
                         "discovery maps and true state form the centralised observation")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES (calibrates the "
                         "HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the environments are independent, so a multi-GPU "
              "run is N independent shards (env-id ranges) with no exchange and its "
              "throughput N times this line's; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_27162_amd import hase, workloads as wl

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}))
        return
    w = wl.WORKLOADS[args.workload]
    specs = wl.workload_specs(args.workload)
    K, W = int(args.steps), int(args.warmup)
    R = int(args.run_steps or w["steps"])
    n_envs = len(specs)
    agents = sum(s["n"] for s in specs)
    lanes = [int(x) for x in args.lanes.split(",")] if args.lanes else None

    g = hase.HaseBatch(specs, device="cuda:0", lanes=lanes)
    stream = g.stream
    g.reset(w["seed"], obs=False)
    if args.autotune:
        lanes = g.autotune(args.autotune)
    maps_on = g.map_words > 0 and not args.no_maps
    state_on = args.true_state == "on" or (args.true_state == "auto" and g.map_words > 0)
    obs, rew, done = g.alloc_outputs(R)
    mp = g.alloc_outputs(R, maps=True)[3] if maps_on else None
    st = g.alloc_state_outputs(R) if state_on else None
    if args.only_per_launch:
        # one kernel launch per env-step only: P launches after a 50-launch warm-up
        P = min(R, 2000)
        g.step_into(obs, rew, done, min(P, 50), mode=hase.PER_LAUNCH, maps=mp, state=st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.step_into(obs, rew, done, P, mode=hase.PER_LAUNCH, maps=mp, state=st)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_pl = e0.elapsed_time(e1)
        print(json.dumps({"per_launch_env_steps": P, "ms_per_env_step": ms_pl / P,
                          "workload": args.workload}), flush=True)
        g.close()
        return
    xa = (torch.randint(0, 5, (R, agents), dtype=torch.int8, device="cuda:0")
          if args.int8_actions else None)
    g.prepare(obs, rew, done, R, actions=xa, maps=mp, state=st)
    for _ in range(W):
        g.step_into(obs, rew, done, R, actions=xa, maps=mp, state=st)
    torch.cuda.synchronize()

    # ---- K runs back to back, an event between consecutive runs
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(K):
        g.step_into(obs, rew, done, R, actions=xa, maps=mp, state=st)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    run_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(K)]
    total_ms = evs[0].elapsed_time(evs[K])
    mean_ms = total_ms / K
    value = agents * R * K / (total_ms / 1e3)

    alg_bytes = (R * out_bytes_per_step(specs, maps_on, actions=xa is not None, state=state_on) +
                 state_bytes_per_launch(specs))
    achieved = alg_bytes / (mean_ms / 1e3) / 1e9
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": mean_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {DESCR[args.workload]}, {R} env-steps per run",
                   "n_envs": n_envs, "agents": agents, "env_steps_per_bench_step": R,
                   "launch": "persistent: one kernel launch per run (per lanes group)",
                   "lanes_per_env": g.get_tiling(), "map_output": maps_on,
                   "true_state_output": state_on,
                   "actions": "external int8" if xa is not None else "counter generator"},
        "env_steps_per_s": n_envs * R * K / (total_ms / 1e3),
        "run_ms": spread(run_ms),
        "wall_s_timed_region": wall_s,
    }
    traffic = traffic_from_profiles(args.workload + ("_int8" if xa is not None else ""), R)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "step kernel (persistent, one launch per run)",
            "alg_bytes_per_launch": alg_bytes, "launch_ms": mean_ms}

    if not args.only_runs:
        # ---- short calls: the fixed cost per call (each call synchronised)
        chunks = {}
        per_step_run_us = mean_ms * 1e3 / R
        for C in (1, 20, 128):
            co, cr, cd = g.alloc_outputs(C)
            g.prepare(co, cr, cd, C)
            g.step_into(co, cr, cd, C)
            ms = []
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for _ in range(30):
                torch.cuda.synchronize()
                e0.record(stream)
                g.step_into(co, cr, cd, C)
                e1.record(stream)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            sp = spread(ms)
            chunks[str(C)] = dict(call_ms=sp, us_per_env_step=sp["median"] * 1e3 / C,
                                  agent_steps_per_s=agents * C / (sp["median"] / 1e3),
                                  vs_run_per_step=sp["median"] * 1e3 / C / per_step_run_us)
            del co, cr, cd
        line["chunks"] = chunks

        # ---- one kernel launch per env-step (the baseline of the metric)
        P = min(R, 2000)
        g2 = hase.HaseBatch(specs, device="cuda:0", lanes=lanes)
        g2.reset(w["seed"], obs=False)
        g2.step_into(obs, rew, done, min(P, 50), mode=hase.PER_LAUNCH, maps=mp, state=st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g2.step_into(obs, rew, done, P, mode=hase.PER_LAUNCH, maps=mp, state=st)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_pl = e0.elapsed_time(e1)
        line["per_launch"] = dict(value=agents * P / (ms_pl / 1e3), ms_per_env_step=ms_pl / P,
                                  env_steps=P, unit="agent-steps/s")
        line["persistent_speedup"] = value / line["per_launch"]["value"]
        g2.close()

        # ---- external int8 actions resident in HBM (one run)
        acts = torch.randint(0, 5, (R, agents), dtype=torch.int8, device="cuda:0")
        g.prepare(obs, rew, done, R, actions=acts, maps=mp, state=st)
        g.step_into(obs, rew, done, R, actions=acts, maps=mp, state=st)
        ms = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            torch.cuda.synchronize()
            e0.record(stream)
            g.step_into(obs, rew, done, R, actions=acts, maps=mp, state=st)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        sp = spread(ms)
        ab = (R * out_bytes_per_step(specs, maps_on, actions=True, state=state_on) +
              state_bytes_per_launch(specs))
        line["int8_actions"] = dict(value=agents * R / (sp["median"] / 1e3), run_ms=sp,
                                    unit="agent-steps/s", alg_bytes_per_launch=ab,
                                    hbm_frac=ab / (sp["median"] / 1e3) / 1e9 / HBM_PEAK_GBS)
        del acts

        # ---- the same roofline against a copy measured on this GPU
        del obs, rew, done, mp, st
        torch.cuda.empty_cache()
        cbw = copy_bandwidth(torch)
        roof["copy_gbs"] = cbw
        roof["frac_of_copy"] = achieved / cbw
    line["roofline"] = roof
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(specs, w["seed"])
    g.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
