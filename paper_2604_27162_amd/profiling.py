"""rocprofv3 measurement of the step kernel, summarised into profiles/.

    python -m paper_2604_27162_amd.profiling --workload single16k

Runs (each as a child process of this one, which never touches the GPU),
every one over bench.py timing runs of the workload's configuration only
(--only-runs: no other launch of the step kernel):
  1. rocprofv3 --kernel-trace --stats (per-kernel durations: the step
     kernel's average is the average run);
  2. rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE (HBM traffic);
  3. rocprofv3 --pmc with eight SQ counters (waves, VALU / SALU / LDS /
     vector-store instructions, cycles waiting to issue, busy cycles, VALU
     active cycles), normalised per wave and per wave-step;
  4. FETCH_SIZE and WRITE_SIZE over bench.py --copy-probe (a plain device
     copy of known size) to calibrate them: scale = true bytes / counted.
Raw output goes to --raw (default rocprof_raw/profile_<workload>); the
summary (--summarize-only can redo it from raw output copied back from the
GPU machine) to profiles/step_kernel_<workload>.md and the HBM traffic per
launch to profiles/traffic.json, keyed by the hash of the device sources so
that bench.py reports it only while the kernel is unchanged.

With --per-launch, one kernel trace of bench.py --only-per-launch (one
launch per env-step) instead, summarised to
profiles/step_kernel_<workload>_per_launch.md: kernel time per launch
against the gaps between launches. With --int8, the same passes over runs
with external int8 actions (bench.py --int8-actions), summarised to
profiles/step_kernel_<workload>_int8.md and keyed <workload>_int8 in
traffic.json.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 4 << 30
SQ = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_WR",
      "SQ_WAIT_INST_ANY", "SQ_BUSY_CYCLES", "SQ_ACTIVE_INST_VALU"]


def _run(cmd, log, timeout):
    print("$ " + " ".join(cmd), flush=True)
    with open(log, "w") as f:
        subprocess.run(cmd, stdout=f, stderr=subprocess.STDOUT, timeout=timeout, check=True,
                       cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"))


def _csv(path_glob):
    files = glob.glob(path_glob)
    if not files:
        raise FileNotFoundError(path_glob)
    return list(csv.DictReader(open(files[0])))


def _counter(rows, name_part, counter):
    """Value of one counter for the longest dispatch of a kernel (the
    counter rows of one dispatch are summed over their instances)."""
    per = {}
    for r in rows:
        if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter:
            d = (r.get("Dispatch_Id") or r.get("Correlation_Id"),
                 int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) if "End_Timestamp" in r else 0)
            per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    (_, dur), val = max(per.items(), key=lambda kv: (kv[0][1], kv[1]))
    return val, dur


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--workload", default="single16k")
    ap.add_argument("--raw", default=None)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--collect-only", action="store_true", help="run rocprofv3 only")
    ap.add_argument("--summarize-only", action="store_true",
                    help="only summarise raw output collected earlier")
    ap.add_argument("--int8", action="store_true",
                    help="profile runs with external int8 actions resident in HBM")
    ap.add_argument("--per-launch", action="store_true",
                    help="profile the run with one kernel launch per env-step instead "
                         "(kernel trace only)")
    args = ap.parse_args(argv)
    if args.per_launch:
        return per_launch(args)
    tag = args.workload + ("_int8" if args.int8 else "")
    raw = os.path.abspath(args.raw or os.path.join(ROOT, "rocprof_raw", f"profile_{tag}"))
    os.makedirs(raw, exist_ok=True)
    os.makedirs(args.out, exist_ok=True)
    py = sys.executable
    bench = [py, os.path.join(ROOT, "bench.py"), "--workload", args.workload, "--only-runs",
             "--no-cpu-baseline"] + (["--int8-actions"] if args.int8 else [])
    timed = bench + ["--steps", "5", "--warmup", "1"]
    one = bench + ["--steps", "1", "--warmup", "0"]
    copy = [py, os.path.join(ROOT, "bench.py"), "--copy-probe", str(COPY_BYTES)]

    def pmc(name, counters, prog):
        return ["rocprofv3", "--pmc", *counters, "--output-format", "csv", "-d", f"{raw}/{name}",
                "-o", "run", "--"] + prog

    cmds = {
        "trace": ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv", "-d",
                  f"{raw}/trace", "-o", "run", "--"] + timed,
        "fetch": pmc("fetch", ["FETCH_SIZE"], one),
        "write": pmc("write", ["WRITE_SIZE"], one),
        "sq": pmc("sq", SQ, one),
        "copy_fetch": pmc("copy_fetch", ["FETCH_SIZE"], copy),
        "copy_write": pmc("copy_write", ["WRITE_SIZE"], copy),
    }
    if not args.summarize_only:
        for name, cmd in cmds.items():
            _run(cmd, f"{raw}/{name}.log", timeout=170)
    if args.collect_only:
        return

    stats = _csv(f"{raw}/trace/*kernel_stats.csv")
    step_rows = [r for r in stats if "step_kernel" in r["Name"]]
    top = max(step_rows, key=lambda r: float(r["TotalDurationNs"]))
    kname = top["Name"]
    # the timed runs: every dispatch of the dominant kernel after the warm-up run
    disp = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                  for r in _csv(f"{raw}/trace/*kernel_trace.csv") if r["Kernel_Name"] == kname)
    timed_ns = [d for _, d in disp[1:]] or [d for _, d in disp]
    avg_ns = sum(timed_ns) / len(timed_ns)
    fetch_kib, _ = _counter(_csv(f"{raw}/fetch/*counter_collection.csv"), "step_kernel", "FETCH_SIZE")
    write_kib, _ = _counter(_csv(f"{raw}/write/*counter_collection.csv"), "step_kernel", "WRITE_SIZE")
    cf_kib, _ = _counter(_csv(f"{raw}/copy_fetch/*counter_collection.csv"), "copyBuffer", "FETCH_SIZE")
    cw_kib, _ = _counter(_csv(f"{raw}/copy_write/*counter_collection.csv"), "copyBuffer", "WRITE_SIZE")
    sf = COPY_BYTES / (cf_kib * 1024.0)
    sw = COPY_BYTES / (cw_kib * 1024.0)
    traffic = fetch_kib * 1024.0 * sf + write_kib * 1024.0 * sw
    sq_rows = _csv(f"{raw}/sq/*counter_collection.csv")
    sq = {c: _counter(sq_rows, "step_kernel", c)[0] for c in SQ}

    sys.path.insert(0, ROOT)
    import bench
    from paper_2604_27162_amd import workloads as wl
    specs = wl.workload_specs(args.workload)
    steps = wl.WORKLOADS[args.workload]["steps"]
    maps = any(s["flags"] & bench.EXPLORE for s in specs)
    # bench.py writes the discovery maps and the true state of exploring
    # workloads by default
    alg = (steps * bench.out_bytes_per_step(specs, maps, actions=args.int8, state=maps) +
           bench.state_bytes_per_launch(specs))
    khash = bench.kernel_source_hash()
    waves = sq["SQ_WAVES"] or 1.0

    tj = os.path.join(args.out, "traffic.json")
    d = json.load(open(tj)) if os.path.exists(tj) else {}
    d[tag] = {"kernel_hash": khash, "steps": steps, "hbm_bytes_per_launch": traffic,
              "fetch_kib": fetch_kib, "write_kib": write_kib, "scale_fetch": sf,
              "scale_write": sw, "alg_bytes_per_launch": alg, "kernel": kname,
              "launch_ns_avg": avg_ns, "sq": sq}
    json.dump(d, open(tj, "w"), indent=1, sort_keys=True)

    md = os.path.join(args.out, f"step_kernel_{tag}.md")
    with open(md, "w") as f:
        f.write(f"# step kernel, workload {args.workload}, {steps} steps per launch"
                f"{', external int8 actions' if args.int8 else ''}\n\n")
        f.write(f"Device sources hash: `{khash}`\n\n## Commands (run from /tmp)\n\n")
        for name, cmd in cmds.items():
            rel = [c.replace(ROOT + "/", "").replace(raw, "<raw>").replace(py, "python3")
                   for c in cmd]
            f.write(f"- {name}: `{' '.join(rel)}`\n")
        f.write("\n## Kernel trace (--stats): every dispatch of the step kernel is one run\n\n")
        f.write("| kernel | calls | total ms | average us | min us | max us |\n"
                "|---|---|---|---|---|---|\n")
        for r in sorted(step_rows, key=lambda r: -float(r["TotalDurationNs"])):
            f.write(f"| `{r['Name'].split('(')[0]}` | {r['Calls']} | "
                    f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.3f} | "
                    f"{float(r['MinNs']) / 1e3:.3f} | {float(r['MaxNs']) / 1e3:.3f} |\n")
        f.write(f"\nTimed runs (every dispatch after the warm-up run): {len(timed_ns)}, "
                f"average {avg_ns / 1e3:.3f} us, min {min(timed_ns) / 1e3:.3f} us, "
                f"max {max(timed_ns) / 1e3:.3f} us\n")
        f.write("\n## HBM traffic (--pmc, one pass per counter, one run)\n\n")
        f.write(f"- copy probe ({COPY_BYTES} bytes read + written): FETCH_SIZE {cf_kib:.0f} KiB, "
                f"WRITE_SIZE {cw_kib:.0f} KiB -> scale fetch {sf:.4f}, write {sw:.4f}\n")
        f.write(f"- step kernel run: FETCH_SIZE {fetch_kib:.1f} KiB, WRITE_SIZE "
                f"{write_kib:.1f} KiB\n")
        f.write(f"- scaled HBM bytes per run: {traffic:.4e} "
                f"(algorithmic {alg:.4e}, ratio {traffic / alg:.4f})\n")
        f.write(f"- achieved (algorithmic bytes / average timed run): "
                f"{alg / (avg_ns * 1e-9) / 1e9:.1f} GB/s of 8000 GB/s\n")
        f.write("\n## SQ counters (--pmc, one pass, one run)\n\n")
        f.write("| counter | total | per wave | per wave-step |\n|---|---|---|---|\n")
        for c in SQ:
            f.write(f"| {c} | {sq[c]:.4e} | {sq[c] / waves:.1f} | {sq[c] / waves / steps:.2f} |\n")
    print(open(md).read())


def per_launch(args):
    """Kernel trace of bench.py --only-per-launch: how the time of one env-step
    launched on its own splits into kernel time and the gaps between
    launches. Written to profiles/step_kernel_<workload>_per_launch.md."""
    raw = os.path.abspath(args.raw or os.path.join(ROOT, "rocprof_raw", f"per_launch_{args.workload}"))
    os.makedirs(raw, exist_ok=True)
    os.makedirs(args.out, exist_ok=True)
    py = sys.executable
    cmd = ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv", "-d", f"{raw}/trace",
           "-o", "run", "--", py, os.path.join(ROOT, "bench.py"), "--workload", args.workload,
           "--only-per-launch", "--no-cpu-baseline"]
    log = f"{raw}/trace.log"
    if not args.summarize_only:
        _run(cmd, log, timeout=170)
    timed = None
    for line in open(log):
        if line.startswith("{") and "ms_per_env_step" in line:
            timed = json.loads(line)
    disp = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                  for r in _csv(f"{raw}/trace/*kernel_trace.csv") if "step_kernel" in r["Kernel_Name"])
    # the timed launches are the last P dispatches
    P = timed["per_launch_env_steps"] if timed else len(disp)
    disp = disp[-P:]
    dur = sorted(e - b for b, e in disp)
    gaps = sorted(disp[i + 1][0] - disp[i][1] for i in range(len(disp) - 1))
    med = lambda v: v[len(v) // 2] if v else 0.0
    sys.path.insert(0, ROOT)
    import bench
    khash = bench.kernel_source_hash()
    span_us = (disp[-1][1] - disp[0][0]) / 1e3 / len(disp) if disp else 0.0
    md = os.path.join(args.out, f"step_kernel_{args.workload}_per_launch.md")
    with open(md, "w") as f:
        f.write(f"# step kernel, workload {args.workload}, one launch per env-step\n\n")
        f.write(f"Device sources hash: `{khash}`\n\n")
        rel = [c.replace(ROOT + "/", "").replace(raw, "<raw>").replace(py, "python3") for c in cmd]
        f.write(f"Command (run from /tmp): `{' '.join(rel)}`\n\n")
        f.write(f"- timed launches: {len(disp)} (after a 50-launch warm-up)\n")
        f.write(f"- kernel duration per launch: median {med(dur) / 1e3:.3f} us, min "
                f"{dur[0] / 1e3:.3f} us, max {dur[-1] / 1e3:.3f} us\n")
        f.write(f"- gap between consecutive launches: median {med(gaps) / 1e3:.3f} us, min "
                f"{gaps[0] / 1e3:.3f} us\n")
        f.write(f"- first start to last end per launch: {span_us:.3f} us\n")
        if timed:
            f.write(f"- bench.py's timed figure (events around the {P} launches): "
                    f"{timed['ms_per_env_step'] * 1e3:.3f} us per env-step\n")
    print(open(md).read())


if __name__ == "__main__":
    main()
