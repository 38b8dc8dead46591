"""rocprofv3 measurement of the step kernel, summarised into profiles/.

    python -m paper_2604_27162_amd.profiling --workload single16k --steps 10000

Runs (each as a child process of this one, which never touches the GPU):
  1. rocprofv3 --kernel-trace --stats over bench.py (per-kernel durations);
  2. rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, over bench.py;
  3. the same two counters over bench.py --copy-probe (a plain device copy
     of known size) to calibrate them: scale = true bytes / counted bytes.
Raw output goes to --raw (default rocprof_raw/profile_<workload>); the summary
(--summarize-only can redo it from raw output copied back from the GPU
machine) to profiles/step_kernel_<workload>.md and the HBM
traffic per launch to profiles/traffic.json, keyed by the hash of the device
sources so that bench.py reports it only while the kernel is unchanged.
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
    vals = [(float(r["Counter_Value"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            for r in rows if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter]
    return max(vals, key=lambda v: v[1])  # the longest dispatch


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--workload", default="single16k")
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--raw", default=None)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--collect-only", action="store_true", help="run rocprofv3 only")
    ap.add_argument("--summarize-only", action="store_true",
                    help="only summarise raw output collected earlier")
    args = ap.parse_args(argv)
    raw = os.path.abspath(args.raw or os.path.join(ROOT, "rocprof_raw", f"profile_{args.workload}"))
    os.makedirs(raw, exist_ok=True)
    os.makedirs(args.out, exist_ok=True)
    py = sys.executable
    bench = [py, os.path.join(ROOT, "bench.py"), "--workload", args.workload, "--steps",
             str(args.steps), "--warmup", "200", "--no-cpu-baseline", "--no-per-launch"]
    copy = [py, os.path.join(ROOT, "bench.py"), "--copy-probe", str(COPY_BYTES)]
    cmds = {
        "trace": ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv", "-d",
                  f"{raw}/trace", "-o", "run", "--"] + bench,
        "fetch": ["rocprofv3", "--pmc", "FETCH_SIZE", "--output-format", "csv", "-d",
                  f"{raw}/fetch", "-o", "run", "--"] + bench,
        "write": ["rocprofv3", "--pmc", "WRITE_SIZE", "--output-format", "csv", "-d",
                  f"{raw}/write", "-o", "run", "--"] + bench,
        "copy_fetch": ["rocprofv3", "--pmc", "FETCH_SIZE", "--output-format", "csv", "-d",
                       f"{raw}/copy_fetch", "-o", "run", "--"] + copy,
        "copy_write": ["rocprofv3", "--pmc", "WRITE_SIZE", "--output-format", "csv", "-d",
                       f"{raw}/copy_write", "-o", "run", "--"] + copy,
    }
    if not args.summarize_only:
        for name, cmd in cmds.items():
            _run(cmd, f"{raw}/{name}.log", timeout=240)
    if args.collect_only:
        return

    stats = _csv(f"{raw}/trace/*kernel_stats.csv")
    step_rows = [r for r in stats if "step_kernel" in r["Name"]]
    top = max(step_rows, key=lambda r: float(r["TotalDurationNs"]))
    trace = _csv(f"{raw}/trace/*kernel_trace.csv")
    durs = sorted((int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), r["Kernel_Name"])
                  for r in trace if "step_kernel" in r["Kernel_Name"])
    longest_ns, kname = durs[-1]
    fetch_kib, _ = _counter(_csv(f"{raw}/fetch/*counter_collection.csv"), "step_kernel", "FETCH_SIZE")
    write_kib, _ = _counter(_csv(f"{raw}/write/*counter_collection.csv"), "step_kernel", "WRITE_SIZE")
    cf_kib, _ = _counter(_csv(f"{raw}/copy_fetch/*counter_collection.csv"), "copyBuffer", "FETCH_SIZE")
    cw_kib, _ = _counter(_csv(f"{raw}/copy_write/*counter_collection.csv"), "copyBuffer", "WRITE_SIZE")
    sf = COPY_BYTES / (cf_kib * 1024.0)
    sw = COPY_BYTES / (cw_kib * 1024.0)
    traffic = fetch_kib * 1024.0 * sf + write_kib * 1024.0 * sw

    sys.path.insert(0, ROOT)
    import bench
    from paper_2604_27162_amd import workloads as wl
    specs = wl.workload_specs(args.workload)
    # bench.py writes the discovery maps of exploring workloads by default
    maps = any(s["flags"] & bench.EXPLORE for s in specs)
    alg = args.steps * bench.out_bytes_per_step(specs, maps) + bench.state_bytes_per_launch(specs)
    khash = bench.kernel_source_hash()

    tj = os.path.join(args.out, "traffic.json")
    d = json.load(open(tj)) if os.path.exists(tj) else {}
    d[args.workload] = {"kernel_hash": khash, "steps": args.steps, "hbm_bytes_per_launch": traffic,
                        "fetch_kib": fetch_kib, "write_kib": write_kib, "scale_fetch": sf,
                        "scale_write": sw, "alg_bytes_per_launch": alg, "kernel": kname,
                        "launch_ns": longest_ns}
    json.dump(d, open(tj, "w"), indent=1, sort_keys=True)

    md = os.path.join(args.out, f"step_kernel_{args.workload}.md")
    with open(md, "w") as f:
        f.write(f"# step kernel, workload {args.workload}, {args.steps} steps per launch\n\n")
        f.write(f"Device sources hash: `{khash}`\n\n## Commands (run from /tmp)\n\n")
        for name, cmd in cmds.items():
            rel = [c.replace(ROOT + "/", "") .replace(raw, "<raw>").replace(py, "python3") for c in cmd]
            f.write(f"- {name}: `{' '.join(rel)}`\n")
        f.write("\n## Kernel trace (--stats), step kernels\n\n")
        f.write("| kernel | calls | total ms | average us |\n|---|---|---|---|\n")
        for r in sorted(step_rows, key=lambda r: -float(r["TotalDurationNs"])):
            f.write(f"| `{r['Name'].split('(')[0]}` | {r['Calls']} | "
                    f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.3f} |\n")
        f.write(f"\nLongest dispatch (the {args.steps}-step persistent launch): "
                f"`{kname.split('(')[0]}` {longest_ns / 1e6:.3f} ms\n\n")
        f.write("## HBM traffic (--pmc, one pass per counter)\n\n")
        f.write(f"- copy probe ({COPY_BYTES} bytes read + written): FETCH_SIZE {cf_kib:.0f} KiB, "
                f"WRITE_SIZE {cw_kib:.0f} KiB -> scale fetch {sf:.4f}, write {sw:.4f}\n")
        f.write(f"- step kernel launch: FETCH_SIZE {fetch_kib:.1f} KiB, WRITE_SIZE "
                f"{write_kib:.1f} KiB\n")
        f.write(f"- scaled HBM bytes per launch: {traffic:.4e} "
                f"(algorithmic {alg:.4e}, ratio {traffic / alg:.4f})\n")
        f.write(f"- achieved (algorithmic bytes / longest dispatch): "
                f"{alg / (longest_ns * 1e-9) / 1e9:.1f} GB/s of 8000 GB/s\n")
    print(open(md).read())


if __name__ == "__main__":
    main()
