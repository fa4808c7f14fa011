"""Throughput of the GPU-resident fork-join runtime on one MI355X.

One step = one persistent launch (gtap_run) over the thread-mode
microbenchmark batch: fib(32) with a task at every call, N-Queens n=13 with one
task per legal column, and an unbalanced tree search (geometric branching of
mean 4, depth limit 13, seed 1) -- three roots of very uneven size sharing one
launch.  `value` is tasks per second over the timed steps (wall clock between
synchronizations, inputs already on the device).  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tasks/s & k-cliques/s at 1 GPU; batched jobs/s + p99 latency vs plain"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes the runtime must move per event (see the roofline section
# of the design notes): a task's frame is written once at spawn (48 B of
# header and payload) and read once when it first runs (48 B); a completion
# adds to the parent's accumulator and decrements its join counter (8 B + 4 B);
# a fork stores the join count and clears the accumulator (12 B) and its
# re-execution reads header and accumulator (24 B); a task ID published to a
# deque is written and later read once (8 B).
BYTES_SPAWN = 48
BYTES_TASK_READ = 48
BYTES_COMPLETION = 12
BYTES_FORK = 12
BYTES_CONT_READ = 24
BYTES_PUSHED = 8


def algorithmic_bytes(st: dict) -> int:
    return (BYTES_SPAWN * st["spawns"] + (BYTES_TASK_READ + BYTES_COMPLETION) * st["tasks"]
            + (BYTES_FORK + BYTES_CONT_READ) * st["conts"] + BYTES_PUSHED * st["pushed"])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "thread_sched_kernel_microbench_traffic.txt")


def kernel_source_sha() -> str:
    """Hash of the HIP sources the scheduler kernel is built from."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_2604_05982_amd", "csrc", "*"))):
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha") != kernel_source_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(nbytes: int, reps: int = 3) -> None:
    """A plain device copy of known size (calibrates FETCH_SIZE/WRITE_SIZE)."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "reps": reps}), flush=True)


def workload_jobs(rt, gtap):
    thr = gtap.uts_threshold(4)
    return [rt.submit_fib(32), rt.submit_nqueens(13), rt.submit_uts(1, thr, 13)]


def cpu_baseline(min_seconds: float = 10.0, max_seconds: float = 30.0) -> dict:
    """The sequential oracle on one host core over the same three roots."""
    import oracle
    thr = oracle.uts_threshold(4)
    reps, tasks = 0, 0
    t0 = time.perf_counter()
    while True:
        for r in (oracle.fib(32), oracle.nqueens(13), oracle.uts(1, thr, 13)):
            tasks += r.tasks
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or el * (reps + 1) / reps > max_seconds:
            break
    return {"value": tasks / el, "unit": "tasks/s", "cores": 1, "kind": "oracle",
            "sample": f"full workload (fib(32) + N-Queens(13) + UTS depth 13) x{reps}, "
                      f"{el:.1f} s on one host thread"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--waves-per-group", type=int, default=4)
    ap.add_argument("--num-waves", type=int, default=1024)
    ap.add_argument("--steal-below", type=int, default=64)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="run only a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return 0
    from paper_2604_05982_amd import gtap

    rt = gtap.Runtime(waves_per_group=args.waves_per_group, num_waves=args.num_waves,
                      steal_below=args.steal_below, small_frames=1 << 25, timeout_ms=60000)
    expect = (2178309, 73712, 102971195)
    for _ in range(args.warmup):
        jobs = workload_jobs(rt, gtap)
        rt.run()
        got = tuple(rt.result(j) for j in jobs)
        if got != expect:
            raise SystemExit(f"wrong results {got}, expected {expect}")
    torch.cuda.synchronize()
    tot = {}
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        jobs = workload_jobs(rt, gtap)
        rt.run()
        st = rt.stats()
        kernel_ms.append(st["kernel_ms"])
        for k, v in st.items():
            if isinstance(v, int):
                tot[k] = tot.get(k, 0) + v
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    got = tuple(rt.result(j) for j in jobs)
    if got != expect:
        raise SystemExit(f"wrong results {got}, expected {expect}")

    tasks = tot["tasks"]
    ms_step = 1000.0 * el / args.steps
    mean_kernel_ms = sum(kernel_ms) / len(kernel_ms)
    alg_bytes_launch = algorithmic_bytes(tot) / args.steps
    achieved = alg_bytes_launch / (mean_kernel_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": tasks / el,
        "unit": "tasks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "thread-mode microbenchmarks in one persistent launch: fib(32), "
                        "N-Queens(13), UTS(mean 4, depth 13, seed 1)",
            "mode": "thread", "queues": 1, "waves": st["num_waves"],
            "waves_per_group": st["waves_per_group"], "steal_below": args.steal_below,
        },
        "tasks_per_step": tasks // args.steps,
        "executions_per_s": (tasks + tot["conts"]) / el,
        "kernel_ms": mean_kernel_ms,
        "kernel_tasks_per_s": tasks / args.steps / (mean_kernel_ms * 1e-3),
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "kernel": "thread_sched_kernel",
            "algorithmic_bytes_per_launch": alg_bytes_launch,
        },
        "runtime_counters_per_step": {k: v // args.steps for k, v in tot.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    rt.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
