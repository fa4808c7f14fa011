"""Throughput of the GPU-resident fork-join runtime on one MI355X.

Default (the combined run): prints ONE JSON line.  Its headline is the
batched job mix -- 20,000 jobs (60 % k-clique counting on induced subgraphs of
a seeded n=10^6 Chung-Lu graph, 40 % unbalanced tree search, trace seed 5) run
by one persistent launch per step; `value` is jobs per second over the K timed
steps (wall clock between synchronizations, inputs already on the device),
every step's 20,000 results compared with the oracle's stored results.  The
same line carries the served open loop (p50/p99 against one launch per job),
the autotuner's choice against the default configuration, and sub-records
for the other configurations under "configs":
  C0  4-cliques of a 2,000-vertex Chung-Lu graph (thread mode, one queue)
  C1  fib(32), N-Queens(13), UTS(mean 4, depth 13) in one launch and alone
  C2  block-mode FMM on 10^6 Plummer points (P2P interactions/s, M2L pairs/s)
  C3  7-cliques of the 10^6-vertex graph, 4 DAQ queues against one, and the
      split search with bitset candidate subgraphs
Every record carries a `roofline` for its dominant kernel and a `cpu_baseline`
(the oracle on one host thread over a bounded sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --workload c0|c1|c2|c3|c4   (one configuration alone)
       python bench.py --workload kclique7|serving|fmm|schedulers|fmm_dtt|cilksort|microbench
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

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "thread_sched_kernel_hbm_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "thread_sched_kernel_kclique7_valu_daq.txt")


# The HIP sources each scheduler kernel is compiled from (the block-mode
# kernel includes the thread-mode headers; the thread-mode kernel does not
# include the block-mode one).
THREAD_KERNEL_SOURCES = ("layout.h", "wave.h", "tasks.h", "kclique_bits.h", "sched_thread.h", "fmm.h", "fmm_lists.h")
BLOCK_KERNEL_SOURCES = THREAD_KERNEL_SOURCES + ("sched_block.h",)


def kernel_source_sha(files=THREAD_KERNEL_SOURCES) -> str:
    """Hash of the HIP sources a scheduler kernel is built from."""
    h = hashlib.sha256()
    for name in sorted(files):
        with open(os.path.join(ROOT, "paper_2604_05982_amd", "csrc", name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_values(path: str) -> dict:
    """key: value lines of a committed profile summary, {} when it is missing
    or was taken from other kernel sources than these."""
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    return vals if vals.get("source_sha") == kernel_source_sha() else {}


def measured_traffic(key: str):
    """HBM bytes per launch of workload `key` from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary (copy-calibrated), or None when the kernel
    sources changed since it was taken or the workload was not profiled."""
    try:
        return float(_profile_values(TRAFFIC_FILE)[f"{key}.hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_valu() -> dict:
    """VALU lane utilisation (percent) of the 7-clique launches from the
    committed rocprofv3 counter summary, or {} when it is stale."""
    vals = _profile_values(VALU_FILE)
    return {k: float(v) for k, v in vals.items() if k.endswith("lane_utilisation_pct")}


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


def kclique_cpu_baseline(g, args, stride: int = 4) -> dict:
    """The oracle on one host thread over the 7-cliques whose lowest vertex is
    0 mod `stride` (a vertex sample of the same graph, 10-30 s)."""
    import oracle
    alg = "pivot" if args.kclique_split == "pivot" else "orient"
    thr = args.split_threshold if args.kclique_split != "none" else 64
    t0 = time.perf_counter()
    r = oracle.kclique_split_roots(g.row_ptr, g.col, 7, stride, 0, threshold=thr, algorithm=alg)
    el = time.perf_counter() - t0
    return {"value": r.value / el, "unit": "k-cliques/s", "cores": 1, "kind": "oracle",
            "sample": f"the {r.value} 7-cliques whose lowest vertex is 0 mod {stride} ({alg}, threshold {thr}), "
                      f"{el:.1f} s on one host thread"}


def bench_kclique7(args, gtap) -> int:
    """7-cliques of the seeded n=10^6, mean degree 40, exponent 2.1 Chung-Lu graph
    (thread mode; DAQ with 4 candidate-size buckets when --queues 4)."""
    import torch
    from synth import graphs
    g = graphs.chung_lu(1000000, 40, 2.1, 0.6, 2)
    want = None
    with open(os.path.join(ROOT, "tests", "golden", "kclique_chung_lu.txt")) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 6 and f[0] == "n1000000_d40_g2.1_cap0.6_s2" and f[2] == "7":
                want = (f[1], int(f[3]))
    opts = dict(num_waves=args.num_waves, waves_per_group=args.waves_per_group, deque_capacity=1 << 17,
                small_frames=1 << 25, big_frames=1 << 23, big_frame_ints=max(320, g.max_outdeg),
                timeout_ms=60000, steal_below=args.steal_below)
    split = args.kclique_split != "none"
    if args.queues > 1:
        opts.update(num_queues=args.queues, daq_policy=2,
                    daq_bounds=[int(b) for b in args.daq_bounds.split(",")][: args.queues - 1],
                    deque_capacity=1 << 19, big_frames=1 << 24)
    if split:  # node-state frames for heavy edges and the nodes that split
        opts.update(waves_per_group=4, big_frames=1 << 23,
                    big_frame_ints=gtap.kclique_split_buffer_ints(g.max_outdeg))
    rt = gtap.Runtime(**opts)
    rp = torch.as_tensor(g.row_ptr32).cuda()
    col = torch.as_tensor(g.col).cuda()
    alg = gtap.GTAP_KCLIQUE_PIVOT if args.kclique_split == "pivot" else gtap.GTAP_KCLIQUE_ORIENT

    def submit():
        if split:
            return rt.submit_kclique_split(rp, col, 7, threshold=args.split_threshold, algorithm=alg,
                                           max_outdeg=g.max_outdeg)
        return rt.submit_kclique(rp, col, 7, max_outdeg=g.max_outdeg)

    for _ in range(args.warmup):
        j = submit()
        rt.run()
    torch.cuda.synchronize()
    tot, kms, counts = {}, [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        j = submit()
        rt.run()
        st = rt.stats()
        kms.append(st["kernel_ms"])
        counts.append(rt.result(j))
        for k, v in st.items():
            if isinstance(v, int):
                tot[k] = tot.get(k, 0) + v
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    count = counts[-1]
    ok = want is not None and all(want == (g.checksum(), c) for c in counts)
    out = {"metric": METRIC, "value": count * args.steps / el, "unit": "k-cliques/s",
           "tasks_per_s": tot["tasks"] / el, "kernel_ms": sum(kms) / len(kms), "count": count,
           "matches_oracle": ok, "queues": args.queues, "waves": st["num_waves"],
           "search": ({"algorithm": args.kclique_split, "split_threshold": args.split_threshold}
                      if split else {"algorithm": "orientation, one task per candidate"}),
           "steps": args.steps, "warmup": args.warmup, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "7-cliques, Chung-Lu n=1e6, mean degree 40, exponent 2.1, cap 0.6, seed 2",
                      "graph_edges": g.m_undirected, "max_outdeg": g.max_outdeg},
           "cpu_baseline": None if args.no_cpu_baseline else kclique_cpu_baseline(g, args),
           "runtime_counters_per_step": {k: v // args.steps for k, v in tot.items()}}
    rt.close()
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def _latency_summary(res, arrivals, classes) -> dict:
    """p50/p99 of host-observed completion minus scheduled arrival (ms)."""
    lat = [1e3 * (r.done_s - a) for r, a in zip(res, arrivals)]
    out = {"p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "max_ms": max(lat) if lat else None}
    for c in sorted(set(classes)):
        lc = [x for x, cc in zip(lat, classes) if cc == c]
        out[c] = {"p50_ms": _pct(lc, 50), "p99_ms": _pct(lc, 99), "jobs": len(lc)}
    return out


def serving_trace(gtap, rt, g, n_jobs, seed, torch):
    """The batched/serving job mix: k-clique jobs on induced subgraphs of g
    (their CSR staged on the device up front) and UTS jobs."""
    import numpy as np
    from synth import graphs, serving
    specs = serving.serving_mix(n_jobs, seed)
    kc = [sp for sp in specs if sp.kind == "kclique"]
    subs = graphs.induced_many(g, [(sp.s, sp.sub_seed) for sp in kc], threads=min(16, os.cpu_count() or 1))
    rp_off = np.cumsum([0] + [h.n + 1 for h in subs])
    col_off = np.cumsum([0] + [h.col.size for h in subs])
    rp_dev = torch.as_tensor(np.concatenate([h.row_ptr.astype(np.int32) for h in subs] or
                                            [np.zeros(1, np.int32)])).cuda()
    col_dev = torch.as_tensor(np.concatenate([h.col for h in subs] + [np.zeros(1, np.int32)])).cuda()
    entries, classes, it = [], [], 0
    for sp in specs:
        if sp.kind == "kclique":
            h = subs[it]
            a = gtap.gtap_kclique_args(rp_dev.data_ptr() + 4 * int(rp_off[it]),
                                       col_dev.data_ptr() + 4 * int(col_off[it]), h.n, sp.k, 64, h.max_outdeg)
            entries.append((gtap.GTAP_KIND_KCLIQUE, a))
            classes.append("kclique")
            it += 1
        else:
            entries.append(gtap.Runtime.uts_args(sp.seed, gtap.uts_threshold(sp.m), sp.depth))
            classes.append("uts")
    staged = {"kclique_jobs": len(kc), "uts_jobs": len(specs) - len(kc),
              "staged_csr_bytes": int(4 * (rp_dev.numel() + col_dev.numel())),
              "subgraph_vertices": int(sum(h.n for h in subs)), "subgraph_edges": int(col_off[-1])}
    return specs, entries, classes, (rp_dev, col_dev), subs, staged


def bench_serving(args, gtap) -> int:
    """Batched and served job mixes against one launch per job (plain)."""
    import numpy as np
    import torch
    from synth import graphs, serving
    say = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    g = graphs.chung_lu(1000000, 40, 2.1, 0.6, 2)
    say(f"graph ready {time.perf_counter() - t0:.1f}s max_outdeg={g.max_outdeg}")
    common = dict(max_jobs=1 << 15, big_frame_ints=max(320, g.max_outdeg), deque_capacity=1 << 18,
                  timeout_ms=300000)
    base = gtap.Runtime(num_waves=args.num_waves, waves_per_group=args.waves_per_group, small_frames=1 << 26,
                        big_frames=1 << 22, **common)
    # calibration trace (its own seed): the autotuner's jobs and the open-loop rate
    _, cal_entries, _, cal_keep, _, _ = serving_trace(gtap, base, g, max(1, args.jobs // 4), 6, torch)
    tune_jobs = base.trace([(0.0, e) for e in cal_entries[: args.calib_jobs]])
    space = gtap.tune_space(num_queues=(1, 2, 4), waves_per_group=(4,), num_waves=(1024, 0),
                            daq_policy=gtap.GTAP_DAQ_BY_KIND, repeats=1)
    tuned, tune_rep = base.autotune(tune_jobs, space)
    base.close()
    say(f"autotuned {tuned} {tune_rep}")
    rt = gtap.Runtime(**tuned, **common)
    headroom = int(tuned["small_frames"]) // 4
    specs, entries, classes, keep, subs, staged = serving_trace(gtap, rt, g, args.jobs, 5, torch)
    n = len(entries)
    say(f"trace ready {time.perf_counter() - t0:.1f}s {staged}")

    def served(arrivals):
        jobs = rt.trace([(t, e) for t, e in zip(arrivals, entries)])
        rt.serve_start(max_inflight=args.inflight, headroom_small=headroom)
        res = rt.trace_run(jobs, timeout_ms=280000)
        rt.serve_stop()
        return res, rt.stats()

    # (i) saturated: every job at t = 0
    zeros = np.zeros(n)
    tb = time.perf_counter()
    ids = []
    for kind, a in entries:
        ids.append(gtap.gtap_submit(rt.ctx, kind, a))
    rt.run()
    batch_s = time.perf_counter() - tb
    res_batch = [rt.result(j) for j in ids]
    st_batch = rt.stats()
    say(f"batch launch {batch_s:.2f}s")
    res_sat, st_sat = served(zeros)
    served_s = max(r.done_s for r in res_sat)
    say(f"served saturated {served_s:.2f}s")
    plain_sat = rt.trace_run_plain(rt.trace([(0.0, e) for e in entries]))
    plain_s = max(r.done_s for r in plain_sat)
    say(f"plain saturated {plain_s:.2f}s")
    r_b, r_s, r_p = res_batch, [r.result for r in res_sat], [r.result for r in plain_sat]
    alone_eq_mix = r_b == r_p and r_s == r_p

    # calibration on another trace seed: saturated served throughput
    cal_jobs = rt.trace([(0.0, e) for e in cal_entries])
    rt.serve_start(max_inflight=args.inflight, headroom_small=headroom)
    cal_res = rt.trace_run(cal_jobs, timeout_ms=280000)
    rt.serve_stop()
    cal_rate = len(cal_entries) / max(r.done_s for r in cal_res)
    del cal_keep
    say(f"calibrated saturated rate {cal_rate:.1f} jobs/s")

    # (ii) open loop at 0.8 x the calibrated saturated rate (and a sweep)
    rhos = [0.8] + ([0.3, 0.5, 0.7, 0.9] if args.sweep else [])
    open_loop = {}
    for rho in rhos:
        arr = serving.poisson_arrivals(n, rho * cal_rate, 55)
        res_o, _ = served(arr)
        ok = [r.result for r in res_o] == r_p
        entry = {"rate_jobs_per_s": rho * cal_rate, "served": _latency_summary(res_o, arr, classes),
                 "served_exact": ok}
        alone_eq_mix = alone_eq_mix and ok
        if rho == 0.8:
            res_po = rt.trace_run_plain(rt.trace([(t, e) for t, e in zip(arr, entries)]))
            entry["plain"] = _latency_summary(res_po, arr, classes)
            alone_eq_mix = alone_eq_mix and [r.result for r in res_po] == r_p
        open_loop[f"rho_{rho}"] = entry
        say(f"open loop rho={rho}: {json.dumps(entry)[:300]}")

    out = {"metric": METRIC, "value": n / batch_s, "unit": "jobs/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic",
           "config": {"workload": f"{n} jobs, trace seed 5: 60% k-clique (k 4..8, induced subgraphs of "
                                  "log-uniform 1e3..2e5 vertices of the n=1e6 Chung-Lu graph), 40% UTS "
                                  "(m 2..4, depth 8..14)", **staged, "max_inflight": args.inflight,
                      "waves": st_batch["num_waves"], "autotuned": tuned, "autotune_report": tune_rep},
           "saturated_jobs_per_s": {"batch_launch": n / batch_s, "served": n / served_s, "plain": n / plain_s},
           "saturated_tasks_per_s_batch": st_batch["tasks"] / batch_s,
           "batch_kernel_ms": st_batch["kernel_ms"], "tasks_total": st_batch["tasks"],
           "open_loop": open_loop, "all_results_equal_alone_vs_mix": alone_eq_mix,
           "served_admitted": st_sat["admitted"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = serving_cpu_baseline(specs, subs, res_batch)
        alone_eq_mix = alone_eq_mix and out["cpu_baseline"]["sample_matches"]
    del keep
    rt.close()
    print(json.dumps(out), flush=True)
    return 0 if alone_eq_mix else 1


def serving_cpu_baseline(specs, subs, gpu_results, budget_s: float = 15.0) -> dict:
    """The oracle over the trace's jobs in order, smallest first, until the
    time budget: jobs/s on one host core, and the sampled results checked."""
    import oracle
    order = []
    it = 0
    for i, sp in enumerate(specs):
        if sp.kind == "kclique":
            order.append((subs[it].col.size, i, it))
            it += 1
        else:
            order.append((sp.m ** sp.depth, i, -1))
    order.sort()
    done, match = 0, True
    t0 = time.perf_counter()
    for _, i, it in order:
        sp = specs[i]
        if sp.kind == "kclique":
            h = subs[it]
            v = oracle.kclique(h.row_ptr, h.col, sp.k).value
        else:
            v = oracle.uts(sp.seed, oracle.uts_threshold(sp.m), sp.depth).value
        match = match and v == gpu_results[i]
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "jobs/s", "cores": 1, "kind": "oracle",
            "sample": f"the {done} smallest of {len(specs)} trace jobs, {el:.1f} s on one host thread "
                      "(a lower bound on the oracle's time for the whole trace)",
            "sample_matches": match}


def bench_fmm(args, gtap) -> int:
    """3D Laplace FMM on 10^6 Plummer points (leaf 64, theta 1/2, order 6).
    --fmm-traversal tasks (default): block-mode traversal tasks with M2L and
    cooperative P2P inside; lists / worklist: the traversal builds M2L and
    P2P lists (thread-mode tasks or the level-synchronous worklist) that sorted
    data-parallel kernels evaluate.  value = P2P interactions per second of the
    interaction phase (traversal, plus sort and list evaluation for lists)."""
    import numpy as np
    import torch
    from synth import points
    n = args.fmm_points
    x, y, z, q = points.plummer(n, 3)
    tx, ty, tz, tq = (torch.as_tensor(a).cuda() for a in (x, y, z, q))
    phi = torch.zeros_like(tx)
    trav = {"tasks": gtap.GTAP_FMM_TASKS, "lists": gtap.GTAP_FMM_LISTS,
            "worklist": gtap.GTAP_FMM_WORKLIST}[args.fmm_traversal]
    if trav == gtap.GTAP_FMM_TASKS:
        rt = gtap.Runtime(mode=gtap.GTAP_MODE_BLOCK, waves_per_group=args.fmm_wpg, small_frames=1 << 24,
                          big_frames=0, timeout_ms=120000,
                          num_waves=args.num_waves if args.num_waves != 1024 else 0)
    else:
        rt = gtap.Runtime(mode=gtap.GTAP_MODE_THREAD, waves_per_group=4, small_frames=1 << 24,
                          big_frames=1 << 10, timeout_ms=120000)
    for _ in range(args.warmup):
        rt.submit_fmm(tx, ty, tz, tq, phi, traversal=trav)
        rt.run()
    torch.cuda.synchronize()
    res, wall = [], []
    for _ in range(args.steps):
        phi.zero_()
        t0 = time.perf_counter()
        j = rt.submit_fmm(tx, ty, tz, tq, phi, traversal=trav)
        rt.run()
        wall.append(time.perf_counter() - t0)
        res.append(rt.fmm_result(j))
    st = rt.stats()
    rt.close()
    med = sorted(range(len(wall)), key=lambda i: wall[i])[len(wall) // 2]
    r = res[med]
    inter_ms = r["traversal_ms"] + r["sort_ms"] + r["m2l_ms"] + r["p2p_ms"]
    trav_s = inter_ms * 1e-3
    e2e = wall[med]
    mode = "block mode, work inside the tasks" if trav == gtap.GTAP_FMM_TASKS else \
        ("thread-mode list-building tasks + list kernels" if trav == gtap.GTAP_FMM_LISTS
         else "level-synchronous worklist + list kernels")
    out = {"metric": METRIC, "value": r["p2p_interactions"] / trav_s, "unit": "P2P interactions/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"FMM dual-tree traversal ({mode}): {n} Plummer points (seed 3), "
                                  "leaf 64, theta 1/2, Cartesian order 6", "waves": st["num_waves"],
                      "waves_per_group": st["waves_per_group"]},
           "interaction_phase_ms": inter_ms,
           "m2l_pairs_per_s": r["m2l_pairs"] / trav_s,
           "traversal_tasks_per_s": st["tasks"] / (r["traversal_ms"] * 1e-3),
           "end_to_end_ms_median": 1e3 * e2e, "end_to_end_ms_min": 1e3 * min(wall),
           "end_to_end_ms_max": 1e3 * max(wall),
           "phase_ms": {k: r[k] for k in ("tree_ms", "upward_ms", "traversal_ms", "sort_ms", "m2l_ms", "p2p_ms",
                                          "downward_ms")},
           "lists": {k: r[k] for k in ("n_cells", "n_leaves", "max_level", "m2l_pairs", "p2p_pairs",
                                       "p2p_interactions", "coincident")},
           "traversal_tasks": st["tasks"], "traversal_conts": st["conts"]}
    if not args.no_cpu_baseline:
        import oracle
        tg = np.random.default_rng(17).choice(n, 256, replace=False)
        t0 = time.perf_counter()
        w = oracle.fmm(x, y, z, q, targets=tg)
        el = time.perf_counter() - t0
        got = phi.cpu().numpy()[tg]
        err = np.linalg.norm(got - w.phi) / np.linalg.norm(w.phi)
        out["cpu_baseline"] = {"value": w.stats["p2p_interactions"] / el, "unit": "P2P interactions/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"oracle FMM (tree, upward pass, full traversal) evaluated at 256 "
                                         f"sampled targets, {el:.1f} s on one host thread"}
        out["parity_sampled"] = {"targets": 256, "rel_l2": err,
                                 "lists_equal": all(r[k] == w.stats[k] for k in
                                                    ("m2l_pairs", "p2p_pairs", "m2l_hash", "p2p_hash"))}
    print(json.dumps(out), flush=True)
    return 0


def bench_schedulers(args, gtap) -> int:
    """Scheduler comparison (Sec. 6.5): fib(n) in thread mode under four queue
    managements over a sweep of grid sizes -- batched work stealing with the
    private LDS stack (this runtime), the same without it (the paper's
    Algorithm 1), non-batched work stealing (one task per pop and per steal)
    and one centralised FIFO queue.  Every run is checked against the closed
    forms F(n), 2F(n+1)-1 calls and F(n+1)-1 continuations."""
    import torch
    n = args.fib_n
    f = [0, 1]
    while len(f) < n + 2:
        f.append(f[-1] + f[-2])
    want = (f[n], 2 * f[n + 1] - 1, f[n + 1] - 1)
    variants = [("batched, LDS stack", 0), ("batched", gtap.GTAP_FLAG_NO_PRIVATE_STACK),
                ("non-batched", gtap.GTAP_FLAG_SCHED_SINGLE), ("central queue", gtap.GTAP_FLAG_SCHED_CENTRAL)]
    grid = [int(w) for w in args.sched_waves.split(",")]
    rows = []
    for name, flag in variants:
        slow = None
        for w in grid:
            if slow is not None:
                rows.append({"variant": name, "waves": w, "skipped": slow})
                continue
            rt = gtap.Runtime(flags=flag, num_waves=w, waves_per_group=4, small_frames=1 << 26,
                              deque_capacity=(1 << 20) if flag == gtap.GTAP_FLAG_SCHED_CENTRAL else (1 << 16),
                              timeout_ms=20000)
            ms = []
            try:
                for it in range(args.warmup + args.steps):
                    jid = rt.submit_fib(n)
                    rt.run()
                    st = rt.stats()
                    got = (rt.result(jid), st["tasks"], st["conts"])
                    if got != want:
                        raise SystemExit(f"{name}, {w} waves: got {got}, expected {want}")
                    if it >= args.warmup:
                        ms.append(st["kernel_ms"])
            except gtap.GtapError as e:
                # a watchdog expiry or a capacity error is a failure, never a table row
                rt.close()
                print(f"# {name:20s} waves {w:5d}: run failed with {gtap.gtap_status_string(e.code)} "
                      f"{e.report}", file=sys.stderr, flush=True)
                return 1
            torch.cuda.synchronize()
            rt.close()
            med = sorted(ms)[len(ms) // 2]
            row = {"variant": name, "waves": st["num_waves"], "kernel_ms_median": med,
                   "kernel_ms_min": min(ms), "tasks_per_s": want[1] / (med * 1e-3),
                   "pushed": st["pushed"], "popped": st["popped"], "stolen": st["stolen"],
                   "pop_batches": st["pop_batches"], "steal_batches": st["steal_batches"],
                   "steal_attempts": st["steal_attempts"], "iterations": st["iterations"]}
            rows.append(row)
            print(f"# {name:20s} waves {row['waves']:5d}: {med:9.3f} ms  {row['tasks_per_s'] / 1e9:7.3f} G tasks/s",
                  file=sys.stderr, flush=True)
            if med > 3000.0:
                slow = f"over 3 s per run at {w} wavefronts"
    best = max(r["tasks_per_s"] for r in rows if r["variant"] == variants[0][0] and "tasks_per_s" in r)
    out = {"metric": METRIC, "value": best, "unit": "tasks/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"scheduler comparison: fib({n}) in thread mode, one launch per run, "
                                  f"grid sweep over {grid} wavefronts (4 per workgroup)"},
           "rows": rows}
    print(json.dumps(out), flush=True)
    return 0


def bench_fmm_dtt(args, gtap) -> int:
    """The paper's FMM experiment (Sec. 6.4.1): uniform points, a theta sweep,
    the dual-tree traversal building M2L / P2P lists either as thread-mode
    tasks of this runtime or as the level-synchronous GPU worklist (one launch
    and one host synchronisation per frontier); both feed the same sort and
    data-parallel M2L / P2P kernels.  Reports the traversal time of each and
    the end-to-end breakdown."""
    import numpy as np
    import torch
    from synth import points
    n = args.fmm_points
    x, y, z, q = points.uniform_cube(n, 21, half=100.0)
    tx, ty, tz, tq = (torch.as_tensor(a).cuda() for a in (x, y, z, q))
    phi = torch.zeros_like(tx)
    thetas = [tuple(int(v) for v in t.split("/")) for t in args.fmm_thetas.split(",")]
    rt = gtap.Runtime(mode=gtap.GTAP_MODE_THREAD, waves_per_group=4, small_frames=1 << 25, big_frames=1 << 10,
                      timeout_ms=120000)
    rows = []
    for th in thetas:
        for name, tr in (("tasks", gtap.GTAP_FMM_LISTS), ("worklist", gtap.GTAP_FMM_WORKLIST)):
            runs = []
            for it in range(args.warmup + args.steps):
                phi.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                j = rt.submit_fmm(tx, ty, tz, tq, phi, leaf_max=64, theta=th, traversal=tr)
                rt.run()
                wall = time.perf_counter() - t0
                r = rt.fmm_result(j)
                r["wall_ms"] = 1e3 * wall
                if it >= args.warmup:
                    runs.append(r)
            runs.sort(key=lambda r: r["traversal_ms"])
            r = runs[len(runs) // 2]
            row = {"theta": f"{th[0]}/{th[1]}", "traversal": name, "dtt_ms": r["traversal_ms"],
                   "dtt_ms_min": runs[0]["traversal_ms"], "end_to_end_ms": r["wall_ms"],
                   "phase_ms": {k: r[k] for k in ("tree_ms", "upward_ms", "traversal_ms", "sort_ms", "m2l_ms",
                                                  "p2p_ms", "downward_ms")},
                   "lists": {k: r[k] for k in ("n_cells", "n_leaves", "max_level", "m2l_pairs", "p2p_pairs",
                                               "p2p_interactions")},
                   "dtt_rounds": r["dtt_rounds"], "list_retries": r["list_retries"],
                   "m2l_hash": r["m2l_hash"], "p2p_hash": r["p2p_hash"]}
            rows.append(row)
            print(f"# theta {row['theta']:5s} {name:8s}: DTT {row['dtt_ms']:9.2f} ms, end to end "
                  f"{row['end_to_end_ms']:9.1f} ms, M2L pairs {r['m2l_pairs']}, P2P pairs {r['p2p_pairs']}",
                  file=sys.stderr, flush=True)
        a, b = rows[-2], rows[-1]
        if (a["m2l_hash"], a["p2p_hash"]) != (b["m2l_hash"], b["p2p_hash"]):
            raise SystemExit(f"theta {a['theta']}: the two traversals built different lists")
    st = rt.stats()
    rt.close()
    best = min(r["dtt_ms"] for r in rows if r["traversal"] == "tasks")
    out = {"metric": METRIC, "value": None, "unit": "ms (DTT list construction)", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"FMM pipeline with list-building DTT: {n} uniform points in [-100, 100)^3 "
                                  f"(seed 21), leaf 64, order 6, theta sweep {args.fmm_thetas}",
                      "waves": st["num_waves"], "waves_per_group": st["waves_per_group"]},
           "rows": rows}
    out["value"] = best
    for r in rows:
        r.pop("m2l_hash")
        r.pop("p2p_hash")
    print(json.dumps(out), flush=True)
    return 0


def bench_cilksort(args, gtap) -> int:
    """Cilksort (Sec. 6.3) of n uniform random 32-bit keys in thread mode,
    sort / merge cutoffs 64 / 256; --queues 3 runs the paper's DAQ setup
    (recursive, serial-sort and serial-merge queues).  value = keys sorted per
    second (kernel time, HIP events); every run is checked for sortedness and
    for the key sum."""
    import torch
    n = args.sort_n
    g = torch.Generator(device="cuda").manual_seed(13)
    src = torch.randint(-2**31, 2**31, (n,), dtype=torch.int64, device="cuda", generator=g).to(torch.int32)
    ssum = int((src.to(torch.int64) & 0xFFFFFFFF).sum())
    kw = dict(num_queues=args.queues, daq_policy=gtap.GTAP_DAQ_CILKSORT) if args.queues > 1 else {}
    rt = gtap.Runtime(waves_per_group=4, small_frames=1 << 25, big_frames=1 << 10, deque_capacity=1 << 18,
                      timeout_ms=120000, **kw)
    keys = torch.empty_like(src)
    tmp = torch.empty_like(src)
    ms = []
    for it in range(args.warmup + args.steps):
        keys.copy_(src)
        torch.cuda.synchronize()
        jid = rt.submit_cilksort(keys, tmp, sort_cutoff=args.sort_cutoff, merge_cutoff=args.merge_cutoff)
        rt.run()
        st = rt.stats()
        v = keys.to(torch.int64) & 0xFFFFFFFF
        if rt.result(jid) != n or not bool((v[1:] >= v[:-1]).all()) or int(v.sum()) != ssum:
            raise SystemExit("cilksort output is not the sorted input")
        if it >= args.warmup:
            ms.append(st["kernel_ms"])
    rt.close()
    med = sorted(ms)[len(ms) // 2]
    out = {"metric": METRIC, "value": n / (med * 1e-3), "unit": "keys/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"Cilksort of {n} uniform random 32-bit keys (seed 13), sort / merge cutoffs "
                                  f"{args.sort_cutoff} / {args.merge_cutoff}, thread mode",
                      "queues": args.queues, "waves": st["num_waves"]},
           "kernel_ms_median": med, "kernel_ms_min": min(ms),
           "runtime_counters_per_run": {k: st[k] for k in ("tasks", "conts", "pushed", "stolen", "iterations",
                                                           "idle_iterations", "local_pushed")}}
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# The combined run (default): one JSON line whose headline is the batched job
# mix (20,000 jobs), with the other configurations as sub-records.

C0_GRAPH = (2000, 16, 2.5, 1.0, 1)
C3_GRAPH = (1000000, 40, 2.1, 0.6, 2)
C3_TAG = "n1000000_d40_g2.1_cap0.6_s2"
C0_TAG = "n2000_d16_g2.5_cap1.0_s1"

# Algorithmic bytes per event for a scheduler launch, priced like the per-task
# table of the runtime's roofline: a spawned task's frame is written (32 B)
# and read (32 B), its result (8 B) and the join update (4 B) reach the
# parent: 76 B per task; a task ID published to a deque is written and read
# once (4 + 4 B); every batch operation on a deque count is one 4-byte RMW.
# Task data the bodies move (k-clique lists) is counted by the kernel itself.
BYTES_PER_TASK = 76
BYTES_PER_PUSHED = 8
BYTES_PER_BATCH = 4
FP64_FLOP_P2P = 20       # per P2P interaction: differences, r^2, 1/r, q/r, accumulate
FP64_FLOP_M2L = 1848     # per M2L pair: 924 multiply-adds of the order-6 Taylor terms
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64


def sched_bytes(st: dict) -> int:
    batches = st["push_batches"] + st["pop_batches"] + st["steal_batches"]
    return (BYTES_PER_TASK * st["tasks"] + BYTES_PER_PUSHED * st["pushed"] + BYTES_PER_BATCH * batches
            + st.get("data_bytes", 0))


def add_stats(tot: dict, st: dict) -> None:
    for k, v in st.items():
        if isinstance(v, int):
            tot[k] = tot.get(k, 0) + v


def sched_roofline(tot: dict, steps: int, kernel_ms: list, probe: dict, traffic_key: str) -> dict:
    """HBM roofline of thread_sched_kernel from the runtime's counters (bytes
    per launch / mean launch time on the launch stream), with the
    device-scope RMW rate beside the probed peak."""
    mean_ms = sum(kernel_ms) / len(kernel_ms)
    per_launch = sched_bytes(tot) / steps
    achieved = per_launch / (mean_ms * 1e-3) / 1e9
    rmw = tot["atomics"] / steps / (mean_ms * 1e-3)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(traffic_key),
            "kernel": "thread_sched_kernel", "kernel_ms": mean_ms, "algorithmic_bytes_per_launch": per_launch,
            "bytes_per_task": per_launch / max(1, tot["tasks"] / steps),
            "atomics": {"achieved_rmw_per_s": rmw, "rmw_per_launch": tot["atomics"] / steps,
                        "peak_distinct_rmw_per_s": probe.get("distinct"),
                        "frac_of_distinct": rmw / probe["distinct"] if probe.get("distinct") else None,
                        "peak_one_word_rmw_per_s": probe.get("one_word")}}


def atomic_probe(gtap) -> dict:
    """Device-scope RMW peaks on this GPU (distinct lines, one word per
    wavefront, one word for the grid), best of three launches each."""
    import torch
    blocks, iters = 2048, 64
    words = torch.zeros(blocks * 256 * 8 + 1, dtype=torch.int64, device="cuda")
    out = {}
    for mode, name in ((gtap.GTAP_PROBE_DISTINCT, "distinct"), (gtap.GTAP_PROBE_PER_WAVE, "per_wave"),
                       (gtap.GTAP_PROBE_ONE_WORD, "one_word")):
        out[name] = max(gtap.gtap_probe_atomics(mode, blocks, iters, words.data_ptr(), words.numel())[0]
                        for _ in range(3))
    del words
    return out


def timed_launches(rt, submit, steps, warmup, check, torch):
    """warmup + steps launches of one batch; returns (wall seconds of the timed
    steps, summed runtime counters, per-launch kernel ms).  check(results) must
    hold after every launch."""
    for _ in range(warmup):
        ids = submit()
        rt.run()
        check([rt.result(j) for j in ids])
    torch.cuda.synchronize()
    tot, kms, res = {}, [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ids = submit()
        rt.run()
        st = rt.stats()
        kms.append(st["kernel_ms"])
        add_stats(tot, st)
        res.append([rt.result(j) for j in ids])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for r in res:
        check(r)
    return el, tot, kms, st


def expect(want):
    def check(got):
        if list(got) != list(want):
            raise SystemExit(f"wrong results {got}, expected {want}")
    return check


def c1_record(args, gtap, probe, torch, steps, warmup) -> dict:
    """Thread-mode microbenchmarks: the three roots in one launch, and each alone."""
    thr = gtap.uts_threshold(4)
    rt = gtap.Runtime(waves_per_group=args.waves_per_group, num_waves=args.num_waves,
                      steal_below=args.steal_below, small_frames=1 << 25, timeout_ms=60000)
    want = {"fib": 2178309, "nqueens": 73712, "uts": 102971195}
    subm = {"fib": lambda: [rt.submit_fib(32)], "nqueens": lambda: [rt.submit_nqueens(13)],
            "uts": lambda: [rt.submit_uts(1, thr, 13)]}
    el, tot, kms, st = timed_launches(rt, lambda: subm["fib"]() + subm["nqueens"]() + subm["uts"](),
                                      steps, warmup, expect(list(want.values())), torch)
    rec = {"workload": "fib(32), N-Queens(13), UTS(mean 4, depth 13, seed 1) in one persistent launch",
           "value": tot["tasks"] / el, "unit": "tasks/s", "steps": steps, "warmup": warmup,
           "ms_per_step": 1e3 * el / steps, "tasks_per_step": tot["tasks"] // steps,
           "executions_per_s": (tot["tasks"] + tot["conts"]) / el, "matches_oracle": True,
           "kernel_tasks_per_s": tot["tasks"] / steps / (sum(kms) / len(kms) * 1e-3),
           "roofline": sched_roofline(tot, steps, kms, probe, "microbench"),
           "waves": st["num_waves"], "runtime_counters_per_step": {k: v // steps for k, v in tot.items()}}
    per = {}
    for name in ("fib", "nqueens", "uts"):
        e, t, k, _ = timed_launches(rt, subm[name], steps, warmup, expect([want[name]]), torch)
        per[name] = {"tasks_per_s": t["tasks"] / e, "ms_per_step": 1e3 * e / steps,
                     "kernel_ms": sum(k) / len(k), "tasks_per_step": t["tasks"] // steps,
                     "conts_per_step": t["conts"] // steps,
                     "roofline_frac": sched_roofline(t, steps, k, probe, "")["frac"]}
    rec["per_workload"] = per
    rt.close()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(min_seconds=3.0, max_seconds=10.0)
        rec["cpu_context_all_cores"] = c1_cpu_all_cores()
    return rec


def c1_cpu_all_cores() -> dict:
    """Context only: the oracle on every host core, one UTS subtree, fib call
    or first-row N-Queens placement per unit (the oracle's C code runs without
    the interpreter lock, so threads run in parallel)."""
    import concurrent.futures as cf
    import oracle
    cores = os.cpu_count() or 1
    thr = oracle.uts_threshold(4)
    units = [lambda: oracle.fib(31), lambda: oracle.fib(30), lambda: oracle.nqueens(13),
             lambda: oracle.uts(1, thr, 13)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        tasks = sum(r.tasks for r in ex.map(lambda f: f(), units))
    el = time.perf_counter() - t0
    return {"value": tasks / el, "unit": "tasks/s", "cores": cores, "kind": "oracle",
            "sample": f"fib(31), fib(30), N-Queens(13) and UTS depth 13 as independent jobs on {cores} threads "
                      f"(whole roots: the oracle has no sub-root entry), {el:.1f} s; the largest root bounds it"}


def golden_kclique(tag: str, k: int):
    with open(os.path.join(ROOT, "tests", "golden", "kclique_chung_lu.txt")) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 6 and f[0] == tag and f[2] == str(k):
                return {"checksum": f[1], "count": int(f[3]), "tasks": int(f[4]), "conts": int(f[5])}
    raise SystemExit(f"no golden k-clique count for {tag} k={k}")


def c0_record(args, gtap, probe, torch, steps, warmup) -> dict:
    """4-cliques of the n=2,000 Chung-Lu graph, thread mode, one queue."""
    from synth import graphs
    g = graphs.chung_lu(*C0_GRAPH)
    want = golden_kclique(C0_TAG, 4)
    if g.checksum() != want["checksum"]:
        raise SystemExit("C0 graph checksum differs from the golden file's")
    rt = gtap.Runtime(waves_per_group=4, num_waves=args.c0_waves, small_frames=1 << 20, big_frames=1 << 16,
                      big_frame_ints=max(64, g.max_outdeg), timeout_ms=30000)
    rp, col = torch.as_tensor(g.row_ptr32).cuda(), torch.as_tensor(g.col).cuda()
    el, tot, kms, st = timed_launches(rt, lambda: [rt.submit_kclique(rp, col, 4, max_outdeg=g.max_outdeg)],
                                      steps, warmup, expect([want["count"]]), torch)
    ok = tot["tasks"] == want["tasks"] * steps and tot["conts"] == want["conts"] * steps
    rec = {"workload": "4-cliques, Chung-Lu n=2000, mean degree 16, exponent 2.5, cap 1.0, seed 1; "
                       "one task per call, one queue",
           "value": want["count"] * steps / el, "unit": "k-cliques/s", "steps": steps, "warmup": warmup,
           "ms_per_step": 1e3 * el / steps, "count": want["count"], "tasks_per_s": tot["tasks"] / el,
           "waves": st["num_waves"], "matches_oracle": ok, "roofline": sched_roofline(tot, steps, kms, probe, ""),
           "runtime_counters_per_step": {k: v // steps for k, v in tot.items()}}
    rt.close()
    if not args.no_cpu_baseline:
        import oracle
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 2.0:
            oracle.kclique(g.row_ptr, g.col, 4)
            reps += 1
        e = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": want["count"] * reps / e, "unit": "k-cliques/s", "cores": 1,
                               "kind": "oracle", "sample": f"the whole count x{reps}, {e:.1f} s on one host thread"}
    if not ok:
        raise SystemExit(f"C0 task counts {tot['tasks'] // steps}/{tot['conts'] // steps} differ from the oracle's")
    return rec


def c3_record(args, gtap, g, probe, torch, steps, warmup) -> dict:
    """7-cliques of the n=10^6 graph with 4 DAQ queues (candidate-set buckets
    8/32/128) against one queue: the split search with bitset candidate
    subgraphs (the record's value) and one task per call."""
    want = golden_kclique(C3_TAG, 7)
    rp, col = torch.as_tensor(g.row_ptr32).cuda(), torch.as_tensor(g.col).cuda()
    out = {"workload": "7-cliques, Chung-Lu n=1e6, mean degree 40, exponent 2.1, cap 0.6, seed 2 "
                       f"({g.m_undirected} edges, max out-degree {g.max_outdeg})", "count": want["count"]}
    variants = {}
    for name, queues, split in (("tree_daq4", 4, False), ("tree_daq1", 1, False),
                                ("split_daq4", 4, True), ("split_daq1", 1, True)):
        opts = dict(num_waves=1024, waves_per_group=4, deque_capacity=1 << 17, small_frames=1 << 25,
                    big_frames=1 << 23, big_frame_ints=max(320, g.max_outdeg), timeout_ms=60000)
        if queues > 1:
            opts.update(num_queues=4, daq_policy=gtap.GTAP_DAQ_KCLIQUE, daq_bounds=[8, 32, 128],
                        deque_capacity=1 << 19, big_frames=1 << 24)
        if split:
            opts.update(big_frames=1 << 23, big_frame_ints=gtap.kclique_split_buffer_ints(g.max_outdeg))
        rt = gtap.Runtime(**opts)
        if split:
            sub = lambda: [rt.submit_kclique_split(rp, col, 7, threshold=64, algorithm=gtap.GTAP_KCLIQUE_ORIENT,
                                                   max_outdeg=g.max_outdeg)]
        else:
            sub = lambda: [rt.submit_kclique(rp, col, 7, max_outdeg=g.max_outdeg)]
        n_steps = steps if split else max(1, min(steps, 3))
        el, tot, kms, st = timed_launches(rt, sub, n_steps, min(warmup, 1), expect([want["count"]]), torch)
        rt.close()
        v = {"value": want["count"] * n_steps / el, "unit": "k-cliques/s", "steps": n_steps,
             "ms_per_step": 1e3 * el / n_steps, "kernel_ms": sum(kms) / len(kms),
             "tasks_per_s": tot["tasks"] / el, "matches_oracle": True,
             "roofline": sched_roofline(tot, n_steps, kms, probe, "kclique7_" + name),
             "runtime_counters_per_step": {k: x // n_steps for k, x in tot.items()}}
        if not split:
            v["task_tree_matches_oracle"] = (tot["tasks"] == want["tasks"] * n_steps and
                                             tot["conts"] == want["conts"] * n_steps)
            if not v["task_tree_matches_oracle"]:
                raise SystemExit(f"C3 {name}: task counts differ from the oracle's")
        variants[name] = v
    out.update(variants["split_daq4"])
    out["search"] = ("bitset candidate subgraphs with cost-threshold splitting (orientation, threshold 64), "
                     "4 DAQ queues by candidate-set bucket 8/32/128")
    out["variants"] = {k: v for k, v in variants.items() if k != "split_daq4"}
    out["daq_speedup"] = {"one_task_per_call": variants["tree_daq1"]["ms_per_step"] / variants["tree_daq4"]["ms_per_step"],
                          "split": variants["split_daq1"]["ms_per_step"] / variants["split_daq4"]["ms_per_step"]}
    out["valu_lane_utilisation"] = measured_valu()
    if not args.no_cpu_baseline:
        a = argparse.Namespace(kclique_split="orient", split_threshold=64)
        out["cpu_baseline"] = kclique_cpu_baseline(g, a)
        out["cpu_context_all_cores"] = kclique_cpu_all_cores(g)
    return out


def kclique_cpu_all_cores(g, stride: int = 4) -> dict:
    """Context only: the same vertex sample (lowest vertex 0 mod stride) split
    over every host core by vertex residue."""
    import concurrent.futures as cf
    import oracle
    cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        parts = list(ex.map(lambda t: oracle.kclique_split_roots(g.row_ptr, g.col, 7, stride * cores, stride * t,
                                                                  threshold=64, algorithm="orient").value,
                            range(cores)))
    el = time.perf_counter() - t0
    return {"value": sum(parts) / el, "unit": "k-cliques/s", "cores": cores, "kind": "oracle",
            "sample": f"the {sum(parts)} 7-cliques whose lowest vertex is 0 mod {stride}, split over {cores} "
                      f"threads by vertex residue, {el:.1f} s"}


def c2_record(args, gtap, steps, warmup) -> dict:
    """Block-mode FMM on 10^6 Plummer points: traversal tasks with M2L and
    cooperative P2P inside."""
    import numpy as np
    import torch
    from synth import points
    n = 1000000
    x, y, z, q = points.plummer(n, 3)
    tx, ty, tz, tq = (torch.as_tensor(a).cuda() for a in (x, y, z, q))
    phi = torch.zeros_like(tx)
    rt = gtap.Runtime(mode=gtap.GTAP_MODE_BLOCK, waves_per_group=2, small_frames=1 << 24, big_frames=0,
                      timeout_ms=120000)
    n_steps = max(1, min(steps, 5))
    for _ in range(min(warmup, 1)):
        rt.submit_fmm(tx, ty, tz, tq, phi)
        rt.run()
    torch.cuda.synchronize()
    res, wall, kms = [], [], []
    t0 = time.perf_counter()
    for _ in range(n_steps):
        phi.zero_()
        t1 = time.perf_counter()
        j = rt.submit_fmm(tx, ty, tz, tq, phi)
        rt.run()
        wall.append(time.perf_counter() - t1)
        res.append(rt.fmm_result(j))
        kms.append(rt.stats()["kernel_ms"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = rt.stats()
    rt.close()
    r = res[-1]
    trav_ms = sum(kms) / len(kms)
    flops = FP64_FLOP_P2P * r["p2p_interactions"] + FP64_FLOP_M2L * r["m2l_pairs"]
    achieved = flops / (trav_ms * 1e-3) / 1e12
    rec = {"workload": "3D Laplace FMM, block mode (work inside the traversal tasks): 1e6 Plummer points "
                       "(seed 3), leaf 64, theta 1/2, Cartesian order 6",
           "value": r["p2p_interactions"] / (trav_ms * 1e-3), "unit": "P2P interactions/s",
           "steps": n_steps, "ms_per_step": 1e3 * el / n_steps, "traversal_ms": trav_ms,
           "m2l_pairs_per_s": r["m2l_pairs"] / (trav_ms * 1e-3),
           "end_to_end_ms_median": 1e3 * sorted(wall)[len(wall) // 2],
           "phase_ms": {k: r[k] for k in ("tree_ms", "upward_ms", "traversal_ms", "downward_ms")},
           "lists": {k: r[k] for k in ("n_cells", "n_leaves", "m2l_pairs", "p2p_pairs", "p2p_interactions")},
           "traversal_tasks": st["tasks"],
           "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel": "block_sched_kernel",
                        "kernel_ms": trav_ms, "algorithmic_flop_per_launch": flops,
                        "flop_per_unit": {"p2p_interaction": FP64_FLOP_P2P, "m2l_pair": FP64_FLOP_M2L}},
           "dtype": "f64"}
    if not args.no_cpu_baseline:
        import oracle
        tg = np.random.default_rng(17).choice(n, 256, replace=False)
        t1 = time.perf_counter()
        w = oracle.fmm(x, y, z, q, targets=tg)
        e = time.perf_counter() - t1
        got = phi.cpu().numpy()[tg]
        err = float(max(np.max(np.abs(got - w.phi)) / np.max(np.abs(w.phi)),
                        np.linalg.norm(got - w.phi) / np.linalg.norm(w.phi)))
        rec["cpu_baseline"] = {"value": w.stats["p2p_interactions"] / e, "unit": "P2P interactions/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"oracle FMM (tree, upward pass, full traversal) evaluated at 256 sampled "
                                         f"targets, {e:.1f} s on one host thread"}
        rec["parity_sampled"] = {"targets": 256, "rel_err": err,
                                 "lists_equal": all(r[k] == w.stats[k] for k in
                                                    ("m2l_pairs", "p2p_pairs", "m2l_hash", "p2p_hash"))}
        rec["matches_oracle"] = err <= 1e-12 and rec["parity_sampled"]["lists_equal"]
        if not rec["matches_oracle"]:
            raise SystemExit(f"C2 parity: {rec['parity_sampled']}")
    return rec


def load_serving_golden(n_jobs: int, seed: int):
    """The oracle's result for every job of serving_mix(n_jobs, seed), written
    by tests/golden/make_serving_golden.py, or None if that trace has none."""
    path = os.path.join(ROOT, "tests", "golden", f"serving_trace_s{seed}.txt")
    if not os.path.exists(path):
        return None
    out = []
    with open(path) as fh:
        head = fh.readline().split()
        if f"serving_mix({n_jobs}," not in " ".join(head):
            return None
        for line in fh:
            if not line.startswith("#"):
                out.append(int(line.split()[3]))
    return out if len(out) == n_jobs else None


def c4_tune_space(gtap):
    """Queue count, DAQ class function and bounds, workgroup shape and grid."""
    return gtap.tune_space(num_queues=(1, 2, 4), waves_per_group=(2, 4, 8), num_waves=(1024, 0),
                           daq_policies=(gtap.GTAP_DAQ_BY_KIND, gtap.GTAP_DAQ_KCLIQUE),
                           bounds=((8, 32, 128), (4, 16, 64)), repeats=1)


def c4_record(args, gtap, g, probe, torch, steps, warmup, say) -> dict:
    """The batched job mix: 20,000 jobs (60 % k-clique on induced subgraphs of
    the n=10^6 graph, 40 % UTS) in one persistent launch per step, against
    one launch per job; then the served open loop."""
    import numpy as np
    from synth import serving
    n_jobs = args.jobs
    golden = load_serving_golden(n_jobs, 5)
    common = dict(max_jobs=1 << 15, big_frame_ints=max(320, g.max_outdeg), deque_capacity=1 << 18,
                  timeout_ms=300000)
    default_cfg = dict(num_waves=1024, waves_per_group=4, small_frames=1 << 26, big_frames=1 << 22)
    base = gtap.Runtime(**default_cfg, **common)
    _, cal_entries, _, cal_keep, _, _ = serving_trace(gtap, base, g, max(1, n_jobs // 4), 6, torch)
    tune_jobs = base.trace([(0.0, e) for e in cal_entries[: args.calib_jobs]])
    tuned, tune_rep = base.autotune(tune_jobs, c4_tune_space(gtap))
    base.close()
    say(f"C4 autotuned {tuned} {tune_rep}")
    specs, entries, classes, keep, subs, staged = serving_trace(gtap, None, g, n_jobs, 5, torch)
    say(f"C4 trace ready {staged}")

    def check(res):
        if golden is not None and res != golden:
            bad = [i for i, (a, b) in enumerate(zip(res, golden)) if a != b]
            raise SystemExit(f"C4: {len(bad)} results differ from the oracle's, first job {bad[0]}")

    def batch_pass(rt):
        ids = [gtap.gtap_submit(rt.ctx, kind, a) for kind, a in entries]
        rt.run()
        return [rt.result(j) for j in ids]

    # the default configuration on the measurement trace, once (context for the tuner)
    rt = gtap.Runtime(**default_cfg, **common)
    batch_pass(rt)
    t1 = time.perf_counter()
    check(batch_pass(rt))
    default_s = time.perf_counter() - t1
    default_kernel_ms = rt.stats()["kernel_ms"]
    rt.close()
    say(f"C4 default configuration: {default_s:.2f} s per batch")

    rt = gtap.Runtime(**tuned, **common)
    el, tot, kms, st = timed_launches(rt, lambda: [gtap.gtap_submit(rt.ctx, kind, a) for kind, a in entries],
                                      steps, warmup, check, torch)
    say(f"C4 batched: {steps} steps, {el / steps:.2f} s per step")
    headroom = int(tuned["small_frames"]) // 4
    if args.c4_batched_only:
        # counter runs: the tuned batched launches alone (one launch per job
        # under per-dispatch counter collection would take minutes)
        rt.close()
        del cal_keep, keep
        return {"value": n_jobs * steps / el, "unit": "jobs/s", "steps": steps, "warmup": warmup,
                "ms_per_step": 1e3 * el / steps, "batched_only": True,
                "workload": f"{n_jobs} jobs, trace seed 5, the tuned batched launches alone",
                "tasks_per_step": tot["tasks"] // steps, "tasks_per_s": tot["tasks"] / el,
                "kernel_ms": sum(kms) / len(kms), "matches_oracle": golden is not None,
                "autotune": {"chosen": {k: v for k, v in tuned.items() if not isinstance(v, (list, tuple))}},
                "roofline": sched_roofline(tot, steps, kms, probe, "serving"),
                "runtime_counters_per_step": {k: v // steps for k, v in tot.items()}}

    def served(arrivals):
        jobs = rt.trace([(t, e) for t, e in zip(arrivals, entries)])
        rt.serve_start(max_inflight=args.inflight, headroom_small=headroom)
        res = rt.trace_run(jobs, timeout_ms=280000)
        rt.serve_stop()
        return res

    res_sat = served(np.zeros(n_jobs))
    served_s = max(r.done_s for r in res_sat)
    check([r.result for r in res_sat])
    plain_sat = rt.trace_run_plain(rt.trace([(0.0, e) for e in entries]))
    plain_s = max(r.done_s for r in plain_sat)
    check([r.result for r in plain_sat])
    say(f"C4 served saturated {served_s:.2f} s, one launch per job {plain_s:.2f} s")
    # open loop at 0.8 x the saturated served rate of the calibration trace
    cal_jobs = rt.trace([(0.0, e) for e in cal_entries])
    rt.serve_start(max_inflight=args.inflight, headroom_small=headroom)
    cal_res = rt.trace_run(cal_jobs, timeout_ms=280000)
    rt.serve_stop()
    cal_rate = len(cal_entries) / max(r.done_s for r in cal_res)
    del cal_keep
    arr = serving.poisson_arrivals(n_jobs, 0.8 * cal_rate, 55)
    res_o = served(arr)
    check([r.result for r in res_o])
    res_po = rt.trace_run_plain(rt.trace([(t, e) for t, e in zip(arr, entries)]))
    check([r.result for r in res_po])
    say(f"C4 open loop at {0.8 * cal_rate:.0f} jobs/s done")
    rt.close()
    rec = {"value": n_jobs * steps / el, "unit": "jobs/s", "steps": steps, "warmup": warmup,
           "ms_per_step": 1e3 * el / steps,
           "workload": f"{n_jobs} jobs, trace seed 5: 60% k-clique (k 4..8, one task per call, induced "
                       "subgraphs of log-uniform 1e3..2e5 vertices of the n=1e6 Chung-Lu graph), 40% UTS "
                       "(m 2..4, depth 8..14); one persistent launch per step",
           "staged": staged, "tasks_per_step": tot["tasks"] // steps,
           "tasks_per_s": tot["tasks"] / el, "kernel_ms": sum(kms) / len(kms),
           "matches_oracle": golden is not None, "jobs_checked_per_step": len(golden) if golden else 0,
           "saturated_jobs_per_s": {"batched": n_jobs * steps / el, "served": n_jobs / served_s,
                                    "one_launch_per_job": n_jobs / plain_s},
           "batched_vs_one_launch_per_job": (n_jobs * steps / el) / (n_jobs / plain_s),
           "open_loop": {"rate_jobs_per_s": 0.8 * cal_rate, "calibrated_saturated_rate": cal_rate,
                         "served": _latency_summary(res_o, arr, classes),
                         "one_launch_per_job": _latency_summary(res_po, arr, classes)},
           "autotune": {"chosen": {k: v for k, v in tuned.items() if not isinstance(v, (list, tuple))},
                        "daq_bounds": list(tuned.get("daq_bounds", []))[:3], "report": tune_rep,
                        "default_config_s_per_batch": default_s, "default_kernel_ms": default_kernel_ms,
                        "tuned_s_per_batch": el / steps},
           "roofline": sched_roofline(tot, steps, kms, probe, "serving"),
           "runtime_counters_per_step": {k: v // steps for k, v in tot.items()}}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = serving_cpu_baseline(specs, subs, golden or [r.result for r in plain_sat])
        rec["cpu_context_all_cores"] = serving_cpu_all_cores(specs, subs)
    del keep
    return rec


def serving_cpu_all_cores(specs, subs, budget_s: float = 8.0) -> dict:
    """Context only: the oracle over the trace's jobs, smallest first, on every
    host core (whole jobs are the units)."""
    import concurrent.futures as cf
    import oracle
    cores = os.cpu_count() or 1
    order, it = [], 0
    for i, sp in enumerate(specs):
        if sp.kind == "kclique":
            order.append((subs[it].col.size, i, it))
            it += 1
        else:
            order.append((sp.m ** sp.depth, i, -1))
    order.sort()
    t0 = time.perf_counter()
    done = [0]

    def one(item):
        if time.perf_counter() - t0 > budget_s:
            return 0
        _, i, it = item
        sp = specs[i]
        if sp.kind == "kclique":
            oracle.kclique(subs[it].row_ptr, subs[it].col, sp.k)
        else:
            oracle.uts(sp.seed, oracle.uts_threshold(sp.m), sp.depth)
        return 1

    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        done = sum(ex.map(one, order))
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "jobs/s", "cores": cores, "kind": "oracle",
            "sample": f"the {done} smallest of {len(specs)} trace jobs on {cores} threads, {el:.1f} s"}


def line_head(value, unit, steps, warmup, ms_per_step, dtype, config) -> dict:
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config}


def bench_one(args, gtap) -> int:
    """One configuration alone (c0..c4, microbench = c1): its record as the line."""
    import torch
    say = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    probe = atomic_probe(gtap)
    w = args.workload
    if w in ("c1", "microbench"):
        rec = c1_record(args, gtap, probe, torch, args.steps, args.warmup)
    elif w == "c0":
        rec = c0_record(args, gtap, probe, torch, args.steps, args.warmup)
    elif w == "c2":
        rec = c2_record(args, gtap, args.steps, args.warmup)
    else:
        from synth import graphs
        g = graphs.chung_lu(*C3_GRAPH)
        if w == "c3":
            rec = c3_record(args, gtap, g, probe, torch, args.steps, args.warmup)
        else:
            rec = c4_record(args, gtap, g, probe, torch, args.steps, args.warmup, say)
    out = line_head(rec.pop("value"), rec.pop("unit"), rec.pop("steps", args.steps), rec.pop("warmup", args.warmup),
                    rec.pop("ms_per_step", None), rec.pop("dtype", "int64"), {"workload": rec.pop("workload")})
    out.update(rec)
    out["atomic_probe_rmw_per_s"] = probe
    print(json.dumps(out), flush=True)
    return 0


def bench_all(args, gtap) -> int:
    """The combined run: C1, C0, C2, C3 as sub-records, C4 as the headline."""
    import torch
    from synth import graphs
    say = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    probe = atomic_probe(gtap)
    say(f"atomic probe {probe}")
    sub = {}
    sub["C1"] = c1_record(args, gtap, probe, torch, args.steps, args.warmup)
    say(f"C1 done {time.perf_counter() - t0:.0f} s: {sub['C1']['value'] / 1e9:.2f} G tasks/s")
    sub["C0"] = c0_record(args, gtap, probe, torch, args.steps, args.warmup)
    say(f"C0 done {time.perf_counter() - t0:.0f} s: {sub['C0']['value'] / 1e6:.2f} M cliques/s")
    sub["C2"] = c2_record(args, gtap, args.steps, args.warmup)
    say(f"C2 done {time.perf_counter() - t0:.0f} s: {sub['C2']['value'] / 1e9:.2f} G interactions/s")
    g = graphs.chung_lu(*C3_GRAPH)
    say(f"graph ready {time.perf_counter() - t0:.0f} s")
    sub["C3"] = c3_record(args, gtap, g, probe, torch, args.steps, args.warmup)
    say(f"C3 done {time.perf_counter() - t0:.0f} s: {sub['C3']['value'] / 1e6:.2f} M cliques/s")
    rec = c4_record(args, gtap, g, probe, torch, args.steps, args.warmup, say)
    say(f"C4 done {time.perf_counter() - t0:.0f} s")
    out = line_head(rec.pop("value"), rec.pop("unit"), rec.pop("steps"), rec.pop("warmup"), rec.pop("ms_per_step"),
                    "int64", {"workload": rec.pop("workload"), "headline": "C4 batched job mix",
                              "mode": "thread", "gpus": 1})
    out.update(rec)
    out["configs"] = sub
    out["atomic_probe_rmw_per_s"] = probe
    out["bench_wall_s"] = time.perf_counter() - t0
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--waves-per-group", type=int, default=4)
    ap.add_argument("--num-waves", type=int, default=1024)
    ap.add_argument("--steal-below", type=int, default=64)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="run only a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--c0-waves", type=int, default=1024, help="c0: wavefronts of the launch (the job is small)")
    ap.add_argument("--fmm-points", type=int, default=1000000, help="fmm: number of points")
    ap.add_argument("--fmm-wpg", type=int, default=2, help="fmm: wavefronts per workgroup (1, 2, 4)")
    ap.add_argument("--fib-n", type=int, default=35, help="schedulers: fib argument")
    ap.add_argument("--fmm-thetas", default="1/2,2/5,1/3", help="fmm_dtt: MAC parameters")
    ap.add_argument("--sort-n", type=int, default=100000000, help="cilksort: number of keys")
    ap.add_argument("--sort-cutoff", type=int, default=64, help="cilksort: serial sort cutoff")
    ap.add_argument("--merge-cutoff", type=int, default=256, help="cilksort: serial merge cutoff")
    ap.add_argument("--fmm-traversal", default="tasks", choices=("tasks", "lists", "worklist"),
                    help="fmm: block-mode tasks with the work inside, or a list-building traversal")
    ap.add_argument("--sched-waves", default="64,128,256,512,1024", help="schedulers: grid sizes (wavefronts)")
    ap.add_argument("--workload", default="all",
                    choices=("all", "c0", "c1", "c2", "c3", "c4", "microbench", "kclique7", "serving", "fmm",
                             "schedulers", "fmm_dtt", "cilksort"),
                    help="kclique7: 7-cliques of the n=10^6 Chung-Lu graph (DAQ comparison); "
                         "serving: batched / served job mix against one launch per job")
    ap.add_argument("--jobs", type=int, default=20000, help="serving: jobs in the trace")
    ap.add_argument("--inflight", type=int, default=4096, help="serving: admission limit")
    ap.add_argument("--calib-jobs", type=int, default=400, help="serving: autotuner calibration jobs")
    ap.add_argument("--c4-batched-only", action="store_true",
                    help="c4: only the autotuner and the batched launches (for counter runs)")
    ap.add_argument("--sweep", action="store_true", help="serving: also rho 0.3/0.5/0.7/0.9")
    ap.add_argument("--queues", type=int, default=1, help="kclique7: DAQ queues (1 = off)")
    ap.add_argument("--kclique-split", default="none", choices=("none", "orient", "pivot"),
                    help="kclique7: bitset candidate subgraphs with cost-threshold splitting")
    ap.add_argument("--daq-bounds", default="8,32,128", help="kclique7 with --queues: class bounds")
    ap.add_argument("--split-threshold", type=int, default=16,
                    help="kclique7 with --kclique-split: split nodes with more candidates than this")
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
    if args.workload == "all":
        return bench_all(args, gtap)
    if args.workload == "kclique7":
        return bench_kclique7(args, gtap)
    if args.workload == "serving":
        return bench_serving(args, gtap)
    if args.workload == "fmm":
        return bench_fmm(args, gtap)
    if args.workload == "schedulers":
        return bench_schedulers(args, gtap)
    if args.workload == "fmm_dtt":
        return bench_fmm_dtt(args, gtap)
    if args.workload == "cilksort":
        return bench_cilksort(args, gtap)

    return bench_one(args, gtap)


if __name__ == "__main__":
    sys.exit(main())
