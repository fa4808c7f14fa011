"""Write the CPU oracle's result for every job of the batched-serving trace.

The trace is synth.serving.serving_mix(20000, 5): 60 % k-clique jobs (k in
4..8) on subgraphs induced by s vertices (log-uniform in [1e3, 2e5]) of the
seeded n=10^6, mean degree 40, exponent 2.1, cap 0.6 Chung-Lu graph, and 40 %
unbalanced tree search jobs (mean branching m in [2, 4], depth 8..14).  Only
oracle/ and synth/ are called: oracle.kclique (the plain recursion) for the
k-clique jobs and oracle.uts for the trees, on a pool of threads (the oracle
is C behind ctypes, so the threads run in parallel).

Output: tests/golden/serving_trace_s5.txt, one line per job
    index kind parameter result
(parameter = k for k-clique jobs, the depth limit for trees), after a header
with the graph checksum and a hash of the job specs.

usage: python tests/golden/make_serving_golden.py [--jobs 20000] [--seed 5] [--threads 8]
"""
import argparse
import concurrent.futures as cf
import hashlib
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import graphs, serving  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def spec_hash(specs) -> str:
    h = hashlib.sha256()
    for sp in specs:
        h.update(repr(sp).encode())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    t0 = time.time()
    g = graphs.chung_lu(1000000, 40, 2.1, 0.6, 2)
    specs = serving.serving_mix(args.jobs, args.seed)
    kc = [i for i, sp in enumerate(specs) if sp.kind == "kclique"]
    subs = graphs.induced_many(g, [(specs[i].s, specs[i].sub_seed) for i in kc], threads=args.threads)
    sub_of = dict(zip(kc, subs))
    print(f"graph and {len(kc)} subgraphs ready in {time.time() - t0:.1f} s", flush=True)

    def one(i):
        sp = specs[i]
        if sp.kind == "kclique":
            h = sub_of[i]
            return i, oracle.kclique(h.row_ptr, h.col, sp.k).value
        return i, oracle.uts(sp.seed, oracle.uts_threshold(sp.m), sp.depth).value

    res = [None] * len(specs)
    # largest trees first, so that the pool ends with small jobs
    order = sorted(range(len(specs)), key=lambda i: -(specs[i].m ** specs[i].depth if specs[i].kind == "uts"
                                                    else sub_of[i].col.size))
    done = 0
    with cf.ThreadPoolExecutor(max_workers=max(1, args.threads)) as ex:
        for i, v in ex.map(one, order):
            res[i] = v
            done += 1
            if done % 2000 == 0:
                print(f"{done} jobs ({time.time() - t0:.1f} s)", flush=True)
    out = os.path.join(HERE, f"serving_trace_s{args.seed}.txt")
    with open(out, "w") as fh:
        fh.write(f"# serving_mix({args.jobs}, {args.seed}) specs {spec_hash(specs)} graph "
                 f"n1000000_d40_g2.1_cap0.6_s2 {g.checksum()}\n")
        fh.write("# index kind k|depth result  (oracle.kclique / oracle.uts)\n")
        for i, sp in enumerate(specs):
            fh.write(f"{i} {sp.kind} {sp.k if sp.kind == 'kclique' else sp.depth} {res[i]}\n")
    print(f"wrote {out} in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
