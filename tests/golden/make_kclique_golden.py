"""Write the CPU oracle's k-clique counts for the seeded Chung-Lu graphs.

Only oracle/ (and the seeded input generator) are called.  Output:
tests/golden/kclique_chung_lu.txt with one line per (graph, k): the graph's
parameters and checksum, the count and the oracle's task counts.

usage: python tests/golden/make_kclique_golden.py [--large]
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import graphs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kclique_chung_lu.txt")

GRAPHS = {
    "n2000_d16_g2.5_cap1.0_s1": (2000, 16, 2.5, 1.0, 1, (3, 4, 5, 6)),
    "n1000000_d40_g2.1_cap0.6_s2": (1000000, 40, 2.1, 0.6, 2, (3, 4, 5, 6, 7)),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--large", action="store_true", help="also the n=10^6 graph (hours of CPU for k=7)")
    args = ap.parse_args()
    lines = ["# graph checksum k count tasks conts  (oracle.kclique, range_leaf 64)\n"]
    for name, (n, d, g, cap, seed, ks) in GRAPHS.items():
        if n > 10000 and not args.large:
            continue
        G = graphs.chung_lu(n, d, g, cap, seed)
        for k in ks:
            t = time.time()
            r = oracle.kclique(G.row_ptr, G.col, k)
            lines.append(f"{name} {G.checksum()} {k} {r.value} {r.tasks} {r.conts}\n")
            print(lines[-1].strip(), f"({time.time() - t:.1f} s)", flush=True)
            with open(OUT, "w") as fh:
                fh.writelines(lines)


if __name__ == "__main__":
    main()
