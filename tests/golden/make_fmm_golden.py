"""Write tests/golden/fmm_plummer_1m.txt: direct-summation and oracle-FMM
potentials at 4,096 sampled targets of the 10^6-point Plummer input (seed 3,
leaf 64, theta 1/2, order 6).  Calls only the CPU oracle and the input
generator; takes about a minute on one core."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import points  # noqa: E402

N, SEED, NT, TSEED = 1000000, 3, 4096, 29


def main():
    x, y, z, q = points.plummer(N, SEED)
    tg = np.sort(np.random.default_rng(TSEED).choice(N, NT, replace=False))
    t0 = time.time()
    d = oracle.direct(x, y, z, q, tg)
    t1 = time.time()
    f = oracle.fmm(x, y, z, q, targets=tg)
    t2 = time.time()
    out = os.path.join(HERE, "fmm_plummer_1m.txt")
    with open(out, "w") as fh:
        fh.write("# FMM potentials at 4,096 sampled targets of 10^6 Plummer points (seed 3), leaf 64,\n")
        fh.write("# theta 1/2, Cartesian order 6.  Written by make_fmm_golden.py from the CPU oracle:\n")
        fh.write("# direct = sum over j != i of q_j / |x_i - x_j|; fmm = the oracle FMM at the target.\n")
        fh.write(f"# targets drawn with numpy default_rng({TSEED}).choice(N, {NT}, replace=False), sorted\n")
        st = f.stats
        fh.write(f"# lists: m2l_pairs {st['m2l_pairs']} p2p_pairs {st['p2p_pairs']} m2l_hash {st['m2l_hash']} "
                 f"p2p_hash {st['p2p_hash']} n_cells {st['n_cells']} n_leaves {st['n_leaves']}\n")
        fh.write("# index direct fmm\n")
        for i, a, b in zip(tg, d, f.phi):
            fh.write(f"{int(i)} {float(a)!r} {float(b)!r}\n")
    print(f"direct {t1 - t0:.1f}s, fmm {t2 - t1:.1f}s -> {out}")


if __name__ == "__main__":
    main()
