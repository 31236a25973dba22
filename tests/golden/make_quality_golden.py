"""Writes the oracle's layout-quality references for the large workloads.

Calls only the oracle (and the seeded input generators): the serial FP64
Algorithm 1 for the 259k-node graph, the FP64 threaded bundle scheme of
Sec. 3.4 for the 4M-node graph (a serial run takes too long; the paper reports
the parallel and serial variants within a few percent of each other, Sec. 4.3),
and both for the 259k-node graph (the "-lockfree" entries).
The "-pmds" entries start from the oracle's Pivot MDS layout (the initial
layout of Sec. 4.1, oracle/pmds.py, 50 pivots) instead of the seeded uniform
draws.  NP and SI are measured on seeded node samples; the GPU tests use the
same samples.  Every entry holds five seeds, as the paper averages five runs
of each stochastic method (Sec. 4.1).  Usage:  python tests/golden/make_quality_golden.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synthgraph as S  # noqa: E402
from oracle import metrics as M  # noqa: E402
from oracle import oracle as O  # noqa: E402
from oracle import pmds as P  # noqa: E402

PLAN = {
    # name: (graph, maker, k, T, runner, seeds, init)
    "orkut-like-259k": ("orkut-like-259k", "orkut_like", 5, 30, "serial", (0, 1, 2, 3, 4),
                        "uniform"),
    "lj-like-4m": ("lj-like-4m", "lj_like", 5, 30, "threaded", (0, 1, 2, 3, 4), "uniform"),
    "orkut-like-259k-pmds": ("orkut-like-259k", "orkut_like", 5, 30, "serial", (0, 1, 2, 3, 4),
                             "pmds"),
    "lj-like-4m-pmds": ("lj-like-4m", "lj_like", 5, 30, "threaded", (0, 1, 2, 3, 4), "pmds"),
    # the paper's lock-free scheme (Sec. 3.4) on the 259k-node graph: the
    # reference for lock-free layouts, next to serial Algorithm 1 above
    "orkut-like-259k-lockfree": ("orkut-like-259k", "orkut_like", 5, 30, "threaded",
                                 (0, 1, 2, 3, 4), "uniform"),
    "orkut-like-259k-pmds-lockfree": ("orkut-like-259k", "orkut_like", 5, 30, "threaded",
                                      (0, 1, 2, 3, 4), "pmds"),
}
NP_SAMPLE, SI_SAMPLE, METRIC_SEED = 2000, 10000, 12345


def main(names):
    for name in names:
        graph, maker, k, T, runner, seeds, init = PLAN[name]
        g = S.cached(graph, getattr(S, maker))
        runs = []
        for seed in seeds:
            t0 = time.time()
            Y0 = P.pmds(g.row_ptr, g.col, g.n, seed) if init == "pmds" else None
            if runner == "serial":
                Y = O.serial_run(g.row_ptr, g.col, g.n, k, T, seed, Y0=Y0)
                desc = "serial Algorithm 1 (shuffled edge order), FP64"
            else:
                threads = os.cpu_count() or 1
                Y = O.threaded_run(g.row_ptr, g.col, g.n, k, T, seed, threads, Y0=Y0)
                desc = f"threaded bundle scheme, FP64, {threads} threads"
            desc += ", from the Pivot MDS layout" if init == "pmds" else ""
            q = {"np": M.np_score(g.row_ptr, g.col, Y, sample=NP_SAMPLE, seed=METRIC_SEED),
                 "si": M.si_score(Y, g.labels, sample=SI_SAMPLE, seed=METRIC_SEED)}
            runs.append({"seed": seed, **q, "seconds": round(time.time() - t0, 1)})
            print(name, seed, q, flush=True)
        out = {"workload": name, "graph": graph, "init": init, "k": k, "epochs": T,
               "eta0": 1.0, "oracle": desc,
               "np_sample": NP_SAMPLE, "si_sample": SI_SAMPLE, "metric_seed": METRIC_SEED,
               "runs": runs}
        with open(os.path.join(HERE, f"quality_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or list(PLAN))
