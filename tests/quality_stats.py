"""Comparison of lock-free layout quality between two configurations.

Lock-free runs are not bit-reproducible, so each configuration is run on the
same seeds and the per-seed differences are compared: the mean difference of
NP and of SI must lie within 0.01 absolute (the paper averages five runs of
each stochastic method, Sec. 4.1).  The standard error of that mean is
reported with every comparison, so that a failure shows whether the gap or
the seed spread is large."""
import numpy as np

BAR = 0.01


def paired_gap(a, b):
    """Mean of a - b over paired seeds and its standard error."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    mean = float(d.mean())
    se = float(d.std(ddof=1) / np.sqrt(d.size)) if d.size > 1 else 0.0
    return mean, se


def assert_paired_close(qa, qm, keys=("np", "si"), label=None, bar=BAR):
    for key in keys:
        mean, se = paired_gap([x[key] for x in qa], [x[key] for x in qm])
        print(f"paired {label} {key}: mean difference {mean:+.4f} (se {se:.4f}, "
              f"{len(qa)} seeds, bar {bar})", flush=True)
        assert abs(mean) <= bar, (label, key, mean, se, qa, qm)
