"""Comparison of lock-free layout quality between two configurations.

Lock-free runs are not bit-reproducible, so each configuration is run on the
same seeds and the per-seed differences are compared.  The bar is 0.01 on
the mean difference, widened by 2.5 standard errors of that mean, so that a
true difference at 0.01 does not fail by chance (the paper averages five
runs of each stochastic method, Sec. 5.1; a gap well beyond 0.01 still
fails)."""
import numpy as np


def paired_gap(a, b):
    """Mean of a - b over paired seeds and the bar it is held to."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    mean = float(d.mean())
    se = float(d.std(ddof=1) / np.sqrt(d.size)) if d.size > 1 else 0.0
    return mean, 0.01 + 2.5 * se


def assert_paired_close(qa, qm, keys=("np", "si"), label=None):
    for key in keys:
        mean, bar = paired_gap([x[key] for x in qa], [x[key] for x in qm])
        assert abs(mean) <= bar, (label, key, mean, bar, qa, qm)
