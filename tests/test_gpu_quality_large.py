"""Final-layout quality of the lock-free GPU path at the workload sizes, against
the oracle's references (tests/golden/quality_*.json, written by
tests/golden/make_quality_golden.py from the oracle only): mean NP and SI
over the reference's seeds within 0.01 absolute of the oracle's lock-free
bundle scheme (Sec. 3.4) on the same seeded node samples, and within 0.02 of
serial Algorithm 1 where that is available, each beyond the sampling error of
the means, from the seeded uniform start and from the Pivot MDS start."""
import json
import os

import numpy as np
import pytest

import synthgraph as S
from oracle import metrics as M

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _mean(runs, key):
    return float(np.mean([r[key] for r in runs]))


def _var_of_mean(runs, key, fallback):
    """Sampling variance of the mean over seeds (a single run borrows the
    other side's per-seed variance)."""
    v = [r[key] for r in runs]
    s2 = float(np.var(v, ddof=1)) if len(v) > 1 else fallback
    return s2 / len(v), s2


def _allowance(got, ref, key, bar):
    """bar + 2.5 standard errors of the difference of the two means."""
    vg, sg = _var_of_mean(got, key, 0.0)
    vr, _ = _var_of_mean(ref, key, sg)
    return bar + 2.5 * float(np.sqrt(vg + vr))


def _check(name, maker, serial=None):
    """Lock-free layouts vary from run to run, and the paper reports the mean
    of five runs of each stochastic method (Sec. 5.1).  The GPU runs every
    seed the reference holds (five on the 4M-node graph) and the means are
    compared: within 0.01 of the reference (the oracle's own lock-free scheme
    where one is given) and within 0.02 of serial Algorithm 1 when that is
    given too, each widened by 2.5 standard errors of the difference of the
    means, so that a true difference at the bar does not fail by chance."""
    ref = json.load(open(os.path.join(GOLDEN, f"quality_{name}.json")))
    g = S.cached(ref.get("graph", name), maker)
    init = SL.LAYOUT_INIT_PMDS if ref.get("init") == "pmds" else SL.LAYOUT_INIT_UNIFORM
    got = []
    for run in ref["runs"]:
        with SL.Layout(g.row_ptr, g.col, g.n, k=ref["k"], epochs=ref["epochs"], seed=run["seed"],
                       init_mode=init) as L:
            L.run()
            Y = L.positions()
            info = L.info()
        assert np.all(np.isfinite(Y))
        got.append({"np": M.np_score(g.row_ptr, g.col, Y, sample=ref["np_sample"],
                                     seed=ref["metric_seed"]),
                    "si": M.si_score(Y, g.labels, sample=ref["si_sample"],
                                     seed=ref["metric_seed"])})
    ser = None
    if serial:
        ser = json.load(open(os.path.join(GOLDEN, f"quality_{serial}.json")))
    for key in ("np", "si"):
        gpu, orc = _mean(got, key), _mean(ref["runs"], key)
        allow = _allowance(got, ref["runs"], key, 0.01)
        line = (f"{name}: {key} gpu {gpu:.4f} oracle {orc:.4f} (difference {gpu - orc:+.4f}, "
                f"allowed {allow:.4f}; {len(got)} seeds, engine {info['engine']}, "
                f"grid {info['grid_blocks']})")
        if ser:
            line += f", serial Algorithm 1 {_mean(ser['runs'], key):.4f}"
        print(line, flush=True)
        assert abs(gpu - orc) <= allow, (key, got, ref["runs"])
        if ser:
            allow_s = _allowance(got, ser["runs"], key, 0.02)
            assert abs(gpu - _mean(ser["runs"], key)) <= allow_s, (key, got, ser["runs"])


def test_quality_orkut_like_259k():
    _check("orkut-like-259k-lockfree", S.orkut_like, serial="orkut-like-259k")


def test_quality_lj_like_4m():
    _check("lj-like-4m", S.lj_like)


def test_quality_orkut_like_259k_from_pmds():
    """From the Pivot MDS start of Sec. 4.1 (the oracle starts from its own
    PMDS layout, which may differ from the device's by a rotation)."""
    _check("orkut-like-259k-pmds-lockfree", S.orkut_like, serial="orkut-like-259k-pmds")


def test_quality_lj_like_4m_from_pmds():
    _check("lj-like-4m-pmds", S.lj_like)
