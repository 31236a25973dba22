"""Replicas merged by summed deltas (the natural way to split one graph over
several devices or XCDs), studied with the oracle on the CPU.

Each of R replicas runs the serial update (Algorithm 1) over its own share
of the rows from the same starting positions, and the replicas' position
changes are then summed into one layout.  With one merge per epoch the early
steps (eta near 1, where one attraction moves a node most of the way to its
neighbour) are summed R times over and the layout collapses; with merges
every 1/m of an epoch, so that only about n/4 edges are processed between
merges, the final quality matches the serial run.  The library therefore
keeps one replica per graph and bounds its lanes in flight instead.
"""
import numpy as np
import pytest

import synthgraph as S
from oracle import metrics as M
from oracle import oracle as O

T, K, SEED = 30, 5, 0


def _rows(rp, col, lo, hi):
    deg = np.diff(rp)
    deg[:lo] = 0
    deg[hi:] = 0
    r2 = np.zeros_like(rp)
    r2[1:] = np.cumsum(deg)
    return r2.astype(np.int32), col[rp[lo]:rp[hi]].copy()


def _replicated(g, R, m):
    rp = g.row_ptr.astype(np.int64)
    n = g.n
    Y = O.init_positions(n, SEED).reshape(n, 2)
    B = R * m
    cuts = [0] + [int(np.searchsorted(rp, g.nnz * b // B)) for b in range(1, B)] + [n]
    parts = [_rows(rp, g.col, cuts[b], cuts[b + 1]) for b in range(B)]
    for t in range(T):
        for u in range(m):
            step = np.zeros_like(Y)
            for x in range(R):
                r2, c2 = parts[u * R + x]
                Yx = O.serial_run(r2, c2, n, K, T, SEED + 1000 * (u * R + x), Y0=Y.copy(),
                                  t_begin=t, t_end=t + 1)
                step += Yx.reshape(n, 2) - Y
            Y = Y + step
    return Y


@pytest.fixture(scope="module")
def graph():
    return S.chung_lu_communities(10_000, 80_000, tau=2.2, dmax=1000.0, n_comm=10, intra=0.9,
                                  seed=3)


@pytest.fixture(scope="module")
def serial_quality(graph):
    g = graph
    Y = O.serial_run(g.row_ptr, g.col, g.n, K, T, SEED).reshape(g.n, 2)
    return M.quality(g.row_ptr, g.col, Y, g.labels)


def test_one_merge_per_epoch_collapses_the_layout(graph, serial_quality):
    g = graph
    q = M.quality(g.row_ptr, g.col, _replicated(g, 8, 1), g.labels)
    print("serial", serial_quality, "8 replicas, one merge per epoch", q)
    assert q["si"] < serial_quality["si"] - 0.3


def test_frequent_merges_match_the_serial_layout(graph, serial_quality):
    g = graph
    m = 2 * g.nnz // g.n  # about n/2 directed edges between merges
    q = M.quality(g.row_ptr, g.col, _replicated(g, 8, m), g.labels)
    print("serial", serial_quality, f"8 replicas, {m} merges per epoch", q)
    assert abs(q["si"] - serial_quality["si"]) <= 0.02
    assert abs(q["np"] - serial_quality["np"]) <= 0.01
