"""Clustering quality (CQ, Sec. 4.1) on the GPU against the oracle's k-means.

* k-means++ start: the chosen points equal the oracle's (same counter-based
  draws; the running D^2 sums are FP64 on both sides, in different summation
  orders, which could move a pick only when a target falls within rounding of
  a boundary);
* Lloyd's iterations from the same centers: identical assignments and pass
  counts (FP64 squared distances without contraction on both sides, lowest
  index on ties);
* the ARI equals the oracle's definition applied to the device's clusters;
* the whole CQ equals the oracle's cq_kmeans;
* coincident points, one cluster, argument errors, and the 4M-node graph
  (time printed).
"""
import time

import numpy as np
import pytest

import synthgraph as S
from oracle import metrics as M

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


@pytest.fixture(scope="module")
def d1():
    return S.sbm_2000(0)


@pytest.fixture(scope="module")
def pl20k():
    return S.chung_lu_communities(20_000, 160_000, tau=2.2, dmax=1500.0, n_comm=20, intra=0.9,
                                  seed=3)


def _layout_after(g, epochs, seed=1):
    L = SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=30, seed=seed)
    if epochs:
        L.run(epochs)
    return L


@pytest.mark.parametrize("which,epochs,seed", [("d1", 0, 3), ("d1", 30, 4), ("pl20k", 10, 5)])
def test_kmeans_pp_and_lloyd_match_oracle(which, epochs, seed, d1, pl20k):
    g = {"d1": d1, "pl20k": pl20k}[which]
    with _layout_after(g, epochs) as L:
        Y = L.positions()
        K = int(np.unique(g.labels).size)
        cq, assign, iters, centers = L.cluster_quality(g.labels, seed=seed)
        # Lloyd alone, from the oracle's own start
        ref_c = M.kmeans_pp(Y, K, seed)
        cq2, assign2, iters2, c2 = L.cluster_quality(g.labels, init_centers=Y[ref_c])
    assert np.array_equal(centers, ref_c)
    assert np.all(c2 == -1)
    ref_a, _, ref_it = M.kmeans_lloyd(Y, Y[ref_c], 300)
    assert np.array_equal(assign2, ref_a) and iters2 == ref_it
    assert np.array_equal(assign, ref_a) and iters == ref_it
    assert abs(cq - M.ari(g.labels, assign)) <= 1e-12
    assert abs(cq - M.cq_kmeans(Y, g.labels, seed)) <= 1e-12
    assert cq2 == cq


def test_cq_edge_cases(d1):
    # every point in one place: D^2 is 0 after the first center (fallback
    # picks), all distances tie (cluster 0), one cluster against 4 labels
    Y0 = np.zeros((d1.n, 2), np.float32)
    with SL.Layout(d1.row_ptr, d1.col, d1.n, k=5, epochs=3, seed=1, init_pos=Y0) as L:
        cq, assign, iters, centers = L.cluster_quality(d1.labels, seed=2)
        assert np.array_equal(centers, M.kmeans_pp(Y0, 4, 2))
        assert np.all(assign == 0) and iters == 2
        assert cq == M.ari(d1.labels, assign) == 0.0
    with _layout_after(d1, 10) as L:
        cq1, a1, _, _ = L.cluster_quality(d1.labels, clusters=1)
        assert np.all(a1 == 0) and cq1 == 0.0
        # labels all equal and one cluster: identical trivial partitions
        one = np.zeros(d1.n, np.int32)
        assert L.cluster_quality(one, clusters=1)[0] == 1.0
        for kw in ({"clusters": d1.n + 1}, {"clusters": 5000}, {"max_iter": 0}):
            with pytest.raises(SL.LayoutError) as ei:
                L.cluster_quality(d1.labels, **kw)
            assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
    with SL.Layout(d1.row_ptr, d1.col, d1.n, k=5, epochs=3, dim=3) as L:
        with pytest.raises(SL.LayoutError) as ei:
            L.cluster_quality(d1.labels)
        assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED


def test_cq_on_the_4m_graph():
    """Full-size CQ (500 clusters over 4M nodes): the device ARI equals the
    oracle's ARI of the device's clusters; time printed."""
    g = S.cached("lj-like-4m", S.lj_like)
    with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=30, seed=0) as L:
        L.run()
        t0 = time.perf_counter()
        cq, assign, iters, centers = L.cluster_quality(g.labels, seed=0, max_iter=100)
        dt = time.perf_counter() - t0
    print(f"CQ of the 4M-node layout: {cq:.4f} ({iters} passes, {dt:.2f} s)", flush=True)
    assert 0.0 < cq <= 1.0 and np.unique(centers).size == centers.size
    assert abs(cq - M.ari(g.labels, assign)) <= 1e-9
