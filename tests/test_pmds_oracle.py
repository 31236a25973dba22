"""Pins of the Pivot MDS oracle (initial layout of Sec. 4.1) against closed
forms and an independent formulation (CPU only).

* path graph: hop distances are Euclidean on a line, so PMDS recovers the
  line exactly (first axis +-(i - mean), second axis 0, fitted distances
  equal to the hop distances) with any
  number of pivots >= 2, and the max/min pivot order is known in closed form;
* cycle graph with every node a pivot: the two leading eigenvectors of a
  circulant matrix are a cosine/sine pair, so the nodes land on a regular
  polygon (equal radii, equal consecutive distances);
* every node a pivot: PMDS equals classical MDS (eigenvectors of
  B = -1/2 J D^2 J scaled by sqrt(lambda)) up to rotation, reflection and
  the scale fit;
* the component layout is centred; nodes outside the first pivot's component
  take the seeded uniform draws scaled to the layout's extent;
* BFS distances against scipy's shortest paths.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import synthgraph as S
from oracle import oracle as O
from oracle import pmds as P


def _path(n):
    return S.csr_from_pairs(np.arange(n - 1), np.arange(1, n), n)


def _cycle(n):
    u = np.arange(n)
    return S.csr_from_pairs(u, (u + 1) % n, n)


def test_bfs_matches_scipy_shortest_paths():
    g = S.chung_lu_communities(3000, 9000, tau=2.3, dmax=200.0, n_comm=10, intra=0.9, seed=4)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    for src in (0, 17, int(np.argmax(g.degrees()))):
        ref = shortest_path(A, method="D", unweighted=True, indices=src)
        got = P.bfs_distances(g.row_ptr, g.col, g.n, src)
        ref = np.where(np.isinf(ref), -1, ref).astype(np.int64)
        assert np.array_equal(got, ref)


def test_path_pivot_order_closed_form():
    rp, col = _path(40)
    piv, _ = P.select_pivots(rp, col, 40, 6)
    # node 1 has the largest degree (first of the ties); then the far end;
    # then the middle of [1, 39]; then the first maximiser of min(i-1, 20-i)
    # and min(i-20, 39-i), which tie at 9 for i = 10, 11, 29, 30
    assert list(piv[:4]) == [1, 39, 20, 10]


@pytest.mark.parametrize("p", [2, 5, 40])
def test_path_is_recovered_exactly(p):
    n = 40
    rp, col = _path(n)
    Y, det = P.pmds(rp, col, n, 0, p=p, want_detail=True)
    x = np.arange(n) - (n - 1) / 2
    sgn = np.sign(Y[:, 0] @ x)
    assert np.abs(sgn * Y[:, 0] - x).max() <= 1e-4  # FP32 rounding of the output
    assert np.abs(Y[:, 1]).max() <= 1e-4
    # the fitted layout reproduces every pivot's hop distances
    Yp = Y[det["pivots"]]
    fit = np.linalg.norm(Y[:, None, :] - Yp[None, :, :], axis=2).T
    assert np.abs(fit - det["dist"]).max() <= 1e-4


def test_cycle_is_a_regular_polygon():
    n = 12
    rp, col = _cycle(n)
    Y = P.pmds(rp, col, n, 0, p=n)
    r = np.linalg.norm(Y, axis=1)
    assert (r.max() - r.min()) <= 1e-5 * r.max()
    step = np.linalg.norm(Y - np.roll(Y, 1, axis=0), axis=1)
    assert (step.max() - step.min()) <= 1e-5 * step.max()


def _procrustes_residual(A, B):
    """min over rotation/reflection R and scale c of |A - c B R| / |A|."""
    A = A - A.mean(0)
    B = B - B.mean(0)
    U, sig, Vt = np.linalg.svd(B.T @ A)
    R = U @ Vt
    c = sig.sum() / (B * B).sum()
    return np.linalg.norm(A - c * B @ R) / np.linalg.norm(A)


def test_all_pivots_equals_classical_mds():
    g = S.chung_lu_communities(300, 900, tau=2.3, dmax=40.0, n_comm=4, intra=0.9, seed=2)
    # keep the giant component so that every node can be a pivot
    d0 = P.bfs_distances(g.row_ptr, g.col, g.n, int(np.argmax(g.degrees())))
    keep = np.flatnonzero(d0 >= 0)
    remap = -np.ones(g.n, dtype=np.int64)
    remap[keep] = np.arange(keep.size)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    m = (d0[src] >= 0)
    rp, col = S.csr_from_pairs(remap[src[m]], remap[g.col[m]], keep.size)
    n = keep.size
    Y = P.pmds(rp, col, n, 0, p=n)
    X = P.classical_mds(rp, col, n)
    assert _procrustes_residual(X, Y) <= 1e-6


def test_component_centred_and_rest_uniform():
    rp1, col1 = _path(30)
    # nodes 30..39: isolated nodes and one separate edge (38, 39)
    u = np.concatenate([np.arange(29), [38]])
    v = np.concatenate([np.arange(1, 30), [39]])
    rp, col = S.csr_from_pairs(u, v, 40)
    Y, det = P.pmds(rp, col, 40, 7, p=5, want_detail=True)
    comp = det["component"]
    assert comp.sum() == 30 and comp[:30].all()
    assert np.abs(Y[comp].mean(0)).max() <= 1e-4
    R = np.float32(np.abs(Y[comp]).max())
    ref = O.init_positions_scaled(40, 7, R)
    assert np.array_equal(Y[~comp], ref[~comp])


def test_power_law_layout_is_centred_and_spread():
    g = S.chung_lu_communities(5000, 20000, tau=2.2, dmax=300.0, n_comm=8, intra=0.9, seed=5)
    Y, det = P.pmds(g.row_ptr, g.col, g.n, 1, p=20, want_detail=True)
    comp = det["component"]
    assert len(det["pivots"]) == 20 and len(set(det["pivots"].tolist())) == 20
    c = Y[comp]
    assert np.abs(c.mean(0)).max() <= 1e-3 * np.abs(c).max()
    lam = det["eigenvalues"]
    assert lam[0] >= lam[1] >= lam[2] >= 0
