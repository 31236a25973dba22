"""Pivot MDS initial layout on the GPU against the FP64 oracle (Sec. 4.1).

* pivots and hop distances: bit-exact (integer work);
* positions: what PMDS fixes is the component's layout up to a
  rotation/reflection of the two eigen-axes (eigenvector signs, and any
  rotation inside a repeated eigenvalue), so the comparison is on invariants:
  all pairwise distances of a sample of component nodes, relative to the
  layout's extent, within 1e-3 (FP32 distances
  in C and FP32 products in C^T C against FP64; the test graphs have a clear
  gap between the second and third eigenvalue, checked first);
* nodes outside the first pivot's component: the seeded uniform draws in
  [-R, R]^2, compared within FP32 rounding of R;
* a layout run from the PMDS start keeps the oracle's quality (NP, SI within
  0.01 of the serial oracle run from the oracle's own PMDS start).
"""
import numpy as np
import pytest

import synthgraph as S
from oracle import metrics as M
from oracle import oracle as O
from oracle import pmds as P

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


def _path(n):
    return S.csr_from_pairs(np.arange(n - 1), np.arange(1, n), n)


def _grid(a, b):
    idx = np.arange(a * b).reshape(a, b)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return S.csr_from_pairs(u, v, a * b)


def _pair_dist_err(Y, R, sample, seed=0):
    rng = np.random.default_rng(seed)
    idx = rng.choice(Y.shape[0], size=min(sample, Y.shape[0]), replace=False)
    dy = np.linalg.norm(Y[idx][:, None] - Y[idx][None], axis=2)
    dr = np.linalg.norm(R[idx][:, None] - R[idx][None], axis=2)
    extent = np.abs(R).max()
    return np.abs(dy - dr).max() / extent


def _graphs():
    g1 = S.chung_lu_communities(20_000, 120_000, tau=2.2, dmax=1500.0, n_comm=12, intra=0.9,
                                seed=3)
    rp, col = _grid(60, 25)
    g2 = S.Graph(rp, col, 1500, np.zeros(1500, np.int32), "grid60x25")
    rp, col = _path(300)
    g3 = S.Graph(rp, col, 300, np.zeros(300, np.int32), "path300")
    return [g1, g2, g3]


@pytest.fixture(scope="module")
def graphs():
    return _graphs()


@pytest.mark.parametrize("which,pivots", [(0, 50), (0, 7), (1, 50), (2, 64), (1, 1)])
def test_pmds_matches_oracle(graphs, which, pivots):
    g = graphs[which]
    Y, piv, dist = SL.layout_pmds(g.row_ptr, g.col, g.n, pivots, seed=3, want_detail=True)
    R, det = P.pmds(g.row_ptr, g.col, g.n, 3, p=pivots, want_detail=True)
    assert np.array_equal(piv, det["pivots"])
    assert np.array_equal(dist, det["dist"])
    assert np.all(np.isfinite(Y))
    lam = det["eigenvalues"]
    if pivots > 1 and lam[1] > 1e-6 * lam[0]:
        assert lam[1] - lam[2] > 1e-3 * lam[0], lam  # the 2D subspace is well separated
    # the component is fixed up to a rotation/reflection; nodes outside it
    # keep their seeded draws, which do not turn with it
    comp = det["component"]
    assert _pair_dist_err(Y[comp].astype(np.float64), R[comp], 1500) <= 1e-3
    if (~comp).any():
        Rg = np.float32(np.abs(Y[comp]).max())
        ref = O.init_positions_scaled(g.n, 3, Rg)
        assert np.array_equal(Y[~comp].astype(np.float64), ref[~comp])


def test_pmds_components_and_rest(graphs):
    # a 30-node path, isolated nodes 30..37, and a separate edge (38, 39)
    u = np.concatenate([np.arange(29), [38]])
    v = np.concatenate([np.arange(1, 30), [39]])
    rp, col = S.csr_from_pairs(u, v, 40)
    Y, piv, dist = SL.layout_pmds(rp, col, 40, 5, seed=7, want_detail=True)
    R, det = P.pmds(rp, col, 40, 7, p=5, want_detail=True)
    assert np.array_equal(piv, det["pivots"]) and np.array_equal(dist, det["dist"])
    comp = det["component"]
    assert _pair_dist_err(Y[comp].astype(np.float64), R[comp], 30) <= 1e-4
    Rg = np.float32(np.abs(Y[comp]).max())
    ref = O.init_positions_scaled(40, 7, Rg)
    assert np.array_equal(Y[~comp].astype(np.float64), ref[~comp])


def test_pmds_edge_cases():
    # no edges: the first pivot (node 0) is alone, everything else uniform in [-1, 1]^2
    rp = np.zeros(6, dtype=np.int32)
    Y, piv, dist = SL.layout_pmds(rp, np.zeros(0, np.int32), 5, 4, seed=2, want_detail=True)
    assert list(piv) == [0] and np.array_equal(dist[0], [0, -1, -1, -1, -1])
    assert np.array_equal(Y[0], [0.0, 0.0])
    ref = O.init_positions_scaled(5, 2, 1.0)
    assert np.array_equal(Y[1:].astype(np.float64), ref[1:])
    # one node
    Y = SL.layout_pmds(np.zeros(2, np.int32), np.zeros(0, np.int32), 1, 0, seed=1)
    assert Y.shape == (1, 2) and np.array_equal(Y[0], [0.0, 0.0])
    # bad arguments and a bad graph
    with pytest.raises(SL.LayoutError) as ei:
        SL.layout_pmds(rp, np.zeros(0, np.int32), 5, 65)
    assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
    with pytest.raises(SL.LayoutError) as ei:
        SL.layout_pmds(np.array([0, 1, 1], np.int32), np.array([1], np.int32), 2, 4)
    assert ei.value.code == SL.LAYOUT_E_BAD_GRAPH


def test_layout_from_pmds_start_keeps_oracle_quality():
    g = S.sbm_2000(0)
    T, seed = 50, 4
    Y0 = P.pmds(g.row_ptr, g.col, g.n, seed)
    ref = O.serial_run(g.row_ptr, g.col, g.n, 5, T, seed, Y0=Y0)
    with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=T, seed=seed,
                   init_mode=SL.LAYOUT_INIT_PMDS) as L:
        start = L.positions()
        # same extent as the oracle's start (the planted blocks make the
        # leading eigenvalues nearly equal, so the axes themselves may rotate)
        ext_g, ext_o = np.abs(start).max(), np.abs(Y0).max()
        assert abs(ext_g - ext_o) <= 0.05 * ext_o
        L.run()
        Y = L.positions()
    qa = M.quality(g.row_ptr, g.col, ref, g.labels, sample=2000)
    qg = M.quality(g.row_ptr, g.col, Y, g.labels, sample=2000)
    assert abs(qa["np"] - qg["np"]) <= 0.01 and abs(qa["si"] - qg["si"]) <= 0.01, (qa, qg)
