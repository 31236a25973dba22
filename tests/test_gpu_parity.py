"""GPU parity of the HIP path against the FP64 oracle (called through the C ABI).

Bars (from the method's requirements):
* initial positions and sampled negatives: bit-exact;
* one synchronous (Jacobi) epoch from identical positions: max error within
  1e-5 x the diameter (bounding-box diagonal) of the oracle's output;
* one epoch run by a single lane (no concurrency) against the serial oracle in
  the same visiting order: same trajectory within FP32 rounding;
* final lock-free layouts: NP and SI within 0.01 of the serial oracle's.
"""
import math

import numpy as np
import pytest

import synthgraph as S
from oracle import oracle as O
from oracle import metrics as M

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


def _diam(Y):
    return float(np.linalg.norm(Y.max(0) - Y.min(0)))


@pytest.fixture(scope="module")
def d1():
    return S.sbm_2000(0)


@pytest.fixture(scope="module")
def pl20k():
    """A 20k-node power-law community graph (several thousand chunks, hubs)."""
    return S.chung_lu_communities(20_000, 160_000, tau=2.2, dmax=1500.0, n_comm=20, intra=0.9,
                                  seed=3)


def _layout(g, k=5, epochs=50, seed=0, **kw):
    return SL.Layout(g.row_ptr, g.col, g.n, k=k, epochs=epochs, seed=seed, **kw)


# ------------------------------------------------------------ bit-exact
@pytest.mark.parametrize("n,seed", [(2000, 0), (777, 5), (1, 3), (100_003, 11)])
def test_init_positions_bit_exact(n, seed):
    rp = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(0, dtype=np.int32)
    with SL.Layout(rp, col, n, k=5, epochs=1, seed=seed) as L:
        Y = L.positions()
    ref = O.init_positions(n, seed).astype(np.float32)
    assert np.array_equal(Y.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("k", [1, 3, 5, 8])
def test_draws_bit_exact_d1(d1, k):
    with _layout(d1, k=k, epochs=50, seed=7) as L:
        for t in (0, 1, 49):
            got = L.draws(t)
            ref = O.draw_negatives(d1.row_ptr, d1.col, d1.n, k, t, 7)
            assert np.array_equal(got, ref), (k, t)


def test_draws_bit_exact_power_law(pl20k):
    with _layout(pl20k, k=5, epochs=30, seed=123) as L:
        for t in (0, 17):
            assert np.array_equal(L.draws(t),
                                  O.draw_negatives(pl20k.row_ptr, pl20k.col, pl20k.n, 5, t, 123))


def test_draws_two_nodes():
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    with SL.Layout(rp, col, 2, k=8, epochs=3, seed=1) as L:
        d = L.draws(2)
    assert np.array_equal(d, np.array([[1] * 8, [0] * 8]))


# ---------------------------------------------------------------- Jacobi
def _jacobi_check(g, k, seed, eta0, t=0, T=30, gamma=2.0):
    Y0 = O.init_positions(g.n, seed).astype(np.float32)
    ref, absd = O.jacobi_epoch(g.row_ptr, g.col, g.n, k, t, T, seed, Y0.astype(np.float64),
                               eta0=eta0, gamma=gamma, want_abs=True)
    with _layout(g, k=k, epochs=T, seed=seed, update_mode=SL.LAYOUT_JACOBI, eta0=eta0,
                 gamma=gamma, engine=SL.LAYOUT_ENGINE_GLOBAL, init_pos=Y0, start_epoch=t) as L:
        L.run(1)
        Y = L.positions().astype(np.float64)
    err = np.abs(Y - ref).max()
    tol = 1e-5 * _diam(ref)
    return err, tol


def test_jacobi_epoch_d1_eta1(d1):
    err, tol = _jacobi_check(d1, 5, 0, 1.0)
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("gamma", [1.5, 3.0])
def test_jacobi_epoch_general_gamma(d1, gamma):
    """Repulsion exponents other than the t-FDP row's 2 (the pow path)."""
    err, tol = _jacobi_check(d1, 5, 6, 1.0, gamma=gamma)
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("t", [0, 13])
def test_jacobi_epoch_power_law(pl20k, t):
    dmax = int(pl20k.degrees().max())
    err, tol = _jacobi_check(pl20k, 5, 2, 1.0 / dmax, t=t)
    assert err <= tol, (err, tol)


# ------------------------------------------------- single-lane trajectory
@pytest.mark.parametrize("mode,engine,gamma", [
    (0, 1, 2.0), (1, 1, 2.0), (0, 2, 2.0), (1, 2, 2.0), (0, 1, 3.0), (1, 2, 1.5), (0, 3, 2.0)])
def test_single_lane_epoch_matches_serial_oracle(d1, mode, engine, gamma):
    """One lane owns every edge (chunk = all edges): the kernel then runs the
    serial algorithm in CSR order; compare with the oracle in that order."""
    seed, T = 4, 50
    Y0 = O.init_positions(d1.n, seed).astype(np.float32)
    ref = O.serial_run(d1.row_ptr, d1.col, d1.n, 5, T, seed, Y0=Y0.astype(np.float64),
                       t_begin=0, t_end=1, order=O.ORDER_CSR, gamma=gamma)
    with _layout(d1, k=5, epochs=T, seed=seed, update_mode=mode, engine=engine, init_pos=Y0,
                 gamma=gamma, bundle_edges=d1.nnz, grid_blocks=1, block_threads=64) as L:
        assert L.info()["n_chunks"] == 1
        L.run(1)
        Y = L.positions().astype(np.float64)
    err = np.abs(Y - ref).max()
    assert err <= 1e-3 * _diam(ref), (err, _diam(ref))


@pytest.mark.parametrize("hot", [1, 12])
def test_single_lane_epoch_with_hot_nodes_matches_serial_oracle(d1, hot):
    """HOGWILD_STORE with the far-end updates of nodes of degree >= hot
    committed as atomic adds of the change (hot = 1: every node): on one lane
    the trajectory is still the serial one, since adding the change to the
    value the lane itself stored differs from storing it by one rounding."""
    seed, T = 4, 50
    Y0 = O.init_positions(d1.n, seed).astype(np.float32)
    ref = O.serial_run(d1.row_ptr, d1.col, d1.n, 5, T, seed, Y0=Y0.astype(np.float64),
                       t_begin=0, t_end=1, order=O.ORDER_CSR)
    with _layout(d1, k=5, epochs=T, seed=seed, update_mode=SL.LAYOUT_HOGWILD_STORE,
                 engine=SL.LAYOUT_ENGINE_GLOBAL, init_pos=Y0, bundle_edges=d1.nnz,
                 grid_blocks=1, block_threads=64, hot_degree=hot) as L:
        assert L.info()["hot_degree"] == hot
        L.run(1)
        Y = L.positions().astype(np.float64)
    err = np.abs(Y - ref).max()
    assert err <= 1e-3 * _diam(ref), (err, _diam(ref))


def test_hot_degree_applies_to_global_store_only(d1):
    for mode, engine in ((SL.LAYOUT_ATOMIC, SL.LAYOUT_ENGINE_GLOBAL),
                         (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_LDS),
                         (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_XCD)):
        with _layout(d1, k=5, epochs=5, update_mode=mode, engine=engine, hot_degree=4) as L:
            assert L.info()["hot_degree"] == 0
    with _layout(d1, k=5, epochs=5, hot_degree=0) as L:  # the default: plain stores only
        assert L.info()["hot_degree"] == 0
    with pytest.raises(SL.LayoutError) as ei:
        _layout(d1, k=5, epochs=5, hot_degree=-1)
    assert ei.value.code == SL.LAYOUT_E_INVALID_ARG


# --------------------------------------------------------- final quality
@pytest.fixture(scope="module")
def d1_oracle_quality(d1):
    Y = O.serial_run(d1.row_ptr, d1.col, d1.n, 5, 50, 0)
    return M.quality(d1.row_ptr, d1.col, Y, d1.labels)


@pytest.mark.parametrize("mode,engine,threads", [
    (SL.LAYOUT_UPDATE_AUTO, SL.LAYOUT_ENGINE_AUTO, 0),
    (SL.LAYOUT_ATOMIC, SL.LAYOUT_ENGINE_GLOBAL, 0),
    (SL.LAYOUT_ATOMIC, SL.LAYOUT_ENGINE_LDS, 0),
    (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_LDS, 64),
    (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_XCD, 0),
    (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_GLOBAL, 0),
])
def test_final_layout_quality_d1(d1, d1_oracle_quality, mode, engine, threads):
    with _layout(d1, k=5, epochs=50, seed=0, update_mode=mode, engine=engine,
                 block_threads=threads) as L:
        L.run()
        Y = L.positions()
    assert np.all(np.isfinite(Y))
    q = M.quality(d1.row_ptr, d1.col, Y, d1.labels)
    assert abs(q["np"] - d1_oracle_quality["np"]) <= 0.01, (q, d1_oracle_quality)
    assert abs(q["si"] - d1_oracle_quality["si"]) <= 0.01, (q, d1_oracle_quality)


def test_xcd_engine_choice_and_limits():
    """Graphs whose positions fit one XCD's L2 and that are too large for LDS
    run on the XCD-local engine by default; it runs HOGWILD_STORE only and
    refuses graphs beyond its 3 MiB position budget."""
    pl50k = S.chung_lu_communities(50_000, 400_000, tau=2.2, dmax=2000.0, n_comm=30, intra=0.9,
                                   seed=6)
    with _layout(pl50k, k=5, epochs=4, seed=1) as L:
        info = L.info()
        assert info["engine"] == SL.LAYOUT_ENGINE_XCD and info["update_mode"] == 0
        Y0 = L.positions()
        L.run()
        Y = L.positions()
    assert np.all(np.isfinite(Y)) and not np.array_equal(Y, Y0)
    with pytest.raises(SL.LayoutError) as ei:
        _layout(pl50k, k=5, epochs=4, engine=SL.LAYOUT_ENGINE_XCD, update_mode=SL.LAYOUT_ATOMIC)
    assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
    n = 400_000
    rp, col = S.csr_from_pairs(np.arange(n - 1), np.arange(1, n), n)
    with pytest.raises(SL.LayoutError) as ei:
        SL.Layout(rp, col, n, k=5, epochs=2, engine=SL.LAYOUT_ENGINE_XCD)
    assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
    # the same graph as ATOMIC falls back to the all-CU global engine
    with _layout(pl50k, k=5, epochs=2, seed=1, update_mode=SL.LAYOUT_ATOMIC) as L:
        assert L.info()["engine"] == SL.LAYOUT_ENGINE_GLOBAL


def test_atomic_mode_conserves_centroid(d1):
    with _layout(d1, k=5, epochs=50, seed=0, update_mode=SL.LAYOUT_ATOMIC,
                 engine=SL.LAYOUT_ENGINE_GLOBAL) as L:
        Y0 = L.positions().astype(np.float64)
        L.run()
        Y = L.positions().astype(np.float64)
    drift = np.abs(Y.mean(0) - Y0.mean(0)).max()
    assert drift < 1e-3, drift


# ------------------------------------------------------ errors and edges
def _bad(rp, col, n):
    with pytest.raises(SL.LayoutError) as ei:
        SL.Layout(np.asarray(rp, np.int32), np.asarray(col, np.int32), n, k=2, epochs=2)
    return ei.value.code


def test_rejects_malformed_graphs():
    assert _bad([0, 1, 1], [1], 2) == SL.LAYOUT_E_BAD_GRAPH            # missing reverse edge
    assert _bad([0, 1, 2], [0, 1], 2) == SL.LAYOUT_E_BAD_GRAPH         # self-loops
    assert _bad([0, 2, 3, 4], [2, 1, 0, 0], 3) == SL.LAYOUT_E_BAD_GRAPH  # unsorted row
    assert _bad([0, 1, 2], [5, 0], 2) == SL.LAYOUT_E_BAD_GRAPH         # column out of range
    assert _bad([1, 1, 2], [1, 0], 2) == SL.LAYOUT_E_BAD_GRAPH         # row_ptr[0] != 0
    assert _bad([0, 2, 1], [1, 1], 2) == SL.LAYOUT_E_BAD_GRAPH         # decreasing row_ptr


def test_rejects_bad_arguments():
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    h = SL.layout_create(rp, col, 2, 2, 5, 3, 0)
    SL.layout_destroy(h)
    for args, code in [((rp, col, 2, 4, 5, 3, 0), SL.LAYOUT_E_UNSUPPORTED),
                       ((rp, col, 2, 2, 9, 3, 0), SL.LAYOUT_E_UNSUPPORTED),
                       ((rp, col, 2, 2, -1, 3, 0), SL.LAYOUT_E_INVALID_ARG),
                       ((rp, col, 2, 2, 5, 0, 0), SL.LAYOUT_E_INVALID_ARG)]:
        with pytest.raises(SL.LayoutError) as ei:
            SL.layout_create(*args)
        assert ei.value.code == code


def test_epochs_run_out_and_resume_is_exact(d1):
    # Jacobi mode is deterministic up to FP32 summation order
    T = 6
    with _layout(d1, k=5, epochs=T, seed=3, update_mode=SL.LAYOUT_JACOBI, eta0=0.2) as L:
        L.run(4)
        mid = L.positions()
        L.run(10)  # only 2 remain
        assert L.status()[0] == T
        end = L.positions()
        with pytest.raises(SL.LayoutError) as ei:
            L.run(1)
        assert ei.value.code == SL.LAYOUT_E_DONE
    with _layout(d1, k=5, epochs=T, seed=3, update_mode=SL.LAYOUT_JACOBI, eta0=0.2,
                 init_pos=mid, start_epoch=4) as L2:
        L2.run()
        end2 = L2.positions()
    assert np.abs(end - end2).max() <= 1e-5 * _diam(end)


def test_empty_and_tiny_graphs():
    # no edges: positions stay at the initial values
    rp = np.zeros(11, dtype=np.int32)
    with SL.Layout(rp, np.zeros(0, np.int32), 10, k=5, epochs=3, seed=2) as L:
        Y0 = L.positions()
        L.run()
        assert np.array_equal(L.positions(), Y0)
    # isolated nodes and k = 0
    rp, col = S.csr_from_pairs(np.array([0, 1]), np.array([1, 2]), 6)
    for k in (0, 5):
        Y0 = O.init_positions(6, 1)
        ref = O.jacobi_epoch(rp, col, 6, k, 0, 4, 1, Y0)
        with SL.Layout(rp, col, 6, k=k, epochs=4, seed=1, update_mode=SL.LAYOUT_JACOBI) as L:
            L.run(1)
            assert np.abs(L.positions() - ref).max() <= 1e-5 * _diam(ref) + 1e-6


def test_ragged_tail_and_bundle_sizes(pl20k):
    """nnz is not a multiple of the chunk length; every bundle size gives the
    same synchronous epoch."""
    g = pl20k
    Y0 = O.init_positions(g.n, 9).astype(np.float32)
    dmax = int(g.degrees().max())
    ref = O.jacobi_epoch(g.row_ptr, g.col, g.n, 3, 0, 10, 9, Y0.astype(np.float64),
                         eta0=1.0 / dmax)
    for b in (1, 7, 16, 61, 1000):
        with _layout(g, k=3, epochs=10, seed=9, update_mode=SL.LAYOUT_JACOBI, eta0=1.0 / dmax,
                     init_pos=Y0, bundle_edges=b) as L:
            L.run(1)
            Y = L.positions()
        assert np.abs(Y - ref).max() <= 1e-5 * _diam(ref), b


# ---------------------------------------------- degree-weighted negatives
@pytest.mark.parametrize("which", ["d1", "pl20k"])
def test_alias_table_and_draws_bit_exact(which, d1, pl20k):
    g = d1 if which == "d1" else pl20k
    thr_o, alias_o = O.alias_build(g.degrees())
    with _layout(g, k=5, epochs=10, seed=31, neg_weights=SL.LAYOUT_NEG_DEGREE) as L:
        thr, alias = SL.layout_debug_alias(L.h, g.n)
        assert np.array_equal(thr, thr_o) and np.array_equal(alias, alias_o)
        for t in (0, 9):
            ref = O.draw_negatives(g.row_ptr, g.col, g.n, 5, t, 31, mode=O.NEG_DEGREE, thr=thr_o,
                                   alias=alias_o)
            assert np.array_equal(L.draws(t), ref)


def test_alias_table_skewed_weights():
    """A star plus a path: one dominant heavy, many lights, chained partial heavies."""
    n = 3000
    u = np.concatenate([np.zeros(1500, dtype=np.int64), np.arange(1500, n - 1)])
    v = np.concatenate([np.arange(1, 1501), np.arange(1501, n)])
    rp, col = S.csr_from_pairs(u, v, n)
    thr_o, alias_o = O.alias_build(np.diff(rp).astype(np.int64))
    with SL.Layout(rp, col, n, k=3, epochs=2, seed=1, neg_weights=SL.LAYOUT_NEG_DEGREE) as L:
        thr, alias = SL.layout_debug_alias(L.h, n)
    assert np.array_equal(thr, thr_o) and np.array_equal(alias, alias_o)


@pytest.mark.parametrize("kind", ["random", "zeros_and_one_heavy", "near_2_32"])
def test_custom_negative_weights_bit_exact(d1, kind):
    """Caller-given integer weights (the flexible negative sampling named as
    future work in the conclusion): alias table and draws bit-exact with the
    oracle's sweep over the same weights, including zero weights, one
    dominant weight (most draws hit it, and its own source rejects) and a
    total just under 2^32."""
    rng = np.random.default_rng(5)
    if kind == "random":
        w = rng.integers(1, 1000, d1.n).astype(np.uint32)
        w[::7] = 0
    elif kind == "zeros_and_one_heavy":
        w = np.zeros(d1.n, np.uint32)
        w[:10] = 1
        w[3] = 100_000
    else:
        w = np.full(d1.n, (2**32 - 1) // d1.n, np.uint32)
    thr_o, alias_o = O.alias_build(w.astype(np.int64))
    with _layout(d1, k=4, epochs=6, seed=3, neg_weights=SL.LAYOUT_NEG_CUSTOM,
                 neg_weight_values=w) as L:
        thr, alias = SL.layout_debug_alias(L.h, d1.n)
        assert np.array_equal(thr, thr_o) and np.array_equal(alias, alias_o)
        for t in (0, 5):
            ref = O.draw_negatives(d1.row_ptr, d1.col, d1.n, 4, t, 3, mode=O.NEG_DEGREE,
                                   thr=thr_o, alias=alias_o)
            assert np.array_equal(L.draws(t), ref)
        L.run()
        assert np.all(np.isfinite(L.positions()))


def test_custom_negative_weights_rejected(d1):
    for w in (np.zeros(d1.n, np.uint32), np.full(d1.n, 2**31, np.uint32)):
        with pytest.raises(SL.LayoutError) as ei:
            _layout(d1, k=4, epochs=2, neg_weights=SL.LAYOUT_NEG_CUSTOM, neg_weight_values=w)
        assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
    with pytest.raises(SL.LayoutError) as ei:
        _layout(d1, k=4, epochs=2, neg_weights=SL.LAYOUT_NEG_CUSTOM)
    assert ei.value.code == SL.LAYOUT_E_INVALID_ARG


def test_jacobi_epoch_degree_weighted(d1):
    thr_o, alias_o = O.alias_build(d1.degrees())
    Y0 = O.init_positions(d1.n, 6).astype(np.float32)
    ref = O.jacobi_epoch(d1.row_ptr, d1.col, d1.n, 5, 0, 20, 6, Y0.astype(np.float64),
                         mode=O.NEG_DEGREE, thr=thr_o, alias=alias_o)
    with _layout(d1, k=5, epochs=20, seed=6, update_mode=SL.LAYOUT_JACOBI, init_pos=Y0,
                 neg_weights=SL.LAYOUT_NEG_DEGREE) as L:
        L.run(1)
        Y = L.positions()
    assert np.abs(Y - ref).max() <= 1e-5 * _diam(ref)


# ------------------------------------------------------------ chunk table
@pytest.mark.parametrize("bundle,hub", [(16, 64), (7, 7), (1, 3), (64, 1000)])
def test_chunk_table_is_row_aligned(pl20k, bundle, hub):
    """Chunks cover [0, nnz) in order; a chunk starts at a row start, or at a
    multiple of `hub` inside a row longer than `hub`; every row starting in a
    bucket [bB, (b+1)B) shares a chunk with the row holding edge bB."""
    g = pl20k
    with _layout(g, k=5, epochs=2, engine=SL.LAYOUT_ENGINE_GLOBAL, bundle_edges=bundle,
                 hub_split_edges=hub) as L:
        begin, src = SL.layout_debug_chunks(L.h)
    rp = g.row_ptr.astype(np.int64)
    assert begin[0] == 0 and begin[-1] == g.nnz
    assert np.all(np.diff(begin) > 0)
    row = np.searchsorted(rp, begin[:-1], side="right") - 1
    assert np.array_equal(row, src)
    deg = np.diff(rp)
    off = begin[:-1] - rp[src]
    assert np.all((off == 0) | ((deg[src] > hub) & (off % hub == 0)))
    # every non-hub row lies inside one chunk
    chunk_of_first = np.searchsorted(begin, rp[:-1], side="right") - 1
    chunk_of_last = np.searchsorted(begin, rp[1:] - 1, side="right") - 1
    nonhub = (deg > 0) & (deg <= hub)
    assert np.all(chunk_of_first[nonhub] == chunk_of_last[nonhub])
    # chunk count: one per B-bucket start row, per hub segment, per row after a hub
    flags = np.zeros(g.n, dtype=bool)
    rows_b = np.searchsorted(rp, np.arange(0, g.nnz, bundle), side="right") - 1
    flags[rows_b] = True
    hubs = np.where(deg > hub)[0]
    flags[hubs] = True
    after = rp[hubs + 1]
    after = after[after < g.nnz]
    flags[np.searchsorted(rp, after, side="right") - 1] = True
    expect = np.where(flags, np.where(deg > hub, (deg + hub - 1) // hub, 1), 0).sum()
    assert begin.size - 1 == expect
