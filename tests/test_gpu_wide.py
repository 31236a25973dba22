"""64-bit row pointers (layout_create64): the paper's full com-friendster shape.

* A small graph through layout_create64 (int64 row_ptr) and through the int32
  entry point give the same chunk table, the same draws, and the same Jacobi
  epoch (within FP32 summation order).
* The full com-friendster shape (65,608,366 nodes, 1.8e9 undirected edges,
  i.e. 3.6e9 directed edges, past int32 offsets), generated on the device:
  the negatives of sampled directed edges, most of them beyond offset 2^31,
  and the initial positions of sampled nodes are bit-exact against the
  oracle; one epoch of the default path keeps every position finite.
"""
import numpy as np
import pytest

import synthgraph as S
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")
torch = pytest.importorskip("torch")


def test_create64_equals_int32_entry():
    g = S.chung_lu_communities(20_000, 160_000, tau=2.2, dmax=1500.0, n_comm=20, intra=0.9,
                               seed=3)
    rp64 = g.row_ptr.astype(np.int64)
    kw = dict(k=5, epochs=20, seed=4, engine=SL.LAYOUT_ENGINE_GLOBAL)
    with SL.Layout(rp64, g.col, g.n, **kw) as A, SL.Layout(g.row_ptr, g.col, g.n, **kw) as B:
        ca, cb = SL.layout_debug_chunks(A.h), SL.layout_debug_chunks(B.h)
        assert np.array_equal(ca[0], cb[0]) and np.array_equal(ca[1], cb[1])
        assert np.array_equal(A.draws(7), B.draws(7))
    kw["update_mode"] = SL.LAYOUT_JACOBI
    with SL.Layout(rp64, g.col, g.n, **kw) as A, SL.Layout(g.row_ptr, g.col, g.n, **kw) as B:
        A.run(1)
        B.run(1)
        ya, yb = A.positions(), B.positions()
    diam = float(np.linalg.norm(yb.max(0) - yb.min(0)))
    assert np.abs(ya - yb).max() <= 1e-5 * diam
    with pytest.raises(SL.LayoutError):  # a torch int32 row_ptr is refused by the 64-bit call
        SL.layout_create64(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(),
                           g.n, 2, 5, 5, 0, None, 1)


@pytest.fixture(scope="module")
def full():
    import time
    from synthgraph import gpu as G
    from conftest import generate_on_device
    t0 = time.perf_counter()
    rp, col, labels = generate_on_device(G.friendster_full_gpu, seed=0)
    del labels
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(f"generated the full com-friendster shape in {time.perf_counter() - t0:.1f} s",
          flush=True)
    yield rp, col
    del rp, col
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_full_friendster_shape_draws_and_init(full):
    rp_d, col_d = full
    n = rp_d.numel() - 1
    assert rp_d.dtype == torch.int64
    row_ptr = rp_d.cpu().numpy()
    nnz = int(row_ptr[-1])
    assert nnz > 2**31 and nnz == col_d.numel()
    rng = np.random.default_rng(8)
    hub = int(np.argmax(np.diff(row_ptr)))
    edges = np.concatenate([
        rng.integers(0, nnz, 20_000), [0, nnz - 1, nnz - 2, 2**31 - 1, 2**31],
        np.arange(row_ptr[hub], min(row_ptr[hub] + 64, row_ptr[hub + 1]))]).astype(np.int64)
    nodes = np.concatenate([rng.choice(n, 20_000, replace=False), [0, n - 1, hub]])
    with SL.Layout(rp_d, col_d, n, k=5, epochs=30, seed=2) as L:
        assert L.info()["engine"] == SL.LAYOUT_ENGINE_GLOBAL
        Y0 = L.positions()
        assert np.array_equal(Y0[nodes], O.init_positions_at(n, 2, nodes).astype(np.float32))
        print("init positions match", flush=True)
        for t in (0, 29):
            got = SL.layout_debug_draws_at(L.h, t, edges, 5)
            assert np.array_equal(got, O.draw_edges(row_ptr, n, 5, t, 2, edges)), t
            print(f"draws of epoch {t} match", flush=True)
        ms = L.run_timed(1)
        assert np.all(np.isfinite(L.positions()))
    print(f"full com-friendster shape: n={n} nnz={nnz}, one epoch {ms:.1f} ms", flush=True)


def test_full_shape_refuses_more_chunks_than_32_bit_counters_hold(full):
    rp_d, col_d = full
    with pytest.raises(SL.LayoutError) as ei:  # 3.6e9 one-edge chunks
        SL.Layout(rp_d, col_d, rp_d.numel() - 1, k=5, epochs=30, bundle_edges=1)
    assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
    print("refused:", ei.value, flush=True)


def test_full_shape_degree_alias_table_and_draws_bit_exact(full):
    """Degree-weighted negatives on the full shape: total weight W = nnz =
    3.6e9, past 2^31 and near the 2^32 limit of the integer alias table.
    The whole table (65.6M entries) and the negatives of sampled edges, most
    past offset 2^31, match the oracle bit for bit."""
    rp_d, col_d = full
    n = rp_d.numel() - 1
    row_ptr = rp_d.cpu().numpy()
    nnz = int(row_ptr[-1])
    assert 2**31 < nnz < 2**32
    thr_o, alias_o = O.alias_build(np.diff(row_ptr))
    rng = np.random.default_rng(9)
    edges = np.concatenate([rng.integers(0, nnz, 20_000), [0, nnz - 1, 2**31]]).astype(np.int64)
    with SL.Layout(rp_d, col_d, n, k=5, epochs=30, seed=6,
                   neg_weights=SL.LAYOUT_NEG_DEGREE) as L:
        thr, alias = SL.layout_debug_alias(L.h, n)
        assert np.array_equal(thr, thr_o) and np.array_equal(alias, alias_o)
        print("alias table of 65.6M entries matches", flush=True)
        for t in (0, 29):
            got = SL.layout_debug_draws_at(L.h, t, edges, 5)
            ref = O.draw_edges(row_ptr, n, 5, t, 6, edges, mode=O.NEG_DEGREE, thr=thr_o,
                               alias=alias_o)
            assert np.array_equal(got, ref), t


def test_full_shape_atomic_epoch_conserves_centroid(full):
    """One ATOMIC epoch over 3.6e9 directed edges: every pair update adds +v
    and -v, so the centroid stays put up to FP32 rounding."""
    rp_d, col_d = full
    n = rp_d.numel() - 1
    with SL.Layout(rp_d, col_d, n, k=5, epochs=30, seed=0, update_mode=SL.LAYOUT_ATOMIC,
                   hub_split_edges=1 << 30) as L:
        Y0 = L.positions().astype(np.float64)
        ms = L.run_timed(1)
        Y1 = L.positions().astype(np.float64)
    extent = float(np.abs(Y0).max())
    drift = float(np.abs(Y1.mean(0) - Y0.mean(0)).max())
    print(f"full shape ATOMIC epoch {ms:.1f} ms, centroid drift {drift:.2e} of extent {extent:.0f}",
          flush=True)
    assert np.all(np.isfinite(Y1)) and drift <= 1e-4 * extent, (drift, extent)
