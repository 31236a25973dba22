"""3D layouts on the GPU against the FP64 oracle (the same force law of Table 1
with q over three coordinates).

Bars as for 2D:
* initial positions (third coordinate from the third word of the init block)
  and negatives: bit-exact;
* one Jacobi epoch: within 1e-5 x the oracle output's diameter;
* one epoch on one lane against the serial oracle in CSR order: within 1e-3 x
  the diameter (FP32 trajectory), on every engine and both policies;
* final lock-free layouts: NP and SI within 0.01 of the serial 3D oracle's;
* a 3D start in the plane z = 0 stays there exactly and follows the 2D run;
* device/host readout, set_positions, and the 2D-only entry points refuse 3D.
"""
import numpy as np
import pytest

import synthgraph as S
from oracle import metrics as M
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


def _diam(Y):
    return float(np.linalg.norm(Y.max(0) - Y.min(0)))


@pytest.fixture(scope="module")
def d1():
    return S.sbm_2000(0)


@pytest.fixture(scope="module")
def pl20k():
    return S.chung_lu_communities(20_000, 160_000, tau=2.2, dmax=1500.0, n_comm=20, intra=0.9,
                                  seed=3)


def _layout(g, **kw):
    kw.setdefault("k", 5)
    kw.setdefault("epochs", 50)
    kw.setdefault("seed", 0)
    k, epochs, seed = kw.pop("k"), kw.pop("epochs"), kw.pop("seed")
    return SL.Layout(g.row_ptr, g.col, g.n, k=k, epochs=epochs, seed=seed, dim=3, **kw)


@pytest.mark.parametrize("n,seed", [(2000, 0), (777, 5), (100_003, 11)])
def test_init_positions_3d_bit_exact(n, seed):
    rp = np.zeros(n + 1, np.int32)
    with SL.Layout(rp, np.zeros(0, np.int32), n, k=5, epochs=3, seed=seed, dim=3) as L:
        Y = L.positions()
    assert Y.shape == (n, 3)
    assert np.array_equal(Y, O.init_positions(n, seed, dim=3).astype(np.float32))


def test_draws_do_not_depend_on_dim(d1):
    with _layout(d1, epochs=10, seed=2) as L:
        assert np.array_equal(L.draws(4), O.draw_negatives(d1.row_ptr, d1.col, d1.n, 5, 4, 2))


@pytest.mark.parametrize("which,t,eta0", [("d1", 0, 1.0), ("d1", 7, 1.0), ("pl20k", 3, None)])
def test_jacobi_epoch_3d(which, t, eta0, d1, pl20k):
    g = {"d1": d1, "pl20k": pl20k}[which]
    if eta0 is None:
        eta0 = 1.0 / float(g.degrees().max())
    seed, T = 3, 20
    Y0 = O.init_positions(g.n, seed, dim=3).astype(np.float32)
    ref = O.jacobi_epoch(g.row_ptr, g.col, g.n, 5, t, T, seed, Y0.astype(np.float64), eta0=eta0)
    with _layout(g, epochs=T, seed=seed, update_mode=SL.LAYOUT_JACOBI, init_pos=Y0, eta0=eta0,
                 start_epoch=t) as L:
        L.run(1)
        Y = L.positions().astype(np.float64)
    err = np.abs(Y - ref).max()
    assert err <= 1e-5 * _diam(ref), (err, _diam(ref))


@pytest.mark.parametrize("mode,engine", [(0, 1), (1, 1), (0, 2), (1, 2), (0, 3)])
def test_single_lane_epoch_3d(d1, mode, engine):
    seed, T = 4, 50
    Y0 = O.init_positions(d1.n, seed, dim=3).astype(np.float32)
    ref = O.serial_run(d1.row_ptr, d1.col, d1.n, 5, T, seed, Y0=Y0.astype(np.float64),
                       t_begin=0, t_end=1, order=O.ORDER_CSR)
    with _layout(d1, epochs=T, seed=seed, update_mode=mode, engine=engine, init_pos=Y0,
                 bundle_edges=d1.nnz, grid_blocks=1, block_threads=64) as L:
        assert L.info()["n_chunks"] == 1
        L.run(1)
        Y = L.positions().astype(np.float64)
    err = np.abs(Y - ref).max()
    assert err <= 1e-3 * _diam(ref), (err, _diam(ref))


@pytest.fixture(scope="module")
def d1_oracle_quality_3d(d1):
    Y = O.serial_run(d1.row_ptr, d1.col, d1.n, 5, 50, 0, dim=3)
    return M.quality(d1.row_ptr, d1.col, Y, d1.labels)


@pytest.mark.parametrize("mode,engine", [
    (SL.LAYOUT_UPDATE_AUTO, SL.LAYOUT_ENGINE_AUTO),
    (SL.LAYOUT_ATOMIC, SL.LAYOUT_ENGINE_GLOBAL),
    (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_GLOBAL),
    (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_XCD),
    (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ENGINE_LDS),
])
def test_final_layout_quality_3d(d1, d1_oracle_quality_3d, mode, engine):
    with _layout(d1, update_mode=mode, engine=engine) as L:
        L.run()
        Y = L.positions()
    assert Y.shape == (d1.n, 3) and np.all(np.isfinite(Y))
    assert np.ptp(Y[:, 2]) > 0.1 * np.ptp(Y[:, 0])  # a genuinely 3D layout
    q = M.quality(d1.row_ptr, d1.col, Y, d1.labels)
    ref = d1_oracle_quality_3d
    assert abs(q["np"] - ref["np"]) <= 0.01, (q, ref)
    assert abs(q["si"] - ref["si"]) <= 0.01, (q, ref)


def test_plane_start_stays_in_the_plane(d1):
    Y2 = O.init_positions(d1.n, 6).astype(np.float32)
    Y3 = np.concatenate([Y2, np.zeros((d1.n, 1), np.float32)], axis=1)
    kw = dict(epochs=50, seed=6, bundle_edges=d1.nnz, grid_blocks=1, block_threads=64,
              engine=SL.LAYOUT_ENGINE_GLOBAL)
    with _layout(d1, init_pos=Y3, **kw) as L:
        L.run(3)
        Y = L.positions()
    with SL.Layout(d1.row_ptr, d1.col, d1.n, k=5, init_pos=Y2, **kw) as L2:
        L2.run(3)
        Yp = L2.positions()
    assert np.all(Y[:, 2] == 0.0)
    assert np.abs(Y[:, :2] - Yp).max() <= 1e-3 * _diam(Yp)


def test_readout_set_positions_and_refusals(d1):
    import torch

    with _layout(d1, epochs=10, seed=1) as L:
        L.run(2)
        Y = L.positions()
        dev = torch.empty((d1.n, 3), dtype=torch.float32, device="cuda:0")
        SL.layout_get_positions_device(L.h, dev)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy(), Y)
        Z = np.arange(d1.n * 3, dtype=np.float32).reshape(d1.n, 3)
        L.set_positions(Z)
        assert np.array_equal(L.positions(), Z)
        for call in (lambda: L.sampled_energy(0), L.effective_energy,
                     lambda: L.silhouette(d1.labels), lambda: L.neighbourhood([0])):
            with pytest.raises(SL.LayoutError) as ei:
                call()
            assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
    with pytest.raises(SL.LayoutError) as ei:
        SL.Layout(d1.row_ptr, d1.col, d1.n, k=5, epochs=5, dim=4)
    assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
    with pytest.raises(SL.LayoutError) as ei:
        _layout(d1, init_mode=SL.LAYOUT_INIT_PMDS)
    assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
    # the LDS engine holds 16 bytes per 3D position
    big = S.chung_lu_communities(12_000, 40_000, tau=2.3, dmax=200.0, n_comm=8, intra=0.9, seed=1)
    with pytest.raises(SL.LayoutError) as ei:
        _layout(big, engine=SL.LAYOUT_ENGINE_LDS)
    assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED


def test_host_transfers_3d_at_scale():
    """3D positions are 16 bytes on the device and rows of 3 floats on the
    host: caller init from host and from device, readout and set_positions
    are exact at 1M nodes, and each host transfer takes well under a second
    (a strided copy with 12-byte rows between device and pageable memory
    would move one row at a time and take minutes)."""
    import time
    import torch

    n = 1_000_000
    rp, col = S.csr_from_pairs(np.arange(n), (np.arange(n) + 1) % n, n)
    rng = np.random.default_rng(4)
    Y0 = rng.standard_normal((n, 3)).astype(np.float32)
    t0 = time.perf_counter()
    with SL.Layout(rp, col, n, k=5, epochs=3, seed=2, dim=3, init_pos=Y0) as L:
        t_create = time.perf_counter() - t0
        t0 = time.perf_counter()
        got = L.positions()
        t_read = time.perf_counter() - t0
        assert np.array_equal(got, Y0)
        Z = rng.standard_normal((n, 3)).astype(np.float32)
        t0 = time.perf_counter()
        L.set_positions(Z)
        t_write = time.perf_counter() - t0
        assert np.array_equal(L.positions(), Z)
        L.run(1)
        assert np.all(np.isfinite(L.positions()))
    print(f"3D host transfers at n = {n}: create {t_create:.3f} s, readout {t_read:.3f} s, "
          f"set {t_write:.3f} s", flush=True)
    assert t_read < 2.0 and t_write < 2.0 and t_create < 5.0
    dev = torch.device("cuda:0")
    with SL.Layout(torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev), n, k=5, epochs=3,
                   seed=2, dim=3, init_pos=torch.from_numpy(Y0).to(dev)) as L:
        assert np.array_equal(L.positions(), Y0)
