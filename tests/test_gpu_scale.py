"""The out-of-last-level-cache regime: a com-friendster-sized node set
(65,608,366 nodes, positions of 525 MB, beyond the 256 MB MALL) with 10^9
undirected edges, generated on the GPU (synthgraph/gpu.py).  The oracle cannot
run epochs at this size, so parity is checked on what it can compute item by
item and on properties that hold at any size:
* the negatives of 20,000 sampled directed edges (including the first and
  last edge and edges of the largest hub) bit-exact for epochs 0 and 29;
* the initial positions of 20,000 sampled nodes bit-exact;
* ATOMIC mode conserves the centroid over an epoch (each pair update adds
  equal and opposite moves), to 1e-4 of the layout's extent; rows are not
  split here, since a split hub commits its mean move (1/S of the sum) by
  design;
* every position stays finite after 30 epochs of the default path.
"""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def big():
    from synthgraph import gpu as G
    if not torch.cuda.is_available():
        pytest.skip("needs the GPU")
    from conftest import generate_on_device
    rp, col, labels = generate_on_device(G.friendster_like_gpu, seed=0)
    torch.cuda.synchronize()
    yield rp, col, labels
    del rp, col, labels
    torch.cuda.empty_cache()


def test_friendster_like_draws_and_init_bit_exact(big):
    rp_d, col_d, _ = big
    n = rp_d.numel() - 1
    rp = rp_d.cpu().numpy()
    nnz = int(rp[-1])
    assert nnz == 2 * 1_000_000_000
    deg = np.diff(rp)
    hub = int(np.argmax(deg))
    rng = np.random.default_rng(3)
    edges = np.concatenate([[0, nnz - 1, rp[hub], rp[hub + 1] - 1],
                            rng.integers(0, nnz, 20_000 - 4)]).astype(np.int64)
    nodes = np.concatenate([[0, n - 1, hub], rng.integers(0, n, 20_000 - 3)]).astype(np.int64)
    with SL.Layout(rp_d, col_d, n, k=5, epochs=30, seed=11) as L:
        info = L.info()
        assert info["engine"] == SL.LAYOUT_ENGINE_GLOBAL
        for t in (0, 29):
            got = SL.layout_debug_draws_at(L.h, t, edges, 5)
            ref = O.draw_edges(rp, n, 5, t, 11, edges)
            assert np.array_equal(got, ref), t
        Y0 = L.positions()
        assert np.array_equal(Y0[nodes].astype(np.float64), O.init_positions_at(n, 11, nodes))
        L.run()
        assert np.all(np.isfinite(L.positions()))


def test_friendster_like_atomic_conserves_centroid(big):
    rp_d, col_d, _ = big
    n = rp_d.numel() - 1
    with SL.Layout(rp_d, col_d, n, k=5, epochs=30, seed=2, update_mode=SL.LAYOUT_ATOMIC,
                   hub_split_edges=1 << 30) as L:
        Y0 = L.positions().astype(np.float64)
        L.run(1)
        Y1 = L.positions().astype(np.float64)
    extent = float(np.abs(Y0).max())
    drift = np.abs(Y1.mean(0) - Y0.mean(0)).max()
    assert np.all(np.isfinite(Y1)) and drift <= 1e-4 * extent, (drift, extent)
