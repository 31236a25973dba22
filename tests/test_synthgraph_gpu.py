"""The torch graph generator (input generation only), run on the CPU: the CSR
it builds without sorting directed keys is a valid symmetric graph, the
excess-drop path used above 2^30 edges keeps exactly the requested count, and
the value-range unique equals torch.unique."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from synthgraph import gpu as G  # noqa: E402


def _valid(rp, col, n, m):
    rp = rp.numpy().astype(np.int64)
    col = col.numpy().astype(np.int64)
    assert rp[0] == 0 and rp[-1] == col.size == 2 * m
    src = np.repeat(np.arange(n), np.diff(rp))
    key = src * n + col
    assert np.all(np.diff(key) > 0)        # rows strictly ascending, no duplicates
    assert np.all(src != col)              # no self-loops
    assert np.array_equal(np.sort(col * n + src), key)  # both directions present


@pytest.mark.parametrize("n,m,seed", [(5000, 40000, 1), (300, 2000, 3)])
def test_generated_csr_is_a_valid_symmetric_graph(n, m, seed):
    rp, col, labels = G.chung_lu_communities_gpu(n, m, tau=2.2, dmax=(2 * m) ** 0.5,
                                                 n_comm=max(1, n // 100), intra=0.9, seed=seed,
                                                 device="cpu")
    assert rp.dtype == torch.int32 and labels.numel() == n
    _valid(rp, col, n, m)


def test_excess_drop_path_keeps_the_requested_count(monkeypatch):
    # the drop path serves graphs of _PERM_MAX edges or more; run it on a small one
    monkeypatch.setattr(G, "_PERM_MAX", 1000)
    n, m = 20000, 300000
    rp, col, _ = G.chung_lu_communities_gpu(n, m, tau=2.2, dmax=(2 * m) ** 0.5, n_comm=20,
                                            intra=0.9, seed=2, device="cpu")
    _valid(rp, col, n, m)


def test_value_range_unique_equals_torch_unique(monkeypatch):
    monkeypatch.setattr(G, "_SORT_MAX", 1000)
    monkeypatch.setattr(G, "_PART_ELEMS", 300)
    gen = torch.Generator().manual_seed(0)
    x = torch.randint(0, 5000, (20000,), generator=gen)
    x[:3000] = 7  # a heavy repeated value
    assert torch.equal(G._unique(torch, x), torch.unique(x))
