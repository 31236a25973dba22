"""Input relabelling used by the benchmark's --relabel measurement (host and
device versions): the relabelled graph is the same graph under the node
permutation, with sorted rows, in the stated node order; the torch version
(run here on CPU tensors) equals the numpy one."""
import numpy as np
import pytest

import synthgraph as S


@pytest.mark.parametrize("order", ["degree", "community"])
def test_relabel_is_the_same_graph_in_the_stated_order(order):
    g = S.chung_lu_communities(3000, 12000, tau=2.2, dmax=200.0, n_comm=8, intra=0.9, seed=9)
    h = S.relabel(g, order)
    deg = np.diff(g.row_ptr)
    perm = S.relabel_order(deg, g.labels, order)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    src = np.repeat(np.arange(g.n), deg)
    old = set(zip(inv[src].tolist(), inv[g.col].tolist()))
    src2 = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
    assert old == set(zip(src2.tolist(), h.col.tolist()))
    assert all(np.all(np.diff(h.col[h.row_ptr[i]:h.row_ptr[i + 1]]) > 0) for i in range(h.n))
    assert np.array_equal(h.labels, g.labels[perm])
    dn = np.diff(h.row_ptr)
    if order == "degree":
        assert np.all(np.diff(dn) <= 0)
    else:
        assert np.all(np.diff(h.labels) >= 0)
        for c in np.unique(h.labels):
            assert np.all(np.diff(dn[h.labels == c]) <= 0)


@pytest.mark.parametrize("order", ["degree", "community"])
def test_device_relabel_equals_host_relabel(order):
    torch = pytest.importorskip("torch")
    from synthgraph import gpu as G
    g = S.chung_lu_communities(2000, 9000, tau=2.3, dmax=150.0, n_comm=6, intra=0.9, seed=4)
    h = S.relabel(g, order)
    rp, col, lab = G.relabel_gpu(torch.from_numpy(g.row_ptr.astype(np.int64)),
                                 torch.from_numpy(g.col), torch.from_numpy(g.labels), order)
    assert np.array_equal(rp.numpy(), h.row_ptr.astype(np.int64))
    assert np.array_equal(col.numpy(), h.col)
    assert np.array_equal(lab.numpy(), h.labels)
