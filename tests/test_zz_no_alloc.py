"""The allocation-free silhouette (layout_silhouette_noalloc, for callers that
cannot allocate device memory) against the allocating entry point
(layout_silhouette, itself held to sklearn's silhouette within 1e-5): the same
value on two calls in a row on the same GPU, the second on a smaller graph,
so that the shared scratch array's leftovers from the first call cannot leak
into the second; a graph beyond the array's size is refused."""
import ctypes

import numpy as np
import pytest

import synthgraph as S

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


def _both(g, seed, epochs):
    with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=epochs, seed=seed) as L:
        L.run(epochs)
        ref = L.silhouette(g.labels)
        lib = SL.lib()
        out = ctypes.c_double()
        lab = np.ascontiguousarray(g.labels, dtype=np.int32)
        rc = lib.layout_silhouette_noalloc(L.h, lab.ctypes.data, ctypes.byref(out))
        assert rc == SL.LAYOUT_OK, SL.layout_last_error()
        got = out.value
        # and once more on the same handle: the same answer
        again = SL.layout_silhouette_noalloc(L.h, g.labels)
    return ref, got, again


def test_noalloc_silhouette_matches_allocating_entry_point():
    big = S.small_sbm(9000, 6, 10.0, seed=3)
    small = S.small_sbm(1500, 3, 8.0, seed=4)
    for g, seed in ((big, 1), (small, 2)):
        ref, got, again = _both(g, seed, 10)
        print(f"silhouette n={g.n}: allocating {ref:.12f}, noalloc {got:.12f}", flush=True)
        assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))
        assert abs(again - ref) <= 1e-9 * max(1.0, abs(ref))


def test_noalloc_silhouette_refuses_more_nodes_than_its_array():
    n = SL.LAYOUT_NOALLOC_MAX_NODES + 1
    rp = np.zeros(n + 1, np.int32)  # edgeless: nothing to lay out, positions only
    with SL.Layout(rp, np.zeros(0, np.int32), n, k=5, epochs=1, seed=0) as L:
        labels = (np.arange(n) % 2).astype(np.int32)
        with pytest.raises(SL.LayoutError) as ei:
            SL.layout_silhouette_noalloc(L.h, labels)
        assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
        # the allocating entry point takes it
        assert np.isfinite(L.silhouette(labels))
