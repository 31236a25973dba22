"""Race diagnostics of the lock-free epoch on the GPU (Sec. 3.4).

* Atomic probe: every lane of a launch over all CUs adds 1 at device scope to
  one counter (and, spread, each to its own): the totals are exact, so atomic
  updates from all XCDs land (the ATOMIC policy relies on it); rates printed.
* Conflict counter: an epoch that runs on one lane has no conflicting write
  (no false positives); with many lanes conflicts appear, grow with the
  number of lanes in flight, and are printed for the 259k- and 4M-node graphs.
"""
import numpy as np
import pytest

import synthgraph as S

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


@pytest.mark.parametrize("spread", [0, 1])
def test_atomic_probe_totals_are_exact(spread):
    fsum, isum, adds, ms = SL.layout_bench_atomics(64, spread)
    assert fsum == float(adds) and isum == adds
    print(f"atomic probe ({'one address per lane' if spread else 'one address'}): "
          f"{2 * adds / (ms * 1e-3) / 1e9:.2f} G atomics/s", flush=True)


@pytest.fixture(scope="module")
def pl20k():
    return S.chung_lu_communities(20_000, 160_000, tau=2.2, dmax=1500.0, n_comm=20, intra=0.9,
                                  seed=3)


@pytest.mark.parametrize("mode", [SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ATOMIC])
def test_single_lane_has_no_conflicts(pl20k, mode):
    g = pl20k
    with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=10, seed=1, update_mode=mode,
                   engine=SL.LAYOUT_ENGINE_GLOBAL, bundle_edges=g.nnz, grid_blocks=1,
                   block_threads=64) as L:
        assert L.info()["n_chunks"] == 1
        stores, conflicts, untracked = SL.layout_debug_conflicts(L.h, 2)
        assert stores > g.nnz and conflicts == 0
        if mode == SL.LAYOUT_HOGWILD_STORE:
            assert untracked == 0  # every whole-row commit reloads its source
        assert L.status()[0] == 2
        assert np.all(np.isfinite(L.positions()))


def test_conflicts_grow_with_lanes_in_flight(pl20k):
    g = pl20k
    rates = []
    for grid in (2, 16, 256):
        with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=10, seed=1,
                       engine=SL.LAYOUT_ENGINE_GLOBAL, grid_blocks=grid, block_threads=256,
                       nodes_per_lane=1) as L:
            stores, conflicts, _ = SL.layout_debug_conflicts(L.h, 3)
        rates.append(conflicts / stores)
    print("conflicting writes per write, 512 / 4096 / 65536 lanes:",
          [f"{r:.2e}" for r in rates], flush=True)
    assert 0 < rates[0] < rates[1] < rates[2] < 1.0


def test_conflict_rate_of_the_default_launch():
    for name, maker in (("orkut-like-259k", S.orkut_like), ("lj-like-4m", S.lj_like)):
        g = S.cached(name, maker)
        out = []
        for mode in (SL.LAYOUT_HOGWILD_STORE, SL.LAYOUT_ATOMIC):
            with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=30, seed=0, update_mode=mode,
                           engine=SL.LAYOUT_ENGINE_GLOBAL) as L:
                L.run(1)
                stores, conflicts, untracked = SL.layout_debug_conflicts(L.h, 1)
            out.append((stores, conflicts, untracked))
            assert 0 <= conflicts < stores
        print(f"{name}: conflicting writes per write, STORE {out[0][1] / out[0][0]:.2e} "
              f"(untracked {out[0][2] / out[0][0]:.1e}), ATOMIC {out[1][1] / out[1][0]:.2e} "
              f"(untracked {out[1][2] / out[1][0]:.1e})", flush=True)


def test_conflict_counter_refusals(pl20k):
    g = pl20k
    with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=5, engine=SL.LAYOUT_ENGINE_XCD) as L:
        with pytest.raises(SL.LayoutError) as ei:
            SL.layout_debug_conflicts(L.h, 1)
        assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
    with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=5, engine=SL.LAYOUT_ENGINE_GLOBAL,
                   dim=3) as L:
        with pytest.raises(SL.LayoutError) as ei:
            SL.layout_debug_conflicts(L.h, 1)
        assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED
