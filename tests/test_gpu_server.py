"""Served layouts (continuous batching): jobs submitted while others run are
admitted as slots and memory free up; each job's result is the same alone
and in the mix (NP and SI of the single-graph path, mean over eight paired
seeds within 0.01); every served job draws the oracle's negatives, whatever
engine serves it; in the synchronous mode a served job's positions after T
epochs are the oracle's T chained synchronous epochs within 1e-5 x diameter;
admission respects the HBM budget; a malformed job fails alone; all-CU jobs
that do not fit the device's lanes together take turns in arrival order while
smaller jobs pass in their own class."""
import threading
import time

import numpy as np
import pytest

import synthgraph as S
from oracle import metrics as M
from quality_stats import assert_paired_close
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SL = pytest.importorskip("paper_2608_01907_amd.snaplayout")


@pytest.fixture(scope="module")
def pool():
    gs = [S.small_sbm(n, 4, 12.0, seed=40 + q) for q, n in enumerate([800, 2500, 6000])]
    gs += [S.chung_lu_communities(n, m, tau=2.2, dmax=600.0, n_comm=16, intra=0.9, seed=50 + q)
           for q, (n, m) in enumerate([(40_000, 320_000), (120_000, 900_000)])]
    return gs


def _alone(g, seed, T, k=5):
    with SL.Layout(g.row_ptr, g.col, g.n, k=k, epochs=T, seed=seed) as L:
        L.run()
        return L.positions()


def _quality(g, Y):
    """NP on 1,000 and SI on 4,000 seeded sample nodes (the same samples for
    every layout of g)."""
    return {"np": M.np_score(g.row_ptr, g.col, Y, sample=1000),
            "si": M.si_score(Y, g.labels, sample=4000)}


def test_server_results_same_alone_and_in_mix(pool):
    T = 30
    srv = SL.layout_server_create(0, 16, 1 << 20)
    try:
        ids = []
        for q, g in enumerate(pool * 8):  # each graph eight times, submitted back to back
            ids.append((q % len(pool), 300 + q,
                        SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, 5, T, 300 + q)))
        results = {}
        for gi, seed, jid in ids:
            SL.layout_server_wait(srv, jid, 120.0)
            Y, lat = SL.layout_server_take(srv, jid, pool[gi].n)
            assert lat > 0 and np.all(np.isfinite(Y))
            results[(gi, seed)] = Y
        st = SL.layout_server_get_stats(srv)
        assert st["completed"] == len(ids) and st["failed"] == 0
        assert st["p99_latency_s"] >= st["p50_latency_s"] > 0
    finally:
        SL.layout_server_destroy(srv)
    # lock-free runs are not bit-reproducible: paired comparison over the
    # eight seeds of each graph, alone and in the mix
    for gi, g in enumerate(pool):
        seeds = sorted(seed for (gj, seed) in results if gj == gi)
        qa = [M.quality(g.row_ptr, g.col, _alone(g, sd, T), g.labels, sample=4000) for sd in seeds]
        qm = [M.quality(g.row_ptr, g.col, results[(gi, sd)], g.labels, sample=4000)
              for sd in seeds]
        assert_paired_close(qa, qm, label=gi)


def test_server_budget_binds_admission_and_jobs_overlap(pool):
    """A budget that fits two of the large jobs at a time: no more is ever
    admitted, and jobs submitted later are still served."""
    g = pool[-1]
    probe = SL.layout_server_create(1 << 40, 1, 0)
    SL.layout_server_destroy(probe)
    per_job = 4 * (g.n + 1) + 4 * g.nnz + 8 * g.n + 8 * (g.nnz // 16 + 2 * (g.nnz // 64) + 2) + 4
    srv = SL.layout_server_create(int(2.5 * per_job), 16, 1 << 18)
    try:
        ids = [SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, 5, 10, q) for q in range(5)]
        seen_running = 0
        t0 = time.time()
        while time.time() - t0 < 120:
            st = SL.layout_server_get_stats(srv)
            assert st["hbm_in_use"] <= st["hbm_budget"]
            seen_running = max(seen_running, st["running"])
            if st["completed"] == 5:
                break
            time.sleep(0.002)
        assert seen_running <= 2
        for jid in ids:
            SL.layout_server_wait(srv, jid, 60.0)
            SL.layout_server_take(srv, jid, g.n)
    finally:
        SL.layout_server_destroy(srv)


def test_server_isolates_a_bad_job_and_refuses_oversized(pool):
    srv = SL.layout_server_create(4 << 20, 4, 0)
    try:
        good = SL.layout_server_submit(srv, pool[0].row_ptr, pool[0].col, pool[0].n, 5, 5, 1)
        bad = SL.layout_server_submit(srv, np.array([0, 1, 1], np.int32),
                                      np.array([1], np.int32), 2, 5, 5, 2)
        with pytest.raises(SL.LayoutError) as ei:
            SL.layout_server_wait(srv, bad, 60.0)
        assert ei.value.code == SL.LAYOUT_E_BAD_GRAPH
        SL.layout_server_wait(srv, good, 60.0)
        Y, _ = SL.layout_server_take(srv, good, pool[0].n)
        assert np.all(np.isfinite(Y))
        big = pool[-1]
        with pytest.raises(SL.LayoutError) as ei:
            SL.layout_server_submit(srv, big.row_ptr, big.col, big.n, 5, 5, 3)
        assert ei.value.code == SL.LAYOUT_E_OOM
        assert SL.layout_server_get_stats(srv)["rejected"] == 1
    finally:
        SL.layout_server_destroy(srv)


def test_server_concurrent_submitters(pool):
    srv = SL.layout_server_create(0, 6, 0)
    errors = []
    done = []

    def client(q):
        try:
            g = pool[q % 3]
            jid = SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, 5, 8, 500 + q)
            SL.layout_server_wait(srv, jid, 120.0)
            Y, _ = SL.layout_server_take(srv, jid, g.n)
            done.append(np.all(np.isfinite(Y)))
        except Exception as exc:  # reported below
            errors.append(exc)

    th = [threading.Thread(target=client, args=(q,)) for q in range(12)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    SL.layout_server_destroy(srv)
    assert not errors and len(done) == 12 and all(done)


def test_server_small_job_moves_and_stays_finite(pool):
    """A job small enough for the LDS engine runs whole in one launch."""
    g = pool[0]
    srv = SL.layout_server_create(0, 2, 0)
    try:
        jid = SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, 5, 20, 9)
        SL.layout_server_wait(srv, jid, 60.0)
        Y, lat = SL.layout_server_take(srv, jid, g.n)
    finally:
        SL.layout_server_destroy(srv)
    Y0 = O.init_positions(g.n, 9)
    assert np.all(np.isfinite(Y)) and not np.allclose(Y, Y0)


# ------------------------------------ caller weights, PMDS starts, cancel
def _server(**kw):
    o = SL.layout_opts_init()
    for k_, v in kw.items():
        setattr(o, k_, v)
    return SL.layout_server_create(0, 16, 1 << 20, o)


def test_server_custom_weights_match_the_plain_path(pool):
    """Weighted negatives through the server: the same layout quality as the
    plain path with the same weights (paired over seeds), and the argument
    rules of layout_server_submit_ex."""
    T = 30
    g = pool[3]
    w = np.diff(g.row_ptr).astype(np.uint32) + 1  # degree + 1
    srv = _server(neg_weights=SL.LAYOUT_NEG_CUSTOM)
    try:
        # degree-like negatives make this layout's SI vary by about 0.02 from
        # seed to seed (alone and served alike), so 32 paired seeds keep the
        # standard error of the mean difference near 0.0035
        ids = [(sd, SL.layout_server_submit_ex(srv, g.row_ptr, g.col, g.n, 5, T, sd,
                                               neg_weight_values=w)) for sd in range(500, 532)]
        res = {}
        for sd, jid in ids:
            SL.layout_server_wait(srv, jid, 120.0)
            res[sd] = SL.layout_server_take(srv, jid, g.n)[0]
        with pytest.raises(SL.LayoutError) as ei:  # weights required
            SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, 5, T, 1)
        assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
        with pytest.raises(SL.LayoutError) as ei:  # zero mass
            SL.layout_server_submit_ex(srv, g.row_ptr, g.col, g.n, 5, T, 1,
                                       neg_weight_values=np.zeros(g.n, np.uint32))
        assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
    finally:
        SL.layout_server_destroy(srv)
    plain = {}
    for sd, _ in ids:
        with SL.Layout(g.row_ptr, g.col, g.n, k=5, epochs=T, seed=sd,
                       neg_weights=SL.LAYOUT_NEG_CUSTOM, neg_weight_values=w) as L:
            L.run()
            plain[sd] = L.positions()
    qa = [_quality(g, plain[sd]) for sd, _ in ids]
    qs = [_quality(g, res[sd]) for sd, _ in ids]
    assert_paired_close(qa, qs, label="custom")
    srv = _server()
    try:
        with pytest.raises(SL.LayoutError) as ei:  # weights without the custom mode
            SL.layout_server_submit_ex(srv, g.row_ptr, g.col, g.n, 5, T, 1, neg_weight_values=w)
        assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
    finally:
        SL.layout_server_destroy(srv)


def test_server_pmds_start_and_caller_init(pool):
    """eta0 = 0 keeps the start: a PMDS server returns each job's Pivot MDS
    layout; a caller's init_pos comes back unchanged."""
    srv = _server(init_mode=SL.LAYOUT_INIT_PMDS, eta0=0.0)
    try:
        jobs = [(gi, SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, 5, 3, 40 + gi))
                for gi, g in enumerate(pool)]
        Y0 = np.random.default_rng(1).standard_normal((pool[0].n, 2)).astype(np.float32)
        own = SL.layout_server_submit_ex(srv, pool[0].row_ptr, pool[0].col, pool[0].n, 5, 3, 7,
                                         init_pos=Y0)
        for gi, jid in jobs:
            SL.layout_server_wait(srv, jid, 120.0)
            Y = SL.layout_server_take(srv, jid, pool[gi].n)[0]
            g = pool[gi]
            ref = SL.layout_pmds(g.row_ptr, g.col, g.n, 0, 40 + gi)
            diam = float(np.linalg.norm(ref.max(0) - ref.min(0)))
            assert np.abs(Y - ref).max() <= 1e-5 * diam, gi
        SL.layout_server_wait(srv, own, 120.0)
        assert np.array_equal(SL.layout_server_take(srv, own, pool[0].n)[0], Y0)
    finally:
        SL.layout_server_destroy(srv)


def test_server_cancel(pool):
    """Cancel a queued job (ends at once) and a running one (retired after its
    round); the other jobs complete, the budget is released, and the
    cancelled ids answer as documented."""
    big = pool[4]
    srv = SL.layout_server_create(0, 1, 1 << 16)  # one slot: jobs queue up
    try:
        # thousands of short rounds: seconds of work, so the cancel lands mid-run
        running = SL.layout_server_submit(srv, big.row_ptr, big.col, big.n, 5, 3000, 1)
        queued = [SL.layout_server_submit(srv, big.row_ptr, big.col, big.n, 5, 10, 2 + q)
                  for q in range(3)]
        deadline = time.time() + 60
        while SL.layout_server_poll(srv, running) != SL.LAYOUT_JOB_RUNNING:
            assert time.time() < deadline
            time.sleep(0.01)
        SL.layout_server_cancel(srv, queued[1])
        assert SL.layout_server_poll(srv, queued[1]) == SL.LAYOUT_JOB_CANCELLED
        SL.layout_server_cancel(srv, running)
        with pytest.raises(SL.LayoutError):
            SL.layout_server_wait(srv, running, 60.0)  # ends cancelled
        assert SL.layout_server_poll(srv, running) == SL.LAYOUT_JOB_CANCELLED
        for jid in (queued[0], queued[2]):
            SL.layout_server_wait(srv, jid, 120.0)
            Y, _ = SL.layout_server_take(srv, jid, big.n)
            assert np.all(np.isfinite(Y))
        for jid in (running, queued[1]):
            with pytest.raises(SL.LayoutError) as ei:
                SL.layout_server_take(srv, jid, big.n)
            assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
            with pytest.raises(SL.LayoutError):  # forgotten after take
                SL.layout_server_poll(srv, jid)
        with pytest.raises(SL.LayoutError) as ei:
            SL.layout_server_cancel(srv, 10**9)
        assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
        st = SL.layout_server_get_stats(srv)
        assert st["cancelled"] == 2 and st["completed"] == 2 and st["hbm_in_use"] == 0
    finally:
        SL.layout_server_destroy(srv)


# ------------------------------------------- served output against the oracle
def _oracle_jacobi_chain(g, k, T, seed, eta0):
    Y = O.init_positions(g.n, seed)
    for t in range(T):
        Y = O.jacobi_epoch(g.row_ptr, g.col, g.n, k, t, T, seed, Y, eta0=eta0)
    return Y


def test_server_jacobi_matches_oracle(pool):
    """Synchronous mode through the server: every job (small and large, all on
    the global engine in this mode; the large ones cut into several epoch
    slices per epoch by a small round budget) ends within 1e-5 x diameter of T
    chained synchronous oracle epochs (Algorithm 1's pairs and draws, Sec. 3.3
    forces) from the same seeded start."""
    T, k, eta0 = 3, 4, 0.05
    srv = _server_jacobi(eta0)
    try:
        jobs = [(gi, 60 + gi, SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, k, T, 60 + gi))
                for gi, g in enumerate(pool)]
        for gi, seed, jid in jobs:
            SL.layout_server_wait(srv, jid, 120.0)
            Y, _ = SL.layout_server_take(srv, jid, pool[gi].n)
            ref = _oracle_jacobi_chain(pool[gi], k, T, seed, eta0)
            diam = float(np.linalg.norm(ref.max(0) - ref.min(0)))
            err = float(np.abs(Y - ref).max())
            print(f"served jacobi job {gi} (n {pool[gi].n}): max error {err:.3e}, "
                  f"tol {1e-5 * diam:.3e}", flush=True)
            assert err <= 1e-5 * diam, (gi, err, diam)
        assert SL.layout_server_get_stats(srv)["rounds"] > T  # slices were taken
    finally:
        SL.layout_server_destroy(srv)


def _server_jacobi(eta0):
    o = SL.layout_opts_init()
    o.update_mode = SL.LAYOUT_JACOBI
    o.eta0 = eta0
    return SL.layout_server_create(0, 16, 1 << 18, o)


def test_server_jacobi_refuses_other_engines():
    o = SL.layout_opts_init()
    o.update_mode = SL.LAYOUT_JACOBI
    o.engine = SL.LAYOUT_ENGINE_LDS
    with pytest.raises(SL.LayoutError) as ei:
        SL.layout_server_create(0, 4, 0, o)
    assert ei.value.code == SL.LAYOUT_E_UNSUPPORTED


@pytest.fixture(scope="module")
def wide_graph():
    """Positions beyond one XCD's L2 (400k nodes x 8 B > 3 MiB): the all-CU
    engine serves it."""
    return S.chung_lu_communities(400_000, 1_200_000, tau=2.2, dmax=1000.0, n_comm=300,
                                  intra=0.9, seed=77)


@pytest.mark.parametrize("weighted", [False, True])
def test_server_draws_match_oracle_on_every_engine(pool, wide_graph, weighted):
    """Held server: jobs of all three classes (LDS-sized SBMs, XCD-bin graphs,
    and a graph served by the all-CU engine) are admitted and set up; the
    negatives each draws in its first and last epoch, computed from its own
    device state, are the oracle's bit for bit (uniform, and caller weights
    through each job's own alias table).  Released, every job completes."""
    T, k = 6, 5
    graphs = list(pool) + [wide_graph]
    o = SL.layout_opts_init()
    if weighted:
        o.neg_weights = SL.LAYOUT_NEG_CUSTOM
    srv = SL.layout_server_create(0, 16, 1 << 20, o)
    try:
        SL.layout_server_hold(srv, True)
        jobs = []
        for gi, g in enumerate(graphs):
            w = None
            if weighted:
                w = (np.random.default_rng(gi).integers(0, 40, g.n) + (np.arange(g.n) % 7 == 0)
                     ).astype(np.uint32)
            jid = SL.layout_server_submit_ex(srv, g.row_ptr, g.col, g.n, k, T, 900 + gi,
                                             neg_weight_values=w)
            jobs.append((gi, 900 + gi, w, jid))
        for gi, seed, w, jid in jobs:
            g = graphs[gi]
            kw = {}
            if weighted:
                thr, alias = O.alias_build(w.astype(np.int64))
                kw = {"mode": O.NEG_DEGREE, "thr": thr, "alias": alias}
            for t in (0, T - 1):
                got = SL.layout_server_debug_draws(srv, jid, t, g.nnz, k)
                ref = O.draw_negatives(g.row_ptr, g.col, g.n, k, t, seed, **kw)
                assert np.array_equal(got, ref), (gi, t)
            assert SL.layout_server_poll(srv, jid) == SL.LAYOUT_JOB_RUNNING
        st = SL.layout_server_get_stats(srv)
        assert st["rounds"] == 0 and st["running"] == len(jobs)  # held: no epoch ran yet
        SL.layout_server_hold(srv, False)
        for gi, seed, w, jid in jobs:
            SL.layout_server_wait(srv, jid, 120.0)
            with pytest.raises(SL.LayoutError) as ei:  # done: no longer on the device
                SL.layout_server_debug_draws(srv, jid, 0, graphs[gi].nnz, k)
            assert ei.value.code == SL.LAYOUT_E_DONE
            Y, _ = SL.layout_server_take(srv, jid, graphs[gi].n)
            assert np.all(np.isfinite(Y))
            with pytest.raises(SL.LayoutError) as ei:  # forgotten after take
                SL.layout_server_debug_draws(srv, jid, 0, graphs[gi].nnz, k)
            assert ei.value.code == SL.LAYOUT_E_INVALID_ARG
    finally:
        SL.layout_server_destroy(srv)


def test_server_all_cu_jobs_take_turns_and_small_jobs_pass():
    """Two jobs whose lane caps (n / 32 each) do not fit the device's lanes
    together run one after the other in arrival order, so the first ends
    well before the second; a small job submitted after both runs in its own
    class and ends before the second.  Every result is finite."""
    n = 1_100_000  # n / 32 = 34,375 lanes; two exceed 256 CUs x 256 lanes
    rp, col = S.csr_from_pairs(np.arange(n), (np.arange(n) + 1) % n, n)
    small = S.small_sbm(2500, 4, 12.0, seed=41)
    srv = SL.layout_server_create(0, 16, 0)
    try:
        a = SL.layout_server_submit(srv, rp, col, n, 5, 400, 1)
        b = SL.layout_server_submit(srv, rp, col, n, 5, 400, 2)
        time.sleep(0.02)
        c = SL.layout_server_submit(srv, small.row_ptr, small.col, small.n, 5, 30, 3)
        lat = {}
        for name, jid, nn in (("a", a, n), ("b", b, n), ("c", c, small.n)):
            SL.layout_server_wait(srv, jid, 120.0)
            Y, lat[name] = SL.layout_server_take(srv, jid, nn)
            assert np.all(np.isfinite(Y)), name
    finally:
        SL.layout_server_destroy(srv)
    print("latencies", {k: round(v, 3) for k, v in lat.items()}, flush=True)
    assert lat["a"] < 0.75 * lat["b"], lat
    assert lat["c"] < lat["b"], lat
