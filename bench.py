"""Throughput benchmark of the SNAP-tFDP layout on one MI355X.

Default workload: the 4M-node / 34M-edge power-law community graph (k = 5,
30 epochs).  A step is one whole layout job with the graph already resident in
HBM: create (device validation, chunk table, seeded init), every epoch of the
schedule, and the readout of the positions into a device buffer.

    value = |E| * (1 + k) * T / step time      (|E| undirected)

The JSON line also carries
  roofline      -- the dominant kernel (the epoch kernel): algorithmic bytes per
                   launch / mean launch time (HIP events on the handle's
                   stream) against the 8 TB/s HBM peak; the measured
                   random-gather ceiling of the same graph (the epoch's
                   position reads alone, gather_roofline_frac = its time over
                   the epoch's, at most 1); HBM traffic from
                   the committed rocprofv3 counter summary when it was taken on
                   the current kernel source (else null);
  cpu_baseline  -- the FP64 oracle's threaded bundle scheme timed on this
                   host's cores on a bounded sample (a few epochs);
  batched_and_served -- short runs of the other two workloads (default run
                   only; --no-extra skips them): the 512-graph batch against
                   one graph per launch (plain time from every 8th graph in
                   size order), and
                   200 served jobs at 0.8 of the plain capacity, p50/p99
                   against FIFO one job at a time.
Other workloads (--workload): batched-512 (512 graphs in one HIP-graph
replay, against one graph per launch) and served (a Poisson stream through
the continuous-batching server, against FIFO one job at a time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PLAIN = {
    # name: (maker, k, epochs)
    "lj-like-4m": ("lj_like", 5, 30),
    "orkut-like-259k": ("orkut_like", 5, 30),
    "sbm-2000": ("sbm_2000", 5, 50),
    "friendster-like-65m": ("gpu:friendster_like", 5, 30),
    "friendster-full-65m": ("gpu:friendster_full", 5, 30),
}
KERNEL_SOURCES = ["paper_2608_01907_amd/csrc/kernels.hpp", "paper_2608_01907_amd/csrc/rng.hpp",
                  "paper_2608_01907_amd/csrc/desc.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(row_ptr: np.ndarray, n: int, k: int, hub: int, n_chunks: int,
                      dim: int = 2) -> int:
    """Bytes one epoch must move at minimum: per directed edge the col entry
    (4 B) and (1 + k) position read-modify-writes (2 x 8 B in 2D, 2 x 16 B for
    the 16-byte 3D positions); per source run (a row, or one segment of a row
    split above `hub` edges) the source read and commit (same); per chunk its
    table entries (an 8-byte first edge and a 4-byte source row); the 64-bit
    row pointers the device holds (8 B per row)."""
    nnz = int(row_ptr[-1])
    rmw = 16 if dim == 2 else 32
    deg = np.diff(row_ptr.astype(np.int64))
    runs = int(np.where(deg > hub, (deg + hub - 1) // hub, (deg > 0).astype(np.int64)).sum())
    return int(nnz * (4 + rmw * (1 + k)) + rmw * runs + 12 * n_chunks + 8 * (n + 1))


def committed_traffic(workload: str):
    """HBM bytes per epoch launch from the committed counter summary, or None
    when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"epoch_{workload}_traffic.json")
    if not os.path.exists(path):
        return None, None
    t = json.load(open(path))
    if t.get("kernel_hash") != kernel_hash():
        return None, t
    return t.get("traffic_bytes_per_launch"), t


def cpu_baseline(g, k, T, seed, budget_s=12.0):
    from oracle import oracle as O

    threads = os.cpu_count() or 1
    Y0 = O.init_positions(g.n, seed)
    t0 = time.perf_counter()
    O.threaded_run(g.row_ptr, g.col, g.n, k, T, seed, threads, Y0=Y0, t_begin=0, t_end=1)
    one = time.perf_counter() - t0
    epochs = max(1, min(T - 1, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    O.threaded_run(g.row_ptr, g.col, g.n, k, T, seed, threads, Y0=Y0, t_begin=1,
                   t_end=1 + epochs)
    dt = time.perf_counter() - t0
    value = g.n_edges * (1 + k) * epochs / dt
    return {"value": value, "unit": "edge-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{epochs} epoch(s) of the same graph, FP64 threaded bundle scheme "
                      f"(lock-free, {threads} threads), after one warm-up epoch"}


# ------------------------------------------------------------------ plain
def bench_plain(args):
    import torch
    import synthgraph as S
    from paper_2608_01907_amd import snaplayout as SL

    maker, k, T = PLAIN[args.workload]
    seed = 0
    t0 = time.perf_counter()
    dev = torch.device("cuda:0")
    if maker.startswith("gpu:"):
        # generated on the device (10^9 or 1.8 x 10^9 edges): inputs never leave HBM
        from synthgraph import gpu as G
        make = G.friendster_full_gpu if maker == "gpu:friendster_full" else G.friendster_like_gpu
        rp_d, col_d, labels_d = make(seed=0)
        if args.relabel != "none":
            rp_d, col_d, labels_d = G.relabel_gpu(rp_d, col_d, labels_d, args.relabel)
        del labels_d
        torch.cuda.empty_cache()
        row_ptr = rp_d.cpu().numpy()
        g = S.Graph(row_ptr, np.zeros(0, np.int32), len(row_ptr) - 1, None, args.workload)
        nnz = int(row_ptr[-1])
    else:
        g = S.cached(args.workload, getattr(S, maker))
        if args.relabel != "none":
            g = S.relabel(g, args.relabel)
        rp_d = torch.from_numpy(g.row_ptr).to(dev)
        col_d = torch.from_numpy(g.col).to(dev)
        nnz = g.nnz
    if args.relabel != "none":
        log(f"[bench] nodes relabelled in {args.relabel} order (input preprocessing; the "
            f"draws are those of the relabelled graph)")
    n_edges = nnz // 2
    log(f"[bench] graph {g.name}: n={g.n} |E|={n_edges} nnz={nnz} "
        f"dmax={int(np.diff(g.row_ptr).max())} ({time.perf_counter() - t0:.1f}s)")
    mode = {"auto": SL.LAYOUT_UPDATE_AUTO, "atomic": SL.LAYOUT_ATOMIC,
            "store": SL.LAYOUT_HOGWILD_STORE}[args.mode]
    dim = args.dim
    out_d = torch.empty((g.n, dim), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    engine = {"auto": SL.LAYOUT_ENGINE_AUTO, "global": SL.LAYOUT_ENGINE_GLOBAL,
              "xcd": SL.LAYOUT_ENGINE_XCD, "lds": SL.LAYOUT_ENGINE_LDS}[args.engine]

    def opts():
        o = SL.layout_opts_init()
        o.update_mode = mode
        o.bundle_edges = args.bundle
        o.grid_blocks = args.grid
        o.engine = engine
        return o

    if args.profile_epochs:
        h = SL.layout_create_ex(rp_d, col_d, g.n, dim, k, T, seed, opts(), 1)
        SL.layout_epoch(h, args.profile_epochs)
        SL.layout_sync(h)
        SL.layout_destroy(h)
        log("[bench] profile run done")
        return None

    def step():
        h = SL.layout_create_ex(rp_d, col_d, g.n, dim, k, T, seed, opts(), 1)
        SL.layout_epoch(h, T)
        SL.layout_get_positions_device(h, out_d)
        SL.layout_sync(h)
        SL.layout_destroy(h)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    value = n_edges * (1 + k) * T / (dt / args.steps)
    log(f"[bench] {args.steps} steps, {ms_step:.2f} ms/step")

    # dominant kernel: the epoch kernel, timed with HIP events on its stream
    # around each whole run of T epochs (the runs above warmed it up); the
    # median of five runs (one on the 65M-node graphs, whose run takes ~20 s)
    reps = 1 if maker.startswith("gpu:") else 5
    runs_ms = []
    for _ in range(reps):
        h = SL.layout_create_ex(rp_d, col_d, g.n, dim, k, T, seed, opts(), 1)
        info = SL.layout_get_info(h)
        runs_ms.append(SL.layout_epoch_timed(h, T) / T)
        Y = SL.layout_get_positions(h, g.n, dim)
        finite = bool(np.all(np.isfinite(Y)))
        SL.layout_destroy(h)
    ms_epoch = float(np.median(runs_ms))

    # phases of one job, timed apart with the host clock between device
    # synchronisations: create from HBM-resident inputs (validation, chunk
    # table, init), the epochs, the readout to host memory, and, for the
    # host-buffer case of the boundary, create from host arrays (PCIe copy
    # of the CSR included; not available for the graphs generated on the
    # device, whose CSR never lives in host memory)
    def phases(src_rp, src_col, on_device):
        t_a = time.perf_counter()
        h = SL.layout_create_ex(src_rp, src_col, g.n, dim, k, T, seed, opts(), on_device)
        SL.layout_sync(h)
        t_b = time.perf_counter()
        SL.layout_epoch(h, T)
        SL.layout_sync(h)
        t_c = time.perf_counter()
        SL.layout_get_positions(h, g.n, dim)
        t_d = time.perf_counter()
        SL.layout_destroy(h)
        return {"create_ms": round((t_b - t_a) * 1e3, 2), "epochs_ms": round((t_c - t_b) * 1e3, 2),
                "readout_to_host_ms": round((t_d - t_c) * 1e3, 2)}
    phase = phases(rp_d, col_d, 1)
    if not maker.startswith("gpu:"):
        phase["create_from_host_ms"] = phases(g.row_ptr, g.col, 0)["create_ms"]
    log(f"[bench] phases {phase}")
    nbytes = algorithmic_bytes(g.row_ptr, g.n, k, info["hub_split_edges"], info["n_chunks"], dim)
    achieved = nbytes / (ms_epoch * 1e-3) / 1e9
    policy = {0: "store", 1: "atomic", 2: "jacobi"}[info["update_mode"]]
    # random-gather ceiling: the epoch's reads alone (col stream, 1 + k random
    # 8-byte device-scope position reads per directed edge, the source per
    # chunk) at the epoch's launch shape; the epoch makes the same reads and
    # more, so it cannot beat this time.  The read-modify-write patterns
    # (every touched position written back, by plain stores or by atomics)
    # are reported beside it.
    gather = {}
    cache_probe = {}
    if info["engine"] == SL.LAYOUT_ENGINE_GLOBAL and dim == 2:
        h = SL.layout_create_ex(rp_d, col_d, g.n, 2, k, T, seed, opts(), 1)
        for name, m in (("read", SL.LAYOUT_GATHER_READ), ("store", SL.LAYOUT_HOGWILD_STORE),
                        ("atomic", SL.LAYOUT_ATOMIC)):
            SL.layout_bench_gather(h, m, 2)
            gather[name] = SL.layout_bench_gather(h, m, 5)
        SL.layout_destroy(h)
    if args.cache_probe and dim == 2:
        # the gather pattern with each cache policy of the position accesses
        # (device-scope as in the epoch, plain, non-temporal), reads alone and
        # read-modify-writes, on a global-engine layout of the same graph
        o = opts()
        o.engine = SL.LAYOUT_ENGINE_GLOBAL
        h = SL.layout_create_ex(rp_d, col_d, g.n, 2, k, T, seed, o, 1)
        per_launch = g.row_ptr[-1] * (1 + k)
        for cname, cbits in (("device", 0), ("plain", SL.LAYOUT_GATHER_PLAIN),
                             ("nontemporal", SL.LAYOUT_GATHER_NONTEMPORAL)):
            for kname, kbits in (("read", SL.LAYOUT_GATHER_READ),
                                 ("rmw", SL.LAYOUT_HOGWILD_STORE)):
                SL.layout_bench_gather(h, kbits | cbits, 1)
                ms = SL.layout_bench_gather(h, kbits | cbits, 5)
                cache_probe[f"{kname}_{cname}"] = {
                    "ms": round(ms, 4),
                    "G_accesses_per_s": round(float(per_launch) / (ms * 1e-3) / 1e9, 2)}
        SL.layout_destroy(h)
        log(f"[bench] cache probe {cache_probe}")
    copy_ms = SL.layout_bench_copy(1 << 30, 5)
    copy_gbs = 2 * (1 << 30) / (copy_ms * 1e-3) / 1e9
    log(f"[bench] epoch {ms_epoch:.3f} ms, {achieved:.1f} GB/s algorithmic, gather {gather}, "
        f"copy {copy_gbs:.0f} GB/s")
    traffic, tinfo = (committed_traffic(args.workload) if dim == 2 and args.relabel == "none"
                      else (None, None))
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": {SL.LAYOUT_ENGINE_GLOBAL: "epoch_global_kernel",
                       SL.LAYOUT_ENGINE_LDS: "epoch_lds_kernel",
                       SL.LAYOUT_ENGINE_XCD: "epoch_xcd_kernel"}[info["engine"]]
                      + f"<{k},{policy}>",
            "algorithmic_bytes_per_launch": nbytes, "ms_per_launch": round(ms_epoch, 4),
            "measured_copy_GBs": round(copy_gbs, 1), "kernel_hash": kernel_hash()}
    if tinfo is not None and traffic is None:
        roof["traffic_note"] = "counter summary predates the current kernel source"
    if info["engine"] == SL.LAYOUT_ENGINE_XCD:
        # positions inside one XCD's L2: the ceiling is that L2's rate of
        # random 8-byte read-modify-writes with plain loads (145 G/s measured
        # over all eight XCDs on a 2 MB array, i.e. 18.1 G/s for one)
        rmw = g.row_ptr[-1] * (1 + k) / (ms_epoch * 1e-3) / 1e9
        roof["xcd_l2_rmw"] = {"achieved_G_per_s": round(float(rmw), 2), "ceiling_G_per_s": 18.1,
                              "frac": round(float(rmw) / 18.1, 3)}
    if gather:
        roof["gather_roofline_ms"] = round(gather["read"], 4)
        roof["gather_roofline_frac"] = round(gather["read"] / ms_epoch, 4)
        roof["gather_pattern_ms"] = {k_: round(v, 4) for k_, v in gather.items()}
    if cache_probe:
        roof["cache_probe"] = cache_probe
    quality = None
    if args.quality:
        quality = layout_quality(SL, rp_d, col_d, g, dim, k, T, opts, args.quality)
        log(f"[bench] quality {quality}")
    cpu = None
    if not args.no_cpu and maker.startswith("gpu:"):
        log("[bench] no CPU baseline for a device-generated workload (headline workload only)")
    elif not args.no_cpu and dim != 2:
        log("[bench] the CPU oracle baseline is timed on the 2D workload only")
    elif not args.no_cpu:
        log("[bench] timing the CPU oracle baseline")
        cpu = cpu_baseline(g, k, T, seed)
        log(f"[bench] cpu baseline {cpu['value']:.3e} edge-updates/s on {cpu['cores']} threads")
    return {
        "metric": "edge-updates/sec (|E|(1+k)/epoch time), whole layout job incl. create",
        "value": value, "unit": "edge-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": g.name, "relabel": args.relabel, "n": g.n, "edges": n_edges,
                   "k": k, "epochs": T,
                   "dim": dim, "update_mode": policy, "engine": info["engine"],
                   "bundle_edges": info["bundle_edges"],
                   "hub_split_edges": info["hub_split_edges"],
                   "grid_blocks": info["grid_blocks"]},
        "epoch_ms": round(ms_epoch, 4),
        "epoch_ms_runs": [round(x, 4) for x in runs_ms],
        "phases": phase,
        "epoch_only_value": n_edges * (1 + k) / (ms_epoch * 1e-3),
        "positions_finite": finite,
        "roofline": roof,
        "cpu_baseline": cpu,
        **({"quality": quality} if quality is not None else {}),
    }


def layout_quality(SL, rp_d, col_d, g, dim, k, T, opts, seeds):
    """NP and SI of whole layouts (seeds 0..seeds-1) from the library's own
    monitors: exact SI over all nodes (O(n^2) on the device) for the planted
    labels, and exact NP (r = 2) at 2,000 seeded sample nodes."""
    if g.labels is None or g.n > 5_000_000 or dim != 2:
        return {"skipped": "needs planted labels, a 2D layout and n <= 5M"}
    rng = np.random.default_rng(12345)
    nodes = np.sort(rng.choice(g.n, size=min(2000, g.n), replace=False)).astype(np.int32)
    runs = []
    for seed in range(seeds):
        h = SL.layout_create_ex(rp_d, col_d, g.n, dim, k, T, seed, opts(), 1)
        SL.layout_epoch(h, T)
        si = SL.layout_silhouette(h, g.labels)
        np_mean, _, _ = SL.layout_neighbourhood(h, nodes, 2)
        SL.layout_destroy(h)
        runs.append({"seed": seed, "np": round(float(np_mean), 5), "si": round(float(si), 5)})
    return {"runs": runs, "np_mean": float(np.mean([r["np"] for r in runs])),
            "si_mean": float(np.mean([r["si"] for r in runs])), "np_sample": int(nodes.size),
            "si": "exact, all nodes"}


# ---------------------------------------------------------------- batched
def bench_batched(args):
    import torch
    import synthgraph as S
    from paper_2608_01907_amd import snaplayout as SL

    k, T, count = 5, 50, args.graphs
    t0 = time.perf_counter()
    gs = S.many_graphs("batch", count, 0)
    edges = sum(g.n_edges for g in gs)
    nodes = sum(g.n for g in gs)
    log(f"[bench] {count} graphs, {nodes} nodes, {edges} edges ({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    rps = [torch.from_numpy(g.row_ptr).to(dev) for g in gs]
    cols = [torch.from_numpy(g.col).to(dev) for g in gs]
    out_d = torch.empty((nodes, 2), dtype=torch.float32, device=dev)
    desc = [{"row_ptr": rps[q], "col_idx": cols[q], "n": g.n, "seed": q}
            for q, g in enumerate(gs)]
    torch.cuda.synchronize()
    # tune once (cached), outside the timed region
    cache = os.path.join(os.environ.get("SNAP_GRAPH_CACHE", "/tmp/snap_graphs"), "tune.txt")
    h = SL.layout_batch_create(desc, k, T, SL.layout_opts_init(), 1)
    tune = SL.layout_batch_autotune(h, 2, cache)
    info = SL.layout_batch_get_info(h)
    SL.layout_batch_destroy(h)
    log(f"[bench] autotune {tune}; lds graphs {info['lds_graphs']}, global {info['global_graphs']}")

    def opts():
        o = SL.layout_opts_init()
        o.bundle_edges = tune["bundle_edges"]
        return o

    def step():
        hb = SL.layout_batch_create(desc, k, T, opts(), 1)
        SL.layout_batch_run(hb)
        SL.layout_batch_get_positions_device(hb, out_d)
        SL.layout_batch_sync(hb)
        SL.layout_batch_destroy(hb)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("[bench] warm-up done")
    t0 = time.perf_counter()
    for q in range(args.steps):
        step()
        log(f"[bench] step {q + 1}/{args.steps}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    value = edges * (1 + k) * T / dt
    hb = SL.layout_batch_create(desc, k, T, opts(), 1)
    replay_ms = SL.layout_batch_run_timed(hb)
    SL.layout_batch_destroy(hb)
    log(f"[bench] batched {dt * 1e3:.1f} ms/step, replay {replay_ms:.1f} ms; timing the plain path")
    # plain path: one graph per launch sequence, same graphs; with a sample
    # stride s > 1 the graphs are ordered by edge count and every s-th of that
    # order runs (a systematic sample over sizes, both graph kinds), the
    # total being s times the sample's
    stride = max(1, args.plain_stride)
    by_size = sorted(range(len(gs)), key=lambda q: (gs[q].nnz, q))
    sample = set(by_size[stride // 2::stride]) if stride > 1 else set(range(len(gs)))
    t0 = time.perf_counter()
    for q, g in enumerate([] if args.no_plain else gs):
        if q not in sample:
            continue
        hp = SL.layout_create_ex(rps[q], cols[q], g.n, 2, k, T, q, SL.layout_opts_init(), 1)
        SL.layout_epoch(hp, T)
        SL.layout_sync(hp)
        SL.layout_destroy(hp)
        if (q + 1) % 64 == 0:
            log(f"[bench] plain path: {q + 1}/{len(gs)} graphs, "
                f"{time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) * len(gs) / max(1, len(sample))
    plain_value = edges * (1 + k) * T / plain_s if not args.no_plain else None
    log(f"[bench] batched {dt * 1e3:.1f} ms/step (replay {replay_ms:.1f} ms), plain "
        f"{plain_s * 1e3:.1f} ms")
    return {
        "metric": "edge-updates/sec (|E|(1+k)/epoch time), batched job of many graphs",
        "value": value, "unit": "edge-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched-{count}", "graphs": count, "nodes": nodes,
                   "edges": edges, "k": k, "epochs": T, "lds_graphs": info["lds_graphs"],
                   "global_graphs": info["global_graphs"], "autotune": tune},
        "replay_ms": round(replay_ms, 3),
        "plain_one_graph_per_launch": (None if args.no_plain else
                                       {"value": plain_value, "seconds": round(plain_s, 3),
                                        "sampled_one_in": stride}),
        "speedup_vs_plain": value / plain_value if plain_value else None,
    }


# ----------------------------------------------------------------- served
def bench_served(args):
    import torch  # noqa: F401  (initialises the device for the library)
    import synthgraph as S
    from paper_2608_01907_amd import snaplayout as SL

    k, T = 5, 30
    rng = np.random.default_rng(1)
    pool = S.many_graphs("served", args.pool, 0)
    sizes = np.array([g.n_edges for g in pool], dtype=np.float64)
    log(f"[bench] pool of {len(pool)} graphs, mean |E| {sizes.mean():.0f}")
    picks = rng.integers(0, len(pool), args.jobs)

    def run_plain(order):
        lat = []
        for q in order:
            g = pool[q]
            t0 = time.perf_counter()
            h = SL.layout_create(g.row_ptr, g.col, g.n, 2, k, T, int(q))
            SL.layout_epoch(h, T)
            SL.layout_get_positions(h, g.n)
            SL.layout_destroy(h)
            lat.append(time.perf_counter() - t0)
            if len(lat) % 50 == 0:
                log(f"[bench] plain path: {len(lat)}/{len(order)} jobs")
        return np.array(lat)

    # plain service time (one job at a time) of every pool graph the stream
    # uses, measured once per graph; job i is then served in the time of its
    # own graph, svc_of[picks[i]]
    used = np.unique(picks)
    svc_of = np.full(len(pool), np.nan)
    # first, untimed: one graph of each engine's size range (the first call of
    # each engine loads its code objects)
    by_n = sorted(used, key=lambda q: pool[q].n)
    run_plain([by_n[0], by_n[len(by_n) // 2], by_n[-1]])
    svc_of[used] = run_plain(used)
    job_svc = svc_of[picks]
    mean_svc = float(job_svc.mean())
    log(f"[bench] plain service time of {used.size} graphs measured; stream mean "
        f"{mean_svc * 1e3:.1f} ms per job")
    results = {}
    for rho in args.rho:
        lam = rho / mean_svc
        arrivals = np.cumsum(rng.exponential(1.0 / lam, args.jobs))
        srv = SL.layout_server_create(args.budget, args.slots, 0)
        t_start = time.perf_counter()
        ids = []
        for q, ta in zip(picks, arrivals):
            while time.perf_counter() - t_start < ta:
                time.sleep(max(0.0, min(0.0005, ta - (time.perf_counter() - t_start))))
            g = pool[q]
            ids.append((SL.layout_server_submit(srv, g.row_ptr, g.col, g.n, k, T, int(q)), g.n))
            if len(ids) % 100 == 0:
                log(f"[bench] rho {rho}: {len(ids)}/{args.jobs} jobs submitted, "
                    f"{time.perf_counter() - t_start:.1f}s")
        log(f"[bench] rho {rho}: {len(ids)} jobs submitted")
        served_lat = []
        for q, (jid, n) in enumerate(ids):
            SL.layout_server_wait(srv, jid, 600.0)
            served_lat.append(SL.layout_server_take(srv, jid, n)[1])
            if (q + 1) % 50 == 0:
                log(f"[bench] rho {rho}: {q + 1}/{len(ids)} jobs done")
        served_lat = np.array(served_lat)
        wall = time.perf_counter() - t_start
        st = SL.layout_server_get_stats(srv)
        SL.layout_server_destroy(srv)
        # plain FIFO at the same arrivals, one job at a time in arrival order,
        # each job taking its own graph's measured plain service time
        t_free, lat = 0.0, []
        for ta, s in zip(arrivals, job_svc):
            start = max(ta, t_free)
            t_free = start + s
            lat.append(t_free - ta)
        lat = np.array(lat)
        # the jobs behind the served tail: nodes, plain service time, served
        # and FIFO latency of the five slowest served jobs
        slow = np.argsort(served_lat)[::-1][:5]
        tail = [[int(pool[picks[i]].n), round(float(job_svc[i]), 3), round(float(served_lat[i]), 3),
                 round(float(lat[i]), 3)] for i in slow]
        results[str(rho)] = {
            "served": {"p50_s": st["p50_latency_s"], "p99_s": st["p99_latency_s"],
                       "edge_updates_per_s": st["edge_updates"] / wall, "wall_s": wall,
                       "rounds": st["rounds"]},
            "plain_fifo": {"p50_s": float(np.percentile(lat, 50)),
                           "p99_s": float(np.percentile(lat, 99))},
            "slowest_served": {"columns": ["nodes", "plain_s", "served_s", "fifo_s"],
                               "jobs": tail},
        }
        log(f"[bench] rho {rho}: {results[str(rho)]}")
    # capacity: the first jobs of the stream submitted at once; makespan
    # against the sum of their plain service times
    sat_jobs = picks[: min(len(picks), 200)]
    srv = SL.layout_server_create(args.budget, args.slots, 0)
    t_start = time.perf_counter()
    ids = [(SL.layout_server_submit(srv, pool[q].row_ptr, pool[q].col, pool[q].n, k, T, int(q)),
            pool[q].n) for q in sat_jobs]
    log(f"[bench] saturation: {len(ids)} jobs submitted")
    for q, (jid, n) in enumerate(ids):
        SL.layout_server_wait(srv, jid, 1200.0)
        SL.layout_server_take(srv, jid, n)
        if (q + 1) % 50 == 0:
            log(f"[bench] saturation: {q + 1}/{len(ids)} jobs done")
    makespan = time.perf_counter() - t_start
    st = SL.layout_server_get_stats(srv)
    SL.layout_server_destroy(srv)
    plain_total = float(svc_of[sat_jobs].sum())
    saturation = {"jobs": len(ids), "makespan_s": makespan,
                  "edge_updates_per_s": st["edge_updates"] / makespan,
                  "plain_sequential_s": plain_total,
                  "plain_edge_updates_per_s": st["edge_updates"] / plain_total,
                  "speedup_vs_plain": plain_total / makespan}
    log(f"[bench] saturation: {saturation}")
    main_rho = str(args.rho[-1])
    return {
        "metric": "edge-updates/sec (|E|(1+k)/epoch time) + p50/p99 job latency, served vs plain",
        "value": results[main_rho]["served"]["edge_updates_per_s"], "unit": "edge-updates/s",
        "n_gpus": 1, "steps": args.jobs, "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "served-stream", "jobs": args.jobs, "pool": len(pool), "k": k,
                   "epochs": T, "slots": args.slots, "budget_bytes": args.budget},
        "plain_mean_service_s": mean_svc,
        "by_load": results,
        "saturation": saturation,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lj-like-4m",
                    choices=sorted(PLAIN) + ["batched-512", "served"])
    ap.add_argument("--mode", default="auto", choices=["auto", "atomic", "store"])
    ap.add_argument("--dim", type=int, default=2, choices=[2, 3],
                    help="layout dimension of the plain workloads (the paper's layouts are 2D)")
    ap.add_argument("--bundle", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--engine", default="auto", choices=["auto", "global", "xcd", "lds"],
                    help="plain workloads: the engine (default: the library's choice)")
    ap.add_argument("--quality", type=int, default=0, metavar="SEEDS",
                    help="plain workloads: also report NP and SI of this many whole layouts "
                         "(seeds 0..SEEDS-1), computed by the library's device monitors")
    ap.add_argument("--relabel", default="none", choices=["none", "degree", "community"],
                    help="plain workloads: renumber the nodes before the run (descending "
                         "degree, or by community then degree) to measure locality")
    ap.add_argument("--cache-probe", action="store_true",
                    help="also time the gather pattern under each cache policy")
    ap.add_argument("--profile-epochs", type=int, default=0,
                    help="only run this many epochs on one handle (for profilers)")
    ap.add_argument("--profile-copy", action="store_true",
                    help="only run the streaming copy (counter calibration)")
    ap.add_argument("--graphs", type=int, default=512)
    ap.add_argument("--no-plain", action="store_true",
                    help="batched workload: skip timing the one-graph-at-a-time path")
    ap.add_argument("--plain-stride", type=int, default=1,
                    help="batched workload: time every n-th graph on the plain path only")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload: skip the short batched and served runs")
    ap.add_argument("--pool", type=int, default=48)
    ap.add_argument("--jobs", type=int, default=200)
    ap.add_argument("--rho", type=float, nargs="+", default=[0.5, 0.8])
    ap.add_argument("--slots", type=int, default=128)
    ap.add_argument("--budget", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.profile_copy:
        import torch  # noqa: F401
        from paper_2608_01907_amd import snaplayout as SL

        ms = SL.layout_bench_copy(1 << 30, 3)
        log(f"[bench] copy of 1 GiB: {ms:.3f} ms per launch")
        return
    if args.workload == "batched-512":
        line = bench_batched(args)
    elif args.workload == "served":
        line = bench_served(args)
    else:
        line = bench_plain(args)
        if line is not None and args.workload == "lj-like-4m" and not args.no_extra:
            line["batched_and_served"] = extra_workloads(args)
    if line is not None:
        print(json.dumps(line), flush=True)


def extra_workloads(args):
    """Short runs of the batched and served workloads next to the headline
    one, so that one default run reports all three (the full-length runs are
    --workload batched-512 and --workload served)."""
    out = {}
    b = argparse.Namespace(**vars(args))
    b.steps, b.warmup, b.graphs, b.no_plain, b.plain_stride = 2, 1, 512, False, 8
    try:
        r = bench_batched(b)
        out["batched-512"] = {
            "value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"],
            "replay_ms": r["replay_ms"], "config": r["config"],
            "plain_one_graph_per_launch": r["plain_one_graph_per_launch"],
            "speedup_vs_plain": r["speedup_vs_plain"]}
    except Exception as exc:  # reported, never hides the headline line
        out["batched-512"] = {"error": f"{type(exc).__name__}: {exc}"}
    v = argparse.Namespace(**vars(args))
    v.jobs, v.pool, v.rho = 200, 48, [0.8]
    try:
        r = bench_served(v)
        out["served"] = {"value": r["value"], "unit": r["unit"], "config": r["config"],
                         "plain_mean_service_s": r["plain_mean_service_s"],
                         "by_load": r["by_load"], "saturation": r["saturation"]}
    except Exception as exc:
        out["served"] = {"error": f"{type(exc).__name__}: {exc}"}
    return out


if __name__ == "__main__":
    main()
