"""Throughput benchmark of the SNAP-tFDP layout on one MI355X.

A step is one whole layout job of the workload with the graph already resident
in HBM: create (device validation, chunk table, seeded init), every epoch of
the schedule, and the readout of the positions into a device buffer.

    value = |E| * (1 + k) * T / step time      (|E| undirected)

The JSON line also carries:
  roofline      -- the dominant kernel (the epoch kernel): algorithmic bytes
                   per launch / mean launch time (HIP events on the handle's
                   stream) against the 8 TB/s HBM peak, plus the measured
                   random-gather roofline of the same graph;
  cpu_baseline  -- the FP64 oracle's threaded bundle scheme timed on this
                   host's cores on a bounded sample (a few epochs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (maker, k, epochs)
    "lj-like-4m": ("lj_like", 5, 30),
    "orkut-like-259k": ("orkut_like", 5, 30),
    "sbm-2000": ("sbm_2000", 5, 50),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(row_ptr: np.ndarray, n: int, k: int, bundle: int) -> int:
    """Bytes one epoch must move at minimum: per directed edge the col entry
    (4 B) and (1 + k) position read-modify-writes (16 B each); per chunk the
    chunk-table entry and the source read + commit (16 B) for each row segment
    it covers; the row pointers of the rows touched (4 B each)."""
    nnz = int(row_ptr[-1])
    deg = np.diff(row_ptr.astype(np.int64))
    chunks = (nnz + bundle - 1) // bundle
    # a row of degree d starting at edge offset o is cut into
    # ceil((o % B + d) / B) segments
    off = row_ptr[:-1].astype(np.int64) % bundle
    segs = np.where(deg > 0, (off + deg + bundle - 1) // bundle, 0).sum()
    return int(nnz * (4 + 16 * (1 + k)) + 16 * segs + 4 * chunks + 4 * (n + 1))


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lj-like-4m", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="atomic", choices=["atomic", "store"])
    ap.add_argument("--bundle", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-epochs", type=int, default=0,
                    help="only run this many epochs on one handle (for profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synthgraph as S
    from paper_2608_01907_amd import snaplayout as SL

    maker, k, T = WORKLOADS[args.workload]
    seed = 0
    t0 = time.perf_counter()
    g = S.cached(args.workload, getattr(S, maker))
    log(f"[bench] graph {g.name}: n={g.n} |E|={g.n_edges} nnz={g.nnz} "
        f"dmax={int(g.degrees().max())} ({time.perf_counter() - t0:.1f}s)")
    mode = SL.LAYOUT_ATOMIC if args.mode == "atomic" else SL.LAYOUT_HOGWILD_STORE

    dev = torch.device("cuda:0")
    rp_d = torch.from_numpy(g.row_ptr).to(dev)
    col_d = torch.from_numpy(g.col).to(dev)
    out_d = torch.empty((g.n, 2), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def opts():
        o = SL.layout_opts_init()
        o.update_mode = mode
        o.engine = SL.LAYOUT_ENGINE_AUTO
        o.bundle_edges = args.bundle
        return o

    if args.profile_epochs:
        h = SL.layout_create_ex(rp_d, col_d, g.n, 2, k, T, seed, opts(), 1)
        SL.layout_epoch(h, args.profile_epochs)
        SL.layout_sync(h)
        SL.layout_destroy(h)
        log("[bench] profile run done")
        return

    def step():
        h = SL.layout_create_ex(rp_d, col_d, g.n, 2, k, T, seed, opts(), 1)
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
    value = g.n_edges * (1 + k) * T / (dt / args.steps)
    log(f"[bench] {args.steps} steps, {ms_step:.2f} ms/step")

    # dominant kernel: the epoch kernel, timed with HIP events on its stream
    h = SL.layout_create_ex(rp_d, col_d, g.n, 2, k, T, seed, opts(), 1)
    info = SL.layout_get_info(h)
    ms_epochs = SL.layout_epoch_timed(h, T)
    ms_epoch = ms_epochs / T
    Y = SL.layout_get_positions(h, g.n)
    finite = bool(np.all(np.isfinite(Y)))
    SL.layout_destroy(h)
    nbytes = algorithmic_bytes(g.row_ptr, g.n, k, info["bundle_edges"])
    achieved = nbytes / (ms_epoch * 1e-3) / 1e9
    # random-gather roofline of the same graph (same memory pattern, no math)
    gather = {}
    if info["engine"] == SL.LAYOUT_ENGINE_GLOBAL:
        h = SL.layout_create_ex(rp_d, col_d, g.n, 2, k, T, seed, opts(), 1)
        for name, m in (("store", SL.LAYOUT_HOGWILD_STORE), ("atomic", SL.LAYOUT_ATOMIC)):
            SL.layout_bench_gather(h, m, 2)
            gather[name] = SL.layout_bench_gather(h, m, 5)
        SL.layout_destroy(h)
    copy_ms = SL.layout_bench_copy(1 << 30, 5)
    copy_gbs = 2 * (1 << 30) / (copy_ms * 1e-3) / 1e9
    log(f"[bench] epoch {ms_epoch:.3f} ms, {achieved:.1f} GB/s algorithmic, gather {gather}, "
        f"copy {copy_gbs:.0f} GB/s")

    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"epoch_global_kernel<{k},{args.mode}>" if info["engine"] == 1 else
                      f"epoch_lds_kernel<{k},{args.mode}>",
            "bytes_per_launch": nbytes, "ms_per_launch": round(ms_epoch, 4),
            "measured_copy_GBs": round(copy_gbs, 1)}
    gkey = "atomic" if args.mode == "atomic" else "store"
    if gather:
        roof["gather_roofline_ms"] = round(gather[gkey], 4)
        roof["gather_roofline_frac"] = round(gather[gkey] / ms_epoch, 4)
        roof["gather_roofline_ms_other_mode"] = round(
            gather["store" if gkey == "atomic" else "atomic"], 4)

    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle baseline")
        cpu = cpu_baseline(g, k, T, seed)
        log(f"[bench] cpu baseline {cpu['value']:.3e} edge-updates/s on {cpu['cores']} threads")

    line = {
        "metric": "edge-updates/sec (|E|(1+k)/epoch time), whole layout job incl. create",
        "value": value, "unit": "edge-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": g.name, "n": g.n, "edges": g.n_edges, "k": k, "epochs": T,
                   "update_mode": args.mode, "engine": info["engine"],
                   "bundle_edges": info["bundle_edges"], "grid_blocks": info["grid_blocks"]},
        "epoch_ms": round(ms_epoch, 4),
        "epoch_only_value": g.n_edges * (1 + k) / (ms_epoch * 1e-3),
        "positions_finite": finite,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
