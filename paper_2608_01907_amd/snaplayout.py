"""Python binding of libsnaplayout.so (the C ABI in include/snaplayout.h).

Argument marshalling only: every step of the layout runs in the HIP library.
The functions keep the C names; numpy arrays are passed as host pointers and
torch CUDA tensors (device memory) as device pointers.  A missing library is
an error, never a fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib

LAYOUT_OK = 0
LAYOUT_E_INVALID_ARG = -1
LAYOUT_E_BAD_GRAPH = -2
LAYOUT_E_OOM = -3
LAYOUT_E_DEVICE = -4
LAYOUT_E_DONE = -5
LAYOUT_E_UNSUPPORTED = -6

LAYOUT_HOGWILD_STORE = 0
LAYOUT_ATOMIC = 1
LAYOUT_JACOBI = 2
LAYOUT_UPDATE_AUTO = 3
LAYOUT_INIT_UNIFORM = 0
LAYOUT_INIT_PMDS = 1
LAYOUT_FORCE_T = 0
LAYOUT_FORCE_GAUSSIAN = 1
LAYOUT_NEG_UNIFORM = 0
LAYOUT_NEG_DEGREE = 1
LAYOUT_NEG_CUSTOM = 2
LAYOUT_ENGINE_AUTO = 0
LAYOUT_ENGINE_GLOBAL = 1
LAYOUT_ENGINE_LDS = 2
LAYOUT_ENGINE_XCD = 3
LAYOUT_NOALLOC_MAX_NODES = 1 << 18
LAYOUT_GATHER_READ = 4
LAYOUT_GATHER_PLAIN = 0x10
LAYOUT_GATHER_NONTEMPORAL = 0x20

_NAMES = {
    LAYOUT_E_INVALID_ARG: "LAYOUT_E_INVALID_ARG", LAYOUT_E_BAD_GRAPH: "LAYOUT_E_BAD_GRAPH",
    LAYOUT_E_OOM: "LAYOUT_E_OOM", LAYOUT_E_DEVICE: "LAYOUT_E_DEVICE",
    LAYOUT_E_DONE: "LAYOUT_E_DONE", LAYOUT_E_UNSUPPORTED: "LAYOUT_E_UNSUPPORTED",
}


class LayoutError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{_NAMES.get(code, code)}: {message}")
        self.code = code


class layout_opts(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_float), ("beta", ctypes.c_float), ("gamma", ctypes.c_float),
        ("eta0", ctypes.c_float),
        ("update_mode", ctypes.c_int32), ("neg_weights", ctypes.c_int32),
        ("engine", ctypes.c_int32), ("start_epoch", ctypes.c_int32),
        ("bundle_edges", ctypes.c_int32), ("block_threads", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("hub_split_edges", ctypes.c_int32), ("nodes_per_lane", ctypes.c_int32),
        ("init_mode", ctypes.c_int32), ("pmds_pivots", ctypes.c_int32),
        ("init_pos", ctypes.c_void_p), ("stream", ctypes.c_void_p),
        ("neg_weight_values", ctypes.c_void_p), ("hot_degree", ctypes.c_int32),
        ("force_kernel", ctypes.c_int32),
    ]


class layout_info(ctypes.Structure):
    _fields_ = [
        ("engine", ctypes.c_int32), ("bundle_edges", ctypes.c_int32),
        ("block_threads", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
        ("n_chunks", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("n", ctypes.c_int32), ("k", ctypes.c_int32),
        ("epochs", ctypes.c_int32), ("update_mode", ctypes.c_int32),
        ("hub_split_edges", ctypes.c_int32), ("hot_degree", ctypes.c_int32),
    ]


class layout_graph(ctypes.Structure):
    _fields_ = [
        ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
        ("n", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("init_pos", ctypes.c_void_p),
        ("neg_weight_values", ctypes.c_void_p),
    ]


class layout_batch_info(ctypes.Structure):
    _fields_ = [
        ("graphs", ctypes.c_int32), ("lds_graphs", ctypes.c_int32),
        ("global_graphs", ctypes.c_int32), ("epochs", ctypes.c_int32),
        ("nodes", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("global_chunks", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
        ("bundle_edges", ctypes.c_int32), ("hub_split_edges", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32), ("block_threads", ctypes.c_int32),
        ("lds_block_threads", ctypes.c_int32), ("update_mode_global", ctypes.c_int32),
        ("update_mode_lds", ctypes.c_int32), ("epochs_done", ctypes.c_int32),
        ("xcd_engine", ctypes.c_int32), ("xcd_grid_blocks", ctypes.c_int32),
    ]


class layout_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64), ("rejected", ctypes.c_int64),
        ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
        ("hbm_in_use", ctypes.c_int64), ("hbm_budget", ctypes.c_int64),
        ("rounds", ctypes.c_int64),
        ("edge_updates", ctypes.c_double), ("busy_seconds", ctypes.c_double),
        ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
        ("mean_latency_s", ctypes.c_double), ("cancelled", ctypes.c_int64),
    ]


LAYOUT_JOB_QUEUED = 0
LAYOUT_JOB_RUNNING = 1
LAYOUT_JOB_DONE = 2
LAYOUT_JOB_FAILED = 3
LAYOUT_JOB_CANCELLED = 4

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_f32p = ctypes.POINTER(ctypes.c_float)

_SIGNATURES = {
    "layout_opts_init": (None, [ctypes.POINTER(layout_opts)]),
    "layout_create": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _i32, _u64, ctypes.POINTER(_vp)]),
    "layout_create_ex": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _i32, _u64,
                                        ctypes.POINTER(layout_opts), _i32, ctypes.POINTER(_vp)]),
    "layout_create64": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _i32, _u64,
                                       ctypes.POINTER(layout_opts), _i32, ctypes.POINTER(_vp)]),
    "layout_epoch": (ctypes.c_int, [_vp, _i32]),
    "layout_epoch_timed": (ctypes.c_int, [_vp, _i32, _f32p]),
    "layout_get_positions": (ctypes.c_int, [_vp, _vp]),
    "layout_get_positions_device": (ctypes.c_int, [_vp, _vp, _vp]),
    "layout_set_positions": (ctypes.c_int, [_vp, _vp]),
    "layout_status": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64)]),
    "layout_sync": (ctypes.c_int, [_vp]),
    "layout_destroy": (None, [_vp]),
    "layout_last_error": (ctypes.c_char_p, []),
    "layout_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(layout_info)]),
    "layout_debug_draws": (ctypes.c_int, [_vp, _i32, _vp]),
    "layout_silhouette": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    "layout_silhouette_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    "layout_neighbourhood": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _vp,
                                            ctypes.POINTER(ctypes.c_double)]),
    "layout_cluster_quality": (ctypes.c_int, [_vp, _vp, _i32, _u64, _i32, _vp,
                                              ctypes.POINTER(ctypes.c_double), _vp,
                                              ctypes.POINTER(_i32), _vp]),
    "layout_pmds": (ctypes.c_int, [_vp, _vp, _i32, _i32, _u64, _i32, _vp, _vp, _vp,
                                   ctypes.POINTER(_i32)]),
    "layout_sampled_energy": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]),
    "layout_effective_energy": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double)]),
    "layout_debug_alias": (ctypes.c_int, [_vp, _vp, _vp]),
    "layout_debug_draws_at": (ctypes.c_int, [_vp, _i32, _vp, _i64, _vp]),
    "layout_debug_chunks": (ctypes.c_int, [_vp, _vp, _vp]),
    "layout_bench_gather": (ctypes.c_int, [_vp, _i32, _i32, _f32p]),
    "layout_bench_copy": (ctypes.c_int, [_i64, _i32, _f32p]),
    "layout_debug_conflicts": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i64),
                                              ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "layout_bench_atomics": (ctypes.c_int, [_i32, _i32, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(_i64), ctypes.POINTER(_i64), _f32p]),
    "layout_batch_create": (ctypes.c_int, [ctypes.POINTER(layout_graph), _i32, _i32, _i32,
                                           ctypes.POINTER(layout_opts), _i32,
                                           ctypes.POINTER(_vp)]),
    "layout_batch_run": (ctypes.c_int, [_vp]),
    "layout_batch_run_timed": (ctypes.c_int, [_vp, _f32p]),
    "layout_batch_get_positions": (ctypes.c_int, [_vp, _i32, _vp]),
    "layout_batch_debug_draws": (ctypes.c_int, [_vp, _i32, _i32, _vp]),
    "layout_batch_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(layout_batch_info)]),
    "layout_batch_autotune": (ctypes.c_int, [_vp, _i32, ctypes.c_char_p,
                                             ctypes.POINTER(_i32), ctypes.POINTER(_i32), _f32p]),
    "layout_batch_destroy": (None, [_vp]),
    "layout_batch_get_positions_device": (ctypes.c_int, [_vp, _vp]),
    "layout_batch_sync": (ctypes.c_int, [_vp]),
    "layout_server_create": (ctypes.c_int, [_i64, _i32, _i64, ctypes.POINTER(layout_opts),
                                            ctypes.POINTER(_vp)]),
    "layout_server_submit": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _i32, _u64,
                                            ctypes.POINTER(_i64)]),
    "layout_server_submit_ex": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _i32, _u64, _vp, _vp,
                                               ctypes.POINTER(_i64)]),
    "layout_server_cancel": (ctypes.c_int, [_vp, _i64]),
    "layout_server_poll": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(_i32)]),
    "layout_server_wait": (ctypes.c_int, [_vp, _i64, ctypes.c_double]),
    "layout_server_take": (ctypes.c_int, [_vp, _i64, _vp, ctypes.POINTER(ctypes.c_double)]),
    "layout_server_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(layout_server_stats)]),
    "layout_server_destroy": (ctypes.c_int, [_vp]),
    "layout_server_hold": (ctypes.c_int, [_vp, _i32]),
    "layout_server_debug_draws": (ctypes.c_int, [_vp, _i64, _i32, _vp]),
}


def lib():
    return _lib.load(_SIGNATURES)


def _check(rc):
    if rc != LAYOUT_OK:
        msg = lib().layout_last_error()
        raise LayoutError(rc, msg.decode() if msg else "")


def _ptr(a, dtype=None):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if a is None:
        return None, False
    if hasattr(a, "data_ptr"):  # torch tensor
        if dtype is not None:
            assert str(a.dtype).endswith(np.dtype(dtype).name), (a.dtype, dtype)
        assert a.is_contiguous()
        return a.data_ptr(), bool(a.is_cuda)
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, False


# ----------------------------------------------------------- C-named calls
def layout_opts_init() -> layout_opts:
    o = layout_opts()
    lib().layout_opts_init(ctypes.byref(o))
    return o


def layout_create(row_ptr, col_idx, n, dim, k, epochs, seed):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    _check_csr_sizes(rp, ci, n)
    h = _vp()
    _check(lib().layout_create(rp.ctypes.data, ci.ctypes.data, n, dim, k, epochs, seed,
                               ctypes.byref(h)))
    return h


def _check_csr_sizes(row_ptr, col_idx, n):
    """Refuses arrays shorter than the library will read: row_ptr[0..n] and
    col_idx[0..row_ptr[n]) (the library validates the values themselves)."""
    def count(a):
        return int(a.numel()) if hasattr(a, "numel") else int(np.size(a))
    if n < 0:
        return  # reported by the library
    if count(row_ptr) < n + 1:
        raise LayoutError(LAYOUT_E_INVALID_ARG,
                          f"row_ptr holds {count(row_ptr)} entries; n + 1 = {n + 1} are read")
    last = row_ptr[n]
    last = int(last.item()) if hasattr(last, "item") else int(last)
    if last < 0 or last > count(col_idx):
        raise LayoutError(LAYOUT_E_INVALID_ARG,
                          f"row_ptr[n] = {last}, but col_idx holds {count(col_idx)} entries")


def _row_is_64(row_ptr):
    return "int64" in str(getattr(row_ptr, "dtype", ""))


def layout_create_ex(row_ptr, col_idx, n, dim, k, epochs, seed, opts=None, inputs_on_device=0):
    """Creates a handle; an int64 row_ptr goes through layout_create64."""
    keep = []
    _check_csr_sizes(row_ptr, col_idx, n)
    wide = _row_is_64(row_ptr)
    if inputs_on_device:
        rp_p, _ = _ptr(row_ptr)
        ci_p, _ = _ptr(col_idx)
    else:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64 if wide else np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        keep += [rp, ci]
        rp_p, ci_p = rp.ctypes.data, ci.ctypes.data
    o = opts if opts is not None else layout_opts_init()
    h = _vp()
    create = lib().layout_create64 if wide else lib().layout_create_ex
    _check(create(rp_p, ci_p, n, dim, k, epochs, seed, ctypes.byref(o), int(inputs_on_device),
                  ctypes.byref(h)))
    del keep
    return h


def layout_create64(row_ptr, col_idx, n, dim, k, epochs, seed, opts=None, inputs_on_device=0):
    """layout_create_ex with 64-bit row pointers (int64 numpy array or tensor)."""
    if not hasattr(row_ptr, "data_ptr"):
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    elif not _row_is_64(row_ptr):
        raise LayoutError(LAYOUT_E_INVALID_ARG, "layout_create64 needs an int64 row_ptr")
    return layout_create_ex(row_ptr, col_idx, n, dim, k, epochs, seed, opts, inputs_on_device)


def layout_epoch(h, count):
    _check(lib().layout_epoch(h, count))


def layout_epoch_timed(h, count):
    ms = ctypes.c_float()
    _check(lib().layout_epoch_timed(h, count, ctypes.byref(ms)))
    return ms.value


def layout_get_positions(h, n, dim=2):
    out = np.zeros((n, dim), dtype=np.float32)
    _check(lib().layout_get_positions(h, out.ctypes.data))
    return out


def layout_get_positions_device(h, dev_out, stream=None):
    p, on_dev = _ptr(dev_out)
    if not on_dev:
        raise LayoutError(LAYOUT_E_INVALID_ARG, "dev_out must be a device tensor")
    _check(lib().layout_get_positions_device(h, p, stream))


def layout_set_positions(h, Y):
    arr = np.ascontiguousarray(Y, dtype=np.float32)
    _check(lib().layout_set_positions(h, arr.ctypes.data))


def layout_status(h):
    t = _i32()
    b = _i64()
    _check(lib().layout_status(h, ctypes.byref(t), ctypes.byref(b)))
    return t.value, b.value


def layout_sync(h):
    _check(lib().layout_sync(h))


def layout_destroy(h):
    lib().layout_destroy(h)


def layout_last_error():
    m = lib().layout_last_error()
    return m.decode() if m else ""


def layout_get_info(h) -> dict:
    info = layout_info()
    _check(lib().layout_get_info(h, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in layout_info._fields_}


def layout_debug_draws(h, epoch, nnz, k):
    out = np.zeros((max(nnz, 1), max(k, 1)), dtype=np.int32)
    _check(lib().layout_debug_draws(h, epoch, out.ctypes.data))
    return out[:nnz, :k]


def layout_pmds(row_ptr, col_idx, n, pivots=0, seed=0, want_detail=False):
    """Pivot MDS layout (n x 2 float32); with want_detail also the pivots and
    their hop distances (pivots x n, -1 = unreachable)."""
    _check_csr_sizes(row_ptr, col_idx, n)
    on_device = hasattr(row_ptr, "data_ptr") and row_ptr.is_cuda
    if on_device:
        rp, ci = row_ptr.data_ptr(), col_idx.data_ptr()
    else:
        rp_a = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci_a = np.ascontiguousarray(col_idx, dtype=np.int32)
        rp, ci = rp_a.ctypes.data, (ci_a.ctypes.data if ci_a.size else rp_a.ctypes.data)
    Y = np.zeros((max(n, 1), 2), dtype=np.float32)
    p = pivots if pivots else 50
    piv = np.zeros(p, dtype=np.int32)
    dist = np.zeros((p, max(n, 1)), dtype=np.int32) if want_detail else None
    used = _i32()
    _check(lib().layout_pmds(rp, ci, int(n), int(pivots), int(seed), int(on_device),
                             Y.ctypes.data, piv.ctypes.data,
                             dist.ctypes.data if dist is not None else None,
                             ctypes.byref(used)))
    Y = Y[:n]
    if not want_detail:
        return Y
    u = used.value
    return Y, piv[:u].copy(), dist[:u, :n].copy()


def layout_silhouette(h, labels):
    """Exact silhouette index of the current positions for the given labels."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = ctypes.c_double()
    _check(lib().layout_silhouette(h, lab.ctypes.data, ctypes.byref(out)))
    return out.value


def layout_silhouette_noalloc(h, labels):
    """As layout_silhouette, with the library's fixed device scratch array
    instead of temporary allocations (at most 2^18 nodes)."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = ctypes.c_double()
    _check(lib().layout_silhouette_noalloc(h, lab.ctypes.data, ctypes.byref(out)))
    return out.value


def layout_neighbourhood(h, nodes, radius=2):
    """(NP mean, k_i, |R_i ∩ K_i|) at the query nodes (exact, FP32 ranking)."""
    q = np.ascontiguousarray(nodes, dtype=np.int32)
    k = np.zeros(max(q.size, 1), dtype=np.int32)
    inter = np.zeros(max(q.size, 1), dtype=np.int32)
    out = ctypes.c_double()
    _check(lib().layout_neighbourhood(h, q.ctypes.data, int(q.size), int(radius), k.ctypes.data,
                                      inter.ctypes.data, ctypes.byref(out)))
    return out.value, k[:q.size], inter[:q.size]


def layout_cluster_quality(h, labels, clusters=0, seed=0, max_iter=300, init_centers=None):
    """(CQ, assignment, iterations, k-means++ center indices) of the layout."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    n = lab.size
    K = clusters if clusters else int(np.unique(lab).size)
    ic = None if init_centers is None else np.ascontiguousarray(init_centers, dtype=np.float32)
    assign = np.zeros(max(n, 1), dtype=np.int32)
    centers = np.zeros(max(K, 1), dtype=np.int32)
    cq, iters = ctypes.c_double(), _i32()
    _check(lib().layout_cluster_quality(h, lab.ctypes.data, int(clusters), int(seed),
                                        int(max_iter), None if ic is None else ic.ctypes.data,
                                        ctypes.byref(cq), assign.ctypes.data, ctypes.byref(iters),
                                        centers.ctypes.data))
    return cq.value, assign[:n], iters.value, centers[:K]


def layout_debug_conflicts(h, count):
    """(writes, conflicting writes, untracked writes) over count epochs."""
    st, cf, un = _i64(), _i64(), _i64()
    _check(lib().layout_debug_conflicts(h, int(count), ctypes.byref(st), ctypes.byref(cf),
                                        ctypes.byref(un)))
    return st.value, cf.value, un.value


def layout_bench_atomics(reps, spread=0):
    """(FP64 total, u64 total, adds per kind, ms) of the atomic probe."""
    f, i, a, ms = ctypes.c_double(), _i64(), _i64(), ctypes.c_float()
    _check(lib().layout_bench_atomics(int(reps), int(spread), ctypes.byref(f), ctypes.byref(i),
                                      ctypes.byref(a), ctypes.byref(ms)))
    return f.value, i.value, a.value, ms.value


def layout_sampled_energy(h, epoch):
    """(attraction, repulsion) energy seen by the samples of `epoch`."""
    a, r = ctypes.c_double(), ctypes.c_double()
    _check(lib().layout_sampled_energy(h, epoch, ctypes.byref(a), ctypes.byref(r)))
    return a.value, r.value


def layout_effective_energy(h):
    """(attraction, weighted repulsion) of the degree-weighted objective."""
    a, r = ctypes.c_double(), ctypes.c_double()
    _check(lib().layout_effective_energy(h, ctypes.byref(a), ctypes.byref(r)))
    return a.value, r.value


def layout_debug_draws_at(h, epoch, edges, k):
    """Negatives of the listed directed edges (len(edges) x k)."""
    e = np.ascontiguousarray(edges, dtype=np.int64)
    out = np.zeros((max(e.size, 1), max(k, 1)), dtype=np.int32)
    _check(lib().layout_debug_draws_at(h, epoch, e.ctypes.data, int(e.size), out.ctypes.data))
    return out[: e.size, :k]


def layout_debug_chunks(h):
    n_chunks = layout_get_info(h)["n_chunks"]
    begin = np.zeros(n_chunks + 1, dtype=np.int64)
    src = np.zeros(max(n_chunks, 1), dtype=np.int32)
    _check(lib().layout_debug_chunks(h, begin.ctypes.data, src.ctypes.data))
    return begin, src[:n_chunks]


def layout_debug_alias(h, n):
    thr = np.zeros(max(n, 1), dtype=np.uint32)
    alias = np.zeros(max(n, 1), dtype=np.uint32)
    _check(lib().layout_debug_alias(h, thr.ctypes.data, alias.ctypes.data))
    return thr[:n], alias[:n]


def layout_bench_gather(h, mode, reps):
    ms = ctypes.c_float()
    _check(lib().layout_bench_gather(h, mode, reps, ctypes.byref(ms)))
    return ms.value


def layout_bench_copy(nbytes, reps):
    ms = ctypes.c_float()
    _check(lib().layout_bench_copy(int(nbytes), reps, ctypes.byref(ms)))
    return ms.value


# ------------------------------------------------------------- batches
def layout_batch_create(graphs, k, epochs, opts=None, inputs_on_device=0):
    """graphs: list of dicts with row_ptr, col_idx, n, seed[, init_pos,
    neg_weight_values]."""
    arr = (layout_graph * len(graphs))()
    keep = []
    for q, g in enumerate(graphs):
        _check_csr_sizes(g["row_ptr"], g["col_idx"], g["n"])
        if inputs_on_device:
            rp_p, ci_p = _ptr(g["row_ptr"])[0], _ptr(g["col_idx"])[0]
            ip = _ptr(g.get("init_pos"))[0]
            wp = _ptr(g.get("neg_weight_values"))[0]
        else:
            rp = np.ascontiguousarray(g["row_ptr"], dtype=np.int32)
            ci = np.ascontiguousarray(g["col_idx"], dtype=np.int32)
            keep += [rp, ci]
            rp_p, ci_p = rp.ctypes.data, ci.ctypes.data
            ip = None
            if g.get("init_pos") is not None:
                a = np.ascontiguousarray(g["init_pos"], dtype=np.float32)
                keep.append(a)
                ip = a.ctypes.data
            wp = None
            if g.get("neg_weight_values") is not None:
                w = np.ascontiguousarray(g["neg_weight_values"], dtype=np.uint32)
                keep.append(w)
                wp = w.ctypes.data
        arr[q].row_ptr, arr[q].col_idx, arr[q].n = rp_p, ci_p, int(g["n"])
        arr[q].seed, arr[q].init_pos = int(g.get("seed", 0)), ip
        arr[q].neg_weight_values = wp
    o = opts if opts is not None else layout_opts_init()
    h = _vp()
    _check(lib().layout_batch_create(arr, len(graphs), k, epochs, ctypes.byref(o),
                                     int(inputs_on_device), ctypes.byref(h)))
    del keep
    return h


def layout_batch_run(h):
    _check(lib().layout_batch_run(h))


def layout_batch_run_timed(h):
    ms = ctypes.c_float()
    _check(lib().layout_batch_run_timed(h, ctypes.byref(ms)))
    return ms.value


def layout_batch_get_positions(h, g, n):
    out = np.zeros((n, 2), dtype=np.float32)
    _check(lib().layout_batch_get_positions(h, g, out.ctypes.data))
    return out


def layout_batch_get_positions_device(h, dev_out):
    p, on_dev = _ptr(dev_out)
    if not on_dev:
        raise LayoutError(LAYOUT_E_INVALID_ARG, "dev_out must be a device tensor")
    _check(lib().layout_batch_get_positions_device(h, p))


def layout_batch_sync(h):
    _check(lib().layout_batch_sync(h))


def layout_batch_debug_draws(h, g, epoch, nnz, k):
    out = np.zeros((max(nnz, 1), max(k, 1)), dtype=np.int32)
    _check(lib().layout_batch_debug_draws(h, g, epoch, out.ctypes.data))
    return out[:nnz, :k]


def layout_batch_get_info(h) -> dict:
    info = layout_batch_info()
    _check(lib().layout_batch_get_info(h, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in layout_batch_info._fields_}


def layout_batch_autotune(h, trial_epochs=2, cache_path=None):
    b, p, ms = _i32(), _i32(), ctypes.c_float()
    cp = cache_path.encode() if cache_path else None
    _check(lib().layout_batch_autotune(h, trial_epochs, cp, ctypes.byref(b), ctypes.byref(p),
                                       ctypes.byref(ms)))
    return {"bundle_edges": b.value, "blocks_per_cu": p.value, "epoch_ms": ms.value}


def layout_batch_destroy(h):
    lib().layout_batch_destroy(h)


# --------------------------------------------------------------- server
def layout_server_create(hbm_budget_bytes=0, max_slots=64, round_edges=0, opts=None):
    o = opts if opts is not None else layout_opts_init()
    h = _vp()
    _check(lib().layout_server_create(int(hbm_budget_bytes), int(max_slots), int(round_edges),
                                      ctypes.byref(o), ctypes.byref(h)))
    return h


def layout_server_submit(h, row_ptr, col_idx, n, k, epochs, seed):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    _check_csr_sizes(rp, ci, n)
    jid = _i64()
    _check(lib().layout_server_submit(h, rp.ctypes.data, ci.ctypes.data, n, k, epochs, seed,
                                      ctypes.byref(jid)))
    return jid.value


def layout_server_submit_ex(h, row_ptr, col_idx, n, k, epochs, seed, neg_weight_values=None,
                            init_pos=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    _check_csr_sizes(rp, ci, n)
    w = None if neg_weight_values is None else np.ascontiguousarray(neg_weight_values,
                                                                    dtype=np.uint32)
    ip = None if init_pos is None else np.ascontiguousarray(init_pos, dtype=np.float32)
    jid = _i64()
    _check(lib().layout_server_submit_ex(h, rp.ctypes.data, ci.ctypes.data, n, k, epochs, seed,
                                         None if w is None else w.ctypes.data,
                                         None if ip is None else ip.ctypes.data,
                                         ctypes.byref(jid)))
    return jid.value


def layout_server_cancel(h, job):
    _check(lib().layout_server_cancel(h, job))


def layout_server_poll(h, job):
    st = _i32()
    _check(lib().layout_server_poll(h, job, ctypes.byref(st)))
    return st.value


def layout_server_wait(h, job, timeout_s=-1.0):
    _check(lib().layout_server_wait(h, job, float(timeout_s)))


def layout_server_take(h, job, n):
    out = np.zeros((max(n, 1), 2), dtype=np.float32)
    lat = ctypes.c_double()
    _check(lib().layout_server_take(h, job, out.ctypes.data, ctypes.byref(lat)))
    return out[:n], lat.value


def layout_server_get_stats(h) -> dict:
    st = layout_server_stats()
    _check(lib().layout_server_get_stats(h, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in layout_server_stats._fields_}


def layout_server_hold(h, hold=True):
    _check(lib().layout_server_hold(h, int(bool(hold))))


def layout_server_debug_draws(h, job, epoch, nnz, k):
    """Negatives of a queued or running job in one epoch, (nnz, k) int32."""
    out = np.zeros(max(int(nnz) * int(k), 1), dtype=np.int32)
    _check(lib().layout_server_debug_draws(h, _i64(job), int(epoch), out.ctypes.data))
    return out[: int(nnz) * int(k)].reshape(int(nnz), int(k))


def layout_server_destroy(h):
    _check(lib().layout_server_destroy(h))


# --------------------------------------------------------- convenience
class Layout:
    """One layout job: owns a handle; positions come back as numpy arrays."""

    def __init__(self, row_ptr, col_idx, n, k=5, epochs=50, seed=0, *,
                 update_mode=LAYOUT_UPDATE_AUTO,
                 neg_weights=LAYOUT_NEG_UNIFORM, engine=LAYOUT_ENGINE_AUTO, eta0=1.0,
                 alpha=0.1, beta=8.0, gamma=2.0, init_pos=None, bundle_edges=0,
                 block_threads=0, grid_blocks=0, start_epoch=0, stream=None,
                 hub_split_edges=0, nodes_per_lane=0, init_mode=LAYOUT_INIT_UNIFORM,
                 pmds_pivots=0, neg_weight_values=None, dim=2, hot_degree=0,
                 force_kernel=LAYOUT_FORCE_T):
        o = layout_opts_init()
        o.hot_degree = hot_degree
        o.force_kernel = force_kernel
        o.init_mode, o.pmds_pivots = init_mode, pmds_pivots
        w_keep = None
        if neg_weight_values is not None:
            if hasattr(neg_weight_values, "data_ptr"):
                o.neg_weight_values = neg_weight_values.data_ptr()
            else:
                w_keep = np.ascontiguousarray(neg_weight_values, dtype=np.uint32)
                o.neg_weight_values = w_keep.ctypes.data
        o.alpha, o.beta, o.gamma, o.eta0 = alpha, beta, gamma, eta0
        o.update_mode, o.neg_weights, o.engine = update_mode, neg_weights, engine
        o.bundle_edges, o.block_threads, o.grid_blocks = bundle_edges, block_threads, grid_blocks
        o.start_epoch = start_epoch
        o.hub_split_edges = hub_split_edges
        o.nodes_per_lane = nodes_per_lane
        on_device = hasattr(row_ptr, "data_ptr") and row_ptr.is_cuda
        init_keep = None
        if init_pos is not None:
            if on_device:
                o.init_pos = init_pos.data_ptr()
            else:
                init_keep = np.ascontiguousarray(init_pos, dtype=np.float32)
                o.init_pos = init_keep.ctypes.data
        if stream is not None:
            o.stream = stream
        self.n, self.k, self.epochs, self.dim = int(n), int(k), int(epochs), int(dim)
        self.nnz = int(row_ptr[-1]) if not on_device else int(row_ptr[-1].item())
        self.h = layout_create_ex(row_ptr, col_idx, self.n, self.dim, self.k, self.epochs, seed,
                                  o, int(on_device))
        del init_keep, w_keep

    def run(self, count=None):
        layout_epoch(self.h, self.epochs if count is None else count)
        return self

    def run_timed(self, count=None):
        return layout_epoch_timed(self.h, self.epochs if count is None else count)

    def positions(self):
        return layout_get_positions(self.h, self.n, self.dim)

    def set_positions(self, Y):
        layout_set_positions(self.h, Y)

    def draws(self, epoch):
        return layout_debug_draws(self.h, epoch, self.nnz, self.k)

    def info(self):
        return layout_get_info(self.h)

    def sampled_energy(self, epoch):
        return layout_sampled_energy(self.h, epoch)

    def silhouette(self, labels):
        return layout_silhouette(self.h, labels)

    def effective_energy(self):
        return layout_effective_energy(self.h)

    def neighbourhood(self, nodes, radius=2):
        return layout_neighbourhood(self.h, nodes, radius)

    def cluster_quality(self, labels, clusters=0, seed=0, max_iter=300, init_centers=None):
        return layout_cluster_quality(self.h, labels, clusters, seed, max_iter, init_centers)

    def status(self):
        return layout_status(self.h)

    def sync(self):
        layout_sync(self.h)

    def close(self):
        if getattr(self, "h", None):
            layout_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BatchLayout:
    """Many graphs laid out together (one HIP graph replay for all epochs)."""

    def __init__(self, graphs, k=5, epochs=50, *, update_mode=LAYOUT_UPDATE_AUTO,
                 engine=LAYOUT_ENGINE_AUTO, eta0=1.0, bundle_edges=0, hub_split_edges=0,
                 block_threads=0, grid_blocks=0, neg_weights=LAYOUT_NEG_UNIFORM,
                 nodes_per_lane=0, init_mode=LAYOUT_INIT_UNIFORM, pmds_pivots=0,
                 force_kernel=LAYOUT_FORCE_T, gamma=2.0):
        o = layout_opts_init()
        o.update_mode, o.engine, o.eta0 = update_mode, engine, eta0
        o.force_kernel, o.gamma = force_kernel, gamma
        o.init_mode, o.pmds_pivots = init_mode, pmds_pivots
        o.bundle_edges, o.hub_split_edges = bundle_edges, hub_split_edges
        o.block_threads, o.grid_blocks, o.neg_weights = block_threads, grid_blocks, neg_weights
        o.nodes_per_lane = nodes_per_lane
        self.n = [int(g["n"]) for g in graphs]
        self.nnz = [int(np.asarray(g["row_ptr"])[-1]) for g in graphs]
        self.k, self.epochs = int(k), int(epochs)
        self.h = layout_batch_create(graphs, self.k, self.epochs, o)

    def autotune(self, trial_epochs=2, cache_path=None):
        return layout_batch_autotune(self.h, trial_epochs, cache_path)

    def run(self):
        layout_batch_run(self.h)
        return self

    def run_timed(self):
        return layout_batch_run_timed(self.h)

    def positions(self, g):
        return layout_batch_get_positions(self.h, g, self.n[g])

    def draws(self, g, epoch):
        return layout_batch_debug_draws(self.h, g, epoch, self.nnz[g], self.k)

    def info(self):
        return layout_batch_get_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            layout_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
