"""SNAP-tFDP CPU oracle (FP64) -- test infrastructure only.

Thin ctypes wrapper around ``snap_oracle.c``.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import this module; the
product path never does.  Every function follows the paper:

* forces: Table 1 (t-FDP row), alpha=0.1, beta=8, gamma=2 (Sec. 3.1, t-FDP
  parameters inherited as stated in Sec. 4.2);
* the stochastic epoch: Algorithm 1 and Sec. 3.3 (immediate updates, directed
  edge duplication, k uniform negatives per directed edge);
* the expectation / effective energy: Sec. 3.3, Eq. (4) with the weight
  k (d_i + d_j) / (|V| - 1);
* the threaded bundle scheme: Sec. 3.4.

The random-number layout (Philox4x64-10 key/counter layout, Lemire reduction,
alias sweep) is documented in the header of ``snap_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "snap_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

NEG_UNIFORM = 0
NEG_DEGREE = 1
ORDER_SHUFFLED = 0
ORDER_CSR = 1

ALPHA, BETA, GAMMA, ETA0 = 0.1, 8.0, 2.0, 1.0
FORCE_T = 0         # Table 1, t-FDP row (Student-t kernel 1/(1+q))
FORCE_GAUSSIAN = 1  # the Gaussian kernel exp(-q/2) in place of 1/(1+q) (see snap_oracle.c)
KEY_DOMAIN = 0x534E41502D744644  # second key word of every draw ("SNAP-tFD")

_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FP contraction, so FP32 init rounds once)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
            "-ffp-contract=off", "-o", tmp, SRC, "-lm", "-lpthread",
        ])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        L.oracle_philox_bulk.argtypes = [ctypes.c_uint64] * 6 + [ctypes.c_int64, _u64p]
        L.oracle_philox_bulk.restype = None
        L.oracle_init_positions.argtypes = [ctypes.c_int64, ctypes.c_uint64, _f64p]
        L.oracle_init_positions.restype = None
        L.oracle_init_positions_scaled.argtypes = [ctypes.c_int64, ctypes.c_uint64,
                                                   ctypes.c_float, _f64p]
        L.oracle_init_positions_scaled.restype = None
        L.oracle_init_positions_dim.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_float,
                                                ctypes.c_int32, _f64p]
        L.oracle_init_positions_dim.restype = None
        L.oracle_init_positions_at.argtypes = [ctypes.c_int64, ctypes.c_uint64, _i64p,
                                               ctypes.c_int64, _f64p]
        L.oracle_init_positions_at.restype = None
        L.oracle_draw_edges.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                        ctypes.c_uint64, ctypes.c_int32, _u32p, _u32p, _i64p,
                                        _i32p, ctypes.c_int64, _i32p]
        L.oracle_draw_edges.restype = ctypes.c_int
        L.oracle_alias_build.argtypes = [_i64p, ctypes.c_int64, _u32p, _u32p]
        L.oracle_alias_build.restype = ctypes.c_int
        L.oracle_draw_negatives.argtypes = [
            _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
            ctypes.c_int32, _u32p, _u32p, _i32p]
        L.oracle_draw_negatives.restype = ctypes.c_int
        L.oracle_force_magnitudes.argtypes = [ctypes.c_double] * 4 + [
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.oracle_force_magnitudes.restype = None
        L.oracle_serial_run.argtypes = [
            _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _u32p, _u32p, ctypes.c_int32, _f64p]
        L.oracle_serial_run.restype = ctypes.c_int
        L.oracle_serial_run_ordered.argtypes = [
            _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_int32, _u32p, _u32p, ctypes.c_int32, _i64p, _f64p]
        L.oracle_serial_run_ordered.restype = ctypes.c_int
        L.oracle_pair_energies.argtypes = [ctypes.c_double] * 4 + [
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.oracle_pair_energies.restype = None
        L.oracle_set_force_kernel.argtypes = [ctypes.c_int32]
        L.oracle_set_force_kernel.restype = None
        L.oracle_jacobi_epoch.argtypes = [
            _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_uint64, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_int32, _u32p, _u32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _f64p,
            _f64p, ctypes.c_void_p]
        L.oracle_jacobi_epoch.restype = ctypes.c_int
        L.oracle_sampled_energy.argtypes = [
            _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _u32p, _u32p,
            _f64p, _f64p]
        L.oracle_sampled_energy.restype = ctypes.c_double
        L.oracle_effective_energy.argtypes = [
            _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, _f64p, _f64p]
        L.oracle_effective_energy.restype = ctypes.c_double
        L.oracle_threaded_run.argtypes = [
            _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_int32, _u32p, _u32p, ctypes.c_int32, _f64p]
        L.oracle_threaded_run.restype = ctypes.c_int
        _lib = L
    return _lib


# ----------------------------------------------------------------- helpers
def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    if c.size == 0:
        c = np.zeros(1, dtype=np.int32)
    return rp, c


def _tables(n, thr, alias):
    if thr is None:
        thr = np.zeros(max(n, 1), dtype=np.uint32)
        alias = np.zeros(max(n, 1), dtype=np.uint32)
    return (np.ascontiguousarray(thr, dtype=np.uint32),
            np.ascontiguousarray(alias, dtype=np.uint32))


def _kernel(kernel):
    """Selects the force kernel for the next oracle call."""
    if kernel not in (FORCE_T, FORCE_GAUSSIAN):
        raise ValueError(f"unknown force kernel {kernel}")
    lib().oracle_set_force_kernel(int(kernel))


# -------------------------------------------------------------------- API
def philox_bulk(key, ctr, count):
    """Philox4x64-10 blocks for counters (ctr0 + r, ctr1, ctr2, ctr3), r < count."""
    out = np.zeros(4 * count, dtype=np.uint64)
    lib().oracle_philox_bulk(int(key[0]), int(key[1]), int(ctr[0]), int(ctr[1]), int(ctr[2]),
                             int(ctr[3]), int(count), out)
    return out.reshape(count, 4)


def init_positions(n, seed, dim=2):
    """Seeded uniform init in [-sqrt(n), sqrt(n)]^dim (FP32 values, widened)."""
    Y = np.zeros(dim * max(n, 1), dtype=np.float64)
    if dim == 2:
        lib().oracle_init_positions(int(n), int(seed), Y)
    else:
        lib().oracle_init_positions_dim(int(n), int(seed), float(np.sqrt(np.float32(n))),
                                        int(dim), Y)
    return Y[: dim * n].reshape(n, dim)


def init_positions_scaled(n, seed, scale):
    """The same uniform draws in [-scale, scale]^2 (scale taken as FP32)."""
    Y = np.zeros(2 * max(n, 1), dtype=np.float64)
    lib().oracle_init_positions_scaled(int(n), int(seed), float(scale), Y)
    return Y[: 2 * n].reshape(n, 2)


def init_positions_at(n, seed, nodes):
    """Initial positions (as init_positions) of the listed nodes only."""
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    Y = np.zeros(2 * max(nodes.size, 1), dtype=np.float64)
    lib().oracle_init_positions_at(int(n), int(seed), nodes, int(nodes.size), Y)
    return Y[: 2 * nodes.size].reshape(-1, 2)


def draw_edges(row_ptr, n, k, t, seed, edges, mode=NEG_UNIFORM, thr=None, alias=None):
    """Negatives (as draw_negatives) of the listed directed edges only."""
    edges = np.ascontiguousarray(edges, dtype=np.int64)
    src = (np.searchsorted(np.asarray(row_ptr, dtype=np.int64), edges, side="right") - 1)
    src = np.ascontiguousarray(src, dtype=np.int32)
    thr, alias = _tables(n, thr, alias)
    out = np.zeros(max(edges.size * k, 1), dtype=np.int32)
    lib().oracle_draw_edges(int(n), int(k), int(t), int(seed), int(mode), thr, alias, edges, src,
                            int(edges.size), out)
    return out[: edges.size * k].reshape(-1, k)


def alias_build(w):
    """Integer alias table (thr, alias) for non-negative integer weights w."""
    w = np.ascontiguousarray(w, dtype=np.int64)
    n = w.size
    thr = np.zeros(n, dtype=np.uint32)
    alias = np.zeros(n, dtype=np.uint32)
    rc = lib().oracle_alias_build(w, n, thr, alias)
    if rc != 0:
        raise ValueError("alias_build: weights must be non-negative with 0 < sum < 2^32")
    return thr, alias


def draw_negatives(row_ptr, col, n, k, t, seed, mode=NEG_UNIFORM, thr=None, alias=None):
    """All negatives of epoch t as an (nnz, k) int32 array."""
    rp, c = _csr(row_ptr, col)
    thr, alias = _tables(n, thr, alias)
    nnz = int(rp[n])
    out = np.zeros(max(nnz * k, 1), dtype=np.int32)
    lib().oracle_draw_negatives(rp, c, int(n), int(k), int(t), int(seed), int(mode), thr, alias,
                                out)
    return out[: nnz * k].reshape(nnz, k)


def force_magnitudes(dist, alpha=ALPHA, beta=BETA, gamma=GAMMA, kernel=FORCE_T):
    _kernel(kernel)
    fa, fr = ctypes.c_double(), ctypes.c_double()
    lib().oracle_force_magnitudes(alpha, beta, gamma, float(dist), ctypes.byref(fa),
                                  ctypes.byref(fr))
    return fa.value, fr.value


def pair_energies(dist, alpha=ALPHA, beta=BETA, gamma=GAMMA, kernel=FORCE_T):
    """(U_a, U_r) at distance dist: the pair energies whose negative gradients
    are the Table 1 forces (Eq. (2))."""
    _kernel(kernel)
    ua, ur = ctypes.c_double(), ctypes.c_double()
    lib().oracle_pair_energies(alpha, beta, gamma, float(dist), ctypes.byref(ua),
                               ctypes.byref(ur))
    return ua.value, ur.value


def serial_run(row_ptr, col, n, k, T, seed, Y0=None, t_begin=0, t_end=None,
               order=ORDER_SHUFFLED, mode=NEG_UNIFORM, thr=None, alias=None,
               alpha=ALPHA, beta=BETA, gamma=GAMMA, kernel=FORCE_T, eta0=ETA0, dim=None):
    """Serial Algorithm 1 in FP64 over epochs [t_begin, t_end) of a T-epoch run;
    dim (2 or 3) defaults to the width of Y0, else 2."""
    _kernel(kernel)
    rp, c = _csr(row_ptr, col)
    thr, alias = _tables(n, thr, alias)
    if t_end is None:
        t_end = T
    if dim is None:
        dim = 2 if Y0 is None else int(np.asarray(Y0).reshape(n, -1).shape[1]) if n else 2
    Y = init_positions(n, seed, dim) if Y0 is None else np.array(Y0, dtype=np.float64)
    Y = np.ascontiguousarray(Y.reshape(-1))
    if Y.size == 0:
        Y = np.zeros(dim, dtype=np.float64)
    lib().oracle_serial_run(rp, c, int(n), int(k), int(t_begin), int(t_end), int(T), int(seed),
                            alpha, beta, gamma, eta0, int(order), int(mode), thr, alias, int(dim),
                            Y)
    return Y[: dim * n].reshape(n, dim)


def serial_run_ordered(row_ptr, col, n, k, T, seed, edge_order, Y0=None, t_begin=0,
                       t_end=None, mode=NEG_UNIFORM, thr=None, alias=None, alpha=ALPHA,
                       beta=BETA, gamma=GAMMA, kernel=FORCE_T, eta0=ETA0):
    """Serial Algorithm 1 (2D) visiting the directed edges in the given order
    (a permutation of [0, nnz)); draws stay keyed by CSR position."""
    _kernel(kernel)
    rp, c = _csr(row_ptr, col)
    thr, alias = _tables(n, thr, alias)
    if t_end is None:
        t_end = T
    order = np.ascontiguousarray(edge_order, dtype=np.int64)
    if order.size == 0:
        order = np.zeros(1, dtype=np.int64)
    Y = init_positions(n, seed) if Y0 is None else np.array(Y0, dtype=np.float64)
    Y = np.ascontiguousarray(Y.reshape(-1))
    rc = lib().oracle_serial_run_ordered(rp, c, int(n), int(k), int(t_begin), int(t_end), int(T),
                                         int(seed), alpha, beta, gamma, eta0, int(mode), thr,
                                         alias, 2, order, Y)
    if rc != 0:
        raise ValueError("serial_run_ordered: edge_order is not a permutation of [0, nnz)")
    return Y[: 2 * n].reshape(n, 2)


def jacobi_epoch(row_ptr, col, n, k, t, T, seed, Y, mode=NEG_UNIFORM, thr=None, alias=None,
                 use_attr=True, use_rep=True, alpha=ALPHA, beta=BETA, gamma=GAMMA, kernel=FORCE_T, eta0=ETA0,
                 want_abs=False):
    """One synchronous epoch from Y (n x 2 or n x 3); returns Y_out (and the
    |contribution| sums)."""
    _kernel(kernel)
    rp, c = _csr(row_ptr, col)
    thr, alias = _tables(n, thr, alias)
    dim = int(np.asarray(Y).reshape(n, -1).shape[1]) if n else 2
    Yin = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(-1))
    Yout = np.zeros_like(Yin)
    absd = np.zeros_like(Yin) if want_abs else None
    lib().oracle_jacobi_epoch(rp, c, int(n), int(k), int(t), int(T), int(seed), alpha, beta,
                              gamma, eta0, int(mode), thr, alias, int(bool(use_attr)),
                              int(bool(use_rep)), dim, Yin, Yout,
                              absd.ctypes.data if want_abs else None)
    if want_abs:
        return Yout.reshape(n, dim), absd.reshape(n, dim)
    return Yout.reshape(n, dim)


def sampled_energy(row_ptr, col, n, k, t, seed, Y, mode=NEG_UNIFORM, thr=None, alias=None,
                   alpha=ALPHA, beta=BETA, gamma=GAMMA, kernel=FORCE_T, parts=False):
    """Energy seen by the samples of epoch t at fixed Y (Sec. 3.3); with
    parts=True the pair (attraction, repulsion)."""
    _kernel(kernel)
    rp, c = _csr(row_ptr, col)
    thr, alias = _tables(n, thr, alias)
    Yin = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(-1))
    out = np.zeros(2, dtype=np.float64)
    total = lib().oracle_sampled_energy(rp, c, int(n), int(k), int(t), int(seed), alpha, beta,
                                        gamma, int(mode), thr, alias, Yin, out)
    return (float(out[0]), float(out[1])) if parts else total


def effective_energy(row_ptr, col, n, k, Y, alpha=ALPHA, beta=BETA, gamma=GAMMA, kernel=FORCE_T, parts=False):
    """Degree-weighted objective of Eq. (4) with the weight of Sec. 3.3; with
    parts=True the pair (attraction, weighted repulsion)."""
    _kernel(kernel)
    rp, c = _csr(row_ptr, col)
    Yin = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(-1))
    out = np.zeros(2, dtype=np.float64)
    total = lib().oracle_effective_energy(rp, c, int(n), int(k), alpha, beta, gamma, Yin, out)
    return (float(out[0]), float(out[1])) if parts else total


def threaded_run(row_ptr, col, n, k, T, seed, nthreads, Y0=None, t_begin=0, t_end=None,
                 mode=NEG_UNIFORM, thr=None, alias=None, alpha=ALPHA, beta=BETA, gamma=GAMMA, kernel=FORCE_T,
                 eta0=ETA0):
    """The paper's lock-free bundle scheme on host threads (FP64)."""
    _kernel(kernel)
    rp, c = _csr(row_ptr, col)
    thr, alias = _tables(n, thr, alias)
    if t_end is None:
        t_end = T
    Y = init_positions(n, seed) if Y0 is None else np.array(Y0, dtype=np.float64)
    Y = np.ascontiguousarray(Y.reshape(-1))
    lib().oracle_threaded_run(rp, c, int(n), int(k), int(t_begin), int(t_end), int(T),
                              int(seed), alpha, beta, gamma, eta0, int(mode), thr, alias,
                              int(nthreads), Y)
    return Y.reshape(n, 2)
