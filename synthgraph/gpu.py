"""Seeded synthetic graphs generated on the GPU with torch (input generation
only: nothing of the layout method is computed here).

The same Chung-Lu planted-partition recipe as ``chung_lu_communities`` in
``synthgraph/__init__.py`` (power-law expected degrees, log-normal community
sizes with the heaviest nodes dealt to the largest communities, a fraction
``intra`` of the edges inside a community, random node ids, duplicates and
self-loops removed), written with torch so that graphs of ~10^9 edges are
generated in seconds on the device.  Results are reproducible for a given
seed on the same device and software (torch's seeded device generator); they
are not bit-identical to the numpy generator's.
"""
from __future__ import annotations

import math

import numpy as np


def _powerlaw_weights(torch, n, total, tau, dmax, device):
    """w_i = dmax * ((i + i0) / i0)^(-1/(tau-1)) with i0 chosen so sum(w) = total."""
    expo = 1.0 / (tau - 1.0)
    idx = torch.arange(n, dtype=torch.float64, device=device)
    lo, hi = 1e-6, 1e12
    for _ in range(64):
        mid = math.sqrt(lo * hi)
        tot = float((dmax * ((idx + mid) / mid) ** (-expo)).sum())
        if tot < total:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return dmax * ((idx + i0) / i0) ** (-expo)


# A torch sort holds at most 2^31 - 1 elements; longer unique passes are cut
# into value ranges of about _PART_ELEMS elements.  A permutation of more
# than _PERM_MAX keys is slow, so larger edge sets drop their excess instead.
_SORT_MAX = 2**31 - 1
_PART_ELEMS = 2**30
_PERM_MAX = 2**30


def _unique(torch, x):
    """Sorted distinct values of x; an x longer than one sort holds is cut
    into value ranges (bounds from a strided sample) and each range is made
    unique on its own."""
    if x.numel() < _SORT_MAX:
        return torch.unique(x)
    parts = 2 * (x.numel() // _PART_ELEMS) + 2
    samp = torch.sort(x[:: max(1, x.numel() // (1 << 20))]).values
    bounds = samp[(torch.arange(1, parts, device=x.device) * samp.numel()) // parts]
    bounds = torch.unique(bounds).tolist()
    out = []
    for lo, hi in zip([None] + bounds, bounds + [None]):
        m = torch.ones_like(x, dtype=torch.bool) if lo is None else x >= lo
        if hi is not None:
            m &= x < hi
        out.append(torch.unique(x[m]))
        del m
    return torch.cat(out)


def chung_lu_communities_gpu(n: int, n_edges: int, tau: float, dmax: float, n_comm: int,
                             intra: float, sigma: float = 1.0, seed: int = 0,
                             device: str = "cuda:0", progress: bool = False):
    """Returns (row_ptr [n+1], col int32 [2*n_edges], labels int32 [n]) as
    device tensors; row_ptr is int32 below 2^31 directed edges, else int64.
    With progress, each phase is timed (after a device sync) on stderr."""
    import sys
    import time

    import torch

    t_start = time.perf_counter()

    def say(what):
        if progress:
            if str(device).startswith("cuda"):
                torch.cuda.synchronize(device)
            print(f"[graph] {what} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr,
                  flush=True)

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    rng = np.random.default_rng(seed)
    w = _powerlaw_weights(torch, n, 2.0 * n_edges, tau, dmax, device)  # descending
    # community sizes (host, small)
    raw = rng.lognormal(0.0, sigma, n_comm)
    sizes = np.maximum(1, np.floor(raw / raw.sum() * n)).astype(np.int64)
    while sizes.sum() < n:
        sizes[rng.integers(0, n_comm)] += 1
    while sizes.sum() > n:
        c = rng.integers(0, n_comm)
        if sizes[c] > 1:
            sizes[c] -= 1
    order_c = np.argsort(-sizes, kind="stable")
    slots = torch.from_numpy(np.repeat(order_c, sizes[order_c]).astype(np.int64)).to(device)
    jitter = torch.rand(n, generator=gen, device=device, dtype=torch.float64) * (n * 0.5)
    rank = torch.argsort(torch.arange(n, device=device, dtype=torch.float64) + jitter, stable=True)
    comm_of_rank = slots[rank]
    del slots, jitter, rank
    node_of_rank = torch.randperm(n, generator=gen, device=device)
    labels = torch.empty(n, dtype=torch.int32, device=device)
    labels[node_of_rank] = comm_of_rank.to(torch.int32)
    # ranks grouped by community, cumulative weights
    comm_sorted, by_comm = torch.sort(comm_of_rank, stable=True)
    cum = torch.cat([torch.zeros(1, dtype=torch.float64, device=device), torch.cumsum(w[by_comm], 0)])
    cids = torch.arange(n_comm, device=device)
    c_start = torch.searchsorted(comm_sorted, cids, side="left")
    c_end = torch.searchsorted(comm_sorted, cids, side="right")
    W_c = cum[c_end] - cum[c_start]
    ccum = torch.cat([torch.zeros(1, dtype=torch.float64, device=device), torch.cumsum(W_c, 0)])
    gcum = torch.cat([torch.zeros(1, dtype=torch.float64, device=device), torch.cumsum(w, 0)])
    del comm_sorted, W_c, comm_of_rank

    def draw_in(cs):
        lo, hi = cum[c_start[cs]], cum[c_end[cs]]
        x = lo + torch.rand(cs.numel(), generator=gen, device=device, dtype=torch.float64) * (hi - lo)
        pos = torch.searchsorted(cum, x, right=True) - 1
        pos = torch.minimum(torch.maximum(pos, c_start[cs]), c_end[cs] - 1)
        return node_of_rank[by_comm[pos]]

    def draw_global(count):
        x = torch.rand(count, generator=gen, device=device, dtype=torch.float64) * gcum[-1]
        r = torch.clamp(torch.searchsorted(gcum, x, right=True) - 1, 0, n - 1)
        return node_of_rank[r]

    keys = torch.zeros(0, dtype=torch.int64, device=device)
    for rounds in range(1, 51):
        if keys.numel() >= n_edges:
            break
        need = int((n_edges - keys.numel()) * (1.15 if rounds == 1 else 1.5)) + 64
        n_in = int(rng.binomial(need, intra))
        parts = []
        for lo in range(0, need, 1 << 27):  # bounded temporaries
            cnt = min(1 << 27, need - lo)
            c_in = min(cnt, max(0, n_in - lo))
            u = torch.empty(cnt, dtype=torch.int64, device=device)
            v = torch.empty(cnt, dtype=torch.int64, device=device)
            if c_in > 0:
                xc = torch.rand(c_in, generator=gen, device=device, dtype=torch.float64) * ccum[-1]
                cs = torch.clamp(torch.searchsorted(ccum, xc, right=True) - 1, 0, n_comm - 1)
                u[:c_in] = draw_in(cs)
                v[:c_in] = draw_in(cs)
            if cnt > c_in:
                u[c_in:] = draw_global(cnt - c_in)
                v[c_in:] = draw_global(cnt - c_in)
            ok = u != v
            a = torch.minimum(u[ok], v[ok])
            b = torch.maximum(u[ok], v[ok])
            parts.append(a * n + b)
            del u, v, ok, a, b
        say(f"round {rounds}: drew {need} candidate pairs")
        keys = _unique(torch, torch.cat([keys] + parts))
        del parts
        say(f"round {rounds}: {keys.numel()} distinct edges of {n_edges}")
    if keys.numel() > n_edges and n_edges < _PERM_MAX:
        pick = torch.randperm(keys.numel(), generator=gen, device=device)[:n_edges]
        keys = torch.sort(keys[pick]).values
        del pick
    elif keys.numel() > n_edges:
        # a permutation of ~2^31 keys is slow: drop a uniform random subset of
        # the excess instead (distinct draws of indices, then a random subset
        # of them; every subset of that size is equally likely by symmetry);
        # the kept keys stay sorted
        excess = keys.numel() - n_edges
        drop = torch.zeros(0, dtype=torch.int64, device=device)
        while drop.numel() < excess:
            more = torch.randint(0, keys.numel(), (excess + excess // 16 + 1024,),
                                 generator=gen, device=device)
            drop = torch.unique(torch.cat([drop, more]))
        drop = drop[torch.randperm(drop.numel(), generator=gen, device=device)[:excess]]
        keep = torch.ones(keys.numel(), dtype=torch.bool, device=device)
        keep[drop] = False
        keys = keys[keep]
        del drop, keep
    # CSR of both directions without sorting the directed keys (a sort holds
    # at most 2^31 - 1 elements): keys are sorted by (a, b) with a < b, so
    # row i is its lower neighbours (edges (a, i), sorted by a) followed by
    # its higher ones (edges (i, b), sorted by b).
    a1 = keys // n
    b1 = keys - a1 * n
    del keys
    say("kept a sorted sample of the edges")
    k2 = torch.sort(b1 * n + a1).values  # (b, a) order
    b2 = k2 // n
    a2 = k2 - b2 * n
    del k2
    ids = torch.arange(n + 1, device=device)
    c1 = torch.diff(torch.searchsorted(a1, ids))  # higher neighbours per row (a1 sorted)
    c2 = torch.diff(torch.searchsorted(b2, ids))  # lower neighbours per row (b2 sorted)
    del ids
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(c1 + c2, 0)
    s1 = torch.cumsum(c1, 0) - c1  # first index of each row's group in (a1, b1)
    s2 = torch.cumsum(c2, 0) - c2
    say("row pointers")
    col = torch.empty(int(row_ptr[-1]), dtype=torch.int32, device=device)
    step = 1 << 28  # bounded temporaries
    for lo in range(0, a2.numel(), step):
        t = torch.arange(lo, min(lo + step, a2.numel()), device=device)
        r = b2[t]
        col[row_ptr[r] + (t - s2[r])] = a2[t].to(torch.int32)
    for lo in range(0, a1.numel(), step):
        t = torch.arange(lo, min(lo + step, a1.numel()), device=device)
        r = a1[t]
        col[row_ptr[r] + c2[r] + (t - s1[r])] = b1[t].to(torch.int32)
    del a1, b1, a2, b2, c1, c2, s1, s2
    say("column indices")
    if 2 * n_edges < 2**31:
        row_ptr = row_ptr.to(torch.int32)
    return row_ptr, col, labels


def friendster_like_gpu(seed: int = 0, device: str = "cuda:0"):
    """Stands in for com-friendster's node count (65,608,366 nodes: positions of
    525 MB, beyond the 256 MB last-level cache) with 1.0e9 undirected edges
    (an int32 CSR: < 2^31 directed edges; friendster_full_gpu has 1.8e9),
    tau = 2.2, top expected degree sqrt(2|E|), communities of ~1300 nodes
    (log-normal sizes), 90% intra."""
    n, m = 65_608_366, 1_000_000_000
    return chung_lu_communities_gpu(n, m, tau=2.2, dmax=math.sqrt(2 * m),
                                    n_comm=n // 1300, intra=0.9, seed=seed, device=device)


def friendster_full_gpu(seed: int = 0, device: str = "cuda:0"):
    """The com-friendster shape of the paper's case study: 65,608,366 nodes and
    1.8e9 undirected edges (3.6e9 directed: a 64-bit CSR), otherwise the
    recipe of friendster_like_gpu."""
    n, m = 65_608_366, 1_800_000_000
    return chung_lu_communities_gpu(n, m, tau=2.2, dmax=math.sqrt(2 * m),
                                    n_comm=n // 1300, intra=0.9, seed=seed, device=device,
                                    progress=True)


def relabel_gpu(rp, col, labels, order: str):
    """Device version of synthgraph.relabel for graphs generated here (torch
    tensors; int64 row pointers, int32 columns; at most 2^31 - 1 directed
    edges, the limit of one torch sort)."""
    import torch

    n = rp.numel() - 1
    nnz = int(rp[-1])
    if nnz >= 2**31 - 1:
        raise ValueError("relabel_gpu sorts the edges at once: nnz < 2^31 - 1")
    dev = rp.device
    deg = (rp[1:] - rp[:-1]).to(torch.int64)
    dmax = int(deg.max()) if n else 0
    if order == "degree":
        key = dmax - deg
    elif order == "community":
        key = labels.to(torch.int64) * (dmax + 1) + (dmax - deg)
    else:
        raise ValueError(f"unknown order {order!r}")
    perm = torch.sort(key, stable=True).indices
    del key
    inv = torch.empty_like(perm)
    inv[perm] = torch.arange(n, device=dev)
    deg_new = deg[perm]
    rp_new = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(deg_new, 0, out=rp_new[1:])
    row_of = torch.repeat_interleave(torch.arange(n, device=dev), deg_new)
    old_e = rp.to(torch.int64)[perm][row_of]
    old_e += torch.arange(nnz, device=dev)
    old_e -= rp_new[row_of]
    c = inv[col[old_e].to(torch.int64)]
    del old_e
    c += row_of * n
    del row_of
    c = torch.sort(c).values
    c -= torch.div(c, n, rounding_mode="floor") * n
    col_new = c.to(torch.int32)
    del c
    return rp_new, col_new, labels[perm]
