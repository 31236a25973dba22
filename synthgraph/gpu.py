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


def chung_lu_communities_gpu(n: int, n_edges: int, tau: float, dmax: float, n_comm: int,
                             intra: float, sigma: float = 1.0, seed: int = 0,
                             device: str = "cuda:0"):
    """Returns (row_ptr int32 [n+1], col int32 [2*n_edges], labels int32 [n]) as
    device tensors.  2 * n_edges must stay below 2^31 (int32 CSR)."""
    import torch

    if 2 * n_edges >= 2**31:
        raise ValueError("2 * n_edges must be < 2^31 for an int32 CSR")
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
        keys = torch.unique(torch.cat([keys] + parts))
        del parts
    if keys.numel() > n_edges:
        pick = torch.randperm(keys.numel(), generator=gen, device=device)[:n_edges]
        keys = torch.sort(keys[pick]).values
        del pick
    u = keys // n
    v = keys - u * n
    del keys
    src = torch.cat([u, v])
    dst = torch.cat([v, u])
    del u, v
    skey = torch.sort(src * n + dst).values
    del src, dst
    row = skey // n
    col = (skey - row * n).to(torch.int32)
    counts = torch.bincount(row, minlength=n)
    del skey, row
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return row_ptr.to(torch.int32), col, labels


def friendster_like_gpu(seed: int = 0, device: str = "cuda:0"):
    """Stands in for com-friendster's node count (65,608,366 nodes: positions of
    525 MB, beyond the 256 MB last-level cache) with 1.0e9 undirected edges
    (the int32 CSR holds < 2^31 directed edges; friendster has 1.8e9),
    tau = 2.2, top expected degree sqrt(2|E|), communities of ~1300 nodes
    (log-normal sizes), 90% intra."""
    n, m = 65_608_366, 1_000_000_000
    return chung_lu_communities_gpu(n, m, tau=2.2, dmax=math.sqrt(2 * m),
                                    n_comm=n // 1300, intra=0.9, seed=seed, device=device)
