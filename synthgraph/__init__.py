"""Seeded synthetic graph generators (input recipes only, no layout arithmetic).

These stand in for the paper's datasets (Sec. 4.1, Table "Test datasets"),
which are not available: a stochastic block model for the small planted-cluster
case, and Chung-Lu power-law graphs with planted communities for the
social-network shapes (an Orkut-communities-like subgraph and an LJ-like
4M-node graph).  Both the oracle-side tests and the GPU path consume the same
CSR produced here.

Every graph is returned as an undirected graph stored with both directions
(each undirected edge {u, v} appears as (u, v) and (v, u), Sec. 3.3), rows
sorted, no self-loops, no duplicates, int32 indices.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_THREADS = max(1, min(16, os.cpu_count() or 1))


def _searchsorted(a: np.ndarray, q: np.ndarray) -> np.ndarray:
    """np.searchsorted(a, q, side="right") split over threads (numpy releases
    the GIL inside searchsorted); identical result to the serial call."""
    out = np.empty(q.size, dtype=np.int64)
    if q.size < 1_000_000 or _THREADS == 1:
        out[:] = np.searchsorted(a, q, side="right")
        return out
    bounds = np.linspace(0, q.size, _THREADS + 1).astype(np.int64)

    def work(t):
        s, e = bounds[t], bounds[t + 1]
        out[s:e] = np.searchsorted(a, q[s:e], side="right")

    with ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(work, range(_THREADS)))
    return out


@dataclasses.dataclass
class Graph:
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    n: int
    labels: np.ndarray  # int32[n], planted community of each node
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        """Undirected edge count |E| (the paper's convention)."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


# ------------------------------------------------------------------ CSR
def csr_from_pairs(u: np.ndarray, v: np.ndarray, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR (both directions, sorted rows) from undirected pairs.

    Self-loops and duplicate pairs are removed."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    dkey = np.sort(src * n + dst)
    src = dkey // n
    dst = (dkey % n).astype(np.int32)
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return row_ptr.astype(np.int32), dst


def _unique_pair_count(u, v, n):
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    keep = a != b
    return np.unique(a[keep] * n + b[keep])


# ------------------------------------------------------------------ SBM
def sbm(n: int, blocks: int, p_in: float, p_out: float, seed: int = 0) -> Graph:
    """Stochastic block model with equal blocks, one Bernoulli trial per pair.

    Exact per-pair sampling; intended for small n (the 2,000-node case)."""
    rng = np.random.default_rng(seed)
    labels = (np.arange(n) * blocks // n).astype(np.int32)
    iu, ju = np.triu_indices(n, k=1)
    same = labels[iu] == labels[ju]
    p = np.where(same, p_in, p_out)
    hit = rng.random(iu.size) < p
    row_ptr, col = csr_from_pairs(iu[hit], ju[hit], n)
    return Graph(row_ptr, col, n, labels, name=f"sbm{n}")


def sbm_fast(n: int, blocks: int, mean_degree: float, intra: float, seed: int = 0) -> Graph:
    """Block model sampled by edge count (for n where per-pair trials are too many).

    The target |E| = n * mean_degree / 2 is split by a binomial draw into intra
    and inter edges; intra edges pick a block with probability proportional to
    its number of pairs and two distinct uniform members, inter edges pick two
    nodes of different blocks.  Duplicates are removed and topped up."""
    rng = np.random.default_rng(seed)
    sizes = np.full(blocks, n // blocks, dtype=np.int64)
    sizes[: n % blocks] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    labels = np.repeat(np.arange(blocks, dtype=np.int32), sizes)
    perm = rng.permutation(n)  # node ids not block-contiguous
    labels = labels[np.argsort(perm)]
    inv = perm  # position p in block order -> node id
    target = int(round(n * mean_degree / 2))
    pairs_w = sizes * (sizes - 1) / 2.0
    pairs_w = pairs_w / pairs_w.sum()
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < target:
        need = int((target - keys.size) * 1.1) + 16
        n_in = rng.binomial(need, intra)
        b = rng.choice(blocks, size=n_in, p=pairs_w)
        x = starts[b] + (rng.random(n_in) * sizes[b]).astype(np.int64)
        y = starts[b] + (rng.random(n_in) * sizes[b]).astype(np.int64)
        n_out = need - n_in
        xo = rng.integers(0, n, n_out)
        yo = rng.integers(0, n, n_out)
        bl = np.repeat(np.arange(blocks), sizes)
        ok = bl[xo] != bl[yo]
        u = inv[np.concatenate([x, xo[ok]])]
        v = inv[np.concatenate([y, yo[ok]])]
        keys = np.union1d(keys, _unique_pair_count(u, v, n))
    if keys.size > target:
        keys = rng.choice(keys, size=target, replace=False)
    row_ptr, col = csr_from_pairs(keys // n, keys % n, n)
    return Graph(row_ptr, col, n, labels, name=f"sbmfast{n}")


# ------------------------------------------------------------ Chung-Lu
def _powerlaw_weights(n: int, total: float, tau: float, dmax: float) -> np.ndarray:
    """w_i = dmax * ((i + i0) / i0)^(-1/(tau-1)) with i0 chosen so sum(w) = total."""
    expo = 1.0 / (tau - 1.0)
    idx = np.arange(n, dtype=np.float64)

    def total_for(i0):
        return float(np.sum(dmax * ((idx + i0) / i0) ** (-expo)))

    lo, hi = 1e-6, 1e12
    for _ in range(64):
        mid = math.sqrt(lo * hi)
        if total_for(mid) < total:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return dmax * ((idx + i0) / i0) ** (-expo)


def chung_lu_communities(n: int, n_edges: int, tau: float, dmax: float, n_comm: int,
                         intra: float, sigma: float = 1.0, seed: int = 0,
                         hubs_to_large: bool = True) -> Graph:
    """Chung-Lu power-law graph with planted communities.

    Expected degrees follow w_i ~ (i + i0)^(-1/(tau-1)) with w_0 = dmax and
    sum(w) = 2|E|.  Community sizes are log-normal(sigma) rescaled to n.  A
    fraction ``intra`` of the edges is drawn inside a community (community
    chosen by its weight sum, both endpoints by weight inside it), the rest
    between weight-proportional endpoints over the whole graph.  With
    ``hubs_to_large`` the heaviest nodes are placed in the largest communities
    (so that hub degrees are not capped by small communities).  Node ids are
    randomly permuted; duplicates and self-loops are removed and topped up to
    exactly ``n_edges``."""
    rng = np.random.default_rng(seed)
    w = _powerlaw_weights(n, 2.0 * n_edges, tau, dmax)  # sorted descending
    # community sizes
    raw = rng.lognormal(0.0, sigma, n_comm)
    sizes = np.maximum(1, np.floor(raw / raw.sum() * n)).astype(np.int64)
    while sizes.sum() < n:
        sizes[rng.integers(0, n_comm)] += 1
    while sizes.sum() > n:
        c = rng.integers(0, n_comm)
        if sizes[c] > 1:
            sizes[c] -= 1
    # assign weight-ranked nodes to communities
    if hubs_to_large:
        order_c = np.argsort(-sizes, kind="stable")
        # deal nodes (heaviest first) to communities with probability
        # proportional to remaining capacity, so big communities get the hubs
        slots = np.repeat(order_c, sizes[order_c])
        # a mild shuffle that keeps hubs near large communities
        jitter = rng.random(n) * n * 0.5
        rank = np.argsort(np.arange(n) + jitter, kind="stable")
        comm_of_rank = slots[rank]
    else:
        comm_of_rank = np.repeat(np.arange(n_comm), sizes)
        rng.shuffle(comm_of_rank)
    # node ids: random permutation of the weight ranks
    node_of_rank = rng.permutation(n)
    labels = np.empty(n, dtype=np.int32)
    labels[node_of_rank] = comm_of_rank.astype(np.int32)
    # nodes grouped by community, with cumulative weights
    by_comm = np.lexsort((np.arange(n), comm_of_rank))  # ranks sorted by community
    wc = w[by_comm]
    cum = np.concatenate([[0.0], np.cumsum(wc)])
    comm_sorted = comm_of_rank[by_comm]
    c_start = np.searchsorted(comm_sorted, np.arange(n_comm), side="left")
    c_end = np.searchsorted(comm_sorted, np.arange(n_comm), side="right")
    W_c = cum[c_end] - cum[c_start]
    p_c = W_c / W_c.sum()
    gcum = np.concatenate([[0.0], np.cumsum(w)])

    def draw_in(cs, count):
        lo = cum[c_start[cs]]
        hi = cum[c_end[cs]]
        x = lo + rng.random(count) * (hi - lo)
        pos = _searchsorted(cum, x) - 1
        pos = np.clip(pos, c_start[cs], c_end[cs] - 1)
        return node_of_rank[by_comm[pos]]

    def draw_global(count):
        x = rng.random(count) * gcum[-1]
        r = np.clip(_searchsorted(gcum, x) - 1, 0, n - 1)
        return node_of_rank[r]

    keys = np.zeros(0, dtype=np.int64)
    rounds = 0
    while keys.size < n_edges and rounds < 50:
        rounds += 1
        need = int((n_edges - keys.size) * (1.15 if rounds == 1 else 1.5)) + 64
        n_in = rng.binomial(need, intra)
        cs = rng.choice(n_comm, size=n_in, p=p_c)
        u_in = draw_in(cs, n_in)
        v_in = draw_in(cs, n_in)
        n_out = need - n_in
        u_out = draw_global(n_out)
        v_out = draw_global(n_out)
        new = _unique_pair_count(np.concatenate([u_in, u_out]),
                                 np.concatenate([v_in, v_out]), n)
        keys = np.union1d(keys, new)
    if keys.size > n_edges:
        keys = rng.choice(keys, size=n_edges, replace=False)
    row_ptr, col = csr_from_pairs(keys // n, keys % n, n)
    return Graph(row_ptr, col, n, labels, name=f"chunglu{n}")


# --------------------------------------------------------- named recipes
def sbm_2000(seed: int = 0) -> Graph:
    """2,000 nodes, 4 equal blocks, p_in = 0.02, p_out = 0.0005 (~10.7k edges)."""
    g = sbm(2000, 4, 0.02, 0.0005, seed)
    g.name = "sbm-2000"
    return g


def orkut_like(seed: int = 0) -> Graph:
    """259,019 nodes, 6,893,156 edges, tau = 2.3, 200 log-normal communities
    (mean ~1.3k nodes), 90% intra-community edges; stands in for the paper's
    Orkut community subgraph (Sec. 1)."""
    n, m = 259_019, 6_893_156
    g = chung_lu_communities(n, m, tau=2.3, dmax=math.sqrt(2 * m), n_comm=200, intra=0.9,
                             sigma=1.0, seed=seed)
    g.name = "orkut-like-259k"
    return g


def lj_like(seed: int = 0) -> Graph:
    """4,000,000 nodes, 34,000,000 edges, tau = 2.1, max degree ~20k, 500
    communities, 90% intra; stands in for com-lj (Table "Test datasets").
    The top expected degree is set above 20k because removing duplicate
    intra-community pairs trims the hubs; the realised maximum is about 20k."""
    g = chung_lu_communities(4_000_000, 34_000_000, tau=2.1, dmax=46_000.0, n_comm=500,
                             intra=0.9, sigma=1.0, seed=seed)
    g.name = "lj-like-4m"
    return g


def cl_350k(seed: int = 21) -> Graph:
    """350,000 nodes, 2,800,000 edges, tau = 2.2, 270 communities, 90%
    intra: a graph whose positions (2.8 MB) fit one XCD's L2 with more than
    one XCD's worth of lanes at n / 32 (the served pool's recipe at that
    size)."""
    g = chung_lu_communities(350_000, 2_800_000, tau=2.2, dmax=2400.0, n_comm=270, intra=0.9,
                             seed=seed)
    g.name = "cl-350k"
    return g


def cached(name: str, maker, cache_dir: str | None = None) -> Graph:
    """Generate once and keep an .npz copy (generation is never timed)."""
    cache_dir = cache_dir or os.environ.get("SNAP_GRAPH_CACHE", "/tmp/snap_graphs")
    os.makedirs(cache_dir, exist_ok=True)
    path = os.path.join(cache_dir, name + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Graph(z["row_ptr"], z["col"], int(z["n"]), z["labels"], name=name)
    g = maker()
    tmp = path + ".tmp.npz"
    np.savez(tmp, row_ptr=g.row_ptr, col=g.col, n=np.int64(g.n), labels=g.labels)
    os.replace(tmp, path)
    return g


def small_sbm(n: int, blocks: int, mean_degree: float, seed: int = 0) -> Graph:
    """Tiny block model for oracle pins (per-pair Bernoulli; 90% of expected
    degree inside the block)."""
    bs = n / blocks
    p_in = min(1.0, 0.9 * mean_degree / max(bs - 1, 1))
    p_out = min(1.0, 0.1 * mean_degree / max(n - bs, 1))
    return sbm(n, blocks, p_in, p_out, seed)


# ----------------------------------------------------- many-graph workloads
def batch_member(index: int, seed: int = 0, n_range=(1_000, 200_000), deg_range=(10.0, 40.0),
                 comm_size: float = 1300.0) -> Graph:
    """Graph `index` of the batched workload: n log-uniform in n_range, mean
    degree uniform in deg_range; even indices are block models, odd ones
    Chung-Lu graphs (tau uniform in [2.1, 2.5]); communities of about
    comm_size nodes, 90% intra-community edges."""
    rng = np.random.default_rng([seed, index, 7])
    n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    md = float(rng.uniform(*deg_range))
    blocks = max(1, int(math.ceil(n / comm_size)))
    sub = int(rng.integers(0, 2**31))
    if index % 2 == 0:
        g = sbm_fast(n, blocks, md, 0.9, seed=sub)
    else:
        tau = float(rng.uniform(2.1, 2.5))
        m = int(round(n * md / 2))
        g = chung_lu_communities(n, m, tau=tau, dmax=math.sqrt(2 * m), n_comm=blocks, intra=0.9,
                                 sigma=1.0, seed=sub)
    g.name = f"batch{seed}-{index}"
    return g


def served_member(index: int, seed: int = 0, n_range=(1_000, 2_000_000),
                  mean_degree: float = 16.0, tau: float = 2.2) -> Graph:
    """Graph `index` of the served stream's pool: n log-uniform in n_range,
    Chung-Lu tau = 2.2, mean degree 16, log-normal communities of mean ~1.3k
    nodes, 90% intra."""
    rng = np.random.default_rng([seed, index, 11])
    n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    m = int(round(n * mean_degree / 2))
    g = chung_lu_communities(n, m, tau=tau, dmax=math.sqrt(2 * m),
                             n_comm=max(1, int(round(n / 1300))), intra=0.9, sigma=1.0,
                             seed=int(rng.integers(0, 2**31)))
    g.name = f"served{seed}-{index}"
    return g


def _member_job(args):
    kind, index, seed, kw = args
    fn = batch_member if kind == "batch" else served_member
    g = fn(index, seed, **kw)
    return g.row_ptr, g.col, g.n, g.labels, g.name


def many_graphs(kind: str, count: int, seed: int = 0, workers: int | None = None,
                cache_dir: str | None = None, progress: bool = True, **kw) -> list[Graph]:
    """Generates `count` members of a workload in a process pool (cached as one
    .npz per member).  With progress=True a line goes to stderr every 32
    members generated, so that a long generation is never silent."""
    import sys
    import time
    from concurrent.futures import ProcessPoolExecutor

    cache_dir = cache_dir or os.environ.get("SNAP_GRAPH_CACHE", "/tmp/snap_graphs")
    os.makedirs(cache_dir, exist_ok=True)
    tag = "" if not kw else "-" + "-".join(f"{k}{v}" for k, v in sorted(kw.items()))
    paths = [os.path.join(cache_dir, f"{kind}{seed}{tag}-{q}.npz") for q in range(count)]
    todo = [q for q in range(count) if not os.path.exists(paths[q])]
    if todo:
        workers = workers or max(1, min(16, os.cpu_count() or 1))
        t0 = time.time()
        with ProcessPoolExecutor(workers) as ex:
            for done, (q, (rp, col, n, lab, name)) in enumerate(zip(
                    todo, ex.map(_member_job, [(kind, q, seed, kw) for q in todo])), 1):
                tmp = paths[q] + ".tmp.npz"
                np.savez(tmp, row_ptr=rp, col=col, n=np.int64(n), labels=lab)
                os.replace(tmp, paths[q])
                if progress and (done % 32 == 0 or done == len(todo)):
                    print(f"[synthgraph] {kind}: {done}/{len(todo)} members generated "
                          f"({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    out = []
    for q in range(count):
        z = np.load(paths[q], allow_pickle=False)
        out.append(Graph(z["row_ptr"], z["col"], int(z["n"]), z["labels"], f"{kind}{seed}-{q}"))
    return out


# ------------------------------------------------------------ relabelling
def relabel_order(deg: np.ndarray, labels: np.ndarray | None, order: str) -> np.ndarray:
    """New-to-old node permutation: 'degree' puts nodes in descending degree
    (ties by old id); 'community' groups nodes by planted community, each
    community in descending degree."""
    idx = np.arange(deg.size)
    if order == "degree":
        return np.lexsort((idx, -deg.astype(np.int64)))
    if order == "community":
        return np.lexsort((idx, -deg.astype(np.int64), labels))
    raise ValueError(f"unknown order {order!r}")


def relabel(g: Graph, order: str) -> Graph:
    """The same graph with nodes renumbered by relabel_order (input
    preprocessing: rows and neighbour lists stay sorted)."""
    deg = np.diff(g.row_ptr.astype(np.int64))
    perm = relabel_order(deg, g.labels, order)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    deg_new = deg[perm]
    rp = np.zeros(g.n + 1, np.int64)
    np.cumsum(deg_new, out=rp[1:])
    row_of = np.repeat(np.arange(g.n, dtype=np.int64), deg_new)
    old_e = g.row_ptr.astype(np.int64)[perm][row_of] + (np.arange(rp[-1]) - rp[row_of])
    col = inv[g.col[old_e]].astype(np.int64)
    col = col[np.lexsort((col, row_of))].astype(np.int32)
    return Graph(rp.astype(g.row_ptr.dtype), col, g.n, g.labels[perm], f"{g.name}-{order}")
