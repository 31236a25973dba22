"""Layout-quality metrics of the paper's evaluation (Sec. 4.1, "Metrics").

Test infrastructure: applied identically to oracle layouts and device layouts.

* NP (neighbourhood preservation): mean over nodes of the Jaccard index of the
  graph r-ring N_G(i, r) (graph distance 1..r, i excluded; r = 2) and the k_i
  nearest layout neighbours of y_i, k_i = |N_G(i, r)|.  Nodes with k_i = 0 are
  skipped.  Ties in layout distance are broken by node index.
* SI (silhouette index) with the planted labels as clusters.
* CQ: adjusted Rand index between the labels and KMeans(Y) with as many
  clusters as labels.

For large graphs a seeded node sample is used, and the same sample is used for
every layout being compared (the paper restricts com-* metrics to a subset of
communities for the same reason, Sec. 4.1).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def sample_nodes(n: int, size: int | None, seed: int = 12345) -> np.ndarray:
    if size is None or size >= n:
        return np.arange(n)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=size, replace=False))


def ring(row_ptr: np.ndarray, col: np.ndarray, i: int, r: int = 2) -> np.ndarray:
    """Nodes at graph distance 1..r from i (i excluded), sorted."""
    frontier = np.array([i], dtype=np.int64)
    seen = {int(i)}
    out = []
    for _ in range(r):
        nxt = []
        for u in frontier:
            nb = col[row_ptr[u]:row_ptr[u + 1]]
            nxt.append(nb)
        if not nxt:
            break
        cand = np.unique(np.concatenate(nxt)) if nxt else np.zeros(0, dtype=np.int64)
        new = [int(v) for v in cand if int(v) not in seen]
        for v in new:
            seen.add(v)
        out.extend(new)
        frontier = np.array(new, dtype=np.int64)
        if frontier.size == 0:
            break
    return np.array(sorted(out), dtype=np.int64)


def _ring_fast(row_ptr, col, i, r=2):
    """Vectorised r-ring (same set as ``ring``)."""
    visited = np.array([i], dtype=np.int64)
    frontier = visited
    for _ in range(r):
        if frontier.size == 0:
            break
        starts = row_ptr[frontier]
        ends = row_ptr[frontier + 1]
        lens = ends - starts
        if lens.sum() == 0:
            break
        idx = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + \
            np.arange(lens.sum())
        nb = np.unique(col[idx])
        frontier = np.setdiff1d(nb, visited, assume_unique=True)
        visited = np.union1d(visited, frontier)
    return np.setdiff1d(visited, [i], assume_unique=True)


def np_score(row_ptr, col, Y, r: int = 2, sample: int | None = None, seed: int = 12345,
             tree: cKDTree | None = None) -> float:
    """Neighbourhood preservation NP (Sec. 4.1), r = 2 by default."""
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nodes = sample_nodes(n, sample, seed)
    tree = tree or cKDTree(Y)
    scores = []
    for i in nodes:
        ng = _ring_fast(row_ptr, col, int(i), r)
        ki = ng.size
        if ki == 0:
            continue
        kq = min(ki + 1, n)
        # query one extra point so that i itself can be dropped; then resolve
        # ties at the k-th distance by node index
        dist, idx = tree.query(Y[i], k=kq)
        dist = np.atleast_1d(dist)
        idx = np.atleast_1d(idx)
        keep = idx != i
        dist, idx = dist[keep], idx[keep]
        if dist.size > ki:
            dist, idx = dist[:ki + 1], idx[:ki + 1]
        if dist.size > ki and dist[ki - 1] == dist[ki]:
            # ties straddle the cut: take all points at that distance and
            # keep the lowest indices
            dk = dist[ki - 1]
            extra = tree.query_ball_point(Y[i], dk * (1 + 1e-12) + 1e-300)
            extra = np.array([v for v in extra if v != i], dtype=np.int64)
            d_extra = np.linalg.norm(Y[extra] - Y[i], axis=1)
            order = np.lexsort((extra, d_extra))
            nl = extra[order][:ki]
        else:
            nl = idx[:ki]
        inter = np.intersect1d(ng, nl, assume_unique=False).size
        union = ki + nl.size - inter
        scores.append(inter / union)
    return float(np.mean(scores)) if scores else 0.0


def np_counts_f32(row_ptr, col, Y, nodes, r: int = 2):
    """k_i = |N_G(i, r)| and |N_G(i, r) ∩ K_i| per query node, K_i the k_i
    nearest layout neighbours of y_i ranked by the FP32 squared distance
    fl(fl(dx*dx) + fl(dy*dy)) with dx = fl(y_l.x - y_i.x), ties by node index
    (the NP metric of Sec. 4.1 with that ranking decided in single precision,
    as a device implementation decides it).  Brute force over all nodes."""
    Y = np.asarray(Y, dtype=np.float32)
    n = Y.shape[0]
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    ks, inters = [], []
    for i in np.asarray(nodes, dtype=np.int64):
        ng = _ring_fast(row_ptr, col, int(i), r)
        k = ng.size
        if k == 0:
            ks.append(0)
            inters.append(0)
            continue
        dx = Y[:, 0] - Y[i, 0]
        dy = Y[:, 1] - Y[i, 1]
        q = dx * dx + dy * dy  # float32 throughout, no fused multiply-add
        q[i] = np.inf
        others = np.delete(np.arange(n), i)
        qo = q[others]
        qk = np.partition(qo, k - 1)[k - 1]
        near = others[qo < qk]
        ties = others[qo == qk]  # ascending node ids
        near = np.concatenate([near, ties[:k - near.size]])
        ks.append(k)
        inters.append(np.intersect1d(ng, near).size)
    return np.array(ks, dtype=np.int64), np.array(inters, dtype=np.int64)


def si_score(Y, labels, sample: int | None = None, seed: int = 12345) -> float:
    """Silhouette index (Sec. 4.1) with the planted labels as clusters."""
    from sklearn.metrics import silhouette_score

    Y = np.asarray(Y, dtype=np.float64)
    labels = np.asarray(labels)
    nodes = sample_nodes(Y.shape[0], sample, seed)
    lab = labels[nodes]
    if np.unique(lab).size < 2:
        return 0.0
    return float(silhouette_score(Y[nodes], lab))


def cq_score(Y, labels, sample: int | None = None, seed: int = 12345) -> float:
    """Clustering quality CQ = ARI(labels, KMeans(Y)) (Sec. 4.1)."""
    from sklearn.cluster import KMeans
    from sklearn.metrics import adjusted_rand_score

    Y = np.asarray(Y, dtype=np.float64)
    labels = np.asarray(labels)
    nodes = sample_nodes(Y.shape[0], sample, seed)
    K = np.unique(labels[nodes]).size
    km = KMeans(n_clusters=K, n_init=1, random_state=0).fit(Y[nodes])
    return float(adjusted_rand_score(labels[nodes], km.labels_))


def quality(row_ptr, col, Y, labels, sample: int | None = None, seed: int = 12345,
            with_cq: bool = False) -> dict:
    out = {"np": np_score(row_ptr, col, Y, sample=sample, seed=seed),
           "si": si_score(Y, labels, sample=sample, seed=seed)}
    if with_cq:
        out["cq"] = cq_score(Y, labels, sample=sample, seed=seed)
    return out
