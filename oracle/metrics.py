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


# ----------------------------------------------- CQ: k-means and the ARI
# The clustering behind CQ written out plainly (seeded k-means++ start, then
# Lloyd's iterations), so that a device implementation can be held to it.
KMEANS_TAG = 4  # generator tag of the k-means++ draws: counter (c, 0, 0, 4)


def kmeans_draws(seed: int, K: int) -> np.ndarray:
    """Word x0 of the Philox block (c, 0, 0, KMEANS_TAG) for c < K."""
    from oracle import oracle as O

    return O.philox_bulk((seed, O.KEY_DOMAIN), (0, 0, 0, KMEANS_TAG), K)[:, 0].copy()


def kmeans_pp(Y, K: int, seed: int) -> np.ndarray:
    """k-means++ (Arthur and Vassilvitskii, SODA 2007) on FP32 points widened
    to FP64: the first center is point floor(x_0 n / 2^64); center c >= 1 is
    the first point i whose running sum of D^2 (squared distance to the
    nearest chosen center) exceeds u_c * sum(D^2), u_c = (x_c >> 11) 2^-53;
    when every D^2 is 0 it is point floor(x_c n / 2^64).  Returns indices."""
    X = np.asarray(Y, dtype=np.float32).astype(np.float64)
    n = X.shape[0]
    words = kmeans_draws(seed, K)
    first = int((int(words[0]) * n) >> 64)
    chosen = [first]
    d2 = np.full(n, np.inf)
    for c in range(1, K):
        cx, cy = X[chosen[-1]]
        dx = X[:, 0] - cx
        dy = X[:, 1] - cy
        d2 = np.minimum(d2, dx * dx + dy * dy)
        total = float(np.sum(d2))
        if total > 0.0:
            t = float(int(words[c]) >> 11) * 2.0 ** -53 * total
            idx = int(np.searchsorted(np.cumsum(d2), t, side="right"))
            chosen.append(min(idx, n - 1))
        else:
            chosen.append(int((int(words[c]) * n) >> 64))
    return np.array(chosen, dtype=np.int64)


def kmeans_lloyd(Y, centers, max_iter: int = 300):
    """Lloyd's iterations from the given centers (FP64): assign each point to
    the nearest center (lowest index on ties), move each center to the mean
    of its points (an empty cluster keeps its center), stop when an
    assignment after the first repeats the previous one or after max_iter.
    Returns (assignment, centers, iterations)."""
    X = np.asarray(Y, dtype=np.float32).astype(np.float64)
    C = np.array(centers, dtype=np.float64).reshape(-1, 2)
    K = C.shape[0]
    prev = None
    it = 0
    for it in range(1, max_iter + 1):
        dx = X[:, 0][:, None] - C[:, 0][None, :]
        dy = X[:, 1][:, None] - C[:, 1][None, :]
        a = np.argmin(dx * dx + dy * dy, axis=1)
        if prev is not None and np.array_equal(a, prev):
            break
        prev = a
        cnt = np.bincount(a, minlength=K)
        sx = np.bincount(a, weights=X[:, 0], minlength=K)
        sy = np.bincount(a, weights=X[:, 1], minlength=K)
        nz = cnt > 0
        C[nz, 0] = sx[nz] / cnt[nz]
        C[nz, 1] = sy[nz] / cnt[nz]
    return a.astype(np.int64), C, it


def ari(labels, assign) -> float:
    """Adjusted Rand index (Hubert and Arabie, 1985) from its definition:
    (index - expected) / (max - expected) over the contingency table, with
    index = sum C(n_ij, 2), expected = sum C(a_i, 2) sum C(b_j, 2) / C(n, 2),
    max = (sum C(a_i, 2) + sum C(b_j, 2)) / 2; 1 when max = expected."""
    _, li = np.unique(np.asarray(labels), return_inverse=True)
    _, ci = np.unique(np.asarray(assign), return_inverse=True)
    n = li.size
    table = np.zeros((li.max() + 1, ci.max() + 1), dtype=np.int64)
    np.add.at(table, (li, ci), 1)

    def c2(x):
        x = np.asarray(x, dtype=np.float64)
        return x * (x - 1) / 2

    index = c2(table).sum()
    sa, sb = c2(table.sum(1)).sum(), c2(table.sum(0)).sum()
    expected = sa * sb / c2(n) if n > 1 else 0.0
    mx = (sa + sb) / 2
    if mx == expected:
        return 1.0
    return float((index - expected) / (mx - expected))


def cq_kmeans(Y, labels, seed: int, max_iter: int = 300) -> float:
    """CQ with the k-means written out above (K = number of labels)."""
    K = np.unique(np.asarray(labels)).size
    X = np.asarray(Y, dtype=np.float32)
    a, _, _ = kmeans_lloyd(X, X[kmeans_pp(X, K, seed)], max_iter)
    return ari(labels, a)


def quality(row_ptr, col, Y, labels, sample: int | None = None, seed: int = 12345,
            with_cq: bool = False) -> dict:
    out = {"np": np_score(row_ptr, col, Y, sample=sample, seed=seed),
           "si": si_score(Y, labels, sample=sample, seed=seed)}
    if with_cq:
        out["cq"] = cq_score(Y, labels, sample=sample, seed=seed)
    return out
