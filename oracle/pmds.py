"""Pivot MDS initial layout, FP64 -- test infrastructure only.

The paper initialises every layout with Pivot MDS (Sec. 4.1; Brandes and Pich,
"Eigensolver methods for progressive multidimensional scaling of large data",
GD 2006).  The paper fixes neither the pivot count nor the pivot rule; the
reading taken here (the HIP path implements the same definition
independently):

1. Pivots.  The first pivot is the node of largest degree (smallest index on
   ties).  Each further pivot is the node of the first pivot's connected
   component that maximises the smallest hop distance to the pivots chosen so
   far (smallest index on ties) -- the max/min rule of Brandes and Pich.  At
   most min(p, component size) pivots.
2. Distances.  d_ij = breadth-first hop distance from pivot j to node i.
3. Double centring over the component's m nodes:
   c_ij = -1/2 (d_ij^2 - mean_i' d_i'j^2 - mean_j' d_ij'^2 + mean_i'j' d_i'j'^2).
4. Eigenvectors v1, v2 of the two largest eigenvalues mu1 >= mu2 of C^T C
   (p x p); sigma_k = sqrt(mu_k) are the singular values of C.
5. Coordinates x_i = (C v1 / sqrt(sigma1), C v2 / sqrt(sigma2))_i, i.e. the
   left singular vectors of C scaled by sqrt(sigma_k): with every node a
   pivot, C is the double-centred matrix B of classical MDS, sigma_k = |lambda_k|
   and this is classical MDS's sqrt(lambda_k) u_k, so the two axes keep
   classical MDS's aspect ratio (C v_k alone would stretch them by
   sqrt(sigma1 / sigma2)).  An axis with mu_k <= 1e-6 mu1 (sigma_k <= 1e-3
   sigma1: below the rounding noise of an FP32 C) is 0.
6. Scale s minimising sum_ij (d_ij - s |x_i - x_pivot_j|)^2 over the
   component and the pivots: s = sum d |dx| / sum |dx|^2 (1 if that is 0/0).
7. Nodes outside the first pivot's component take the seeded uniform draws of
   the plain initial layout, in [-R, R]^2 with R the largest |coordinate| of
   the scaled component layout (1 if that is 0).

Only the test suite may import this module.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

DEFAULT_PIVOTS = 50


def bfs_distances(row_ptr, col, n, src):
    """Hop distances from src (-1 = unreachable), level by level."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    dist = np.full(n, -1, dtype=np.int64)
    dist[src] = 0
    frontier = np.array([src], dtype=np.int64)
    level = 0
    while frontier.size:
        starts, ends = rp[frontier], rp[frontier + 1]
        lens = ends - starts
        if lens.sum() == 0:
            break
        # edge indices of every frontier row
        offs = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens)
        nb = col[np.arange(lens.sum()) + offs]
        nb = np.unique(nb[dist[nb] < 0])
        level += 1
        dist[nb] = level
        frontier = nb
    return dist


def select_pivots(row_ptr, col, n, p):
    """Pivots by the max/min rule; returns (pivots, distances p' x n)."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    first = int(np.argmax(deg))  # argmax returns the smallest index on ties
    d0 = bfs_distances(row_ptr, col, n, first)
    comp = d0 >= 0
    p = min(p, int(comp.sum()))
    pivots, dists = [first], [d0]
    mind = np.where(comp, d0, -1)
    while len(pivots) < p:
        nxt = int(np.argmax(mind))
        d = bfs_distances(row_ptr, col, n, nxt)
        pivots.append(nxt)
        dists.append(d)
        mind = np.where(comp, np.minimum(mind, d), -1)
    return np.array(pivots, dtype=np.int64), np.array(dists, dtype=np.int64)


def pmds(row_ptr, col, n, seed, p=DEFAULT_PIVOTS, want_detail=False):
    """Pivot MDS positions (n x 2, FP64; values rounded to FP32 like the
    device's output)."""
    Y = np.zeros((n, 2), dtype=np.float64)
    if n == 0:
        return (Y, {}) if want_detail else Y
    pivots, D = select_pivots(row_ptr, col, n, p)
    comp = D[0] >= 0
    Dc = D[:, comp].T.astype(np.float64)  # m x p'
    D2 = Dc * Dc
    C = -0.5 * (D2 - D2.mean(axis=0, keepdims=True) - D2.mean(axis=1, keepdims=True) + D2.mean())
    G = C.T @ C
    lam, V = np.linalg.eigh(G)  # ascending
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    if V.shape[1] == 1:
        V = np.concatenate([V, np.zeros_like(V)], axis=1)
    mu = np.concatenate([np.maximum(lam, 0.0), [0.0, 0.0]])[:2]
    X = C @ V[:, :2]  # m x 2
    for a in range(2):
        keep = mu[a] > 0 and mu[a] > 1e-6 * mu[0]
        X[:, a] = X[:, a] / np.sqrt(np.sqrt(mu[a])) if keep else 0.0
    # least-squares scale over (component node, pivot) pairs
    idx = np.flatnonzero(comp)
    pos_of = {int(v): q for q, v in enumerate(idx)}
    Xp = X[[pos_of[int(v)] for v in pivots]]
    diff = np.linalg.norm(X[:, None, :] - Xp[None, :, :], axis=2)  # m x p'
    num, den = float((Dc * diff).sum()), float((diff * diff).sum())
    s = num / den if den > 0 else 1.0
    Yc = (s * X).astype(np.float32).astype(np.float64)
    Y[comp] = Yc
    if (~comp).any():
        R = float(np.abs(Yc).max()) if Yc.size else 0.0
        R = np.float32(R if R > 0 else 1.0)
        rest = O.init_positions_scaled(n, seed, R)
        Y[~comp] = rest[~comp]
    if want_detail:
        ev = lam[:3] if lam.size >= 3 else np.concatenate([lam, np.zeros(3 - lam.size)])
        return Y, {"pivots": pivots, "dist": D, "component": comp, "scale": s,
                   "eigenvalues": ev, "G": G}
    return Y


def classical_mds(row_ptr, col, n):
    """Classical MDS of the whole (connected) graph from all-pairs hop
    distances: eigenvectors of B = -1/2 J D^2 J, coordinates sqrt(lambda) u.
    A different formulation, used to pin PMDS with every node a pivot."""
    D = np.array([bfs_distances(row_ptr, col, n, s) for s in range(n)], dtype=np.float64)
    J = np.eye(n) - 1.0 / n
    B = -0.5 * J @ (D * D) @ J
    lam, U = np.linalg.eigh(B)
    order = np.argsort(lam)[::-1][:2]
    return U[:, order] * np.sqrt(np.maximum(lam[order], 0.0))
