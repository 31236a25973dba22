"""Pins of the layout-quality metrics (NP, SI, CQ of Sec. 4.1), which every
quality comparison applies to oracle and device layouts alike (CPU only).

* r-rings against breadth-first distances from scipy's shortest paths, and
  the two ring implementations against each other;
* NP against its definition written out by brute force (all pairwise layout
  distances, ties by index), and NP = 1 exactly for a path laid on a line
  (the 2-ring of every node is its set of nearest layout neighbours);
* SI against a brute-force silhouette;
* CQ = 1 for labels that are well-separated blobs, and about 0 for noise.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import synthgraph as S
from oracle import metrics as M


@pytest.fixture(scope="module")
def small():
    return S.chung_lu_communities(300, 900, tau=2.3, dmax=40.0, n_comm=4, intra=0.85, seed=6)


def test_rings_match_bfs_distances(small):
    g = small
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    D = shortest_path(A, method="D", unweighted=True)
    for i in (0, 5, 77, int(np.argmax(g.degrees()))):
        ref = np.flatnonzero((D[i] >= 1) & (D[i] <= 2))
        assert np.array_equal(M.ring(g.row_ptr, g.col, i, 2), ref)
        assert np.array_equal(M._ring_fast(g.row_ptr, g.col, i, 2), ref)


def _np_brute(row_ptr, col, Y):
    n = Y.shape[0]
    A = sp.csr_matrix((np.ones(row_ptr[-1]), col, row_ptr), shape=(n, n))
    D = shortest_path(A, method="D", unweighted=True)
    dist = np.linalg.norm(Y[:, None, :] - Y[None, :, :], axis=2)
    vals = []
    for i in range(n):
        ring = set(np.flatnonzero((D[i] >= 1) & (D[i] <= 2)).tolist())
        k = len(ring)
        if k == 0:
            continue
        order = sorted((j for j in range(n) if j != i), key=lambda j: (dist[i, j], j))
        knn = set(order[:k])
        vals.append(len(ring & knn) / len(ring | knn))
    return float(np.mean(vals))


def test_np_matches_brute_force(small):
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((small.n, 2))
    assert abs(M.np_score(small.row_ptr, small.col, Y) - _np_brute(small.row_ptr, small.col, Y)) \
        <= 1e-12


def test_np_is_one_for_a_path_on_a_line():
    n = 50
    rp, col = S.csr_from_pairs(np.arange(n - 1), np.arange(1, n), n)
    Y = np.stack([np.arange(n, dtype=np.float64), np.zeros(n)], axis=1)
    assert M.np_score(rp, col, Y) == 1.0


def _si_brute(Y, labels):
    n = Y.shape[0]
    dist = np.linalg.norm(Y[:, None, :] - Y[None, :, :], axis=2)
    s = np.zeros(n)
    for i in range(n):
        own = labels == labels[i]
        if own.sum() <= 1:
            continue
        a = dist[i, own].sum() / (own.sum() - 1)
        b = min(dist[i, labels == c].mean() for c in np.unique(labels) if c != labels[i])
        s[i] = (b - a) / max(a, b)
    return float(s.mean())


def test_si_matches_brute_force(small):
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((small.n, 2)) + 3.0 * small.labels[:, None]
    assert abs(M.si_score(Y, small.labels) - _si_brute(Y, small.labels)) <= 1e-12


def test_cq_extremes():
    rng = np.random.default_rng(4)
    labels = np.repeat(np.arange(4), 100)
    centres = np.array([[0, 0], [50, 0], [0, 50], [50, 50]], dtype=np.float64)
    Y = centres[labels] + rng.standard_normal((400, 2))
    assert M.cq_score(Y, labels) == pytest.approx(1.0)
    noise = rng.standard_normal((400, 2))
    assert abs(M.cq_score(noise, labels)) < 0.05


# ------------------------------------------------- NP ranked in single precision
def test_np_counts_f32_line_and_coincident_positions():
    # a path laid on a line: every 2-ring is exactly the nearest set
    n = 40
    rp, col = S.csr_from_pairs(np.arange(n - 1), np.arange(1, n), n)
    Y = np.stack([np.arange(n, dtype=np.float32), np.zeros(n, np.float32)], axis=1)
    k, inter = M.np_counts_f32(rp, col, Y, np.arange(n))
    assert np.array_equal(k, inter)
    assert k[0] == 2 and k[1] == 3 and np.all(k[2:n - 2] == 4)
    # all nodes at one point: every distance ties, so K_i is the k_i smallest
    # ids other than i
    g = S.chung_lu_communities(200, 600, tau=2.3, dmax=30.0, n_comm=3, intra=0.8, seed=1)
    Y0 = np.zeros((g.n, 2), np.float32)
    nodes = np.arange(0, g.n, 7)
    k, inter = M.np_counts_f32(g.row_ptr, g.col, Y0, nodes)
    for i, ki, ii in zip(nodes, k, inter):
        ring = M.ring(g.row_ptr, g.col, int(i), 2)
        assert ki == ring.size
        smallest = np.delete(np.arange(g.n), i)[:ki]
        assert ii == np.intersect1d(ring, smallest).size


def test_np_counts_f32_agree_with_the_fp64_metric(small):
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((small.n, 2)).astype(np.float32)
    k, inter = M.np_counts_f32(small.row_ptr, small.col, Y, np.arange(small.n))
    used = k > 0
    mean = float(np.mean(inter[used] / (2 * k[used] - inter[used])))
    assert abs(mean - M.np_score(small.row_ptr, small.col, Y.astype(np.float64))) <= 1e-12
    # radius 1 against the brute force of the definition with 1-rings
    k1, i1 = M.np_counts_f32(small.row_ptr, small.col, Y, np.arange(small.n), r=1)
    assert np.array_equal(k1, np.diff(small.row_ptr))
    assert abs(float(np.mean(i1[k1 > 0] / (2 * k1[k1 > 0] - i1[k1 > 0])))
               - M.np_score(small.row_ptr, small.col, Y.astype(np.float64), r=1)) <= 1e-12


# --------------------------------------------------------- CQ: k-means, ARI
def test_ari_matches_sklearn_and_degenerate_cases():
    from sklearn.metrics import adjusted_rand_score

    rng = np.random.default_rng(8)
    for _ in range(5):
        a = rng.integers(0, 6, 500)
        b = np.where(rng.random(500) < 0.7, a, rng.integers(0, 9, 500))
        assert abs(M.ari(a, b) - adjusted_rand_score(a, b)) <= 1e-12
    a = rng.integers(0, 4, 50)
    assert M.ari(a, a + 10) == 1.0  # a relabelling is perfect agreement
    for x, y in [(np.zeros(7), np.zeros(7)), (np.arange(7), np.arange(7)),
                 (np.zeros(7), np.arange(7))]:
        assert abs(M.ari(x, y) - adjusted_rand_score(x, y)) <= 1e-12


def test_kmeans_pp_first_center_and_d2_rule():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((400, 2)).astype(np.float32)
    seed, K = 5, 6
    words = M.kmeans_draws(seed, K)
    c = M.kmeans_pp(Y, K, seed)
    assert c[0] == (int(words[0]) * 400) >> 64
    assert np.unique(c).size == K  # a chosen point has D^2 = 0 and is never drawn again
    # center 1 by brute force over the cumulative D^2 from center 0
    X = Y.astype(np.float64)
    d2 = ((X - X[c[0]]) ** 2).sum(1)
    t = (int(words[1]) >> 11) * 2.0 ** -53 * d2.sum()
    cum = 0.0
    for i in range(400):
        cum += d2[i]
        if cum > t:
            break
    assert c[1] == i


def test_kmeans_pp_samples_in_proportion_to_d2():
    """Two tight groups, one far point: the second center lands in the group
    far from the first center with the D^2 share it carries."""
    Y = np.concatenate([np.zeros((50, 2)), np.full((50, 2), 10.0)]).astype(np.float32)
    hits = 0
    for seed in range(400):
        c = M.kmeans_pp(Y, 2, seed)
        hits += (c[0] < 50) != (c[1] < 50)
    assert hits == 400  # all of D^2 sits in the other group


def test_lloyd_recovers_separated_blobs_and_converges():
    rng = np.random.default_rng(3)
    labels = np.repeat(np.arange(5), 80)
    centres = rng.uniform(-100, 100, (5, 2))
    Y = (centres[labels] + rng.standard_normal((400, 2))).astype(np.float32)
    a, C, it = M.kmeans_lloyd(Y, Y[[0, 80, 160, 240, 320]], 100)
    assert M.ari(labels, a) == 1.0 and it <= 3
    assert np.allclose(np.sort(C, axis=0), np.sort(centres, axis=0), atol=0.5)
    assert M.cq_kmeans(Y, labels, seed=0) > 0.9
    # an empty cluster keeps its center
    a2, C2, _ = M.kmeans_lloyd(Y[:80], np.array([[0.0, 0.0], [1e6, 1e6]]), 10)
    assert np.all(a2 == 0) and tuple(C2[1]) == (1e6, 1e6)
