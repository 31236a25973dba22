"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something it does not compute the same way:
an independent library implementation of the generator (numpy's Philox4x64-10),
closed forms of the Table 1 t-forces (at gamma = 2 and at other exponents),
the expectation identity of Sec. 3.3 evaluated by O(n^2) brute force, a scalar
recursion for the two-node graph, exact rational reconstruction of the alias
table, invariants of pair updates, chi-square tests of the samplers, the
threaded bundle scheme of Sec. 3.4 against serial Algorithm 1 in the bundle
order that numpy's generator gives, and the energies against the forces by
central differences (Eq. (2)).
"""
from fractions import Fraction
import math

import numpy as np
import pytest
from scipy import stats

import synthgraph as S
from oracle import oracle as O

ALPHA, BETA, GAMMA = 0.1, 8.0, 2.0
KEY_DOMAIN = 0x534E41502D744644


# ------------------------------------------------------------ generator
@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (5, 7, 9, 11)),
    ((2**64 - 1, 12345), (2**40, 3, 2**63, 7)),
    ((42, KEY_DOMAIN), (1000, 17, 0, 2)),
])
def test_philox_matches_numpy_library(key, ctr):
    """Philox4x64-10 equals numpy's independent implementation (numpy advances
    the counter by one before each block)."""
    count = 2000
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    ref = bg.random_raw(4 * count).reshape(count, 4)
    mine = O.philox_bulk(key, ((ctr[0] + 1) % 2**64, ctr[1], ctr[2], ctr[3]), count)
    assert np.array_equal(ref, mine)


def test_philox_uniform_top_bits():
    words = O.philox_bulk((7, KEY_DOMAIN), (0, 0, 0, 2), 250_000).reshape(-1)
    top = (words >> np.uint64(56)).astype(np.int64)
    hist = np.bincount(top, minlength=256)
    _, p = stats.chisquare(hist)
    assert p > 1e-3


def _numpy_block(seed, a, b, c, tag):
    """One Philox block from numpy's implementation.  numpy adds one to the
    256-bit counter (with carry) before each block, so pass counter - 1."""
    value = a + (b << 64) + (c << 128) + (tag << 192) - 1
    words = [(value >> (64 * q)) & (2**64 - 1) for q in range(4)]
    bg = np.random.Philox(key=np.array([seed, KEY_DOMAIN], dtype=np.uint64),
                          counter=np.array(words, dtype=np.uint64))
    return bg.random_raw(4)


def _numpy_words(seed, e, t, nblocks=2):
    words = []
    for blk in range(nblocks):
        x = _numpy_block(seed, e, t, blk, 2)
        for q in range(4):
            words.append(int(x[q]) & 0xFFFFFFFF)
            words.append(int(x[q]) >> 32)
    return words


# ------------------------------------------------------------------ init
def test_init_positions_match_library_generator():
    n, seed = 777, 3
    Y = O.init_positions(n, seed)
    s = np.float32(math.sqrt(n))
    assert s == np.sqrt(np.float32(n))
    for i in range(0, n, 37):
        x = _numpy_block(seed, i, 0, 0, 1)
        for c in range(2):
            v = np.int64(int(x[c]) >> 40) - (1 << 23)
            expect = np.float32(np.float32(v) * np.float32(2.0**-23)) * s
            assert Y[i, c] == float(np.float32(expect))


def test_init_positions_range_uniform_fp32():
    n = 20000
    Y = O.init_positions(n, 0)
    s = math.sqrt(n)
    assert np.all(np.abs(Y) <= s)
    assert np.array_equal(Y, Y.astype(np.float32).astype(np.float64))
    for c in range(2):
        hist, _ = np.histogram(Y[:, c], bins=40, range=(-s, s))
        assert stats.chisquare(hist)[1] > 1e-3
    # the coordinates come from different words of the block
    assert abs(np.corrcoef(Y[:, 0], Y[:, 1])[0, 1]) < 0.03


# ------------------------------------------------------------- t-forces
@pytest.mark.parametrize("d,fa,fr", [
    (0.0, 0.0, 0.0),
    (0.5, 0.37, 0.32),
    (1.0, 0.5, 0.25),
    (2.0, 0.52, 0.08),
    (10.0, 0.1 * (10 + 80 / 101), 10 / 101**2),
])
def test_tforce_closed_form(d, fa, fr):
    """Table 1, t-FDP row, alpha=0.1, beta=8, gamma=2, at chosen distances."""
    a, r = O.force_magnitudes(d)
    assert a == pytest.approx(fa, abs=1e-12)
    assert r == pytest.approx(fr, abs=1e-12)


def test_tforce_extrema():
    # the repulsion magnitude d/(1+d^2)^2 peaks at d = 1/sqrt(3) with 9/(16 sqrt 3)
    d0 = 1 / math.sqrt(3)
    _, r0 = O.force_magnitudes(d0)
    assert r0 == pytest.approx(9 / (16 * math.sqrt(3)), abs=1e-12)
    for eps in (1e-3, -1e-3):
        assert O.force_magnitudes(d0 + eps)[1] < r0
    # the attraction magnitude has a stationary point at d = sqrt(3): 0.3 sqrt(3)
    d1 = math.sqrt(3)
    a1, _ = O.force_magnitudes(d1)
    assert a1 == pytest.approx(0.3 * math.sqrt(3), abs=1e-12)
    h = 1e-5
    deriv = (O.force_magnitudes(d1 + h)[0] - O.force_magnitudes(d1 - h)[0]) / (2 * h)
    assert abs(deriv) < 1e-8


# --------------------------------------------------------------- sampler
def _tiny_graph(seed=0):
    return S.small_sbm(60, 2, 6.0, seed)


def test_uniform_draws_match_library_generator():
    """The word-stream/Lemire/exclusion definition, evaluated on numpy's
    Philox words, gives the oracle's draws."""
    g = _tiny_graph()
    seed, t, k = 9, 4, 5
    neg = O.draw_negatives(g.row_ptr, g.col, g.n, k, t, seed)
    src = np.repeat(np.arange(g.n), g.degrees())
    m = g.n - 1
    reject_below = (1 << 32) % m
    for e in range(0, g.nnz, 7):
        words = _numpy_words(seed, e, t)
        w = iter(words)
        i = int(src[e])
        for mm in range(k):
            while True:
                u = next(w)
                p = u * m
                if (p & 0xFFFFFFFF) >= reject_below:
                    break
            sp = p >> 32
            s = sp + (1 if sp >= i else 0)
            assert neg[e, mm] == s


def test_uniform_draws_exclude_source_and_are_uniform():
    # star-free ring so that every node is a source
    n = 50
    u = np.arange(n)
    rp, col = S.csr_from_pairs(u, (u + 1) % n, n)
    src = np.repeat(np.arange(n), np.diff(rp))
    counts = np.zeros((n, n), dtype=np.int64)
    for t in range(400):
        neg = O.draw_negatives(rp, col, n, 5, t, 1)
        np.add.at(counts, (np.repeat(src, 5), neg.reshape(-1)), 1)
    assert np.all(np.diag(counts) == 0)
    for i in (0, 17, 49):
        row = np.delete(counts[i], i)
        assert stats.chisquare(row)[1] > 1e-3


def test_two_node_draws_are_partner():
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    for t in range(5):
        neg = O.draw_negatives(rp, col, 2, 7, t, 123)
        assert np.array_equal(neg[0], np.ones(7)) and np.array_equal(neg[1], np.zeros(7))


# ------------------------------------------------------------------ alias
def _exact_alias_probs(thr, alias):
    n = thr.size
    P = [Fraction(0)] * n
    for c in range(n):
        a = Fraction(int(thr[c]), 2**32)
        P[c] += a / n
        P[int(alias[c])] += (1 - a) / n
    return P


@pytest.mark.parametrize("weights", [
    [1, 1, 1, 1],
    [0, 5, 1, 2, 0, 9, 3],
    [1000, 1, 1, 1, 1, 1, 1, 1],
    list(np.random.default_rng(0).integers(0, 50, 300)),
    list(np.diff(S.small_sbm(200, 3, 8.0, 1).row_ptr)),
])
def test_alias_table_exact_probabilities(weights):
    w = np.array(weights, dtype=np.int64)
    thr, alias = O.alias_build(w)
    P = _exact_alias_probs(thr, alias)
    W = int(w.sum())
    for s in range(w.size):
        assert abs(float(P[s] - Fraction(int(w[s]), W))) <= 2.0**-31
        if w[s] == 0:
            assert P[s] == 0
    assert sum(P) == 1


def test_alias_uniform_is_identity():
    thr, alias = O.alias_build(np.full(37, 4))
    assert np.all(alias == np.arange(37)) and np.all(thr == 0xFFFFFFFF)


def test_alias_rejects_bad_weights():
    with pytest.raises(ValueError):
        O.alias_build(np.zeros(5, dtype=np.int64))
    with pytest.raises(ValueError):
        O.alias_build(np.array([1, -1, 3]))


def test_degree_draws_chi_square():
    """DEGREE negatives follow q_i(s) = w_s / (W - w_i), zero weight never drawn."""
    rng = np.random.default_rng(5)
    n = 80
    u = rng.integers(0, n, 200)
    v = rng.integers(0, n, 200)
    rp, col = S.csr_from_pairs(u, v, n)
    w = np.diff(rp).astype(np.int64)
    thr, alias = O.alias_build(w)
    src = np.repeat(np.arange(n), w)
    W = w.sum()
    obs = np.zeros(n)
    exp = np.zeros(n)
    k = 5
    for t in range(300):
        neg = O.draw_negatives(rp, col, n, k, t, 2, mode=O.NEG_DEGREE, thr=thr, alias=alias)
        np.add.at(obs, neg.reshape(-1), 1)
        assert np.all(neg != src[:, None])
    for i in range(n):
        if w[i] == 0:
            continue
        q = w / (W - w[i])
        q[i] = 0
        exp += 300 * k * w[i] * q
    assert np.all(obs[w == 0] == 0)
    pos = exp > 0
    _, p = stats.chisquare(obs[pos], exp[pos] * obs.sum() / exp[pos].sum())
    assert p > 1e-3


# --------------------------------------------------- Algorithm 1 closed form
@pytest.mark.parametrize("order", [O.ORDER_CSR, O.ORDER_SHUFFLED])
def test_two_node_trajectory_closed_form(order):
    """One edge, both directions, k negatives that are always the partner.
    The separation x follows, per directed edge, x <- x(1 - 2 eta alpha
    (1 + beta/(1+x^2))) then k times x <- x(1 + 2 eta / (1+x^2)^2)."""
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    k, T = 3, 40
    Y0 = np.array([[3.0, -1.0], [-2.0, 4.0]])
    Y = O.serial_run(rp, col, 2, k, T, 11, Y0=Y0, order=order)
    d = Y0[0] - Y0[1]
    for t in range(T):
        eta = 1.0 * (1 - t / T)
        for _ in range(2):
            q = d @ d
            d = d * (1 - 2 * eta * ALPHA * (1 + BETA / (1 + q)))
            for _ in range(k):
                q = d @ d
                d = d * (1 + 2 * eta / (1 + q) ** 2)
    got = Y[0] - Y[1]
    assert np.allclose(got, d, rtol=1e-10, atol=1e-12)
    assert np.allclose(Y.sum(0), Y0.sum(0), atol=1e-12)


def test_attraction_pulls_and_repulsion_pushes():
    """Sign convention: one attraction step shortens the edge, one repulsion
    step lengthens the pair (Sec. 3.1: adjacent vertices are drawn together,
    all vertices repel)."""
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    Y0 = np.array([[2.0, 0.0], [-2.0, 0.0]])
    ya = O.jacobi_epoch(rp, col, 2, 0, 0, 10, 0, Y0, use_rep=False)
    assert np.linalg.norm(ya[0] - ya[1]) < 4.0
    yr = O.jacobi_epoch(rp, col, 2, 1, 0, 10, 0, Y0, use_attr=False)
    assert np.linalg.norm(yr[0] - yr[1]) > 4.0


# ------------------------------------------------------------- invariants
def test_serial_centroid_and_translation():
    g = S.small_sbm(300, 3, 8.0, 4)
    Y0 = O.init_positions(g.n, 4)
    Y = O.serial_run(g.row_ptr, g.col, g.n, 5, 10, 4, Y0=Y0)
    assert np.allclose(Y.mean(0), Y0.mean(0), atol=1e-9 * (1 + np.abs(Y0).max()))
    shift = np.array([123.25, -77.5])
    Ys = O.serial_run(g.row_ptr, g.col, g.n, 5, 10, 4, Y0=Y0 + shift)
    assert np.allclose(Ys - shift, Y, atol=1e-9)


def test_k0_components_contract_about_their_centroid():
    a = S.small_sbm(40, 1, 5.0, 7)
    b = S.small_sbm(30, 1, 5.0, 8)
    # disjoint union
    rp = np.concatenate([a.row_ptr, a.row_ptr[-1] + b.row_ptr[1:]]).astype(np.int32)
    col = np.concatenate([a.col, b.col + a.n]).astype(np.int32)
    n = a.n + b.n
    Y0 = O.init_positions(n, 1) * 5
    Y = O.serial_run(rp, col, n, 0, 20, 1, Y0=Y0)
    comp = [np.arange(a.n), a.n + np.arange(b.n)]
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    _, lab = connected_components(csr_matrix((np.ones(col.size), col, rp), shape=(n, n)))
    for c in np.unique(lab):
        idx = np.where(lab == c)[0]
        assert np.allclose(Y[idx].mean(0), Y0[idx].mean(0), atol=1e-9)
        if idx.size > 1:
            spread0 = np.linalg.norm(Y0[idx] - Y0[idx].mean(0), axis=1).mean()
            spread1 = np.linalg.norm(Y[idx] - Y[idx].mean(0), axis=1).mean()
            assert spread1 < spread0
    assert len(comp) == 2


# ------------------------------------------- expectation identity (Sec. 3.3)
def _brute_force_repulsion(Y, deg, k, q=None):
    """sum_j (k/(n-1)) (d_i + d_j) R(y_i - y_j), or with pair weights q."""
    n = Y.shape[0]
    D = Y[:, None, :] - Y[None, :, :]
    qd = (D ** 2).sum(-1)
    R = D / ((1 + qd) ** GAMMA)[..., None]
    if q is None:
        wgt = k / (n - 1) * (deg[:, None] + deg[None, :]).astype(np.float64)
    else:
        wgt = q
    np.fill_diagonal(wgt, 0.0)
    return (wgt[..., None] * R).sum(1)


def _hub_graph():
    g = S.small_sbm(50, 2, 5.0, 3)
    u = np.repeat(np.arange(g.n), g.degrees())
    extra = np.arange(1, 26)
    uu = np.concatenate([u, np.zeros(extra.size, dtype=np.int64)])
    vv = np.concatenate([g.col, extra])
    rp, col = S.csr_from_pairs(uu, vv, g.n)
    return rp, col, g.n


def _mean_repulsion_displacement(rp, col, n, k, Y, M, mode=O.NEG_UNIFORM, thr=None, alias=None):
    T = 10**9
    acc = np.zeros((M, n, 2))
    for t in range(M):
        eta = 1.0 - t / T
        Yo = O.jacobi_epoch(rp, col, n, k, t, T, 77, Y, mode=mode, thr=thr, alias=alias,
                            use_attr=False)
        acc[t] = (Yo - Y) / eta
    return acc.mean(0), acc.std(0, ddof=1) / math.sqrt(M)


def test_edge_centric_expectation_reconstructs_linear_degree_weight():
    """Averaged over draws, the sampled repulsion equals
    (k/(n-1)) sum_{j != i} (d_i + d_j) R(y_i - y_j) (Sec. 3.3)."""
    rp, col, n = _hub_graph()
    deg = np.diff(rp)
    k = 5
    Y = O.init_positions(n, 5) * 0.4
    mean, se = _mean_repulsion_displacement(rp, col, n, k, Y, 6000)
    ref = _brute_force_repulsion(Y, deg, k)
    z = np.abs(mean - ref) / np.maximum(se, 1e-15)
    assert z.max() < 5.0, z.max()


def test_degree_weighted_negatives_give_product_weight_not_linear():
    """Control: degree-proportional negatives realise the weight
    k (d_i q_i(j) + d_j q_j(i)) (close to the product weighting the paper
    rejects in Sec. 3.2), and fail the linear weight of Eq. (5)."""
    rp, col, n = _hub_graph()
    deg = np.diff(rp).astype(np.int64)
    k = 5
    thr, alias = O.alias_build(deg)
    Y = O.init_positions(n, 5) * 0.4
    mean, se = _mean_repulsion_displacement(rp, col, n, k, Y, 6000, mode=O.NEG_DEGREE, thr=thr,
                                            alias=alias)
    W = deg.sum()
    q = deg[None, :] / (W - deg[:, None]).astype(np.float64)  # q_i(j)
    wgt = k * (deg[:, None] * q + deg[None, :] * q.T)
    ref = _brute_force_repulsion(Y, deg, k, q=wgt)
    z = np.abs(mean - ref) / np.maximum(se, 1e-15)
    assert z.max() < 5.0, z.max()
    lin = _brute_force_repulsion(Y, deg, k)
    z_lin = np.abs(mean - lin) / np.maximum(se, 1e-15)
    assert z_lin.max() > 20.0


def test_jacobi_attraction_is_exact_double_sum():
    """Attraction-only synchronous displacement: -2 eta sum_{j in N(i)} A(y_i - y_j)
    (each undirected edge visited in both directions, Sec. 3.3)."""
    rp, col, n = _hub_graph()
    Y = O.init_positions(n, 8)
    Yo = O.jacobi_epoch(rp, col, n, 5, 3, 10, 1, Y, use_rep=False)
    eta = 1.0 * (1 - 3 / 10)
    src = np.repeat(np.arange(n), np.diff(rp))
    D = Y[src] - Y[col]
    qd = (D ** 2).sum(1)
    A = ALPHA * (1 + BETA / (1 + qd))[:, None] * D
    ref = np.zeros_like(Y)
    np.add.at(ref, src, -2 * eta * A)
    assert np.allclose(Yo - Y, ref, rtol=1e-12, atol=1e-12)


def test_effective_energy_is_mean_sampled_energy():
    """At fixed Y the energy sampled in an epoch averages to
    2 sum_E U_a + (k/(n-1)) sum_{i<j} (d_i+d_j) U_r (Sec. 3.3, Eq. (2))."""
    rp, col, n = _hub_graph()
    Y = O.init_positions(n, 2) * 0.5
    k = 5
    vals = np.array([O.sampled_energy(rp, col, n, k, t, 3, Y) for t in range(4000)])
    ueff = O.effective_energy(rp, col, n, k, Y)
    z = abs(vals.mean() - ueff) / (vals.std(ddof=1) / math.sqrt(vals.size))
    assert z < 5.0
    # energy of the closed form: U_r at q is 1/(2(1+q)) for gamma = 2, and the
    # attraction part is exactly twice the undirected sum
    src = np.repeat(np.arange(n), np.diff(rp))
    qd = ((Y[src] - Y[col]) ** 2).sum(1)
    ua = (ALPHA * (qd / 2 + BETA / 2 * np.log1p(qd))).sum()
    deg = np.diff(rp)
    Dm = Y[:, None, :] - Y[None, :, :]
    qq = (Dm ** 2).sum(-1)
    ur = np.triu((deg[:, None] + deg[None, :]) / (2 * (1 + qq)), 1).sum()
    assert ueff == pytest.approx(ua + k / (n - 1) * ur, rel=1e-12)


# ---------------------------------------------------------- layout sanity
def test_serial_layout_separates_planted_blocks():
    """Parity unpinned beyond the oracle: no dataset numbers apply; sanity only
    (the four planted blocks of the 2,000-node SBM come out separated)."""
    from oracle import metrics as M
    g = S.sbm_2000(0)
    Y = O.serial_run(g.row_ptr, g.col, g.n, 5, 50, 0)
    q = M.quality(g.row_ptr, g.col, Y, g.labels, with_cq=True)
    assert q["si"] > 0.5 and q["cq"] > 0.9 and q["np"] > 0.1


def test_threaded_single_thread_is_deterministic_and_clusters():
    from oracle import metrics as M
    g = S.sbm_2000(1)
    Y1 = O.threaded_run(g.row_ptr, g.col, g.n, 5, 50, 1, nthreads=1)
    Y2 = O.threaded_run(g.row_ptr, g.col, g.n, 5, 50, 1, nthreads=1)
    assert np.array_equal(Y1, Y2)
    Y4 = O.threaded_run(g.row_ptr, g.col, g.n, 5, 50, 1, nthreads=4)
    q1 = M.quality(g.row_ptr, g.col, Y1, g.labels)
    q4 = M.quality(g.row_ptr, g.col, Y4, g.labels)
    assert abs(q1["si"] - q4["si"]) < 0.02 and abs(q1["np"] - q4["np"]) < 0.02


def test_sampled_draws_and_init_match_full_ones():
    """The per-edge and per-node oracle functions used at sizes where the full
    ones cannot run agree with the full ones (same definitions, listed items)."""
    g = S.chung_lu_communities(3000, 12000, tau=2.2, dmax=200.0, n_comm=8, intra=0.9, seed=9)
    rng = np.random.default_rng(1)
    edges = np.concatenate([[0, g.nnz - 1], rng.integers(0, g.nnz, 500)])
    for t in (0, 17):
        full = O.draw_negatives(g.row_ptr, g.col, g.n, 6, t, 21)
        assert np.array_equal(O.draw_edges(g.row_ptr, g.n, 6, t, 21, edges), full[edges])
    thr, alias = O.alias_build(g.degrees())
    full = O.draw_negatives(g.row_ptr, g.col, g.n, 3, 2, 8, mode=O.NEG_DEGREE, thr=thr,
                            alias=alias)
    got = O.draw_edges(g.row_ptr, g.n, 3, 2, 8, edges, mode=O.NEG_DEGREE, thr=thr, alias=alias)
    assert np.array_equal(got, full[edges])
    nodes = np.concatenate([[0, g.n - 1], rng.integers(0, g.n, 300)])
    assert np.array_equal(O.init_positions_at(g.n, 5, nodes), O.init_positions(g.n, 5)[nodes])


# ------------------------------------------------------------ 3D positions
def test_init_positions_3d_match_library_generator():
    """3D init: coordinate c from word x_c of the same block (c = 0, 1, 2); the
    first two coordinates are the 2D init."""
    n, seed = 501, 6
    Y3 = O.init_positions(n, seed, dim=3)
    assert np.array_equal(Y3[:, :2], O.init_positions(n, seed))
    s = np.sqrt(np.float32(n))
    for i in range(0, n, 41):
        x = _numpy_block(seed, i, 0, 0, 1)
        v = np.int64(int(x[2]) >> 40) - (1 << 23)
        assert Y3[i, 2] == float(np.float32(np.float32(np.float32(v) * np.float32(2.0**-23)) * s))


@pytest.mark.parametrize("order", [O.ORDER_CSR, O.ORDER_SHUFFLED])
def test_two_node_trajectory_closed_form_3d(order):
    """The scalar recursion of the two-node graph holds for a 3D separation."""
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    k, T = 2, 30
    Y0 = np.array([[1.0, -2.0, 2.5], [0.5, 1.0, -1.0]])
    Y = O.serial_run(rp, col, 2, k, T, 5, Y0=Y0, order=order)
    d = Y0[0] - Y0[1]
    for t in range(T):
        eta = 1.0 * (1 - t / T)
        for _ in range(2):
            d = d * (1 - 2 * eta * ALPHA * (1 + BETA / (1 + d @ d)))
            for _ in range(k):
                d = d * (1 + 2 * eta / (1 + d @ d) ** 2)
    assert np.allclose(Y[0] - Y[1], d, rtol=1e-10, atol=1e-12)
    assert np.allclose(Y.sum(0), Y0.sum(0), atol=1e-12)


def test_3d_run_in_the_plane_is_the_2d_run():
    """With every z = 0, a 3D run never leaves the plane and equals the 2D run
    bit for bit (q gains +0, each z update is 0)."""
    g = S.small_sbm(200, 2, 6.0, 3)
    Y2 = O.init_positions(g.n, 2)
    Y3 = np.concatenate([Y2, np.zeros((g.n, 1))], axis=1)
    a = O.serial_run(g.row_ptr, g.col, g.n, 5, 8, 2, Y0=Y2)
    b = O.serial_run(g.row_ptr, g.col, g.n, 5, 8, 2, Y0=Y3)
    assert np.array_equal(b[:, :2], a) and np.all(b[:, 2] == 0.0)
    ja = O.jacobi_epoch(g.row_ptr, g.col, g.n, 5, 1, 8, 2, Y2)
    jb = O.jacobi_epoch(g.row_ptr, g.col, g.n, 5, 1, 8, 2, Y3)
    assert np.array_equal(jb[:, :2], ja) and np.all(jb[:, 2] == 0.0)


def test_3d_rotation_equivariance():
    """Rotating the start rotates the result (forces depend on |d| only and act
    along d), which a dropped or misplaced z term would break."""
    g = S.small_sbm(150, 3, 5.0, 9)
    Y0 = O.init_positions(g.n, 1, dim=3)
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((3, 3)))
    a = O.serial_run(g.row_ptr, g.col, g.n, 4, 6, 1, Y0=Y0)
    b = O.serial_run(g.row_ptr, g.col, g.n, 4, 6, 1, Y0=Y0 @ Q.T)
    scale = 1 + np.abs(a).max()
    assert np.allclose(b, a @ Q.T, atol=1e-9 * scale)
    ja = O.jacobi_epoch(g.row_ptr, g.col, g.n, 4, 2, 6, 1, Y0)
    jb = O.jacobi_epoch(g.row_ptr, g.col, g.n, 4, 2, 6, 1, Y0 @ Q.T)
    assert np.allclose(jb, ja @ Q.T, atol=1e-9 * scale)


def test_jacobi_attraction_is_exact_double_sum_3d():
    rp, col, n = _hub_graph()
    Y = O.init_positions(n, 8, dim=3)
    Yo = O.jacobi_epoch(rp, col, n, 5, 3, 10, 1, Y, use_rep=False)
    eta = 1.0 * (1 - 3 / 10)
    src = np.repeat(np.arange(n), np.diff(rp))
    D = Y[src] - Y[col]
    A = ALPHA * (1 + BETA / (1 + (D ** 2).sum(1)))[:, None] * D
    ref = np.zeros_like(Y)
    np.add.at(ref, src, -2 * eta * A)
    assert np.allclose(Yo - Y, ref, rtol=1e-12, atol=1e-12)


# --------------------------------------- the threaded bundle scheme (Sec. 3.4)
def _numpy_row_order(seed, n):
    """The bundle order of the threaded scheme, computed from numpy's own
    Philox4x64-10 (not the oracle's): rows sorted by the first word of block
    (i, 1, 0, 3), ties by row index."""
    keys = np.array([_numpy_block(seed, i, 1, 0, 3)[0] for i in range(n)], dtype=np.uint64)
    return np.lexsort((np.arange(n), keys))


@pytest.mark.parametrize("seed,t_begin,t_end,T,k", [(1, 0, 6, 6, 5), (4, 3, 7, 9, 3), (7, 0, 2, 2, 0)])
def test_threaded_single_thread_is_serial_in_bundle_order(seed, t_begin, t_end, T, k):
    """On one thread the lock-free bundle scheme is serial Algorithm 1 with the
    directed edges visited bundle by bundle (all out-edges of one source, CSR
    order) in the seeded bundle order: same eta schedule, same draws, the
    source re-read before every pair step.  Bit for bit."""
    g = S.small_sbm(400, 4, 8.0, seed)
    rows = _numpy_row_order(seed, g.n)
    edge_order = np.concatenate([np.arange(g.row_ptr[i], g.row_ptr[i + 1]) for i in rows])
    Y0 = O.init_positions(g.n, seed)
    ref = O.serial_run_ordered(g.row_ptr, g.col, g.n, k, T, seed, edge_order, Y0=Y0,
                               t_begin=t_begin, t_end=t_end)
    got = O.threaded_run(g.row_ptr, g.col, g.n, k, T, seed, nthreads=1, Y0=Y0,
                         t_begin=t_begin, t_end=t_end)
    assert np.array_equal(got, ref)
    # and the order matters: the plain CSR order gives another trajectory
    csr = O.serial_run_ordered(g.row_ptr, g.col, g.n, k, T, seed, np.arange(g.nnz), Y0=Y0,
                               t_begin=t_begin, t_end=t_end)
    assert not np.array_equal(csr, ref)


def test_threaded_single_thread_two_nodes_closed_form():
    """Two nodes, one edge: the threaded scheme follows the scalar recursion
    of the separation, independent of any order (compare the serial pin)."""
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    k, T = 2, 15
    Y0 = np.array([[1.5, 0.5], [-0.5, 2.0]])
    Y = O.threaded_run(rp, col, 2, k, T, 3, nthreads=1, Y0=Y0)
    d = Y0[0] - Y0[1]
    for t in range(T):
        eta = 1.0 - t / T
        for _ in range(2):
            d = d * (1 - 2 * eta * ALPHA * (1 + BETA / (1 + d @ d)))
            for _ in range(k):
                d = d * (1 + 2 * eta / (1 + d @ d) ** 2)
    assert np.allclose(Y[0] - Y[1], d, rtol=1e-10, atol=1e-12)


def test_serial_run_ordered_refuses_non_permutation():
    g = S.small_sbm(60, 2, 6.0, 0)
    bad = np.arange(g.nnz)
    bad[1] = bad[0]
    with pytest.raises(ValueError):
        O.serial_run_ordered(g.row_ptr, g.col, g.n, 5, 2, 0, bad)


# ------------------------------------------------------- general gamma
@pytest.mark.parametrize("gamma,d,fr", [
    (1.5, 1.0, 2.0 ** -1.5),                      # 1 / 2^1.5
    (1.5, math.sqrt(3.0), math.sqrt(3.0) / 8.0),  # sqrt3 / 4^1.5
    (3.0, 1.0, 0.125),                            # 1 / 2^3
    (3.0, 2.0, 2.0 / 125.0),                      # 2 / 5^3
    (1.0, 3.0, 0.3),                              # 3 / 10
    (4.0, 0.5, 0.5 / 1.25 ** 4),
])
def test_tforce_repulsion_general_gamma_closed_form(gamma, d, fr):
    """Table 1, t-FDP row with a free exponent: |R| = d / (1 + d^2)^gamma;
    the attraction does not depend on gamma."""
    a, r = O.force_magnitudes(d, gamma=gamma)
    assert r == pytest.approx(fr, rel=1e-13, abs=1e-15)
    assert a == pytest.approx(O.force_magnitudes(d, gamma=2.0)[0], rel=1e-15)


@pytest.mark.parametrize("gamma", [1.5, 3.0])
def test_tforce_repulsion_peak_general_gamma(gamma):
    """d (1+d^2)^-gamma peaks where 1 + d^2 = 2 gamma d^2, i.e. d = 1/sqrt(2 gamma - 1),
    with value (2 gamma - 1)^(gamma - 1/2) / (2 gamma)^gamma."""
    d0 = 1.0 / math.sqrt(2 * gamma - 1)
    peak = (2 * gamma - 1) ** (gamma - 0.5) / (2 * gamma) ** gamma
    r0 = O.force_magnitudes(d0, gamma=gamma)[1]
    assert r0 == pytest.approx(peak, rel=1e-13)
    for eps in (1e-3, -1e-3):
        assert O.force_magnitudes(d0 + eps, gamma=gamma)[1] < r0


@pytest.mark.parametrize("gamma", [1.5, 3.0])
def test_two_node_trajectory_general_gamma(gamma):
    """The two-node recursion with x <- x(1 + 2 eta / (1+x^2)^gamma) per
    negative, through the serial run and through one synchronous epoch."""
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    k, T = 2, 12
    Y0 = np.array([[0.75, -0.25], [-0.5, 0.5]])
    Y = O.serial_run(rp, col, 2, k, T, 5, Y0=Y0, order=O.ORDER_CSR, gamma=gamma)
    d = Y0[0] - Y0[1]
    for t in range(T):
        eta = 1.0 - t / T
        for _ in range(2):
            d = d * (1 - 2 * eta * ALPHA * (1 + BETA / (1 + d @ d)))
            for _ in range(k):
                d = d * (1 + 2 * eta / (1 + d @ d) ** gamma)
    assert np.allclose(Y[0] - Y[1], d, rtol=1e-10, atol=1e-12)
    # one synchronous epoch at t = 0 (eta = 1): every pair force from Y0;
    # node 0 moves by -2A(d) + 2k R(d) with d = y0 - y1 (both directions)
    Yj = O.jacobi_epoch(rp, col, 2, k, 0, T, 5, Y0, gamma=gamma)
    d0 = Y0[0] - Y0[1]
    q = d0 @ d0
    move = -2 * ALPHA * (1 + BETA / (1 + q)) * d0 + 2 * k * d0 / (1 + q) ** gamma
    assert np.allclose(Yj[0] - Y0[0], move, rtol=1e-12, atol=1e-14)
    assert np.allclose(Yj[1] - Y0[1], -move, rtol=1e-12, atol=1e-14)


# ------------------------------------------- energies and forces (Eq. (2))
@pytest.mark.parametrize("kernel", [O.FORCE_T, O.FORCE_GAUSSIAN])
@pytest.mark.parametrize("gamma", [1.5, 2.0, 3.0])
@pytest.mark.parametrize("d", [0.05, 0.4, 1.0, 1.7, 6.0])
def test_pair_energies_are_force_potentials(gamma, d, kernel):
    """F = -grad U (Eq. (2)): the distance derivative of U_a is the attraction
    magnitude and minus that of U_r the repulsion magnitude of Table 1 (and of
    its Gaussian-kernel variant), by central differences."""
    h = 1e-5 * max(d, 1.0)
    ua_p, ur_p = O.pair_energies(d + h, gamma=gamma, kernel=kernel)
    ua_m, ur_m = O.pair_energies(d - h, gamma=gamma, kernel=kernel)
    fa, fr = O.force_magnitudes(d, gamma=gamma, kernel=kernel)
    if fr < 1e-12:
        assert abs((ur_p - ur_m) / (2 * h)) < 1e-12
        fr = None
    assert (ua_p - ua_m) / (2 * h) == pytest.approx(fa, rel=1e-8)
    if fr is not None:
        assert -(ur_p - ur_m) / (2 * h) == pytest.approx(fr, rel=1e-8)


def test_pair_energies_values():
    """U_a(1) = alpha (1/2 + (beta/2) ln 2); U_r(d) = 1/(2(1+d^2)) at gamma = 2 and
    (1+d^2)^-2/4 at gamma = 3; at d = 0, U_a = 0 and U_r = 1/(2(gamma-1))."""
    ua, ur = O.pair_energies(1.0)
    assert ua == pytest.approx(0.1 * (0.5 + 4.0 * math.log(2.0)), rel=1e-14)
    assert ur == pytest.approx(0.25, rel=1e-14)
    assert O.pair_energies(2.0, gamma=3.0)[1] == pytest.approx(1.0 / 100.0, rel=1e-14)
    ua0, ur0 = O.pair_energies(0.0, gamma=1.5)
    assert ua0 == 0.0 and ur0 == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("kernel", [O.FORCE_T, O.FORCE_GAUSSIAN])
@pytest.mark.parametrize("gamma", [1.5, 2.0, 3.0])
def test_jacobi_step_is_gradient_step_on_sampled_energy(gamma, kernel):
    """With the draws of epoch t fixed, the synchronous epoch moves every node by
    -eta times the gradient of that epoch's sampled energy (Eq. (2) summed over
    the sampled pairs): the energies and the forces of the oracle, written
    separately, agree through central differences in every coordinate."""
    g = S.small_sbm(24, 2, 5.0, 11)
    k, t, T, seed = 3, 2, 8, 19
    Y = O.init_positions(g.n, 6) * 0.35
    Yj = O.jacobi_epoch(g.row_ptr, g.col, g.n, k, t, T, seed, Y, gamma=gamma, kernel=kernel)
    eta = 1.0 - t / T
    grad = np.zeros_like(Y)
    h = 1e-6
    for i in range(g.n):
        for c in range(2):
            Yp = Y.copy()
            Ym = Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            ep = O.sampled_energy(g.row_ptr, g.col, g.n, k, t, seed, Yp, gamma=gamma,
                                  kernel=kernel)
            em = O.sampled_energy(g.row_ptr, g.col, g.n, k, t, seed, Ym, gamma=gamma,
                                  kernel=kernel)
            grad[i, c] = (ep - em) / (2 * h)
    move = Yj - Y
    scale = np.abs(move).max()
    assert scale > 0
    assert np.abs(move + eta * grad).max() <= 1e-6 * scale


@pytest.mark.parametrize("kernel", [O.FORCE_T, O.FORCE_GAUSSIAN])
@pytest.mark.parametrize("gamma", [1.5, 2.0, 3.0])
def test_effective_energy_gradient_is_expected_force(gamma, kernel):
    """-grad U_eff equals the expected synchronous force: attraction
    -2 sum_{j in N(i)} A(y_i - y_j) and weighted repulsion
    (k/(n-1)) sum_j (d_i + d_j) R(y_i - y_j) (Sec. 3.3, Eq. (4)), the weight
    that the brute-force expectation pin reconstructs from the draws."""
    g = S.small_sbm(20, 2, 4.0, 12)
    k = 5
    n = g.n
    Y = O.init_positions(n, 2) * 0.4
    deg = np.diff(g.row_ptr).astype(np.float64)
    h = 1e-6
    grad = np.zeros_like(Y)
    for i in range(n):
        for c in range(2):
            Yp = Y.copy()
            Ym = Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            grad[i, c] = (O.effective_energy(g.row_ptr, g.col, n, k, Yp, gamma=gamma,
                                             kernel=kernel)
                          - O.effective_energy(g.row_ptr, g.col, n, k, Ym, gamma=gamma,
                                               kernel=kernel)) / (2 * h)
    # expected force from the closed-form magnitudes, pair by pair
    force = np.zeros_like(Y)
    for i in range(n):
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = g.col[e]
            d = Y[i] - Y[j]
            dist = float(np.linalg.norm(d))
            fa, _ = O.force_magnitudes(dist, gamma=gamma, kernel=kernel)
            force[i] -= 2 * fa * d / dist
        for j in range(n):
            if j == i:
                continue
            d = Y[i] - Y[j]
            dist = float(np.linalg.norm(d))
            _, fr = O.force_magnitudes(dist, gamma=gamma, kernel=kernel)
            force[i] += k / (n - 1) * (deg[i] + deg[j]) * fr * d / dist
    assert np.abs(force + grad).max() <= 1e-6 * np.abs(force).max()


# ------------------------------------------- Gaussian-kernel forces (variant)
@pytest.mark.parametrize("gamma,d,fa,fr", [
    (2.0, 0.0, 0.0, 0.0),
    (2.0, 1.0, 0.1 * (1 + 8 * math.exp(-0.5)), math.exp(-1.0)),
    (2.0, 2.0, 0.1 * (2 + 16 * math.exp(-2.0)), 2 * math.exp(-4.0)),
    (1.0, 3.0, 0.1 * (3 + 24 * math.exp(-4.5)), 3 * math.exp(-4.5)),
    (3.0, 0.5, 0.1 * (0.5 + 4 * math.exp(-0.125)), 0.5 * math.exp(-0.375)),
])
def test_gaussian_force_closed_form(gamma, d, fa, fr):
    """The Gaussian variant: |A| = alpha (d + beta d exp(-d^2/2)),
    |R| = d exp(-gamma d^2 / 2), hand-evaluated."""
    a, r = O.force_magnitudes(d, gamma=gamma, kernel=O.FORCE_GAUSSIAN)
    assert a == pytest.approx(fa, rel=1e-13, abs=1e-15)
    assert r == pytest.approx(fr, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("gamma", [1.0, 2.0, 3.0])
def test_gaussian_repulsion_peak(gamma):
    """d exp(-gamma d^2/2) peaks at d = 1/sqrt(gamma) with value exp(-1/2)/sqrt(gamma)."""
    d0 = 1.0 / math.sqrt(gamma)
    r0 = O.force_magnitudes(d0, gamma=gamma, kernel=O.FORCE_GAUSSIAN)[1]
    assert r0 == pytest.approx(math.exp(-0.5) / math.sqrt(gamma), rel=1e-13)
    for eps in (1e-3, -1e-3):
        assert O.force_magnitudes(d0 + eps, gamma=gamma, kernel=O.FORCE_GAUSSIAN)[1] < r0


def test_gaussian_two_node_trajectory():
    """Two nodes with the Gaussian kernel: per directed edge
    x <- x(1 - 2 eta alpha (1 + beta exp(-x^2/2))), then k times
    x <- x(1 + 2 eta exp(-gamma x^2 / 2))."""
    rp, col = S.csr_from_pairs(np.array([0]), np.array([1]), 2)
    k, T, gamma = 3, 20, 2.0
    Y0 = np.array([[0.6, -0.2], [-0.4, 0.3]])
    Y = O.serial_run(rp, col, 2, k, T, 2, Y0=Y0, order=O.ORDER_CSR, kernel=O.FORCE_GAUSSIAN)
    d = Y0[0] - Y0[1]
    for t in range(T):
        eta = 1.0 - t / T
        for _ in range(2):
            d = d * (1 - 2 * eta * ALPHA * (1 + BETA * math.exp(-(d @ d) / 2)))
            for _ in range(k):
                d = d * (1 + 2 * eta * math.exp(-gamma * (d @ d) / 2))
    assert np.allclose(Y[0] - Y[1], d, rtol=1e-10, atol=1e-12)


def test_gaussian_kernel_is_selected_per_call():
    """Selecting the Gaussian kernel for one call leaves the next default call
    on the t-FDP forces."""
    g = O.force_magnitudes(1.0, kernel=O.FORCE_GAUSSIAN)
    t = O.force_magnitudes(1.0)
    assert t == (0.5, 0.25) and g != t
    with pytest.raises(ValueError):
        O.force_magnitudes(1.0, kernel=7)
