"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: hand-worked closed forms of
eqs. (3)-(5) (tests/golden/hand_cases.json), finite differences of the
objective, brute-force affinities by an independent root finder, special
cases with closed forms, and invariants of the mathematics.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_2310_11186_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")


def frac(s: str) -> float:
    return float(Fraction(s))


def rows_of(row_ptr):
    return np.repeat(np.arange(row_ptr.shape[0] - 1), np.diff(row_ptr))


def entry(row_ptr, col, i, j):
    seg = col[row_ptr[i]:row_ptr[i + 1]]
    k = np.searchsorted(seg, j)
    assert k < seg.shape[0] and seg[k] == j
    return row_ptr[i] + k


# ---------------------------------------------------------------------------
# Hand-worked cases (closed forms of eqs. (3)-(5))
# ---------------------------------------------------------------------------

def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_cases(case):
    n = case["n"]
    row_ptr, col = oracle.csr_from_edges(n, np.array(case["edges"]))
    X = np.random.default_rng(0).standard_normal((n, 5)).astype(np.float32)
    P, beta = oracle.build_P(row_ptr, col, X, 30.0)
    assert col.shape[0] == len(case["P"])
    for key, val in case["P"].items():
        i, j = map(int, key.split(","))
        assert P[entry(row_ptr, col, i, j)] == pytest.approx(frac(val), rel=1e-15)
    Y = np.array(case["Y"], np.float64)
    g, Z = oracle.gradient(row_ptr, col, P, Y, 1.0)
    if case["Z"] == "2/(1+d2)":
        d2 = float(((Y[0] - Y[1]) ** 2).sum())
        assert Z == pytest.approx(2.0 / (1.0 + d2), rel=1e-15)
    else:
        assert Z == pytest.approx(frac(case["Z"]), rel=1e-14)
    kl_expected = sum(frac(c) * math.log(frac(r)) for c, r in case["kl_terms"])
    assert oracle.kl(row_ptr, col, P, Y) == pytest.approx(kl_expected, rel=1e-13, abs=1e-15)
    g_expected = np.array([[frac(a), frac(b)] for a, b in case["grad"]])
    np.testing.assert_allclose(g, g_expected, rtol=1e-13, atol=1e-15)


def test_Z_all_coincident_positions():
    # Y == 0: every w_ij = 1, so Z = n(n-1) exactly (denominator of eq. (4)).
    for n in (1, 2, 7, 64):
        assert oracle.Z(np.zeros((n, 2))) == float(n * (n - 1))


# ---------------------------------------------------------------------------
# Gradient: finite differences of the objective
# ---------------------------------------------------------------------------

def _small_graph(n, avg_deg, seed, d=6):
    g = synth.small_sbm(n, 2, avg_deg, d, seed)
    row_ptr, col = oracle.csr_from_edges(n, g.edges)
    return g, row_ptr, col


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_finite_differences_of_kl(seed):
    g, row_ptr, col = _small_graph(10, 5.0, seed)
    P, _ = oracle.build_P(row_ptr, col, g.X, 2.5)     # low perplexity: the search runs on most rows
    Y = np.random.default_rng(seed).standard_normal((10, 2))
    grad, _ = oracle.gradient(row_ptr, col, P, Y, 1.0)
    h = 1e-6
    fd = np.zeros_like(Y)
    for i in range(Y.shape[0]):
        for c in range(2):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            fd[i, c] = (oracle.kl(row_ptr, col, P, Yp) - oracle.kl(row_ptr, col, P, Ym)) / (2 * h)
    np.testing.assert_allclose(grad, fd, rtol=1e-6, atol=1e-9)


def test_exaggerated_gradient_matches_finite_differences():
    # With P scaled by alpha the gradient is that of F = -alpha sum p log w + log Z
    # (KL up to constants when alpha = 1); F is evaluated here directly.
    g, row_ptr, col = _small_graph(9, 4.0, 11)
    P, _ = oracle.build_P(row_ptr, col, g.X, 2.0)
    rows = rows_of(row_ptr)
    alpha = 12.0

    def F(Y):
        d2 = ((Y[rows] - Y[col]) ** 2).sum(1)
        diff = Y[:, None, :] - Y[None, :, :]
        W = 1.0 / (1.0 + (diff ** 2).sum(-1))
        np.fill_diagonal(W, 0.0)
        return alpha * float((P * np.log1p(d2)).sum()) + math.log(W.sum())

    Y = np.random.default_rng(5).standard_normal((9, 2)) * 2.0
    grad, _ = oracle.gradient(row_ptr, col, P, Y, alpha)
    h = 1e-6
    for i in range(9):
        for c in range(2):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            assert grad[i, c] == pytest.approx((F(Yp) - F(Ym)) / (2 * h), rel=1e-6, abs=1e-9)


def test_gradient_invariants():
    g, row_ptr, col = _small_graph(40, 6.0, 7)
    P, _ = oracle.build_P(row_ptr, col, g.X, 5.0)
    Y = np.random.default_rng(1).standard_normal((40, 2)) * 3.0
    for alpha in (1.0, 12.0):
        grad, Z = oracle.gradient(row_ptr, col, P, Y, alpha)
        # pairwise forces are antisymmetric, so they sum to zero
        assert np.abs(grad.sum(0)).max() < 1e-14 * max(1.0, np.abs(grad).sum())
        # translation invariance
        g2, Z2 = oracle.gradient(row_ptr, col, P, Y + np.array([3.5, -7.25]), alpha)
        np.testing.assert_allclose(g2, grad, rtol=1e-9, atol=1e-13)
        assert Z2 == pytest.approx(Z, rel=1e-12)
        # rotation equivariance
        th = 0.7
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        g3, _ = oracle.gradient(row_ptr, col, P, Y @ R.T, alpha)
        np.testing.assert_allclose(g3, grad @ R.T, rtol=1e-9, atol=1e-13)


def test_gradient_rows_subset_equals_full_gradient_rows():
    # The row-subset gradient (the checker of sampled rows on large graphs)
    # must return, in the listed order, exactly the rows of the full gradient
    # (itself pinned by finite differences above): same Z, same arithmetic per
    # row, so bitwise equal.  The rows cover the first, the last and a partial
    # last block of any tile length, unsorted and with a repeat.
    n = 3001
    gi = synth.small_dcsbm(n, 9003, 2.4, 15, 6, 5)
    row_ptr, col = oracle.csr_from_edges(n, gi.edges)
    P, _ = oracle.build_P(row_ptr, col, gi.X, 5.0)
    Y = np.random.default_rng(4).standard_normal((n, 2)) * 2.0
    rng = np.random.default_rng(9)
    rows = np.concatenate([[n - 1, 0, 2688, 2999], rng.choice(n, 60, replace=False), [n - 1]]).astype(np.int32)
    for alpha in (1.0, 12.0):
        full, Zf = oracle.gradient(row_ptr, col, P, Y, alpha)
        sub, Zs = oracle.gradient_rows(row_ptr, col, P, Y, rows, alpha)
        assert sub.shape == (rows.shape[0], 2)
        assert Zs == Zf
        np.testing.assert_array_equal(sub, full[rows])
    # an empty subset still returns the full Z
    sub, Zs = oracle.gradient_rows(row_ptr, col, P, Y, np.zeros(0, np.int32), 1.0)
    assert sub.shape == (0, 2) and Zs == Zf


def test_two_nodes_are_stationary():
    row_ptr, col = oracle.csr_from_edges(2, np.array([[0, 1]]))
    P, _ = oracle.build_P(row_ptr, col, np.zeros((2, 3), np.float32), 30.0)
    for Y in (np.array([[0.0, 0.0], [1.0, 2.0]]), np.array([[-3.0, 5.0], [0.1, 0.2]])):
        grad, _ = oracle.gradient(row_ptr, col, P, Y)
        assert np.abs(grad).max() < 1e-16
        assert abs(oracle.kl(row_ptr, col, P, Y)) < 1e-16


def test_kl_translation_invariant():
    g, row_ptr, col = _small_graph(30, 5.0, 9)
    P, _ = oracle.build_P(row_ptr, col, g.X, 4.0)
    Y = np.random.default_rng(2).standard_normal((30, 2))
    a = oracle.kl(row_ptr, col, P, Y)
    b = oracle.kl(row_ptr, col, P, Y - np.array([100.0, 0.5]))
    assert a == pytest.approx(b, rel=1e-10)
    assert a > 0


# ---------------------------------------------------------------------------
# Affinities: brute force with an independent root finder, closed forms
# ---------------------------------------------------------------------------

def brute_conditional(Dn, perp):
    """p_{j|i} over one neighbour set by solving 2^{H_bits} = perp for sigma
    with Brent's method on log(sigma) (eq. (2) in its sigma form)."""
    Dn = np.asarray(Dn, np.float64)
    deg = Dn.shape[0]
    if deg <= perp:
        return np.full(deg, 1.0 / deg)

    def p_of(log_sigma):
        s2 = math.exp(2 * log_sigma)
        a = -(Dn - Dn.min()) / (2 * s2)
        e = np.exp(a)
        return e / e.sum()

    def f(log_sigma):
        p = p_of(log_sigma)
        nz = p[p > 0]
        return 2.0 ** (-(nz * np.log2(nz)).sum()) - perp

    root = brentq(f, -40.0, 40.0, xtol=1e-15, rtol=1e-15, maxiter=500)
    return p_of(root)


@pytest.mark.parametrize("perp", [1.5, 2.5, 3.7, 30.0])
def test_affinities_against_brute_force(perp):
    g = synth.small_sbm(12, 2, 6.0, 4, seed=21)
    row_ptr, col = oracle.csr_from_edges(12, g.edges)
    X = g.X.astype(np.float64)
    n = 12
    Pc = np.zeros((n, n))
    for i in range(n):
        nb = col[row_ptr[i]:row_ptr[i + 1]]
        if nb.size == 0:
            continue
        Dn = ((X[i] - X[nb]) ** 2).sum(1)
        Pc[i, nb] = brute_conditional(Dn, perp)
    nonisolated = int((np.diff(row_ptr) > 0).sum())
    Pd = (Pc + Pc.T) / (2 * nonisolated)
    P, _ = oracle.build_P(row_ptr, col, g.X, perp)
    rows = rows_of(row_ptr)
    np.testing.assert_allclose(P, Pd[rows, col], rtol=2e-9, atol=1e-15)
    # and nothing outside the pattern
    mask = np.zeros((n, n), bool)
    mask[rows, col] = True
    assert np.all(Pd[~mask] == 0)


def test_degree_two_row_closed_form():
    # A node with two neighbours at squared distances D1 < D2 and 1 < perp < 2:
    # its row is (p, 1-p) with binary entropy h(p) = ln perp, and
    # beta = ln(p/(1-p)) / (D2 - D1).
    X = np.array([[0, 0], [1, 0], [0, 2.0], [5, 5]], np.float32)
    edges = np.array([[0, 1], [0, 2], [2, 3]])
    row_ptr, col = oracle.csr_from_edges(4, edges)
    D = oracle.edge_sqdist(row_ptr, col, X)
    for perp in (1.2, 1.5, 1.9):
        pc, beta = oracle.calibrate(row_ptr, D, perp)
        p = brentq(lambda q: -(q * math.log(q) + (1 - q) * math.log(1 - q)) - math.log(perp), 0.5, 1 - 1e-15,
                   xtol=1e-16, rtol=1e-15)
        e01, e02 = entry(row_ptr, col, 0, 1), entry(row_ptr, col, 0, 2)
        assert D[e01] == 1.0 and D[e02] == 4.0
        assert pc[e01] == pytest.approx(p, rel=1e-11)
        assert pc[e02] == pytest.approx(1 - p, rel=1e-9)
        assert beta[0] == pytest.approx(math.log(p / (1 - p)) / 3.0, rel=1e-10)


def test_affinity_invariants():
    g = synth.small_sbm(300, 6, 9.0, 8, seed=4)
    row_ptr, col = oracle.csr_from_edges(300, g.edges)
    perp = 5.0
    D = oracle.edge_sqdist(row_ptr, col, g.X)
    pc, beta = oracle.calibrate(row_ptr, D, perp)
    P = oracle.symmetrise(row_ptr, col, pc)
    mir = oracle.mirror(row_ptr, col)
    assert np.array_equal(P, P[mir])                       # symmetric bit for bit
    assert P.sum() == pytest.approx(1.0, abs=1e-12)
    deg = np.diff(row_ptr)
    calibrated = 0
    for i in range(300):
        seg = pc[row_ptr[i]:row_ptr[i + 1]]
        if deg[i] == 0:
            continue
        assert seg.sum() == pytest.approx(1.0, abs=1e-13)
        if deg[i] <= perp:
            assert np.all(seg == 1.0 / deg[i])
        else:
            calibrated += 1
            H = -(seg[seg > 0] * np.log(seg[seg > 0])).sum()
            assert H == pytest.approx(math.log(perp), abs=1e-10)
    assert calibrated > 100


def test_isolated_nodes_and_normaliser():
    # nodes 3 and 5 are isolated: their rows are empty and S = 2 * 4
    edges = np.array([[0, 1], [1, 2], [2, 4], [4, 0]])
    row_ptr, col = oracle.csr_from_edges(6, edges)
    X = np.random.default_rng(3).standard_normal((6, 3)).astype(np.float32)
    P, _ = oracle.build_P(row_ptr, col, X, 30.0)
    assert np.diff(row_ptr)[3] == 0 and np.diff(row_ptr)[5] == 0
    assert P.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.all(P == 1.0 / 8.0)            # 4-cycle, all rows uniform 1/2: (1/2+1/2)/8


def test_ties_at_minimum_distance():
    # node 0 has 5 neighbours; 3 share the minimum distance; with perp <= 3
    # the row is uniform over those three (beta -> infinity limit).
    X = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [3, 0], [0, 4]], np.float32)
    edges = np.array([[0, k] for k in range(1, 6)])
    row_ptr, col = oracle.csr_from_edges(6, edges)
    D = oracle.edge_sqdist(row_ptr, col, X)
    pc, beta = oracle.calibrate(row_ptr, D, 2.5)
    np.testing.assert_array_equal(pc[0:5], [1 / 3, 1 / 3, 1 / 3, 0, 0])
    assert math.isinf(beta[0])
    pc, beta = oracle.calibrate(row_ptr, D, 4.0)     # reachable: a finite beta
    assert math.isfinite(beta[0]) and beta[0] > 0
    H = -(pc[0:5] * np.log(pc[0:5])).sum()
    assert H == pytest.approx(math.log(4.0), abs=1e-10)


# ---------------------------------------------------------------------------
# CSR construction and mirror index
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_csr_against_dense_adjacency(seed):
    rng = np.random.default_rng(seed)
    n = 37
    uv = rng.integers(0, n, size=(150, 2))      # includes self-loops and repeats
    row_ptr, col = oracle.csr_from_edges(n, uv)
    A = np.zeros((n, n), bool)
    for u, v in uv:
        if u != v:
            A[u, v] = A[v, u] = True
    r, c = np.nonzero(A)                          # row-major: sorted by (row, col)
    assert np.array_equal(col, c)
    assert np.array_equal(row_ptr, np.concatenate([[0], np.cumsum(A.sum(1))]))
    mir = oracle.mirror(row_ptr, col)
    rows = rows_of(row_ptr)
    assert np.array_equal(col[mir], rows)
    assert np.array_equal(rows[mir], col)
    assert np.array_equal(mir[mir], np.arange(col.shape[0]))


def test_mirror_rejects_non_canonical():
    row_ptr = np.array([0, 1, 1], np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.mirror(row_ptr, np.array([1], np.int32))          # (0,1) without (1,0)
    with pytest.raises(oracle.OracleError):
        oracle.mirror(np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32))   # repeated column
    with pytest.raises(oracle.OracleError):
        oracle.mirror(np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32))        # self-loops


# ---------------------------------------------------------------------------
# Update rule (reading: momentum + gains; the paper gives no optimiser)
# ---------------------------------------------------------------------------

def test_update_single_step_by_hand():
    Y = np.array([[1.0, -2.0]])
    U = np.array([[0.5, 0.25]])
    gains = np.array([[1.0, 0.02]])
    g = np.array([[-0.1, 0.4]])
    Y1, U1, G1 = oracle.update(Y, U, gains, g, momentum=0.8, eta=10.0, min_gain=0.01)
    # x: g*u = -0.05 < 0 -> gain 1.2; u = 0.4 + 1.2 = 1.6; y = 2.6
    # y: g*u = 0.1 >= 0 -> gain 0.016; u = 0.2 - 0.064 = 0.136; y = -1.864
    np.testing.assert_allclose(G1, [[1.2, 0.016]], rtol=1e-15)
    np.testing.assert_allclose(U1, [[1.6, 0.136]], rtol=1e-14)
    np.testing.assert_allclose(Y1, [[2.6, -1.864]], rtol=1e-14)
    # zero product (first step, u = 0) shrinks the gain; the clamp holds min_gain
    _, _, G2 = oracle.update(Y, np.zeros_like(U), np.array([[0.011, 1.0]]), g, 0.5, 1.0, 0.01)
    np.testing.assert_allclose(G2, [[0.01, 0.8]], rtol=1e-15)


def test_run_switches_exaggeration_and_momentum():
    g, row_ptr, col = _small_graph(20, 5.0, 13)
    P, _ = oracle.build_P(row_ptr, col, g.X, 4.0)
    Y0 = g.Y0.astype(np.float64) * 100
    Y, U, G, _ = oracle.run(row_ptr, col, P, Y0, n_steps=4, early_exaggeration=4.0, exaggeration_iters=2,
                            momentum_early=0.5, momentum_late=0.8, eta=20.0)
    y, u, gn = Y0.copy(), np.zeros_like(Y0), np.ones_like(Y0)
    for t in range(4):
        gr, _ = oracle.gradient(row_ptr, col, P, y, 4.0 if t < 2 else 1.0)
        y, u, gn = oracle.update(y, u, gn, gr, 0.5 if t < 2 else 0.8, 20.0)
    np.testing.assert_array_equal(Y, y)
    np.testing.assert_array_equal(U, u)
    np.testing.assert_array_equal(G, gn)


def test_oracle_threads_do_not_change_results():
    g, row_ptr, col = _small_graph(200, 6.0, 17)
    P, _ = oracle.build_P(row_ptr, col, g.X, 5.0)
    Y = np.random.default_rng(4).standard_normal((200, 2))
    k = oracle.num_threads()
    oracle.set_threads(1)
    a, za = oracle.gradient(row_ptr, col, P, Y)
    oracle.set_threads(max(k, 2))
    b, zb = oracle.gradient(row_ptr, col, P, Y)
    oracle.set_threads(k)
    assert np.array_equal(a, b) and za == zb


# ---------------------------------------------------------------------------
# Neighbourhood graph G_knn,G (§2.2, eq. (7))
# ---------------------------------------------------------------------------

def brute_knn(n, edges, k):
    """N_k(i) from all-pairs hop distances (scipy's BFS), sorted by (dist, id)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path
    e = np.asarray(edges).reshape(-1, 2)
    A = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    D = shortest_path(A, directed=False, unweighted=True)
    adj = np.zeros((n, n), bool)
    for i in range(n):
        cand = [(D[i, j], j) for j in range(n) if j != i and np.isfinite(D[i, j])]
        cand.sort()
        for _, j in cand[:k]:
            adj[i, j] = adj[j, i] = True
    return adj


@pytest.mark.parametrize("seed,n,k", [(0, 30, 3), (1, 40, 6), (2, 25, 30), (3, 60, 1)])
def test_knn_graph_against_all_pairs_hop_distances(seed, n, k):
    g = synth.small_sbm(n, 3, 3.0, 2, seed)
    edges = np.concatenate([g.edges, [[0, n - 1]]])       # a chain link across communities
    rp, col = oracle.csr_from_edges(n, edges)
    krp, kcol = oracle.knn_graph(rp, col, k)
    adj = brute_knn(n, edges, k)
    r, c = np.nonzero(adj)
    assert np.array_equal(kcol, c)
    assert np.array_equal(krp, np.concatenate([[0], np.cumsum(adj.sum(1))]))


def test_knn_graph_special_cases():
    # path 0-1-2-3-4: k = 1 keeps the path; k = 2 adds the 2-hop chords; k >= 4 is complete
    edges = np.array([[0, 1], [1, 2], [2, 3], [3, 4]])
    rp, col = oracle.csr_from_edges(5, edges)
    krp, kcol = oracle.knn_graph(rp, col, 1)
    # node 1's nearest is 0 (tie with 2, smaller id), node 2's is 1, node 3's is 2, node 4's is 3
    assert np.array_equal(krp, rp) and np.array_equal(kcol, col)
    krp, kcol = oracle.knn_graph(rp, col, 4)
    assert np.array_equal(np.diff(krp), [4] * 5)
    # isolated nodes stay isolated; an edge's two ends always join
    rp, col = oracle.csr_from_edges(4, np.array([[1, 2]]))
    krp, kcol = oracle.knn_graph(rp, col, 3)
    assert np.array_equal(krp, [0, 0, 1, 2, 2]) and np.array_equal(kcol, [2, 1])


# ---------------------------------------------------------------------------
# ShortestPath embedding (§2.3, eq. (8))
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,l0", [(0, 50, 2.5), (1, 80, 100.0), (2, 40, 1.0)])
def test_shortest_path_embedding_against_scipy(seed, n, l0):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path
    g = synth.small_sbm(n, 3, 2.5, 2, seed)            # sparse enough to leave some nodes unreachable
    rp, col = oracle.csr_from_edges(n, g.edges)
    targets = np.random.default_rng(seed).choice(n, 7, replace=False).astype(np.int32)
    X = oracle.shortest_path_embedding(rp, col, targets, l0)
    e = g.edges
    A = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    D = shortest_path(A, directed=False, unweighted=True, indices=targets)   # [d, n]
    expect = np.where(np.isfinite(D) & (D <= l0), D, l0 + 1.0).T.astype(np.float32)
    assert np.array_equal(X, expect)
    assert np.all(X[targets, np.arange(7)] == 0)


# ---------------------------------------------------------------------------
# Layout quality: NMI (section 2.5, eq. (11)), k-means on the layout
# (section 2.5, read as Lloyd from given centres), AQ (section 2.6)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,ka,kb,seed", [(50, 3, 4, 0), (1000, 10, 7, 1), (5000, 40, 40, 2), (300, 1, 5, 3)])
def test_nmi_against_sklearn(n, ka, kb, seed):
    from sklearn.metrics import normalized_mutual_info_score
    rng = np.random.default_rng(seed)
    a = rng.integers(0, ka, n).astype(np.int32)
    b = np.where(rng.random(n) < 0.6, a % kb, rng.integers(0, kb, n)).astype(np.int32)   # correlated
    ref = normalized_mutual_info_score(a, b, average_method="arithmetic")
    assert abs(oracle.nmi(a, ka, b, kb) - ref) <= 1e-12


def test_nmi_special_cases():
    a = np.repeat(np.arange(4, dtype=np.int32), 25)
    perm = np.array([2, 0, 3, 1], np.int32)
    assert oracle.nmi(a, 4, perm[a], 4) == pytest.approx(1.0, abs=1e-15)      # same partition, renamed
    x = np.arange(400, dtype=np.int32)
    assert abs(oracle.nmi(x % 2, 2, (x // 2) % 2, 2)) <= 1e-15                # independent: I = 0
    z = np.zeros(10, np.int32)
    assert oracle.nmi(z, 1, z, 1) == 1.0                                       # both single-cluster
    assert np.isnan(oracle.nmi(z, 1, np.full(10, 5, np.int32), 3))             # label out of range


def quantised(Y):
    # the grid the clustering runs on: 2^24 steps over each axis' range
    Y = Y.astype(np.float64)
    lo, hi = Y.min(0), Y.max(0)
    q = np.floor((Y - lo) / (hi - lo) * 2.0 ** 24)
    return np.minimum(q, 2.0 ** 24 - 1)


def blobs(n, k, seed, spread=0.3):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-50, 50, (k, 2))
    lab = rng.integers(0, k, n)
    return (centres[lab] + spread * rng.standard_normal((n, 2))).astype(np.float32), lab


@pytest.mark.parametrize("n,k,seed", [(500, 3, 0), (4000, 12, 1), (20000, 30, 2)])
def test_kmeans_against_sklearn_lloyd(n, k, seed):
    from sklearn.cluster import KMeans
    Y, _ = blobs(n, k, seed, spread=2.0)
    seeds = np.random.default_rng(seed + 7).choice(n, k, replace=False).astype(np.int32)
    labels, iters = oracle.kmeans(Y, seeds, max_iter=300)
    q = quantised(Y)
    km = KMeans(n_clusters=k, init=q[seeds], n_init=1, max_iter=300, tol=0.0, algorithm="lloyd").fit(q)
    assert np.array_equal(labels, km.labels_)
    assert iters < 300


def test_kmeans_fixed_point_and_hand_case():
    Y, _ = blobs(3000, 8, 5, spread=6.0)          # overlapping blobs
    seeds = np.arange(8, dtype=np.int32) * 100
    labels, iters = oracle.kmeans(Y, seeds, max_iter=500)
    assert iters < 500
    q = quantised(Y)
    cent = np.stack([q[labels == c].mean(0) for c in range(8)])
    d2 = ((q[:, None, :] - cent[None]) ** 2).sum(-1)
    assert np.array_equal(labels, d2.argmin(1))     # every point at its nearest mean
    # hand-worked: x = 0, 1, 10, 11 from centres at the first two points:
    # pass 1 gives [0, 1, 1, 1], pass 2 [0, 0, 1, 1], pass 3 changes nothing
    H = np.array([[0, 0], [1, 0], [10, 0], [11, 0]], np.float32)
    labels, iters = oracle.kmeans(H, np.array([0, 1], np.int32))
    assert labels.tolist() == [0, 0, 1, 1] and iters == 3
    # coincident points: every tie goes to the lower index
    labels, iters = oracle.kmeans(np.ones((5, 2), np.float32), np.array([0, 3, 4], np.int32))
    assert labels.tolist() == [0] * 5 and iters == 2
    with pytest.raises(oracle.OracleError):
        oracle.kmeans(H, np.array([0, 4], np.int32))


def test_aq_hand_cases():
    corners = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], np.float32)
    lab = np.array([0, 0, 1, 1], np.int32)
    assert oracle.aq(corners, lab, 2, 2, 0.5) == 1.0     # one point per cell
    assert oracle.aq(corners, lab, 2, 1, 0.5) == 0.0     # one cell, half and half: not > 0.5
    assert oracle.aq(corners, lab, 2, 1, 0.4) == 1.0
    # x = 0..3 on a 3 x 3 grid: x = 3 lies on the upper edge and joins the last
    # column; y = 0 for all, so only the bottom row is used
    line = np.array([[0, 0], [1, 0], [2, 0], [3, 0]], np.float32)
    # cells: col 0 {0}, col 1 {1}, col 2 {2, 3}; labels 0, 1, 0, 1 -> col 2 is 1:1
    assert oracle.aq(line, np.array([0, 1, 0, 1], np.int32), 2, 3, 0.5) == pytest.approx(2 / 9)
    # 3 x 3: a 9-point pattern with two mixed cells
    pts, labs = [], []
    for cx in range(3):
        for cy in range(3):
            for r in range(3):
                pts.append([cx + 0.2 + 0.3 * r, cy + 0.5])
                labs.append(0 if (cx, cy) not in ((1, 1), (2, 0)) else r % 2)
    pts = np.array(pts + [[0, 0], [3, 3]], np.float32)          # corners fix the box to [0, 3]^2
    labs = np.array(labs + [0, 0], np.int32)
    # mixed cells hold labels (0, 1, 0): fraction 2/3 -> good at p = 0.5, not at p = 0.7
    assert oracle.aq(pts, labs, 2, 3, 0.5) == 1.0
    assert oracle.aq(pts, labs, 2, 3, 0.7) == pytest.approx(7 / 9)


def test_aq_invariants():
    Y, lab = blobs(2000, 5, 11, spread=3.0)
    lab = lab.astype(np.int32)
    a = oracle.aq(Y, lab, 5, 10, 0.6)
    assert 0.0 <= a <= 1.0
    assert oracle.aq(Y * np.float32(4.0), lab, 5, 10, 0.6) == a            # exact rescaling
    one = np.zeros_like(lab)
    q = np.floor((Y.astype(np.float64) - Y.min(0)) / ((Y.max(0) - Y.min(0)) / 10.0))
    occupied = len({(min(int(x), 9), min(int(y), 9)) for x, y in q})
    assert oracle.aq(Y, one, 1, 10, 0.99) == pytest.approx(occupied / 100)  # single label: every occupied cell
    assert oracle.aq(Y, lab, 5, 10, 1.0) == 0.0                             # fraction never exceeds 1


# ---------------------------------------------------------------------------
# Random-walk P (section 2.1) and its generator
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    kat = json.load(open(os.path.join(os.path.dirname(GOLDEN), "philox4x32_10_kat.json")))
    for case in kat["cases"]:
        out = oracle.philox4x32_10([int(x, 16) for x in case["ctr"]], [int(x, 16) for x in case["key"]])
        assert [int(x) for x in out] == [int(x, 16) for x in case["out"]]


def transition_matrix(rp, col, X):
    # exp(-||x_u - x_v||^2) over each node's neighbours, normalised per row
    n = rp.shape[0] - 1
    T = np.zeros((n, n))
    Xd = X.astype(np.float64)
    for u in range(n):
        nb = col[rp[u]:rp[u + 1]]
        if len(nb) == 0:
            T[u, u] = 1.0               # a walk from an isolated node stays put
            continue
        D = ((Xd[u] - Xd[nb]) ** 2).sum(1)
        w = np.exp(-(D - D.min()))
        T[u, nb] = w / w.sum()
    return T


def walk_frequencies(rp, col, X, walks, length, seed):
    orp, ocol, P = oracle.walk_P(rp, col, X, walks, length, seed)
    n = rp.shape[0] - 1
    dense = np.zeros((n, n))
    for i in range(n):
        dense[i, ocol[orp[i]:orp[i + 1]]] = P[orp[i]:orp[i + 1]]
    return dense


@pytest.mark.parametrize("length", [1, 2, 3])
def test_walk_P_converges_to_transition_powers(length):
    # a small graph with distinct edge weights; many walks per node
    rng = np.random.default_rng(length)
    n = 9
    edges = np.array([[0, 1], [1, 2], [2, 3], [3, 0], [1, 4], [4, 5], [5, 6], [6, 4], [2, 7]], np.int32)
    rp, col = oracle.csr_from_edges(n, edges)          # node 8 isolated
    X = rng.standard_normal((n, 3)).astype(np.float32)
    walks = 40000
    dense = walk_frequencies(rp, col, X, walks, length, 1234 + length)
    T = transition_matrix(rp, col, X)
    Tl = np.linalg.matrix_power(T, length)
    c = Tl.copy()
    np.fill_diagonal(c, 0.0)                            # walks ending where they started do not count
    M = c.sum()                                         # expected non-returning walks per (walk index)
    expect = (c + c.T) / (2 * M)
    # binomial noise of a pair count over n * walks walks
    sigma = np.sqrt(np.maximum(expect * (1 - expect), 1e-12) / (n * walks)) * 2 + 1e-7
    assert np.all(np.abs(dense - expect) <= 6 * sigma)
    assert np.all(dense[8] == 0) and np.all(dense[:, 8] == 0)


def test_walk_P_invariants():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path
    gi = synth.small_sbm(400, 4, 3.0, 6, 21)
    rp, col = oracle.csr_from_edges(gi.n, gi.edges)
    orp, ocol, P = oracle.walk_P(rp, col, gi.X, 20, 4, 99)
    n = gi.n
    dense = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(orp))
    dense[rows, ocol] = P
    assert np.array_equal(dense, dense.T)                              # symmetric, bitwise
    assert abs(P.astype(np.float64).sum() - 1.0) <= 1e-6
    assert np.all(np.diff(orp) >= 0) and all(np.all(np.diff(ocol[orp[i]:orp[i + 1]]) > 0) for i in range(n))
    assert np.all(ocol != rows)                                        # no diagonal
    A = coo_matrix((np.ones(len(col)), (np.repeat(np.arange(n), np.diff(rp)), col)), shape=(n, n))
    hops = shortest_path(A, unweighted=True)
    assert np.all(hops[rows, ocol] <= 4)                                # within `length` hops
    again = oracle.walk_P(rp, col, gi.X, 20, 4, 99)
    assert np.array_equal(again[1], ocol) and np.array_equal(again[2], P)
    other = oracle.walk_P(rp, col, gi.X, 20, 4, 100)
    assert not (len(other[1]) == len(ocol) and np.array_equal(other[1], ocol) and np.array_equal(other[2], P))


# ---------------------------------------------------------------------------
# Locality order: Morton order of the leading embedding coordinates
# ---------------------------------------------------------------------------

def test_locality_order_one_coordinate_is_sorting():
    x = np.random.default_rng(0).standard_normal((1000, 1)).astype(np.float32)
    x[10] = x[20]                                   # a tie: lower id first
    assert np.array_equal(oracle.locality_order(x), np.argsort(x[:, 0], kind="stable"))


def test_locality_order_z_curve():
    # a 4 x 4 grid: the Z curve visits quadrants (coordinate 0 first), then
    # the points inside each quadrant in the same pattern
    pts = np.array([[a, b] for a in range(4) for b in range(4)], np.float32)
    order = [tuple(int(v) for v in pts[i]) for i in oracle.locality_order(pts)]
    assert order == [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (0, 3), (1, 2), (1, 3),
                     (2, 0), (2, 1), (3, 0), (3, 1), (2, 2), (2, 3), (3, 2), (3, 3)]
    corners = np.array([[0, 0], [1, 1], [0, 1], [1, 0]], np.float32)
    assert oracle.locality_order(corners).tolist() == [0, 2, 3, 1]


def test_locality_order_brings_graph_neighbours_together():
    gi = synth.small_sbm(20000, 40, 8.0, 8, 3)
    perm = oracle.locality_order(gi.X)
    assert np.array_equal(np.sort(perm), np.arange(gi.n))
    rank = np.empty(gi.n, np.int64)
    rank[perm] = np.arange(gi.n)
    gap = np.abs(rank[gi.edges[:, 0]] - rank[gi.edges[:, 1]])
    before = np.abs(gi.edges[:, 0].astype(np.int64) - gi.edges[:, 1])        # the generator's random numbering
    intra = gi.labels[gi.edges[:, 0]] == gi.labels[gi.edges[:, 1]]
    assert np.median(gap[intra]) < 0.5 * np.median(before[intra])          # measured: 1727 against about 6700
    assert np.mean(gap < gi.n // 20) > 2 * np.mean(before < gi.n // 20)
    x = np.random.default_rng(1).standard_normal((50, 12)).astype(np.float32)
    assert np.array_equal(np.sort(oracle.locality_order(x)), np.arange(50))    # d > 8: leading 8 used


# ---------------------------------------------------------------------------
# Repulsive sums over a subset of the pairs (one share of a split run)
# ---------------------------------------------------------------------------

def test_repulsion_terms_hand_cases():
    # path (-1,0), (0,0), (1,0): w01 = w12 = 1/2, w02 = 1/5 (eq. (4)), so
    # F_0 = (1/4)(-1, 0) + (1/25)(-2, 0) = (-33/100, 0), Z = 2 (1/2 + 1/5 + 1/2)
    Y = np.array([[-1.0, 0.0], [0.0, 0.0], [1.0, 0.0]])
    F, Z = oracle.repulsion_terms(Y)
    np.testing.assert_allclose(F, [[-0.33, 0.0], [0.0, 0.0], [0.33, 0.0]], rtol=1e-15, atol=1e-17)
    assert Z == pytest.approx(2.4, rel=1e-15)
    # counting only pairs whose lower group is 0, groups (0, 1, 1): {0,1} and
    # {0,2} count, {1,2} does not: F_1 = (1/4)(1, 0), F_2 = (1/25)(2, 0), Z = 2 (1/2 + 1/5)
    F, Z = oracle.repulsion_terms(Y, group=[0, 1, 1], counted=[1, 0])
    np.testing.assert_allclose(F, [[-0.33, 0.0], [0.25, 0.0], [0.08, 0.0]], rtol=1e-15, atol=1e-17)
    assert Z == pytest.approx(1.4, rel=1e-15)
    # the complement: only {1,2}
    F, Z = oracle.repulsion_terms(Y, group=[0, 1, 1], counted=[0, 1])
    np.testing.assert_allclose(F, [[0.0, 0.0], [-0.25, 0.0], [0.25, 0.0]], rtol=1e-15, atol=1e-17)
    assert Z == pytest.approx(1.0, rel=1e-15)
    # unit square: sides w = 1/2, diagonals w = 1/3:
    # F_0 = (1/4)(-1, 0) + (1/9)(-1, -1) + (1/4)(0, -1) = (-13/36, -13/36)
    Y = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    F, Z = oracle.repulsion_terms(Y)
    np.testing.assert_allclose(F[0], [-13 / 36, -13 / 36], rtol=1e-15)
    assert Z == pytest.approx(16 / 3, rel=1e-15)


def test_repulsion_terms_against_gradient_and_invariants():
    rng = np.random.default_rng(11)
    n = 150
    Y = rng.standard_normal((n, 2)) * 4.0
    F, Z = oracle.repulsion_terms(Y)
    # with no edges the (finite-difference pinned) gradient is the repulsion alone: g = -4 F / Z
    row_ptr = np.zeros(n + 1, np.int32)
    g, Zg = oracle.gradient(row_ptr, np.zeros(0, np.int32), np.zeros(0), Y, 1.0)
    assert Z == pytest.approx(Zg, rel=1e-13)
    np.testing.assert_allclose(-4.0 * F / Z, g, rtol=1e-11, atol=1e-15)
    # a partition of the pairs by lower group adds up to the whole
    group = np.arange(n) // 16
    owner = rng.integers(0, 3, size=group.max() + 1)
    Fs, Zs = np.zeros_like(F), 0.0
    for s in range(3):
        Fk, Zk = oracle.repulsion_terms(Y, group=group, counted=(owner == s))
        # each counted pair acts on both its nodes with opposite forces
        assert np.abs(Fk.sum(0)).max() < 1e-12 * max(1.0, np.abs(Fk).sum())
        Fs += Fk
        Zs += Zk
    np.testing.assert_allclose(Fs, F, rtol=1e-12, atol=1e-14)
    assert Zs == pytest.approx(Z, rel=1e-13)
    # translation invariance and a row subset
    F2, Z2 = oracle.repulsion_terms(Y + np.array([2.5, -1.0]))
    np.testing.assert_allclose(F2, F, rtol=1e-9, atol=1e-13)
    assert Z2 == pytest.approx(Z, rel=1e-12)
    rows = np.array([149, 3, 77])
    Fr, Zr = oracle.repulsion_terms(Y, rows=rows, with_Z=False)
    assert Zr is None
    np.testing.assert_array_equal(Fr, F[rows])
