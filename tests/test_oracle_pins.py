"""Pins for the CPU oracle: closed forms, exact special cases, invariants and
cross-route agreement.  None of these compares the oracle with a retyped copy
of its own formula; each pin comes from mathematics the paper's definition
(section 3.1) fixes independently of how the oracle computes it."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from nvdgen import (path_graph, cycle_graph, complete_graph, star_graph,
                    complete_bipartite, random_tree, barabasi_albert,
                    watts_strogatz, grid_graph, Graph)


def unit_pairs(n, pairs):
    P = np.zeros((n, len(pairs)))
    Q = np.zeros((n, len(pairs)))
    for j, (a, b) in enumerate(pairs):
        P[a, j] = 1.0
        Q[b, j] = 1.0
    return P, Q


def resist(route, g, pairs):
    P, Q = unit_pairs(g.n, pairs)
    if route == "dense":
        r = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    elif route == "grounded":
        r = oracle.ge_grounded(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    elif route == "pcg":
        r = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    elif route == "tree":
        r = oracle.ge_tree(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    else:
        raise ValueError(route)
    return r["dsq"]


ROUTES = ["dense", "grounded", "pcg"]


@pytest.mark.parametrize("route", ROUTES + ["tree"])
def test_path_closed_form(route):
    n = 13
    g = path_graph(n)
    pairs = list(itertools.combinations(range(n), 2))
    R = resist(route, g, pairs)
    want = np.array([cf.path(i, j) for i, j in pairs])
    np.testing.assert_allclose(R, want, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("route", ROUTES)
def test_cycle_closed_form(route):
    n = 11
    g = cycle_graph(n)
    pairs = [(0, j) for j in range(1, n)] + [(3, 9), (5, 6)]
    R = resist(route, g, pairs)
    want = np.array([cf.cycle(n, i, j) for i, j in pairs])
    np.testing.assert_allclose(R, want, rtol=1e-11)


@pytest.mark.parametrize("route", ROUTES)
def test_complete_closed_form(route):
    n = 9
    g = complete_graph(n)
    pairs = list(itertools.combinations(range(n), 2))
    R = resist(route, g, pairs)
    np.testing.assert_allclose(R, cf.complete(n), rtol=1e-11)


@pytest.mark.parametrize("route", ROUTES + ["tree"])
def test_star_closed_form(route):
    g = star_graph(7)
    R = resist(route, g, [(0, 3), (2, 5), (6, 1)])
    np.testing.assert_allclose(
        R, [cf.star_center_leaf(), cf.star_leaf_leaf(), cf.star_leaf_leaf()], rtol=1e-11)


@pytest.mark.parametrize("route", ROUTES)
def test_complete_bipartite_closed_form(route):
    a, b = 4, 6
    g = complete_bipartite(a, b)
    pairs = [(0, 1), (2, 3), (a, a + 1), (a + 2, a + 5), (0, a), (3, a + 4)]
    R = resist(route, g, pairs)
    want = [cf.bipartite_same_side(a, b)] * 2 + [cf.bipartite_same_side(b, a)] * 2 \
        + [cf.bipartite_across(a, b)] * 2
    np.testing.assert_allclose(R, want, rtol=1e-11)


@pytest.mark.parametrize("route", ROUTES + ["tree"])
def test_weighted_tree_series_sum(route):
    rng = np.random.default_rng(5)
    n = 40
    w = rng.uniform(0.2, 3.0, size=n - 1)
    g = random_tree(n, rng, w)
    # unique path via parent pointers in the edge list
    adj = {i: [] for i in range(n)}
    for e, (u, v) in enumerate(zip(g.eu, g.ev)):
        adj[u].append((v, w[e]))
        adj[v].append((u, w[e]))

    def path_weights(s, t):
        stack = [(s, -1, [])]
        while stack:
            v, p, acc = stack.pop()
            if v == t:
                return acc
            for u, ww in adj[v]:
                if u != p:
                    stack.append((u, v, acc + [ww]))

    pairs = [(0, 39), (5, 17), (22, 3), (11, 30)]
    R = resist(route, g, pairs)
    want = [cf.tree_path(path_weights(i, j)) for i, j in pairs]
    np.testing.assert_allclose(R, want, rtol=1e-11)


def test_cycle_fft_route_closed_form_and_dense():
    n = 17
    pairs = [(0, j) for j in range(1, n)]
    P, Q = unit_pairs(n, pairs)
    r = oracle.ge_cycle(n, P, Q, w=2.5)
    np.testing.assert_allclose(r["dsq"], [cf.cycle(n, i, j, 2.5) for i, j in pairs], rtol=1e-12)
    g = cycle_graph(n, np.full(n, 2.5))
    rng = np.random.default_rng(0)
    P, Q = rng.random((n, 3)), rng.random((n, 3))
    np.testing.assert_allclose(oracle.ge_cycle(n, P, Q, w=2.5)["d"],
                               oracle.ge_dense(n, g.row_ptr, g.col_idx, g.w, P, Q)["d"], rtol=1e-12)


def _rand_vectors(n, k, rng):
    P = np.where(rng.random((n, k)) < 0.3, rng.random((n, k)), 0.0)
    Q = np.where(rng.random((n, k)) < 0.3, rng.random((n, k)), 0.0)
    return P, Q


@pytest.mark.parametrize("kind", ["ba", "ws", "grid", "weighted_ba"])
def test_routes_agree(kind):
    rng = np.random.default_rng(11)
    if kind == "ba":
        g = barabasi_albert(300, 3, rng)
    elif kind == "ws":
        g = watts_strogatz(300, 6, 0.1, rng)
    elif kind == "grid":
        g = grid_graph(12, 15)
    else:
        g = barabasi_albert(250, 2, rng)
        g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    P, Q = _rand_vectors(g.n, 4, rng)
    a = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    b = oracle.ge_grounded(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    c = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    np.testing.assert_allclose(b["d"], a["d"], rtol=1e-10)
    np.testing.assert_allclose(c["d"], a["d"], rtol=1e-10)
    np.testing.assert_allclose(b["x"], a["x"], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(c["x"], a["x"], rtol=1e-7, atol=1e-9)


def test_pcg_matches_exact_tree_at_large_n():
    rng = np.random.default_rng(3)
    g = barabasi_albert(20000, 1, rng)        # BA with m = 1 is a tree
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    P, Q = _rand_vectors(g.n, 2, rng)
    t = oracle.ge_tree(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    c = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    np.testing.assert_allclose(c["d"], t["d"], rtol=1e-11)


def test_pcg_matches_exact_cycle_high_condition():
    n = 800                                     # kappa ~ n^2
    g = cycle_graph(n)
    rng = np.random.default_rng(4)
    P, Q = _rand_vectors(n, 2, rng)
    e = oracle.ge_cycle(n, P, Q)
    c = oracle.ge_pcg(n, g.row_ptr, g.col_idx, None, P, Q)
    np.testing.assert_allclose(c["d"], e["d"], rtol=1e-10)


def test_cycle_closed_form_keeps_digits_at_large_n():
    """At n = 2e5 the smallest cycle eigenvalue is ~1e-9; the closed form must
    not lose it to cancellation (2 - 2 cos does, by ~3e-8 on d).  Against the
    grounded sparse solve of the same cycle."""
    n = 200_000
    g = cycle_graph(n)
    rng = np.random.default_rng(2)
    P = np.where(rng.random((n, 3)) < 0.01, rng.random((n, 3)), 0.0)
    Q = np.where(rng.random((n, 3)) < 0.01, rng.random((n, 3)), 0.0)
    e = oracle.ge_cycle(n, P, Q)
    gr = oracle.ge_grounded(n, g.row_ptr, g.col_idx, None, P, Q, sparse=True)
    np.testing.assert_allclose(e["d"], gr["d"], rtol=5e-9)


def test_foster_theorem():
    """sum_e w_e R_e = n - c (Foster's theorem)."""
    rng = np.random.default_rng(8)
    g1 = barabasi_albert(60, 2, rng)
    g2 = path_graph(10)
    # disjoint union plus two isolated nodes -> c = 4
    n = g1.n + g2.n + 2
    w = np.concatenate([rng.lognormal(0, 1, g1.num_edges), rng.uniform(0.5, 2, g2.num_edges)])
    g = Graph(n, np.concatenate([g1.eu, g2.eu + g1.n]), np.concatenate([g1.ev, g2.ev + g1.n]), w)
    R = resist("dense", g, list(zip(g.eu, g.ev)))
    assert abs(np.sum(w * R) - (n - 4)) < 1e-10
    R2 = resist("grounded", g, list(zip(g.eu, g.ev)))
    assert abs(np.sum(w * R2) - (n - 4)) < 1e-10


def test_kirchhoff_index_trace():
    """sum_{i<j} R_ij = n * sum_{lam>0} 1/lam for a connected graph."""
    g = barabasi_albert(50, 3, np.random.default_rng(2))
    pairs = list(itertools.combinations(range(g.n), 2))
    R = resist("grounded", g, pairs)
    L = oracle.laplacian_dense(g.n, g.row_ptr, g.col_idx)
    lam = np.linalg.eigvalsh(L)[1:]
    assert abs(R.sum() - g.n * np.sum(1 / lam)) < 1e-9 * R.sum()


def test_invariants():
    rng = np.random.default_rng(21)
    g = barabasi_albert(120, 3, rng)
    w = rng.uniform(0.5, 2.0, g.num_edges)
    g = g.with_weights(w)
    n = g.n
    A = rng.random((n, 3))
    B = rng.random((n, 3))
    C = rng.random((n, 3))

    def d(P, Q, gg=g):
        return oracle.ge_dense(gg.n, gg.row_ptr, gg.col_idx, gg.w, P, Q)["d"]

    dab = d(A, B)
    assert np.all(dab > 0)
    np.testing.assert_allclose(d(B, A), dab, rtol=1e-13)               # symmetry
    assert np.all(d(A, A) == 0.0)                                      # identity
    np.testing.assert_allclose(d(A + 3.7, B), dab, rtol=1e-10)         # constant shift
    np.testing.assert_allclose(d(-2.5 * A, -2.5 * B), 2.5 * dab, rtol=1e-12)  # homogeneity
    assert np.all(d(A, C) <= d(A, B) + d(B, C) + 1e-12)                # triangle inequality
    np.testing.assert_allclose(d(A, B, g.with_weights(4.0 * w)), dab / 2.0, rtol=1e-12)
    # Rayleigh monotonicity: raising one edge weight never raises the distance
    w2 = w.copy()
    w2[rng.integers(0, w.size, 20)] *= 3.0
    assert np.all(d(A, B, g.with_weights(w2)) <= dab + 1e-12)
    # relabelling nodes
    perm = rng.permutation(n)
    inv = np.argsort(perm)
    gp = Graph(n, inv[g.eu], inv[g.ev], w)
    np.testing.assert_allclose(d(A[perm], B[perm], gp), dab, rtol=1e-11)


def test_disconnected_is_sum_over_components():
    rng = np.random.default_rng(9)
    g1 = barabasi_albert(40, 2, rng)
    g2 = cycle_graph(15)
    n = g1.n + g2.n + 3   # 3 isolated nodes
    g = Graph(n, np.concatenate([g1.eu, g2.eu + g1.n]), np.concatenate([g1.ev, g2.ev + g1.n]))
    P, Q = rng.random((n, 2)), rng.random((n, 2))
    full = oracle.ge_dense(n, g.row_ptr, g.col_idx, None, P, Q)
    a = oracle.ge_dense(g1.n, g1.row_ptr, g1.col_idx, None, P[:40], Q[:40])
    b = oracle.ge_cycle(15, P[40:55], Q[40:55])
    np.testing.assert_allclose(full["dsq"], a["dsq"] + b["dsq"], rtol=1e-11)
    for route in ("grounded", "pcg"):
        r = getattr(oracle, "ge_" + route)(n, g.row_ptr, g.col_idx, None, P, Q)
        np.testing.assert_allclose(r["d"], full["d"], rtol=1e-10)
    # x is mean-zero on every component and zero on isolated nodes
    lab = full["labels"]
    for c in range(lab.max() + 1):
        assert np.all(np.abs(full["x"][lab == c].sum(axis=0)) < 1e-10)
    assert np.all(full["x"][-3:] == 0) or np.allclose(full["x"][-3:], 0, atol=1e-14)


def test_components_bfs_partition():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(1)
    n = 300
    u = rng.integers(0, n, 200)
    v = rng.integers(0, n, 200)
    keep = u != v
    keys = np.unique(np.minimum(u[keep], v[keep]) * n + np.maximum(u[keep], v[keep]))
    g = Graph(n, keys // n, keys % n)
    lab = oracle.components(n, g.row_ptr, g.col_idx)
    nc, ref = connected_components(csr_matrix((np.ones(g.num_edges), (g.eu, g.ev)), shape=(n, n)),
                                   directed=False)
    assert lab.max() + 1 == nc
    # same partition: the label maps are bijective
    pairs = set(zip(lab.tolist(), ref.tolist()))
    assert len(pairs) == nc


def test_pcg_galerkin_monotone_lower_bound():
    """For CG from zero, delta_bar^T x_k is non-decreasing and below d^2."""
    rng = np.random.default_rng(12)
    g = barabasi_albert(500, 3, rng)
    P, Q = _rand_vectors(g.n, 1, rng)
    exact = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, None, P, Q)["dsq"][0]
    vals = []
    for it in range(1, 25):
        r = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, None, P, Q, rtol=0.0, max_iter=it)
        vals.append(r["dsq"][0])
    vals = np.array(vals)
    assert np.all(np.diff(vals) >= -1e-12 * exact)
    assert np.all(vals <= exact * (1 + 1e-12))
    assert abs(vals[-1] - exact) < 1e-6 * exact
