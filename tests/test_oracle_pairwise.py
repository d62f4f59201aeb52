"""Pins of the all-pairs oracle (CPU): closed forms, the two routes against
each other and against per-pair routes, and the properties every distance
matrix of this kind has (it is a Euclidean distance matrix: the points are
L^+^(1/2) v_i)."""
import itertools

import numpy as np

import oracle
from oracle import closed_forms as cf
from nvdgen import barabasi_albert, complete_graph, random_tree, ws_connected


def test_complete_graph_unit_vectors():
    n = 12
    g = complete_graph(n)
    D = oracle.pairwise_dense(n, g.row_ptr, g.col_idx, None, np.eye(n)[:, :6])
    want = np.sqrt(cf.complete(n)) * (1 - np.eye(6))
    np.testing.assert_allclose(D, want, rtol=1e-12, atol=1e-14)


def test_weighted_tree_series_law_by_routes():
    rng = np.random.default_rng(3)
    t = random_tree(40, rng, rng.uniform(0.2, 4.0, 39))
    V = rng.random((40, 6))
    Dd = oracle.pairwise_dense(t.n, t.row_ptr, t.col_idx, t.w, V)
    Dp = oracle.pairwise_pcg(t.n, t.row_ptr, t.col_idx, t.w, V)
    iu, ju = np.triu_indices(6, 1)
    Dt = oracle.ge_tree(t.n, t.row_ptr, t.col_idx, t.w, V[:, iu], V[:, ju])["d"]
    np.testing.assert_allclose(Dd[iu, ju], Dt, rtol=1e-10)
    np.testing.assert_allclose(Dp, Dd, rtol=1e-9, atol=1e-12)


def test_matches_per_pair_dense_and_edm_properties():
    rng = np.random.default_rng(5)
    g = barabasi_albert(300, 3, rng)
    g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    V = np.where(rng.random((300, 9)) < 0.3, rng.standard_normal((300, 9)), 0.0)
    D = oracle.pairwise_dense(g.n, g.row_ptr, g.col_idx, g.w, V)
    iu, ju = np.triu_indices(9, 1)
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, V[:, iu], V[:, ju])["d"]
    np.testing.assert_allclose(D[iu, ju], ref, rtol=1e-11)
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0.0)
    # Euclidean distance matrix: -1/2 J D^2 J is positive semidefinite
    m = 9
    J = np.eye(m) - np.ones((m, m)) / m
    B = -0.5 * J @ (D * D) @ J
    assert np.linalg.eigvalsh(B).min() >= -1e-9 * np.abs(B).max()
    for i, j, k in itertools.permutations(range(m), 3):
        assert D[i, j] <= D[i, k] + D[k, j] + 1e-12


def test_constant_shift_and_repeated_vectors():
    """Adding a constant to a vector does not move it (L^+ 1 = 0); a repeated
    vector is at distance 0."""
    rng = np.random.default_rng(7)
    g = ws_connected(200, 4, 0.2, np.random.SeedSequence(8))
    V = rng.random((200, 4))
    V2 = np.column_stack([V, V[:, 1] + 3.5, V[:, 2]])
    D = oracle.pairwise_dense(g.n, g.row_ptr, g.col_idx, None, V2)
    assert D[1, 4] < 1e-7 and D[2, 5] < 1e-7
    np.testing.assert_allclose(D[:4, 4], D[:4, 1], rtol=1e-9, atol=1e-9)
