"""Seeded input generators: structure, sizes and reproducibility."""
import numpy as np
import pytest

from nvdgen import (barabasi_albert, watts_strogatz, erdos_renyi,
                    configuration_model_powerlaw, giant_component, is_connected,
                    stochastic_block_model, sparse_support_pairs, workload, Graph)


def _simple(g: Graph):
    assert np.all(g.eu < g.ev)
    keys = g.eu * g.n + g.ev
    assert np.unique(keys).size == keys.size
    # CSR symmetric, sorted rows, matches the edge list
    assert g.nnz == 2 * g.num_edges
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    fwd = set(zip(rows.tolist(), g.col_idx.tolist()))
    assert all((c, r) in fwd for r, c in fwd)
    for i in range(min(g.n, 50)):
        seg = g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


@pytest.mark.parametrize("n,m", [(1000, 3), (50, 1), (200, 5)])
def test_ba(n, m):
    g = barabasi_albert(n, m, np.random.default_rng(7))
    assert g.num_edges == m * (n - m)
    _simple(g)
    assert is_connected(g.n, g.eu, g.ev)
    deg = np.diff(g.row_ptr)
    assert deg.min() >= 1 if m == 1 else deg.min() >= m
    g2 = barabasi_albert(n, m, np.random.default_rng(7))
    assert np.array_equal(g.col_idx, g2.col_idx)


def test_ba_heavy_tail():
    g = barabasi_albert(100_000, 3, np.random.default_rng(1))
    deg = np.diff(g.row_ptr)
    # preferential attachment: hubs near m*sqrt(n)
    assert deg.max() > 300
    assert np.median(deg) <= 5


def test_ws():
    g = watts_strogatz(2000, 6, 0.1, np.random.default_rng(3))
    assert g.num_edges == 3 * 2000
    _simple(g)


def test_er_sbm():
    g = erdos_renyi(500, 2000, np.random.default_rng(2))
    assert g.num_edges == 2000
    _simple(g)
    s = stochastic_block_model([30, 40], 0.3, 0.01, np.random.default_rng(2))
    _simple(s)


def test_configuration_model_gc():
    rng = np.random.default_rng(4)
    g = configuration_model_powerlaw(20000, 2.5, 3, int(20000 ** (1 / 1.5)), rng)
    _simple(g)
    gc = giant_component(g)
    assert is_connected(gc.n, gc.eu, gc.ev)
    assert gc.n > 0.95 * 20000
    mean_deg = 2 * gc.num_edges / gc.n
    assert 5.5 < mean_deg < 9.5


def test_pairs():
    P, Q = sparse_support_pairs(1000, 4, 0.1, np.random.default_rng(0))
    assert P.shape == (1000, 4) and P.flags.c_contiguous
    assert np.all((P > 0).sum(axis=0) <= 100) and np.all((P > 0).sum(axis=0) >= 95)
    assert np.all((P >= 0) & (P < 1))


def test_workloads_small_scale():
    w1 = workload(1)
    assert w1.graphs[0].n == 1000 and w1.graphs[0].num_edges == 2991
    assert w1.P[0].shape == (1000, 1)
    w3 = workload(3, scale=0.05, num_graphs=6)
    assert len(w3.graphs) == 6
    for g, P in zip(w3.graphs, w3.P):
        assert is_connected(g.n, g.eu, g.ev)
        assert g.w is not None and np.all((g.w >= 0.5) & (g.w < 2.0))
        assert P.shape == (g.n, 8)
    w4 = workload(4, scale=0.01)
    assert w4.graphs[0].w is not None
    w5 = workload(5, scale=0.001)
    assert is_connected(w5.graphs[0].n, w5.graphs[0].eu, w5.graphs[0].ev)
    # determinism
    again = workload(1)
    assert np.array_equal(again.P[0], w1.P[0])


def test_density_sweep_graphs():
    """Section 4.2 density sweep recipe: n = 10^4, average degree on target
    (BA and WS cannot go below 2), seeded (same call, same graph)."""
    from nvdgen import density_graph, DENSITY_MODELS, DENSITY_N
    for model in DENSITY_MODELS:
        for d in (1, 4, 16):
            g, P, Q = density_graph(model, d)
            assert g.n == DENSITY_N and P.shape == (DENSITY_N, 8) and Q.shape == P.shape
            avg = 2 * g.num_edges / g.n
            want = max(d, 2) if model in ("ba", "ws") else d
            assert abs(avg - want) <= 0.05 * want + 0.05, (model, d, avg)
            assert np.all(g.eu < g.ev) or np.all(g.eu != g.ev)
    g1, P1, _ = density_graph("sbm", 8)
    g2, P2, _ = density_graph("sbm", 8)
    assert np.array_equal(g1.row_ptr, g2.row_ptr) and np.array_equal(g1.col_idx, g2.col_idx)
    assert np.array_equal(P1, P2)


def test_sbm_sparse_edge_counts():
    """The sparse SBM draw keeps the Bernoulli model's expected counts: inside
    and across blocks, within 5 standard deviations."""
    from nvdgen import sbm_sparse
    rng = np.random.default_rng(3)
    sizes = [300, 500, 200]
    p_in, p_out = 0.05, 0.004
    g = sbm_sparse(sizes, p_in, p_out, rng)
    blk = np.repeat(np.arange(3), sizes)
    same = blk[g.eu] == blk[g.ev]
    n_in = sum(s * (s - 1) // 2 for s in sizes)
    n_out = (sum(sizes) ** 2 - sum(s * s for s in sizes)) // 2
    for cnt, npairs, p in ((same.sum(), n_in, p_in), ((~same).sum(), n_out, p_out)):
        mu, sd = npairs * p, np.sqrt(npairs * p * (1 - p))
        assert abs(cnt - mu) <= 5 * sd, (cnt, mu, sd)
    keys = np.minimum(g.eu, g.ev) * g.n + np.maximum(g.eu, g.ev)
    assert np.unique(keys).size == keys.size and np.all(g.eu != g.ev)
