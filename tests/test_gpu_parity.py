"""GPU parity: the HIP path (called through the C ABI) against the CPU
oracle, element by element on the same seeded inputs.

Tolerances: FP64 path <= 1e-8 relative error per distance, mixed path
<= 1e-6 (the targets the workloads state).  Laplacian apply, per element:
|Y_ic - (L X)_ic| <= tol * (|L| |X|)_ic with tol = 1e-13 (FP64) and 2e-6
(FP32).  (|L| |X|)_ic = sum_u w_iu (|x_ic| + |x_uc|) bounds every term of
the row's sum, so this is the backward-error form of a summation of deg_i + 1
terms: deg * eps is 2.9e-13 (FP64) and 1.6e-4 (FP32) at the hub's 2,600
neighbours in the worst case; the bounds used hold with the error growing
like sqrt(deg) * eps, as in a summation with independent roundings."""
import numpy as np
import pytest

import oracle
from nvdgen import (barabasi_albert, watts_strogatz, path_graph, cycle_graph,
                    complete_graph, star_graph, Graph, workload, grid_graph)
from oracle import closed_forms as cf

from gpu_helpers import say, dev_graph, to_dev, rel_err

pytestmark = pytest.mark.gpu


def _hub_graph(seed=0, n=3000, hub_deg=2600):
    """BA graph on nodes 0..n-1, plus hub node n joined to hub_deg of them
    (exercises the split-row path with several segments), plus three isolated
    nodes n+1..n+3."""
    rng = np.random.default_rng(seed)
    g = barabasi_albert(n, 3, rng)
    hub = n
    nb = rng.choice(n, hub_deg, replace=False)
    eu = np.concatenate([g.eu, nb])
    ev = np.concatenate([g.ev, np.full(hub_deg, hub)])
    return Graph(n + 4, np.minimum(eu, ev), np.maximum(eu, ev))


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("k", [1, 3, 8, 16, 64, 100])
def test_laplacian_apply_matches_oracle(weighted, k):
    import torch
    g = _hub_graph()
    rng = np.random.default_rng(k)
    if weighted:
        g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    say("laplacian_apply", g.n, g.nnz, k, weighted)
    dg = dev_graph(g)
    assert dg.stats()["n_long_rows"] >= 1
    X = rng.standard_normal((g.n, k))
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.w)
    want = L @ X
    absL = abs(L)
    scale64 = absL @ np.abs(X)
    Y = dg.laplacian_apply(to_dev(X)).cpu().numpy()
    bad = np.abs(Y - want) > 1e-13 * scale64
    assert not bad.any(), (np.argwhere(bad)[:5], np.max(np.abs(Y - want) / np.maximum(scale64, 1e-300)))
    # FP32: input and weights are rounded to FP32 first, as the kernel sees them
    X32 = X.astype(np.float32).astype(np.float64)
    w32 = None if g.w is None else g.w.astype(np.float32).astype(np.float64)
    L32 = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w32)
    want32 = L32 @ X32
    Y32 = dg.laplacian_apply(to_dev(X).float()).cpu().numpy()
    scale32 = abs(L32) @ np.abs(X32)
    bad = np.abs(Y32 - want32) > 2e-6 * scale32
    assert not bad.any(), (np.argwhere(bad)[:5], np.max(np.abs(Y32 - want32) / np.maximum(scale32, 1e-300)))
    # strided input / output (leading dimension > k)
    Xs = torch.zeros((g.n, k + 5), dtype=torch.float64, device="cuda")
    Xs[:, :k] = to_dev(X)
    Ys = torch.full((g.n, k + 3), 7.0, dtype=torch.float64, device="cuda")
    dg.laplacian_apply(Xs[:, :k], out=Ys[:, :k])
    Ys = Ys.cpu().numpy()
    assert not (np.abs(Ys[:, :k] - want) > 1e-13 * scale64).any()
    assert np.all(Ys[:, k:] == 7.0)


def test_graph_setup_degrees_and_components():
    g = _hub_graph(1)
    rng = np.random.default_rng(2)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    say("graph_setup", g.n)
    dg = dev_graph(g)
    lab, deg = dg.query()
    L = oracle.laplacian_dense(g.n, g.row_ptr, g.col_idx, g.w)
    np.testing.assert_allclose(deg, np.diag(L), rtol=1e-15)
    ref = oracle.components(g.n, g.row_ptr, g.col_idx)
    assert np.array_equal(lab, ref)           # same numbering convention
    st = dg.stats()
    assert st["n_comp"] == ref.max() + 1 and st["n_isolated"] == 3   # nodes n+1..n+3


def test_large_disconnected_components_and_solve():
    """Set-up of a graph large enough for the parallel host passes: three BA
    components of uneven size plus isolated nodes, randomly relabelled and
    given unsorted rows; labels (numbered by smallest node), degrees and a
    mixed solve against the oracle's per-component definition."""
    rng = np.random.default_rng(21)
    parts = [barabasi_albert(n, 3, rng) for n in (150000, 90000, 40000)]
    offs = np.cumsum([0] + [p.n for p in parts])
    n = int(offs[-1]) + 5                         # 5 isolated nodes
    eu = np.concatenate([p.eu + o for p, o in zip(parts, offs[:-1])])
    ev = np.concatenate([p.ev + o for p, o in zip(parts, offs[:-1])])
    perm = rng.permutation(n)
    g0 = Graph(n, perm[eu], perm[ev])
    # shuffle the entries inside every row (the library sorts them)
    ci = g0.col_idx.copy()
    for i in rng.choice(n, 2000, replace=False):
        a, b = g0.row_ptr[i], g0.row_ptr[i + 1]
        ci[a:b] = rng.permutation(ci[a:b])
    say("large disconnected", n, g0.nnz)
    import paper_2310_11222_amd as nvd
    dg = nvd.Graph(g0.row_ptr, ci, None)
    lab, deg = dg.query()
    ref = oracle.components(n, g0.row_ptr, g0.col_idx)
    assert np.array_equal(lab, ref)
    np.testing.assert_array_equal(deg, np.diff(g0.row_ptr).astype(np.float64))
    st = dg.stats()
    assert st["n_comp"] == 3 + 5 and st["n_isolated"] == 5
    k = 4
    P = np.where(rng.random((n, k)) < 0.05, rng.random((n, k)), 0.0)
    Q = np.where(rng.random((n, k)) < 0.05, rng.random((n, k)), 0.0)
    d, _, info = dg.distances(P, Q, precision="mixed", rtol=1e-8)
    r = oracle.ge_pcg(n, g0.row_ptr, g0.col_idx, None, P, Q)
    assert rel_err(d.cpu().numpy(), r["d"]).max() <= 1e-6
    assert all(i["status"] == 0 for i in info)


@pytest.mark.parametrize("k", [1, 5, 64])
def test_project_matches_oracle(k):
    g = _hub_graph(3)
    rng = np.random.default_rng(4)
    P, Q = rng.random((g.n, k)), rng.random((g.n, k))
    say("project", k)
    dg = dev_graph(g)
    D, norms = dg.project(to_dev(P), to_dev(Q))
    want = oracle.project(P - Q, oracle.components(g.n, g.row_ptr, g.col_idx))
    np.testing.assert_allclose(D.cpu().numpy(), want, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(norms.cpu().numpy(), np.linalg.norm(want, axis=0), rtol=1e-12)


def test_c1_fp64_against_dense_oracle():
    w = workload(1)
    g = w.graphs[0]
    say("C1 fp64", g.n)
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, w.P[0], w.Q[0])
    dg = dev_graph(g)
    d, X, info = dg.distances(w.P[0], w.Q[0], precision="fp64", rtol=1e-10, return_x=True)
    d = d.cpu().numpy()
    assert np.all(rel_err(d, ref["d"]) <= 1e-8), (d, ref["d"])
    assert info[0]["status"] == 0 and info[0]["rel_res"] <= 1e-10
    np.testing.assert_allclose(X.cpu().numpy(), ref["x"], rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("k,tile", [(1, 0), (7, 0), (37, 8), (64, 64), (20, 4)])
def test_distances_ba_weighted(precision, tol, k, tile):
    rng = np.random.default_rng(100 + k)
    g = barabasi_albert(2500, 3, rng)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    P = np.where(rng.random((g.n, k)) < 0.1, rng.random((g.n, k)), 0.0)
    Q = np.where(rng.random((g.n, k)) < 0.1, rng.random((g.n, k)), 0.0)
    say("ba weighted", precision, k, tile)
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    dg = dev_graph(g)
    d, _, info = dg.distances(P, Q, precision=precision, rtol=1e-10 if precision == "fp64" else 1e-8,
                              tile_k=tile)
    e = rel_err(d.cpu().numpy(), ref["d"])
    assert e.max() <= tol, e.max()
    assert all(i["status"] == 0 for i in info)
    if precision == "mixed":
        assert all(i["refine_steps"] >= 1 for i in info)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_disconnected_with_isolated_nodes(precision):
    g = _hub_graph(5, n=800, hub_deg=300)
    rng = np.random.default_rng(6)
    # add a separate WS component
    w2 = watts_strogatz(300, 6, 0.1, rng)
    n = g.n + w2.n
    gg = Graph(n, np.concatenate([g.eu, w2.eu + g.n]), np.concatenate([g.ev, w2.ev + g.n]))
    P, Q = rng.random((n, 6)), rng.random((n, 6))
    say("disconnected", precision, n)
    ref = oracle.ge_dense(n, gg.row_ptr, gg.col_idx, None, P, Q)
    dg = dev_graph(gg)
    d, X, info = dg.distances(P, Q, precision=precision, rtol=1e-10, return_x=True)
    e = rel_err(d.cpu().numpy(), ref["d"])
    assert e.max() <= (1e-8 if precision == "fp64" else 1e-6)
    np.testing.assert_allclose(X.cpu().numpy(), ref["x"], rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_closed_forms_on_gpu(precision):
    say("closed forms", precision)
    for g, pairs, want in [
        (path_graph(60), [(0, 59), (3, 40), (10, 11)], [59, 37, 1]),
        (cycle_graph(41), [(0, 20), (5, 6), (0, 13)],
         [cf.cycle(41, 0, 20), cf.cycle(41, 5, 6), cf.cycle(41, 0, 13)]),
        (complete_graph(30), [(0, 1), (7, 29)], [cf.complete(30)] * 2),
        (star_graph(40), [(0, 5), (3, 9)], [1.0, 2.0]),
    ]:
        P = np.zeros((g.n, len(pairs)))
        Q = np.zeros((g.n, len(pairs)))
        for j, (a, b) in enumerate(pairs):
            P[a, j] = 1.0
            Q[b, j] = 1.0
        dg = dev_graph(g)
        d, _, _ = dg.distances(P, Q, precision=precision, rtol=1e-12 if precision == "fp64" else 1e-10)
        dsq = d.cpu().numpy() ** 2
        np.testing.assert_allclose(dsq, want, rtol=1e-8 if precision == "fp64" else 1e-6)


def test_degenerate_pairs():
    g = barabasi_albert(500, 2, np.random.default_rng(7))
    rng = np.random.default_rng(8)
    P = rng.random((g.n, 4))
    Q = P.copy()
    Q[:, 1] = P[:, 1] + 3.25          # constant shift: delta_bar = 0
    Q[:, 2] = 0.0                     # an ordinary pair
    say("degenerate")
    dg = dev_graph(g)
    for prec in ("fp64", "mixed"):
        d, _, info = dg.distances(P, Q, precision=prec)
        d = d.cpu().numpy()
        assert d[0] == 0.0 and info[0]["iters"] == 0
        assert d[1] == 0.0 or d[1] < 1e-12
        assert d[3] == 0.0
        ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, None, P[:, 2:3], Q[:, 2:3])["d"][0]
        assert abs(d[2] - ref) <= (1e-8 if prec == "fp64" else 1e-6) * ref


def test_single_node_and_edge():
    say("tiny graphs")
    g1 = Graph(1, np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64))
    dg = dev_graph(g1)
    d, _, _ = dg.distances(np.array([[2.0]]), np.array([[5.0]]))
    assert d.cpu().numpy()[0] == 0.0
    g2 = path_graph(2)
    dg = dev_graph(g2)
    d, _, _ = dg.distances(np.array([[1.0], [0.0]]), np.array([[0.0], [1.0]]))
    assert abs(d.cpu().numpy()[0] ** 2 - 1.0) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_tree_exact(precision):
    """BA with m = 1 is a tree: exact O(n) oracle at n = 2e5."""
    rng = np.random.default_rng(9)
    g = barabasi_albert(200_000, 1, rng)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    P = np.where(rng.random((g.n, 4)) < 0.05, rng.random((g.n, 4)), 0.0)
    Q = np.where(rng.random((g.n, 4)) < 0.05, rng.random((g.n, 4)), 0.0)
    say("large tree", precision)
    ref = oracle.ge_tree(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    dg = dev_graph(g)
    d, _, info = dg.distances(P, Q, precision=precision, rtol=1e-10 if precision == "fp64" else 1e-8)
    e = rel_err(d.cpu().numpy(), ref["d"])
    assert e.max() <= (1e-8 if precision == "fp64" else 1e-6), (e, info)


def test_grad_weights_matches_oracle():
    import torch
    rng = np.random.default_rng(10)
    g = barabasi_albert(400, 3, rng)
    g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    P, Q = rng.random((g.n, 5)), rng.random((g.n, 5))
    gs = rng.standard_normal(5)
    say("grad weights")
    dg = dev_graph(g)
    d, X, _ = dg.distances(P, Q, precision="fp64", rtol=1e-12, return_x=True)
    gw = dg.grad_weights(X, torch.as_tensor(gs)).cpu().numpy()
    want = oracle.grad_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q, gscale=gs)["grad_w_csr"]
    np.testing.assert_allclose(gw, want, rtol=1e-7, atol=1e-10 * np.abs(want).max())


def test_repeatable_bitwise():
    rng = np.random.default_rng(11)
    g = barabasi_albert(5000, 3, rng)
    P, Q = rng.random((g.n, 16)), rng.random((g.n, 16))
    say("repeatable")
    dg = dev_graph(g)
    a = dg.distances(P, Q, precision="fp64")[0].cpu().numpy()
    b = dg.distances(P, Q, precision="fp64")[0].cpu().numpy()
    assert np.array_equal(a, b)
    a = dg.distances(P, Q, precision="mixed")[0].cpu().numpy()
    b = dg.distances(P, Q, precision="mixed")[0].cpu().numpy()
    assert np.array_equal(a, b)


def test_noconv_reported():
    g = path_graph(3000)
    P = np.zeros((g.n, 1)); Q = np.zeros((g.n, 1))
    P[0] = 1.0; Q[-1] = 1.0
    say("noconv")
    dg = dev_graph(g)
    d, _, info = dg.distances(P, Q, precision="fp64", max_iter=5)
    assert info[0]["status"] == 4          # NVD_E_NOCONV
    assert d.cpu().numpy()[0] > 0
