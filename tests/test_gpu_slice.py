"""GPU parity of the one-column apply by XCD-pinned column slices.  Graphs of
2^20 nodes and more use it where it times faster; here it is forced on small graphs
with small slices (NVD_SLICE=1, NVD_SLICE_NODES), so that every case spans
several slices and row chunks with a ragged last chunk, short items and
hub rows with long items, and compared with the CPU oracle:
  * the apply per element, FP64 and FP32, unit and weighted, strided, with
    the bounds of test_gpu_parity (|Y - L X| <= tol (|L| |X|) per entry);
  * bit-for-bit repeats and agreement with the row-wise apply;
  * distances solved one column at a time, both precisions, against the
    oracle's PCG and grounded routes;
  * new weights after the slices were built;
  * the timed choice on graphs of 2^20 nodes (BA and power-law), against the
    row-wise apply;
  * tree- and approximate-Cholesky-preconditioned solves (smooth directions);
  * a warm start from the oracle's x, the squared output and the returned x.
The single-launch solve is switched off (NVD_SMALL=0) so that the solves go
through the sliced apply.  The 10^7-node case runs in test_gpu_full_size."""
import numpy as np
import pytest

import oracle
from nvdgen import Graph, barabasi_albert, configuration_model_powerlaw, giant_component

from gpu_helpers import say, dev_graph, to_dev, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture
def sliced(monkeypatch):
    def on(nodes):
        monkeypatch.setenv("NVD_SLICE", "1")
        monkeypatch.setenv("NVD_SLICE_NODES", str(nodes))
        monkeypatch.setenv("NVD_SMALL", "0")
    return on


def _hub_graph(seed=0, n=9000, hub_deg=5000):
    """BA graph plus hub node n joined to hub_deg nodes plus three isolated
    nodes: n + 4 = 9004 rows (4 full chunks of 2048 and a ragged one)."""
    rng = np.random.default_rng(seed)
    g = barabasi_albert(n, 3, rng)
    nb = rng.choice(n, hub_deg, replace=False)
    eu = np.concatenate([g.eu, nb])
    ev = np.concatenate([g.ev, np.full(hub_deg, n)])
    return Graph(n + 4, np.minimum(eu, ev), np.maximum(eu, ev))


def _powerlaw(seed=1, n=30000):
    rng = np.random.default_rng(seed)
    kmax = int(np.floor(n ** (1.0 / 1.5)))
    return giant_component(configuration_model_powerlaw(n, 2.5, 3, kmax, rng))


def _check_apply(dg, g, X):
    import torch
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.w)
    want = L @ X
    scale64 = abs(L) @ np.abs(X)
    Y = dg.laplacian_apply(to_dev(X)).cpu().numpy()
    bad = np.abs(Y - want) > 1e-13 * scale64
    assert not bad.any(), (np.argwhere(bad)[:5], np.max(np.abs(Y - want) / np.maximum(scale64, 1e-300)))
    X32 = X.astype(np.float32).astype(np.float64)
    w32 = None if g.w is None else g.w.astype(np.float32).astype(np.float64)
    L32 = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w32)
    want32 = L32 @ X32
    Y32 = dg.laplacian_apply(to_dev(X).float()).cpu().numpy()
    scale32 = abs(L32) @ np.abs(X32)
    bad = np.abs(Y32 - want32) > 2e-6 * scale32
    assert not bad.any(), (np.argwhere(bad)[:5], np.max(np.abs(Y32 - want32) / np.maximum(scale32, 1e-300)))
    # strided column of a wider matrix; the rest of the output is untouched
    Xs = torch.zeros((g.n, 6), dtype=torch.float64, device="cuda")
    Xs[:, 2] = to_dev(X[:, 0])
    Ys = torch.full((g.n, 4), 7.0, dtype=torch.float64, device="cuda")
    dg.laplacian_apply(Xs[:, 2:3], out=Ys[:, 1:2])
    Ys = Ys.cpu().numpy()
    assert not (np.abs(Ys[:, 1] - want[:, 0]) > 1e-13 * scale64[:, 0]).any()
    assert np.all(Ys[:, [0, 2, 3]] == 7.0)
    return Y, Y32


@pytest.mark.parametrize("graph", ["hub", "powerlaw"])
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("nodes", [700, 4000])
def test_sliced_apply_matches_oracle(sliced, graph, weighted, nodes):
    sliced(nodes)
    g = _hub_graph() if graph == "hub" else _powerlaw()
    rng = np.random.default_rng(nodes + weighted)
    if weighted:
        g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    say("sliced apply", graph, g.n, g.nnz, weighted, nodes)
    dg = dev_graph(g)
    b0 = dg.stats()["device_bytes"]
    X = rng.standard_normal((g.n, 1))
    Y, Y32 = _check_apply(dg, g, X)
    assert dg.stats()["device_bytes"] > b0        # the slices were built and used
    # repeats are bit for bit
    assert np.array_equal(dg.laplacian_apply(to_dev(X)).cpu().numpy(), Y)
    assert np.array_equal(dg.laplacian_apply(to_dev(X).float()).cpu().numpy(), Y32)


def test_sliced_apply_against_row_wise(sliced, monkeypatch):
    """Same graph, slices on and off: both within the per-element bound of the
    oracle, and within a few FP64 roundings of each other."""
    g = _powerlaw(3)
    rng = np.random.default_rng(5)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    X = rng.standard_normal((g.n, 1))
    say("sliced vs row-wise", g.n)
    sliced(1000)
    dg = dev_graph(g)
    Ys = dg.laplacian_apply(to_dev(X)).cpu().numpy()
    monkeypatch.setenv("NVD_SLICE", "0")
    Yr = dg.laplacian_apply(to_dev(X)).cpu().numpy()
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.w)
    scale = abs(L) @ np.abs(X)
    assert np.all(np.abs(Ys - Yr) <= 2e-13 * scale)


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-10, 1e-8), ("mixed", 1e-8, 1e-6)])
def test_sliced_distances(sliced, precision, rtol, tol):
    """Three pairs solved in tiles of one column on the power-law graph
    (connected) and on the hub graph (isolated nodes, a hub of 5,000
    neighbours), against the oracle."""
    sliced(1500)
    for name, g in (("powerlaw", _powerlaw(7)), ("hub", _hub_graph(8))):
        rng = np.random.default_rng(11)
        P = np.where(rng.random((g.n, 3)) < 0.1, rng.random((g.n, 3)), 0.0)
        Q = np.where(rng.random((g.n, 3)) < 0.1, rng.random((g.n, 3)), 0.0)
        say("sliced distances", name, g.n, precision)
        dg = dev_graph(g)
        b0 = dg.stats()["device_bytes"]
        d, _, info = dg.distances(P, Q, precision=precision, rtol=rtol, tile_k=1)
        assert dg.stats()["device_bytes"] > b0
        assert all(i["status"] == 0 for i in info), info
        ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
        assert rel_err(d.cpu().numpy(), ref).max() <= tol
        if name == "hub":
            gr = oracle.ge_grounded(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
            assert rel_err(d.cpu().numpy(), gr).max() <= tol


def test_sliced_apply_after_new_weights(sliced):
    """The slices hold copies of the weights: a weight change drops them and
    the next apply uses the new weights."""
    sliced(900)
    g = _hub_graph(2)
    rng = np.random.default_rng(9)
    g1 = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    X = rng.standard_normal((g.n, 1))
    say("sliced new weights", g.n)
    dg = dev_graph(g1)
    _check_apply(dg, g1, X)
    w2 = rng.lognormal(0, 1, g.num_edges)
    g2 = g.with_weights(w2)
    dg.set_weights(g2.w)
    _check_apply(dg, g2, X)


@pytest.mark.parametrize("kind", ["ba", "powerlaw"])
def test_auto_choice_at_1e6_nodes(monkeypatch, kind):
    """Default mode on graphs of 2^20 nodes and more: the first one-column
    call of each precision times both applies and keeps the faster.  Either
    choice must give the distances of the row-wise apply (NVD_SLICE=0) and an
    apply within the per-row bound, on sampled rows, of the definition."""
    import torch
    monkeypatch.delenv("NVD_SLICE", raising=False)
    monkeypatch.setenv("NVD_SMALL", "0")
    rng = np.random.default_rng(17)
    n = (1 << 20) + 1000
    if kind == "ba":
        g = barabasi_albert(n, 3, rng)
    else:
        g = giant_component(configuration_model_powerlaw(n, 2.5, 3, int(n ** (1 / 1.5)), rng))
    say("auto choice", kind, g.n, g.nnz)
    dg = dev_graph(g)
    P = np.where(rng.random((g.n, 1)) < 0.01, rng.random((g.n, 1)), 0.0)
    Q = np.where(rng.random((g.n, 1)) < 0.01, rng.random((g.n, 1)), 0.0)
    d_auto, _, info = dg.distances(P, Q, precision="mixed", rtol=1e-8, tile_k=1)
    assert info[0]["status"] == 0
    x = rng.standard_normal(g.n)
    y32 = dg.laplacian_apply(torch.as_tensor(x).float().cuda()).cpu().numpy().ravel()
    monkeypatch.setenv("NVD_SLICE", "0")
    d_row, _, _ = dg.distances(P, Q, precision="mixed", rtol=1e-8, tile_k=1)
    assert rel_err(d_auto.cpu().numpy(), d_row.cpu().numpy()).max() <= 1e-6
    x32 = x.astype(np.float32).astype(np.float64)
    for i in np.concatenate([rng.choice(g.n, 2000, replace=False), np.argsort(np.diff(g.row_ptr))[-10:]]):
        nb = g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]
        want = np.sum(x32[i] - x32[nb])
        scale = np.sum(np.abs(x32[i]) + np.abs(x32[nb]))
        assert abs(y32[i] - want) <= 2e-6 * scale, i


@pytest.mark.parametrize("precond", ["tree", "achol"])
@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-10, 1e-8), ("mixed", 1e-8, 1e-6)])
def test_sliced_apply_with_strong_preconditioners(sliced, precond, precision, rtol, tol):
    """A preconditioner close to L^+ (the augmented forest, the approximate
    Cholesky factor) makes the CG directions smooth, with a large spread on
    a long near-tree: the case where a plain sum d x_v - sum w x_u would lose
    FP32 digits.  The sliced FP32 apply sums the partials in FP64, so these
    solves must reach the same accuracy as with the row-wise apply.  A
    2,000-node random tree with 30 extra edges and lognormal weights, plus a
    path of 3,000 nodes (its own component), one pair per tile."""
    sliced(500)
    rng = np.random.default_rng(23)
    n1 = 2000
    parent = np.array([rng.integers(0, i) for i in range(1, n1)])
    eu = [np.arange(1, n1), rng.integers(0, n1, 30)]
    ev = [parent, rng.integers(0, n1, 30)]
    n2 = 3000
    eu.append(np.arange(n1, n1 + n2 - 1))
    ev.append(np.arange(n1 + 1, n1 + n2))
    eu = np.concatenate(eu)
    ev = np.concatenate(ev)
    keep = eu != ev
    eu, ev = eu[keep], ev[keep]
    key = np.unique(np.minimum(eu, ev).astype(np.int64) * (n1 + n2) + np.maximum(eu, ev))
    eu, ev = key // (n1 + n2), key % (n1 + n2)
    g = Graph(n1 + n2, eu, ev, rng.lognormal(0.0, 1.0, eu.size))
    P = np.where(rng.random((g.n, 2)) < 0.1, rng.random((g.n, 2)), 0.0)
    Q = np.where(rng.random((g.n, 2)) < 0.1, rng.random((g.n, 2)), 0.0)
    say("sliced with", precond, precision, g.n, g.nnz)
    dg = dev_graph(g)
    b0 = dg.stats()["device_bytes"]
    d, _, info = dg.distances(P, Q, precision=precision, rtol=rtol, tile_k=1, precond=precond)
    assert dg.stats()["device_bytes"] > b0
    assert all(i["status"] == 0 for i in info), info
    ref = oracle.ge_grounded(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    assert rel_err(d.cpu().numpy(), ref).max() <= tol


def test_sliced_warm_start_and_squared_output(sliced):
    """Tiles of one column through the sliced apply: a warm start from the
    oracle's solution converges at once to the oracle's distances, and the
    squared output and the returned x match the oracle (FP64)."""
    sliced(1200)
    g = _powerlaw(29)
    rng = np.random.default_rng(31)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    P = np.where(rng.random((g.n, 2)) < 0.1, rng.random((g.n, 2)), 0.0)
    Q = np.where(rng.random((g.n, 2)) < 0.1, rng.random((g.n, 2)), 0.0)
    # the PCG route (an LU of this expander's grounded Laplacian fills in)
    ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    say("sliced warm start", g.n)
    dg = dev_graph(g)
    dsq, X, info = dg.distances(P, Q, precision="fp64", rtol=1e-10, tile_k=1, return_x=True, out="dsq")
    assert rel_err(dsq.cpu().numpy(), ref["dsq"]).max() <= 1e-8
    np.testing.assert_allclose(X.cpu().numpy(), ref["x"], rtol=0, atol=1e-7 * np.abs(ref["x"]).max())
    d, _, info = dg.distances(P, Q, precision="fp64", rtol=1e-10, tile_k=1, X0=ref["x"])
    assert rel_err(d.cpu().numpy(), ref["d"]).max() <= 1e-8
    assert all(i["iters"] <= 2 for i in info), [i["iters"] for i in info]
