"""GPU parity of the batched solvers (many uneven graphs per call: the sweep
solver over the block-diagonal operator, and the single persistent launch)
against the CPU oracle, and against the same pairs solved one graph at a
time."""
import numpy as np
import pytest

import oracle
from nvdgen import barabasi_albert, ws_connected, workload, Graph, cycle_graph

from gpu_helpers import say, dev_graph, rel_err

pytestmark = pytest.mark.gpu


def _mk_batch(seed, sizes, k_list, weighted=True):
    rng = np.random.default_rng(seed)
    graphs, Ps, Qs = [], [], []
    for i, (n, k) in enumerate(zip(sizes, k_list)):
        if i % 2 == 0:
            g = ws_connected(n, 6, 0.1, np.random.SeedSequence([seed, i]))
        else:
            g = barabasi_albert(n, 4, rng)
        if weighted:
            g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
        P = np.where(rng.random((g.n, k)) < 0.2, rng.standard_normal((g.n, k)), 0.0)
        Q = np.where(rng.random((g.n, k)) < 0.2, rng.standard_normal((g.n, k)), 0.0)
        graphs.append(g)
        Ps.append(P)
        Qs.append(Q)
    return graphs, Ps, Qs


def _oracle(g, P, Q):
    if g.n <= 4000:
        return oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    return oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]


def _run(graphs, Ps, Qs, precision, **kw):
    import paper_2310_11222_amd as nvd
    dgs = [dev_graph(g) for g in graphs]
    batch = nvd.Batch(dgs)
    d, X, info = batch.distances(Ps, Qs, precision=precision, **kw)
    return d.cpu().numpy(), X, info, dgs


SOLVERS = [pytest.param(False, id="sweep"), pytest.param(True, id="persistent")]


@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("precision,tol", [("mixed", 1e-6), ("fp64", 1e-8)])
def test_small_batch_matches_oracle(precision, tol, persistent):
    sizes = [300, 1200, 3500, 800, 2000, 450, 3000, 900, 1500, 600]
    ks = [8] * len(sizes)
    graphs, Ps, Qs = _mk_batch(1, sizes, ks)
    say("batch small", precision, "persistent" if persistent else "sweep")
    d, X, info, _ = _run(graphs, Ps, Qs, precision, rtol=1e-10 if precision == "fp64" else 1e-8,
                         return_x=True, persistent=persistent)
    off = 0
    xoff = 0
    for g, P, Q in zip(graphs, Ps, Qs):
        ref = _oracle(g, P, Q)
        e = rel_err(d[off:off + P.shape[1]], ref)
        assert e.max() <= tol, (g.n, e)
        xr = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["x"]
        xg = X[xoff:xoff + g.n * P.shape[1]].cpu().numpy().reshape(g.n, -1)
        np.testing.assert_allclose(xg, xr, rtol=1e-4, atol=1e-6 * np.abs(xr).max())
        off += P.shape[1]
        xoff += g.n * P.shape[1]
    assert all(i["status"] == 0 for i in info)


@pytest.mark.parametrize("persistent", SOLVERS)
def test_uneven_k_and_equivalence_with_single_solves(persistent):
    sizes = [700, 1600, 400, 2500, 1000]
    ks = [1, 8, 3, 5, 2]
    graphs, Ps, Qs = _mk_batch(2, sizes, ks)
    say("batch uneven k", "persistent" if persistent else "sweep")
    d, _, info, dgs = _run(graphs, Ps, Qs, "mixed", rtol=1e-8, persistent=persistent)
    off = 0
    for dg, g, P, Q in zip(dgs, graphs, Ps, Qs):
        single, _, _ = dg.distances(P, Q, precision="mixed", rtol=1e-8)
        single = single.cpu().numpy()
        ref = _oracle(g, P, Q)
        assert rel_err(d[off:off + P.shape[1]], single).max() <= 2e-6
        assert rel_err(d[off:off + P.shape[1]], ref).max() <= 1e-6
        off += P.shape[1]


@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("precision,tol", [("mixed", 1e-6), ("fp64", 1e-8)])
def test_team_path_large_graph_among_small(precision, tol, persistent):
    """One graph far above a block's share of the work: in the persistent
    solver it gets a multi-block team (barriers, coherent shared vectors) and
    the rest go to the pool; in the sweep it is just more chunks."""
    sizes = [60000] + [400] * 30
    ks = [8] * len(sizes)
    graphs, Ps, Qs = _mk_batch(3, sizes, ks)
    say("batch team", precision, "persistent" if persistent else "sweep")
    d, _, info, _ = _run(graphs, Ps, Qs, precision, rtol=1e-10 if precision == "fp64" else 1e-8,
                         persistent=persistent)
    ref0 = oracle.ge_pcg(graphs[0].n, graphs[0].row_ptr, graphs[0].col_idx, graphs[0].w,
                         Ps[0], Qs[0])["d"]
    assert rel_err(d[:8], ref0).max() <= tol
    off = 8
    for g, P, Q in zip(graphs[1:], Ps[1:], Qs[1:]):
        assert rel_err(d[off:off + 8], _oracle(g, P, Q)).max() <= tol
        off += 8


@pytest.mark.parametrize("persistent", SOLVERS)
def test_workload_shape_reduced_scale(persistent):
    """The 512-graph workload's recipe at 1/10 of the node counts, 64 graphs."""
    w = workload(3, scale=0.1, num_graphs=64)
    say("batch c3 reduced", sum(g.n for g in w.graphs), "persistent" if persistent else "sweep")
    d, _, info, _ = _run(w.graphs, w.P, w.Q, "mixed", rtol=1e-8, persistent=persistent)
    off = 0
    worst = 0.0
    for g, P, Q in zip(w.graphs, w.P, w.Q):
        worst = max(worst, rel_err(d[off:off + 8], _oracle(g, P, Q)).max())
        off += 8
    assert worst <= 1e-6, worst


def test_batch_rejects_disconnected_graph():
    import paper_2310_11222_amd as nvd
    g1 = barabasi_albert(200, 2, np.random.default_rng(4))
    g2 = Graph(10, np.array([0, 5]), np.array([1, 6]))
    say("batch reject")
    with pytest.raises(nvd.NvdError) as ei:
        nvd.Batch([dev_graph(g1), dev_graph(g2)])
    assert ei.value.status == 8


def test_graph_capture_replays_match_eager():
    """The persistent launch is captured once and replayed; every replay (with
    the program's own eager GPU work and synchronisations in between) must
    reproduce the direct-launch result bit for bit."""
    import os
    import torch
    import paper_2310_11222_amd as nvd
    sizes = [900, 2500, 400, 1800, 60000]
    ks = [8, 8, 4, 8, 8]
    graphs, Ps, Qs = _mk_batch(6, sizes, ks)
    say("batch graph replay")
    dgs = [dev_graph(g) for g in graphs]
    batch = nvd.Batch(dgs)
    packed = batch.pack(Ps, Qs)
    K = int(sum(ks))
    os.environ["NVD_BATCH_GRAPH"] = "0"
    try:
        # the first call measures per-graph iteration counts, which set the
        # work plan (team sizes, hence summation order) of the calls after it
        batch.distances(None, None, packed=packed, persistent=True)
        eager = batch.distances(None, None, packed=packed, persistent=True)[0].cpu().numpy()
    finally:
        del os.environ["NVD_BATCH_GRAPH"]
    out = torch.empty(K, dtype=torch.float64, device="cuda")
    for rep in range(4):
        out.fill_(-1.0)
        d = batch.distances(None, None, packed=packed, out=out, persistent=True)[0].cpu().numpy()
        assert np.array_equal(d, eager), (rep, np.abs(d - eager).max())
        # unrelated eager work between replays
        dgs[1].distances(Ps[1], Qs[1], precision="fp64")
        torch.cuda.synchronize()
    q = batch.query()
    print("[batch-graph]", q, flush=True)
    assert q["eager"] == 2
    assert q["captures"] == 1 and q["replays"] == 3, q


def test_sweep_captured_chunks_match_eager():
    """The sweep solver's inner iterations run as captured chunks of 8
    (apply, update, direction) replayed from a hipGraph; with the program's
    own eager work and synchronisations between calls, every call must
    reproduce the direct-launch result bit for bit."""
    import os
    import torch
    import paper_2310_11222_amd as nvd
    sizes = [900, 2500, 400, 1800, 30000]
    ks = [8, 8, 4, 8, 8]
    graphs, Ps, Qs = _mk_batch(7, sizes, ks)
    say("sweep graph replay")
    dgs = [dev_graph(g) for g in graphs]
    batch = nvd.Batch(dgs)
    packed = batch.pack(Ps, Qs)
    K = int(sum(ks))
    os.environ["NVD_BATCH_GRAPH"] = "0"
    try:
        batch.distances(None, None, packed=packed)
        eager = batch.distances(None, None, packed=packed)[0].cpu().numpy()
    finally:
        del os.environ["NVD_BATCH_GRAPH"]
    q0 = batch.query()
    out = torch.empty(K, dtype=torch.float64, device="cuda")
    for rep in range(4):
        out.fill_(-1.0)
        d = batch.distances(None, None, packed=packed, out=out)[0].cpu().numpy()
        assert np.array_equal(d, eager), (rep, np.abs(d - eager).max())
        dgs[1].distances(Ps[1], Qs[1], precision="fp64")
        torch.cuda.synchronize()
    q = batch.query()
    print("[sweep-graph]", q0, q, flush=True)
    assert q["captures"] - q0["captures"] >= 1 and q["replays"] - q0["replays"] >= 4, (q0, q)
    ref = [_oracle(g, P, Q) for g, P, Q in zip(graphs, Ps, Qs)]
    assert rel_err(eager, np.concatenate(ref)).max() <= 1e-6
    batch.close()


def test_sweep_repeatable_and_close_to_persistent():
    """The sweep sums every graph's chunk partials in chunk order: two calls
    agree bit for bit; it agrees with the persistent solver to the mixed
    tolerance and with the oracle, and returns mean-zero x per graph.  The
    40000-node BA graph has hubs above 128 neighbours (chunks of one row
    applied by a whole block)."""
    sizes = [5000, 300, 12000, 800, 2500, 40000, 1000]
    ks = [8, 4, 8, 1, 8, 8, 2]
    graphs, Ps, Qs = _mk_batch(7, sizes, ks)
    assert np.diff(graphs[5].row_ptr).max() > 128
    import paper_2310_11222_amd as nvd
    say("batch sweep repeat")
    batch = nvd.Batch([dev_graph(g) for g in graphs])
    packed = batch.pack(Ps, Qs)
    d1, X1, _ = batch.distances(None, None, packed=packed, return_x=True)
    d2, X2, _ = batch.distances(None, None, packed=packed, return_x=True)
    assert np.array_equal(d1.cpu().numpy(), d2.cpu().numpy())
    assert np.array_equal(X1.cpu().numpy(), X2.cpu().numpy())
    dp, _, _ = batch.distances(None, None, packed=packed, persistent=True)
    assert rel_err(d1.cpu().numpy(), dp.cpu().numpy()).max() <= 2e-6
    off = 0
    for g, P, Q in zip(graphs, Ps, Qs):
        k = P.shape[1]
        assert rel_err(d1.cpu().numpy()[off:off + k], _oracle(g, P, Q)).max() <= 1e-6
        off += k
    X = X1.cpu().numpy()
    off = 0
    for g, k in zip(graphs, ks):
        xg = X[off:off + g.n * k].reshape(g.n, k)
        assert np.abs(xg.sum(axis=0)).max() <= 1e-9 * np.abs(xg).sum()
        off += g.n * k


@pytest.mark.parametrize("persistent", SOLVERS)
@pytest.mark.parametrize("k,precision", [(1, "mixed"), (2, "fp64"), (3, "mixed"), (16, "fp64"),
                                         (33, "mixed"), (64, "mixed")])
def test_tiles_across_widths(k, precision, persistent):
    """Every tile width the batched solvers instantiate (T = 1, 2, 4, 16, 64:
    scalar, 8-byte and 16-byte row accesses), unweighted and weighted graphs
    mixed, against the dense oracle."""
    sizes = [900, 2100, 350, 1600]
    graphs, Ps, Qs = _mk_batch(11 + k, sizes, [k] * len(sizes), weighted=(k % 2 == 1))
    say("batch tiles", k, precision, "persistent" if persistent else "sweep")
    tol = 1e-8 if precision == "fp64" else 1e-6
    d, _, info, _ = _run(graphs, Ps, Qs, precision, rtol=1e-10 if precision == "fp64" else 1e-8,
                         persistent=persistent)
    off = 0
    for g, P, Q in zip(graphs, Ps, Qs):
        ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
        assert rel_err(d[off:off + k], ref).max() <= tol, (g.n, k)
        off += k
    assert all(i["status"] == 0 for i in info)


def test_persistent_barrier_failure_is_reported(monkeypatch):
    """A team barrier that gives up (forced from the host: a spin limit of 0
    makes the first barrier of a multi-block team fail at once) ends every
    loop of the launch, which then exits normally; the call reports
    NVD_E_DEVICE.  The next call, with the default limit, is correct again."""
    import paper_2310_11222_amd as nvd
    sizes = [60000] + [400] * 6
    ks = [8] * len(sizes)
    graphs, Ps, Qs = _mk_batch(31, sizes, ks)
    dgs = [dev_graph(g) for g in graphs]
    batch = nvd.Batch(dgs)
    say("batch barrier failure")
    monkeypatch.setenv("NVD_BATCH_SPIN_LIMIT", "0")
    with pytest.raises(nvd.NvdError) as ei:
        batch.distances(Ps, Qs, precision="mixed", rtol=1e-8, persistent=True)
    assert ei.value.status == 6          # NVD_E_DEVICE
    monkeypatch.delenv("NVD_BATCH_SPIN_LIMIT")
    say("batch after barrier failure")
    d, _, info = batch.distances(Ps, Qs, precision="mixed", rtol=1e-8, persistent=True)
    d = d.cpu().numpy()
    ref0 = oracle.ge_pcg(graphs[0].n, graphs[0].row_ptr, graphs[0].col_idx, graphs[0].w,
                         Ps[0], Qs[0])["d"]
    assert rel_err(d[:8], ref0).max() <= 1e-6
    assert all(i["status"] == 0 for i in info)
    batch.close()
    for dg in dgs:
        dg.close()
