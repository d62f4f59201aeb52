"""GPU parity of the approximate-Cholesky preconditioner (sparse approximate
Gaussian elimination with sampled cliques, section 3.2 / Table 2's solver)
against the CPU oracle: trees and cycles (where every elimination is exact,
so PCG converges at once), the density-sweep graphs, a weighted disconnected
graph, a 2e5-node BA graph, both precisions and several tiles.  The
preconditioner changes the iterations, never the answer: FP64 <= 1e-8 and
mixed <= 1e-6 relative error per distance."""
import numpy as np
import pytest

import oracle
from nvdgen import (barabasi_albert, watts_strogatz, random_tree, cycle_graph, path_graph,
                    density_graph, DENSITY_MODELS, Graph)

from gpu_helpers import say, dev_graph, rel_err

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-8, "mixed": 1e-6}


def _run(g, P, Q, precision, ref, **kw):
    dg = dev_graph(g)
    d, X, info = dg.distances(P, Q, precision=precision, precond="achol",
                              rtol=1e-10 if precision == "fp64" else 1e-8, return_x=True, **kw)
    e = rel_err(d.cpu().numpy(), ref)
    assert e.max() <= TOL[precision], (e.max(), info[:2])
    assert all(i["status"] == 0 for i in info), info
    return dg, X, info


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trees_and_cycles_exact_factor(precision):
    """Leaves and degree-2 vertices are eliminated exactly: a tree or a cycle
    gets an exact factor, and PCG stops after a few iterations."""
    rng = np.random.default_rng(101)
    for g in (random_tree(3000, rng), path_graph(5000), cycle_graph(4001)):
        g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
        P = np.where(rng.random((g.n, 4)) < 0.1, rng.random((g.n, 4)), 0.0)
        Q = np.where(rng.random((g.n, 4)) < 0.1, rng.random((g.n, 4)), 0.0)
        say("achol tree/cycle", precision, g.n)
        ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
        dg, _, info = _run(g, P, Q, precision, ref)
        st = dg.stats()
        assert st["achol_remainder"] == 0 and st["achol_rounds"] > 0
        assert max(i["iters"] for i in info) <= (3 if precision == "fp64" else 8), info


@pytest.mark.parametrize("model", DENSITY_MODELS)
@pytest.mark.parametrize("deg", [1, 4, 16])
def test_density_graphs(model, deg):
    g, P, Q = density_graph(model, deg, n=2000)
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    for precision in ("fp64", "mixed"):
        say("achol density", model, deg, precision)
        _run(g, P, Q, precision, ref)


@pytest.mark.parametrize("tile", [1, 4, 16])
def test_weighted_disconnected(tile):
    rng = np.random.default_rng(102)
    a = barabasi_albert(1500, 3, rng)
    b = watts_strogatz(900, 6, 0.1, rng)
    n = a.n + b.n + 4                                   # plus isolated nodes
    g = Graph(n, np.concatenate([a.eu, b.eu + a.n]), np.concatenate([a.ev, b.ev + a.n]))
    g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    P, Q = rng.random((n, 16)), rng.random((n, 16))
    say("achol disconnected", tile)
    ref = oracle.ge_dense(n, g.row_ptr, g.col_idx, g.w, P, Q)
    for precision in ("fp64", "mixed"):
        _, X, _ = _run(g, P, Q, precision, ref["d"], tile_k=tile)
        if precision == "fp64":
            np.testing.assert_allclose(X.cpu().numpy(), ref["x"], rtol=1e-6,
                                       atol=1e-8 * np.abs(ref["x"]).max())


def test_large_ba_matches_jacobi_and_oracle():
    rng = np.random.default_rng(103)
    g = barabasi_albert(200_000, 3, rng)
    P = np.where(rng.random((g.n, 8)) < 0.05, rng.random((g.n, 8)), 0.0)
    Q = np.where(rng.random((g.n, 8)) < 0.05, rng.random((g.n, 8)), 0.0)
    say("achol BA 2e5")
    ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    for precision in ("fp64", "mixed"):
        dg, _, info = _run(g, P, Q, precision, ref)
        dj, _, infoj = dg.distances(P, Q, precision=precision, rtol=1e-8)
        assert rel_err(dj.cpu().numpy(), ref).max() <= TOL[precision]
    st = dg.stats()
    assert st["achol_factor_nnz"] > 0


def test_reweighting_rebuilds_factor():
    import torch
    rng = np.random.default_rng(104)
    g = barabasi_albert(2000, 3, rng)
    ew = rng.uniform(0.5, 2.0, g.num_edges)
    g = g.with_weights(ew)
    P, Q = rng.random((g.n, 4)), rng.random((g.n, 4))
    say("achol reweight")
    dg = dev_graph(g)
    dg.distances(P, Q, precision="fp64", precond="achol")
    ew2 = rng.lognormal(0, 1, g.num_edges)
    dg.set_weights(torch.as_tensor(ew2[g.csr_edge], device="cuda"))
    d, _, info = dg.distances(P, Q, precision="fp64", precond="achol")
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, ew2[g.csr_edge], P, Q)["d"]
    assert rel_err(d.cpu().numpy(), ref).max() <= 1e-8


def test_batches_reject_achol():
    import ctypes as C
    import torch
    import paper_2310_11222_amd as nvd
    g = barabasi_albert(300, 2, np.random.default_rng(105))
    dg = dev_graph(g)
    b = nvd.Batch([dg])
    P = np.random.default_rng(0).random((g.n, 2))
    ks, Pf, Qf = b.pack([P], [P[::-1].copy()])
    d = torch.empty(2, dtype=torch.float64, device="cuda")
    o = nvd.opts("mixed", 1e-8, precond="achol")
    say("achol batch rejected")
    st = nvd.load().nvd_batch_distances(b._h, ks.ctypes.data_as(C.c_void_p), nvd._ptr(Pf),
                                        nvd._ptr(Qf), C.byref(o), nvd._ptr(d), None, None,
                                        nvd._stream())
    assert st == 8                       # NVD_E_UNSUPPORTED
    b.close()
