"""nvd_distances_noalloc (the solve over the library's fixed per-GPU scratch
array, for callers that cannot allocate) against nvd_distances on the same
inputs and tile: two calls in a row, the second on a smaller input, both
precisions, a disconnected graph, and the size limit.  Bar: FP64 <= 1e-8 and
mixed <= 1e-6 relative error per distance against both nvd_distances and
the oracle."""
import numpy as np
import pytest

import oracle
from nvdgen import barabasi_albert, watts_strogatz, path_graph, Graph

from gpu_helpers import say, dev_graph, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-8, "mixed": 1e-6}


def _pairs(n, k, rng):
    P = np.where(rng.random((n, k)) < 0.1, rng.random((n, k)), 0.0)
    Q = np.where(rng.random((n, k)) < 0.1, rng.random((n, k)), 0.0)
    return P, Q


def _compare(dg, P, Q, precision, tile, ref):
    rtol = 1e-10 if precision == "fp64" else 1e-8
    d0, X0, i0 = dg.distances(P, Q, precision=precision, rtol=rtol, tile_k=tile, return_x=True)
    d1, X1, i1 = dg.distances(P, Q, precision=precision, rtol=rtol, tile_k=tile, return_x=True,
                              noalloc=True)
    d0, d1 = d0.cpu().numpy(), d1.cpu().numpy()
    tol = TOL[precision]
    assert rel_err(d1, d0).max() <= tol, rel_err(d1, d0).max()
    assert rel_err(d1, ref).max() <= tol, rel_err(d1, ref).max()
    assert all(i["status"] == 0 for i in i1)
    np.testing.assert_allclose(X1.cpu().numpy(), X0.cpu().numpy(), rtol=1e-6,
                               atol=1e-8 * np.abs(X0.cpu().numpy()).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_distances_two_calls(precision):
    rng = np.random.default_rng(91)
    gA = barabasi_albert(2500, 3, rng)
    gA = gA.with_weights(rng.uniform(0.5, 2.0, gA.num_edges))
    PA, QA = _pairs(gA.n, 8, rng)
    gB = barabasi_albert(700, 2, rng)
    PB, QB = _pairs(gB.n, 3, rng)
    refA = oracle.ge_dense(gA.n, gA.row_ptr, gA.col_idx, gA.w, PA, QA)["d"]
    refB = oracle.ge_dense(gB.n, gB.row_ptr, gB.col_idx, gB.w, PB, QB)["d"]
    say("noalloc call 1", precision, gA.n, 8)
    _compare(dev_graph(gA), PA, QA, precision, 8, refA)
    say("noalloc call 2 (smaller)", precision, gB.n, 3)
    _compare(dev_graph(gB), PB, QB, precision, 0, refB)


def test_noalloc_disconnected_and_tiles():
    """Two components plus isolated nodes (per-component means carved from
    the scratch array) and k = 13 pairs in tiles 8, 4, 1."""
    rng = np.random.default_rng(92)
    a = barabasi_albert(900, 3, rng)
    b = watts_strogatz(400, 6, 0.1, rng)
    n = a.n + b.n + 3
    g = Graph(n, np.concatenate([a.eu, b.eu + a.n]), np.concatenate([a.ev, b.ev + a.n]))
    P, Q = rng.random((n, 13)), rng.random((n, 13))
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, None, P, Q)["d"]
    say("noalloc disconnected", n)
    dg = dev_graph(g)
    for precision in ("fp64", "mixed"):
        _compare(dg, P, Q, precision, 8, ref)


def test_noalloc_rejects_beyond_limit_and_tree():
    import paper_2310_11222_amd as nvd
    g = path_graph(1_300_000)
    P = np.zeros((g.n, 1))
    Q = np.zeros((g.n, 1))
    P[0, 0] = 1.0
    Q[-1, 0] = 1.0
    say("noalloc limits")
    dg = dev_graph(g)
    with pytest.raises(nvd.NvdError) as ei:
        dg.distances(P, Q, precision="mixed", noalloc=True)
    assert ei.value.status == 8           # NVD_E_UNSUPPORTED
    assert "MiB" in str(ei.value)
    small = path_graph(50)
    dgs = dev_graph(small)
    Ps = np.zeros((50, 1)); Qs = np.zeros((50, 1))
    Ps[0, 0] = 1.0; Qs[-1, 0] = 1.0
    with pytest.raises(nvd.NvdError) as ei:
        dgs.distances(Ps, Qs, precision="fp64", precond="tree", noalloc=True)
    assert ei.value.status == 8
    d, _, _ = dgs.distances(Ps, Qs, precision="fp64", noalloc=True)
    assert abs(d.cpu().numpy()[0] ** 2 - 49.0) <= 1e-8 * 49.0
