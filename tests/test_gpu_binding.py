"""GPU checks of the boundary: graphs given with unsorted rows (the map back
to input order used by set_weights and grad_weights), weights rejected
without side effects, graphs built from device arrays, the vector adjoint
and the distance (not squared) adjoint, and the binding's refusal of
mis-shaped or misplaced buffers before anything reaches the library."""
import numpy as np
import pytest

import oracle
from nvdgen import barabasi_albert

from gpu_helpers import say, dev_graph, to_dev, rel_err

pytestmark = pytest.mark.gpu


def _shuffled_rows(g, rng):
    """The same CSR with the entries of every row in a random order; returns
    (col_idx, w, perm) with perm[k] = position in g's (sorted) CSR of the
    shuffled entry k."""
    perm = np.arange(g.nnz)
    for i in range(g.n):
        a, b = g.row_ptr[i], g.row_ptr[i + 1]
        perm[a:b] = a + rng.permutation(b - a)
    return g.col_idx[perm], (None if g.w is None else g.w[perm]), perm


def test_unsorted_rows_grad_and_set_weights():
    import torch
    import paper_2310_11222_amd as nvd
    rng = np.random.default_rng(61)
    g = barabasi_albert(1500, 3, rng)
    ew = rng.lognormal(0, 1, g.num_edges)
    g = g.with_weights(ew)
    ci_s, w_s, perm = _shuffled_rows(g, rng)
    P, Q = rng.random((g.n, 3)), rng.random((g.n, 3))
    gs = torch.as_tensor(rng.standard_normal(3), device="cuda")
    say("unsorted rows: grad_weights")
    dg_sorted = dev_graph(g)
    dg_shuf = nvd.Graph(g.row_ptr, ci_s, w_s)
    d0, X0, _ = dg_sorted.distances(P, Q, precision="fp64", rtol=1e-12, return_x=True)
    d1, X1, _ = dg_shuf.distances(P, Q, precision="fp64", rtol=1e-12, return_x=True)
    assert rel_err(d1.cpu().numpy(), d0.cpu().numpy()).max() <= 1e-12
    gw0 = dg_sorted.grad_weights(X0, gs).cpu().numpy()
    gw1 = dg_shuf.grad_weights(X0, gs).cpu().numpy()
    # entry k of the shuffled input is entry perm[k] of the sorted CSR
    np.testing.assert_array_equal(gw1, gw0[perm])
    # new weights, given in the shuffled input order
    ew2 = rng.uniform(0.5, 3.0, g.num_edges)
    w2_sorted = ew2[g.csr_edge]
    say("unsorted rows: set_weights")
    dg_shuf.set_weights(torch.as_tensor(w2_sorted[perm], device="cuda"))
    d2, _, _ = dg_shuf.distances(P, Q, precision="fp64", rtol=1e-12)
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, w2_sorted, P, Q)["d"]
    assert rel_err(d2.cpu().numpy(), ref).max() <= 1e-8


def test_rejected_weights_leave_graph_unchanged():
    import torch
    import paper_2310_11222_amd as nvd
    rng = np.random.default_rng(62)
    g = barabasi_albert(800, 3, rng)
    ew = rng.uniform(0.5, 2.0, g.num_edges)
    g = g.with_weights(ew)
    P, Q = rng.random((g.n, 2)), rng.random((g.n, 2))
    say("rejected weights")
    dg = dev_graph(g)
    bad = torch.as_tensor(ew[g.csr_edge], device="cuda").clone()
    bad[3] = -1.0
    with pytest.raises(nvd.NvdError):
        dg.set_weights(bad)
    bad = torch.as_tensor(ew[g.csr_edge], device="cuda").clone()
    bad[3] *= 2.0                                  # mirror differs
    with pytest.raises(nvd.NvdError):
        dg.set_weights(bad)
    d, _, _ = dg.distances(P, Q, precision="fp64")
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    assert rel_err(d.cpu().numpy(), ref).max() <= 1e-8
    # a unit-weight graph stays unit-weight after a rejected call
    dgu = nvd.Graph(g.row_ptr, g.col_idx, None)
    ones = torch.ones(g.nnz, dtype=torch.float64, device="cuda")
    ones[0] = float("nan")
    with pytest.raises(nvd.NvdError):
        dgu.set_weights(ones)
    assert dgu.stats()["weighted"] == 0
    d, _, _ = dgu.distances(P, Q, precision="fp64")
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, None, P, Q)["d"]
    assert rel_err(d.cpu().numpy(), ref).max() <= 1e-8


def test_graph_from_device_arrays():
    import torch
    import paper_2310_11222_amd as nvd
    rng = np.random.default_rng(63)
    g = barabasi_albert(1200, 3, rng)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    P, Q = rng.random((g.n, 4)), rng.random((g.n, 4))
    say("graph from device arrays")
    dg = nvd.Graph(torch.as_tensor(g.row_ptr, device="cuda"),
                   torch.as_tensor(g.col_idx, device="cuda"),
                   torch.as_tensor(g.w, device="cuda"))
    st = dg.stats()
    assert st["n"] == g.n and st["nnz"] == g.nnz and st["weighted"] == 1
    d, _, _ = dg.distances(P, Q, precision="fp64")
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    assert rel_err(d.cpu().numpy(), ref).max() <= 1e-8
    # an invalid device CSR is rejected like a host one
    ci = torch.as_tensor(g.col_idx, device="cuda").clone()
    ci[0] = g.n + 5
    with pytest.raises(nvd.NvdError):
        nvd.Graph(torch.as_tensor(g.row_ptr, device="cuda"), ci, None)


def test_dsq_output_and_vector_adjoint():
    import torch
    rng = np.random.default_rng(64)
    g = barabasi_albert(900, 3, rng)
    g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    P = np.where(rng.random((g.n, 5)) < 0.2, rng.random((g.n, 5)), 0.0)
    Q = np.where(rng.random((g.n, 5)) < 0.2, rng.random((g.n, 5)), 0.0)
    Q[:, 4] = P[:, 4]                              # d = 0
    gs = rng.standard_normal(5)
    say("dsq output, vector adjoint")
    dg = dev_graph(g)
    ref = oracle.grad_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q, gscale=gs)
    dsq, X, info = dg.distances(P, Q, precision="fp64", rtol=1e-12, return_x=True, out="dsq")
    dsq = dsq.cpu().numpy()
    assert rel_err(dsq[:4], ref["dsq"][:4]).max() <= 1e-8 and dsq[4] == 0.0
    assert np.array_equal(dsq, np.array([max(i["dsq"], 0.0) for i in info]))
    GP, GQ = dg.grad_vectors(X, torch.as_tensor(gs))
    np.testing.assert_array_equal(GQ.cpu().numpy(), -GP.cpu().numpy())
    np.testing.assert_allclose(GP.cpu().numpy(), ref["grad_p"], rtol=1e-7,
                               atol=1e-9 * np.abs(ref["grad_p"]).max())


def test_distance_adjoint():
    """Gradients of sum_j g_j d_j through Distance: the d^2 gradients times
    1 / (2 d_j), and zero for a pair with d = 0."""
    import torch
    import paper_2310_11222_amd as nvd
    rng = np.random.default_rng(65)
    g = barabasi_albert(700, 3, rng)
    ew = rng.uniform(0.5, 2.0, g.num_edges)
    g = g.with_weights(ew)
    P = rng.random((g.n, 3))
    Q = rng.random((g.n, 3))
    Q[:, 2] = P[:, 2] + 0.5                        # delta_bar = 0: d = 0
    gd = rng.standard_normal(3)
    say("distance adjoint")
    dg = dev_graph(g)
    idx = torch.as_tensor(g.csr_edge, device="cuda")
    Pt = torch.tensor(P, device="cuda", requires_grad=True)
    Qt = torch.tensor(Q, device="cuda", requires_grad=True)
    Wt = torch.tensor(ew, device="cuda", requires_grad=True)
    d = nvd.distance_t(Pt, Qt, dg, Wt[idx], precision="fp64", rtol=1e-12)
    (d * torch.as_tensor(gd, device="cuda")).sum().backward()
    dn = d.detach().cpu().numpy()
    assert dn[2] == 0.0
    scale = np.array([gd[0] / (2 * dn[0]), gd[1] / (2 * dn[1]), 0.0])
    ref = oracle.grad_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q, gscale=scale)
    ref_ge = np.zeros(g.num_edges)
    np.add.at(ref_ge, g.csr_edge, ref["grad_w_csr"])
    np.testing.assert_allclose(Pt.grad.cpu().numpy(), ref["grad_p"], rtol=1e-7,
                               atol=1e-9 * np.abs(ref["grad_p"]).max())
    np.testing.assert_allclose(Qt.grad.cpu().numpy(), ref["grad_q"], rtol=1e-7,
                               atol=1e-9 * np.abs(ref["grad_q"]).max())
    np.testing.assert_allclose(Wt.grad.cpu().numpy(), ref_ge, rtol=1e-7,
                               atol=1e-9 * np.abs(ref_ge).max())
    assert np.all(Pt.grad.cpu().numpy()[:, 2] == 0.0)


def test_binding_rejects_bad_buffers():
    import torch
    import paper_2310_11222_amd as nvd
    rng = np.random.default_rng(66)
    g = barabasi_albert(300, 2, rng)
    P, Q = rng.random((g.n, 4)), rng.random((g.n, 4))
    say("binding argument checks")
    dg = dev_graph(g)
    for X0 in (torch.zeros((g.n, 3), dtype=torch.float64, device="cuda"),     # wrong k
               torch.zeros((g.n - 1, 4), dtype=torch.float64, device="cuda"),  # wrong n
               torch.zeros((g.n, 4, 1), dtype=torch.float64, device="cuda")):  # 3-D
        with pytest.raises(ValueError):
            dg.distances(P, Q, X0=X0)
    # a float32 or host starting guess is converted, not passed through
    for X0 in (torch.zeros((g.n, 4), dtype=torch.float32, device="cuda"),
               np.zeros((g.n, 4))):
        d, X, _ = dg.distances(P, Q, X0=X0)
        assert X.dtype == torch.float64 and X.is_cuda and X.shape == (g.n, 4)
    X = to_dev(P)
    for out in (torch.empty((g.n, 3), dtype=torch.float64, device="cuda"),
                torch.empty((g.n, 4), dtype=torch.float32, device="cuda"),
                torch.empty((g.n, 4), dtype=torch.float64),
                torch.empty((4, g.n), dtype=torch.float64, device="cuda").t()):
        with pytest.raises(ValueError):
            dg.laplacian_apply(X, out=out)
    with pytest.raises(ValueError):
        dg.laplacian_apply(torch.as_tensor(P))       # host tensor
    with pytest.raises(ValueError):
        dg.grad_weights(X, torch.ones(3, dtype=torch.float64))   # wrong number of scales
    batch = nvd.Batch([dg])
    packed = batch.pack([P], [Q])
    for out in (torch.empty(3, dtype=torch.float64, device="cuda"),
                torch.empty(4, dtype=torch.float64),
                torch.empty(4, dtype=torch.float32, device="cuda")):
        with pytest.raises(ValueError):
            batch.distances(None, None, packed=packed, out=out)
    batch.close()
