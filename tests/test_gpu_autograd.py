"""GPU checks of the hand-written adjoint behind DistanceSq:
torch.autograd.gradcheck on tiny graphs, the dense oracle's gradient,
the exact rank-one (Sherman-Morrison) update, and central finite
differences on 100 random edges of the 2e5-node lognormal BA workload."""
import json
import os

import numpy as np
import pytest

import oracle
from nvdgen import barabasi_albert, workload

from gpu_helpers import say, rel_err

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _setup(g):
    import torch
    import paper_2310_11222_amd as nvd
    dg = nvd.Graph(g.row_ptr, g.col_idx, g.w)
    idx = torch.as_tensor(g.csr_edge, device="cuda")
    return dg, idx


def test_gradcheck_tiny():
    import torch
    import paper_2310_11222_amd as nvd
    rng = np.random.default_rng(0)
    g = barabasi_albert(24, 2, rng)
    ew = rng.uniform(0.5, 2.0, g.num_edges)
    g = g.with_weights(ew)
    dg, idx = _setup(g)
    say("gradcheck")
    P = torch.tensor(rng.random((g.n, 2)), device="cuda", requires_grad=True)
    Q = torch.tensor(rng.random((g.n, 2)), device="cuda", requires_grad=True)
    W = torch.tensor(ew, device="cuda", requires_grad=True)

    def f(P, Q, W):
        return nvd.distance_sq(P, Q, dg, W[idx], precision="fp64", rtol=1e-14, max_iter=5000)

    assert torch.autograd.gradcheck(f, (P, Q, W), eps=1e-6, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gradient_matches_dense_oracle(precision):
    import torch
    import paper_2310_11222_amd as nvd
    rng = np.random.default_rng(1)
    g = barabasi_albert(2000, 3, rng)
    ew = rng.lognormal(0, 1, g.num_edges)
    g = g.with_weights(ew)
    P = np.where(rng.random((g.n, 4)) < 0.1, rng.random((g.n, 4)), 0.0)
    Q = np.where(rng.random((g.n, 4)) < 0.1, rng.random((g.n, 4)), 0.0)
    gs = rng.standard_normal(4)
    say("grad vs dense", precision)
    ref = oracle.grad_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q, gscale=gs)
    ref_ge = np.zeros(g.num_edges)
    np.add.at(ref_ge, g.csr_edge, ref["grad_w_csr"])
    dg, idx = _setup(g)
    Pt = torch.tensor(P, device="cuda", requires_grad=True)
    Qt = torch.tensor(Q, device="cuda", requires_grad=True)
    Wt = torch.tensor(ew, device="cuda", requires_grad=True)
    dsq = nvd.distance_sq(Pt, Qt, dg, Wt[idx], precision=precision, rtol=1e-12 if precision == "fp64" else 1e-10)
    (dsq * torch.tensor(gs, device="cuda")).sum().backward()
    tol = 1e-7 if precision == "fp64" else 1e-5
    np.testing.assert_allclose(dsq.detach().cpu().numpy(), ref["dsq"], rtol=tol)
    np.testing.assert_allclose(Pt.grad.cpu().numpy(), ref["grad_p"], rtol=tol, atol=tol * np.abs(ref["grad_p"]).max())
    np.testing.assert_allclose(Qt.grad.cpu().numpy(), ref["grad_q"], rtol=tol, atol=tol * np.abs(ref["grad_q"]).max())
    np.testing.assert_allclose(Wt.grad.cpu().numpy(), ref_ge, rtol=tol, atol=tol * np.abs(ref_ge).max())


def test_sherman_morrison_on_gpu():
    """d^2(w_e + t) = d^2 - t g^2 / (1 + t R_e): exact, from GPU solves only."""
    import torch
    rng = np.random.default_rng(2)
    g = barabasi_albert(3000, 3, rng)
    ew = rng.uniform(0.5, 2.0, g.num_edges)
    g = g.with_weights(ew)
    dg, idx = _setup(g)
    P = rng.random((g.n, 1))
    Q = rng.random((g.n, 1))
    say("sherman-morrison gpu")
    d, X, _ = dg.distances(P, Q, precision="fp64", rtol=1e-13, return_x=True)
    base = float(d.cpu().numpy()[0]) ** 2
    X = X.cpu().numpy()
    for e in [5, 100, 2000]:
        i, j = g.eu[e], g.ev[e]
        U = np.zeros((g.n, 1)); V = np.zeros((g.n, 1))
        U[i] = 1.0; V[j] = 1.0
        Re = float(dg.distances(U, V, precision="fp64", rtol=1e-13)[0].cpu().numpy()[0]) ** 2
        t = 0.7
        w2 = ew.copy()
        w2[e] += t
        dg.set_weights(torch.tensor(w2[g.csr_edge], device="cuda"))
        got = float(dg.distances(P, Q, precision="fp64", rtol=1e-13)[0].cpu().numpy()[0]) ** 2
        dg.set_weights(torch.tensor(ew[g.csr_edge], device="cuda"))
        gij = X[i, 0] - X[j, 0]
        want = base - t * gij ** 2 / (1 + t * Re)
        assert abs(got - want) <= 1e-9 * base, (got, want)


def test_set_weights_rejects_asymmetric_and_nonpositive():
    import torch
    import paper_2310_11222_amd as nvd
    g = barabasi_albert(100, 2, np.random.default_rng(3))
    dg = nvd.Graph(g.row_ptr, g.col_idx)
    say("set_weights errors")
    w = torch.ones(g.nnz, dtype=torch.float64, device="cuda")
    w[0] = 2.0                                   # mirror keeps 1.0
    with pytest.raises(nvd.NvdError):
        dg.set_weights(w)
    w = torch.ones(g.nnz, dtype=torch.float64, device="cuda")
    w[g.csr_edge == 0] = -1.0
    with pytest.raises(nvd.NvdError):
        dg.set_weights(w)


def test_full_size_loss_gradient_finite_differences():
    """BA n=2e5, m=5, lognormal weights, 32 pairs; loss = sum of d^2.
    Forward distances against the stored oracle values; adjoint edge
    gradients against central differences on 100 random edges."""
    import torch
    import paper_2310_11222_amd as nvd
    w = workload(4)
    g = w.graphs[0]
    # per-edge weights: recover them from the CSR (both entries equal)
    ew = np.zeros(g.num_edges)
    ew[g.csr_edge] = g.w
    say("full-size FD", g.n, g.nnz)
    dg, idx = _setup(g)
    Pt = torch.tensor(w.P[0], device="cuda", requires_grad=True)
    Qt = torch.tensor(w.Q[0], device="cuda", requires_grad=True)
    Wt = torch.tensor(ew, device="cuda", requires_grad=True)
    opts = dict(precision="fp64", rtol=1e-11)
    dsq = nvd.distance_sq(Pt, Qt, dg, Wt[idx], **opts)
    loss = dsq.sum()
    loss.backward()
    gw = Wt.grad.cpu().numpy()
    golden = os.path.join(HERE, "golden", "c4_expected.json")
    if os.path.exists(golden):
        ref = np.array([float(v) for v in json.load(open(golden))["d"]])
        got = np.sqrt(dsq.detach().cpu().numpy())
        assert rel_err(got, ref).max() <= 1e-8
    L0 = float(loss.detach())
    rng = np.random.default_rng(44)
    edges = rng.choice(g.num_edges, 100, replace=False)
    bad = []
    for e in edges:
        h = 1e-3 * ew[e]
        vals = []
        for sgn in (1.0, -1.0):
            w2 = ew.copy()
            w2[e] += sgn * h
            dg.set_weights(torch.tensor(w2[g.csr_edge], device="cuda"))
            d, _, _ = dg.distances(Pt.detach(), Qt.detach(), **opts)
            vals.append(float((d * d).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        if abs(gw[e] - fd) > 1e-5 * abs(gw[e]) + 1e-10 * L0 / ew[e]:
            bad.append((int(e), gw[e], fd))
    dg.set_weights(torch.tensor(ew[g.csr_edge], device="cuda"))
    assert not bad, bad[:5]
