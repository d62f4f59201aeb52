"""Pins for the oracle's gradients of d^2 (with respect to a, b and the edge
weights): finite differences of the exact dense route, the tree closed form
dR/dw_e = -1/w_e^2, and the exact rank-one (Sherman-Morrison) update."""
import numpy as np

import oracle
from oracle.grad import grad_dense, grad_from_x
from nvdgen import barabasi_albert, random_tree, Graph


def _dsq(g, w, P, Q):
    return oracle.ge_dense(g.n, g.row_ptr, g.col_idx, w, P, Q)["dsq"]


def _csr_w(g, ew):
    return np.asarray(ew)[g.csr_edge]


def test_grad_vectors_finite_difference():
    rng = np.random.default_rng(0)
    g = barabasi_albert(30, 2, rng)
    w = _csr_w(g, rng.uniform(0.5, 2.0, g.num_edges))
    P, Q = rng.random((g.n, 2)), rng.random((g.n, 2))
    r = grad_dense(g.n, g.row_ptr, g.col_idx, w, P, Q)
    h = 1e-6
    for i in [0, 5, 17, 29]:
        for j in range(2):
            Pp, Pm = P.copy(), P.copy()
            Pp[i, j] += h
            Pm[i, j] -= h
            fd = (_dsq(g, w, Pp, Q)[j] - _dsq(g, w, Pm, Q)[j]) / (2 * h)
            assert abs(fd - r["grad_p"][i, j]) < 1e-7
            Qp, Qm = Q.copy(), Q.copy()
            Qp[i, j] += h
            Qm[i, j] -= h
            fd = (_dsq(g, w, P, Qp)[j] - _dsq(g, w, P, Qm)[j]) / (2 * h)
            assert abs(fd - r["grad_q"][i, j]) < 1e-7


def test_grad_weights_finite_difference_per_edge():
    rng = np.random.default_rng(1)
    g = barabasi_albert(40, 3, rng)
    ew = rng.lognormal(0, 1, g.num_edges)
    P, Q = rng.random((g.n, 3)), rng.random((g.n, 3))
    gs = np.array([1.0, -0.5, 2.0])
    r = grad_dense(g.n, g.row_ptr, g.col_idx, _csr_w(g, ew), P, Q, gscale=gs)
    # per-edge gradient = sum of the two CSR entries
    ge = np.zeros(g.num_edges)
    np.add.at(ge, g.csr_edge, r["grad_w_csr"])
    for e in rng.choice(g.num_edges, 12, replace=False):
        h = 1e-5 * ew[e]
        wp, wm = ew.copy(), ew.copy()
        wp[e] += h
        wm[e] -= h
        fp = np.dot(gs, _dsq(g, _csr_w(g, wp), P, Q))
        fm = np.dot(gs, _dsq(g, _csr_w(g, wm), P, Q))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - ge[e]) < 1e-6 * max(1.0, abs(ge[e]))


def test_grad_tree_closed_form():
    """On a tree, R_ij = sum_{e on path} 1/w_e, so dR_ij/dw_e = -1/w_e^2 on the
    path and 0 off it."""
    rng = np.random.default_rng(2)
    n = 25
    ew = rng.uniform(0.5, 2.0, n - 1)
    g = random_tree(n, rng, ew)
    i, j = 3, 21
    P = np.zeros((n, 1)); Q = np.zeros((n, 1))
    P[i] = 1.0; Q[j] = 1.0
    r = grad_dense(g.n, g.row_ptr, g.col_idx, _csr_w(g, ew), P, Q)
    ge = np.zeros(g.num_edges)
    np.add.at(ge, g.csr_edge, r["grad_w_csr"])
    # path edges: those whose removal separates i from j
    t = oracle.ge_tree(g.n, g.row_ptr, g.col_idx, _csr_w(g, ew), P, Q)
    par = t["parent"]

    def anc(v):
        out = [v]
        while par[v] >= 0:
            v = par[v]
            out.append(v)
        return out

    ai, aj = anc(i), anc(j)
    common = set(ai) & set(aj)
    on_path = set()
    for chain in (ai, aj):
        for v in chain:
            if v in common:
                break
            on_path.add((min(v, par[v]), max(v, par[v])))
    for e in range(g.num_edges):
        key = (g.eu[e], g.ev[e])
        want = -1.0 / ew[e] ** 2 if key in on_path else 0.0
        assert abs(ge[e] - want) < 1e-10


def test_sherman_morrison_exact_weight_update():
    """d^2(w_e + t) = d^2 - t g^2 / (1 + t R_e), g = x_i - x_j, R_e the edge's
    effective resistance: exact for a rank-one change of L."""
    rng = np.random.default_rng(3)
    g = barabasi_albert(60, 2, rng)
    ew = rng.uniform(0.5, 2.0, g.num_edges)
    P, Q = rng.random((g.n, 1)), rng.random((g.n, 1))
    base = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, _csr_w(g, ew), P, Q)
    for e in [0, 7, 33]:
        i, j = g.eu[e], g.ev[e]
        gij = base["x"][i, 0] - base["x"][j, 0]
        U = np.zeros((g.n, 1)); V = np.zeros((g.n, 1))
        U[i] = 1.0; V[j] = 1.0
        Re = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, _csr_w(g, ew), U, V)["dsq"][0]
        for t in [0.3, 2.0]:
            w2 = ew.copy()
            w2[e] += t
            got = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, _csr_w(g, w2), P, Q)["dsq"][0]
            want = base["dsq"][0] - t * gij ** 2 / (1 + t * Re)
            assert abs(got - want) < 1e-12 * base["dsq"][0]


def test_grad_from_x_matches_per_edge_definition():
    """Directly: -(x_i - x_j)^2 per edge when both CSR halves are summed."""
    g = barabasi_albert(20, 2, np.random.default_rng(4))
    x = np.random.default_rng(5).random((g.n, 1))
    _, gw = grad_from_x(g.n, g.row_ptr, g.col_idx, x)
    ge = np.zeros(g.num_edges)
    np.add.at(ge, g.csr_edge, gw)
    np.testing.assert_allclose(ge, -(x[g.eu, 0] - x[g.ev, 0]) ** 2, rtol=1e-14)
