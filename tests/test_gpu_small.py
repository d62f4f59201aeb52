"""GPU checks of the single-launch path for small and mid-size connected
graphs (the whole solve in one block, or in one cooperative launch of
several blocks meeting at grid barriers): against the oracle and against
the multi-kernel path (NVD_SMALL=0) on the same inputs, both precisions,
unit and weighted graphs, several tiles and block counts, x, d^2,
degenerate pairs, a pair that runs out of iterations, the hand-over to FP64
forced from the host, and a barrier that gives up (forced from the host
with a spin limit of zero, so every block still exits)."""
import numpy as np
import pytest

import oracle
from nvdgen import barabasi_albert, watts_strogatz, path_graph, workload

from gpu_helpers import say, dev_graph, rel_err

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-8, "mixed": 1e-6}


def _both(monkeypatch, dg, P, Q, **kw):
    a = dg.distances(P, Q, return_x=True, **kw)
    monkeypatch.setenv("NVD_SMALL", "0")
    b = dg.distances(P, Q, return_x=True, **kw)
    monkeypatch.delenv("NVD_SMALL")
    return a, b


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("k,tile", [(1, 0), (5, 0), (16, 16), (12, 4)])
def test_small_path_matches_oracle_and_multikernel(monkeypatch, precision, weighted, k, tile):
    rng = np.random.default_rng(200 + k + (7 if weighted else 0))
    g = barabasi_albert(1500, 3, rng)
    if weighted:
        g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    P = np.where(rng.random((g.n, k)) < 0.1, rng.random((g.n, k)), 0.0)
    Q = np.where(rng.random((g.n, k)) < 0.1, rng.random((g.n, k)), 0.0)
    say("small path", precision, weighted, k, tile)
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    dg = dev_graph(g)
    rtol = 1e-10 if precision == "fp64" else 1e-8
    (d1, X1, i1), (d2, X2, i2) = _both(monkeypatch, dg, P, Q, precision=precision, rtol=rtol,
                                       tile_k=tile)
    d1, d2 = d1.cpu().numpy(), d2.cpu().numpy()
    assert rel_err(d1, ref["d"]).max() <= TOL[precision]
    assert rel_err(d1, d2).max() <= TOL[precision]
    assert all(i["status"] == 0 for i in i1)
    # same recurrences and stopping rules; sums in another order can move a
    # stopping decision by one iteration
    assert all(abs(a["iters"] - b["iters"]) <= 2 for a, b in zip(i1, i2)), (i1, i2)
    assert all(abs(a["refine_steps"] - b["refine_steps"]) <= 1 for a, b in zip(i1, i2))
    np.testing.assert_allclose(X1.cpu().numpy(), ref["x"], rtol=1e-6,
                               atol=(1e-8 if precision == "fp64" else 1e-6) * np.abs(ref["x"]).max())
    assert all(i["rel_res"] <= rtol * 1.01 for i in i1)


def test_small_path_c1_and_repeatable(monkeypatch):
    w = workload(1)
    g = w.graphs[0]
    say("small path C1")
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, w.P[0], w.Q[0])["d"]
    dg = dev_graph(g)
    for prec in ("fp64", "mixed"):
        d, _, info = dg.distances(w.P[0], w.Q[0], precision=prec, rtol=1e-10)
        d2, _, _ = dg.distances(w.P[0], w.Q[0], precision=prec, rtol=1e-10)
        assert np.array_equal(d.cpu().numpy(), d2.cpu().numpy())
        assert rel_err(d.cpu().numpy(), ref).max() <= TOL[prec]
        dsq, _, _ = dg.distances(w.P[0], w.Q[0], precision=prec, rtol=1e-10, out="dsq")
        assert dsq.cpu().numpy()[0] == max(info[0]["dsq"], 0.0)


def test_small_path_degenerate_and_noconv(monkeypatch):
    g = barabasi_albert(800, 2, np.random.default_rng(201))
    rng = np.random.default_rng(202)
    P = rng.random((g.n, 4))
    Q = P.copy()
    Q[:, 1] = P[:, 1] + 3.25          # constant shift: delta_bar = 0
    Q[:, 2] = 0.0
    say("small path degenerate")
    dg = dev_graph(g)
    for prec in ("fp64", "mixed"):
        d, _, info = dg.distances(P, Q, precision=prec)
        d = d.cpu().numpy()
        assert d[0] == 0.0 and d[1] == 0.0 and d[3] == 0.0 and info[0]["iters"] == 0
        ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, None, P[:, 2:3], Q[:, 2:3])["d"][0]
        assert abs(d[2] - ref) <= TOL[prec] * ref
    gp = path_graph(2000)
    Pp = np.zeros((gp.n, 1)); Qp = np.zeros((gp.n, 1))
    Pp[10, 0] = 1.0; Qp[1500, 0] = 1.0
    dgp = dev_graph(gp)
    (d1, _, i1), (d2, _, i2) = _both(monkeypatch, dgp, Pp, Qp, precision="fp64", max_iter=5)
    assert i1[0]["status"] == 4 and i2[0]["status"] == 4       # NVD_E_NOCONV both ways
    assert d1.cpu().numpy()[0] > 0


def test_small_path_forced_fp64_handover(monkeypatch):
    rng = np.random.default_rng(203)
    g = watts_strogatz(1200, 6, 0.1, rng)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    P, Q = rng.random((g.n, 4)), rng.random((g.n, 4))
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    say("small path forced stall")
    dg = dev_graph(g)
    monkeypatch.setenv("NVD_REFINE_STALL_RATIO2", "0")
    d, _, info = dg.distances(P, Q, precision="mixed", rtol=1e-10, inner_rtol=1e-2)
    monkeypatch.delenv("NVD_REFINE_STALL_RATIO2")
    assert rel_err(d.cpu().numpy(), ref).max() <= 1e-8
    assert all(i["flags"] & 1 and i["status"] == 0 for i in info)


# ---- several blocks (cooperative launch with grid barriers) ----------------

def _mid_case(seed, n, k, weighted, model="ba"):
    rng = np.random.default_rng(seed)
    g = barabasi_albert(n, 3, rng) if model == "ba" else watts_strogatz(n, 6, 0.1, rng)
    if weighted:
        g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    P = np.where(rng.random((g.n, k)) < 0.05, rng.random((g.n, k)), 0.0)
    Q = np.where(rng.random((g.n, k)) < 0.05, rng.random((g.n, k)), 0.0)
    return g, P, Q


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("n,k,tile,blocks", [(30000, 1, 0, None), (30000, 8, 8, None),
                                             (10000, 16, 16, "80"), (30000, 12, 4, "64"),
                                             (30000, 3, 2, "240")])
def test_mid_path_matches_oracle_and_multikernel(monkeypatch, precision, weighted, n, k, tile,
                                                 blocks):
    """n T from 3e4 to 2.4e5 elements: one element per thread on up to 128
    blocks, or two on fewer; forced block counts cover ragged last blocks
    and many nearly empty ones."""
    g, P, Q = _mid_case(300 + k, n, k, weighted)
    say("mid path", precision, weighted, n, k, tile, blocks)
    ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
    dg = dev_graph(g)
    if blocks:
        monkeypatch.setenv("NVD_MID_BLOCKS", blocks)
    rtol = 1e-10 if precision == "fp64" else 1e-8
    (d1, X1, i1), (d2, X2, i2) = _both(monkeypatch, dg, P, Q, precision=precision, rtol=rtol,
                                       tile_k=tile)
    d1, d2 = d1.cpu().numpy(), d2.cpu().numpy()
    assert rel_err(d1, ref["d"]).max() <= TOL[precision]
    assert rel_err(d1, d2).max() <= TOL[precision]
    assert all(i["status"] == 0 for i in i1), i1
    assert all(abs(a["iters"] - b["iters"]) <= 2 for a, b in zip(i1, i2)), (i1, i2)
    np.testing.assert_allclose(X1.cpu().numpy(), ref["x"], rtol=1e-6,
                               atol=(1e-8 if precision == "fp64" else 1e-6) * np.abs(ref["x"]).max())
    assert all(i["rel_res"] <= rtol * 1.01 for i in i1)


def test_mid_path_repeatable_degenerate_and_dsq(monkeypatch):
    g, P, Q = _mid_case(310, 25000, 8, True, model="ws")
    Q[:, 1] = P[:, 1] - 1.5            # constant shift: delta_bar = 0
    Q[:, 5] = P[:, 5]
    say("mid path repeat")
    ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    dg = dev_graph(g)
    for prec in ("fp64", "mixed"):
        d, X, info = dg.distances(P, Q, precision=prec, rtol=1e-10, return_x=True)
        d2, X2, _ = dg.distances(P, Q, precision=prec, rtol=1e-10, return_x=True)
        assert np.array_equal(d.cpu().numpy(), d2.cpu().numpy())
        assert np.array_equal(X.cpu().numpy(), X2.cpu().numpy())
        dn = d.cpu().numpy()
        assert dn[1] == 0.0 and dn[5] == 0.0 and info[1]["iters"] == 0
        assert rel_err(dn, ref).max() <= TOL[prec]
        dsq, _, _ = dg.distances(P, Q, precision=prec, rtol=1e-10, out="dsq")
        np.testing.assert_array_equal(dsq.cpu().numpy(), [max(i["dsq"], 0.0) for i in info])


def test_mid_path_noconv_and_forced_handover(monkeypatch):
    g, P, Q = _mid_case(320, 30000, 4, True, model="ws")
    say("mid path noconv / stall")
    ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    dg = dev_graph(g)
    (d1, _, i1), (d2, _, i2) = _both(monkeypatch, dg, P, Q, precision="fp64", max_iter=5)
    assert all(i["status"] == 4 for i in i1) and all(i["status"] == 4 for i in i2)
    monkeypatch.setenv("NVD_REFINE_STALL_RATIO2", "0")
    d, _, info = dg.distances(P, Q, precision="mixed", rtol=1e-10, inner_rtol=1e-2)
    monkeypatch.delenv("NVD_REFINE_STALL_RATIO2")
    assert rel_err(d.cpu().numpy(), ref).max() <= 1e-8
    assert all(i["flags"] & 1 and i["status"] == 0 for i in info)


def test_mid_path_barrier_failure_is_reported(monkeypatch):
    from paper_2310_11222_amd._abi import NvdError, NVD_E_DEVICE
    g, P, Q = _mid_case(330, 30000, 4, False)
    say("mid path barrier failure")
    dg = dev_graph(g)
    monkeypatch.setenv("NVD_MID_BLOCKS", "64")
    monkeypatch.setenv("NVD_MID_SPIN_LIMIT", "0")
    with pytest.raises(NvdError) as exc:
        dg.distances(P, Q, precision="mixed")
    assert exc.value.status == NVD_E_DEVICE
    monkeypatch.delenv("NVD_MID_SPIN_LIMIT")
    # the graph stays usable
    ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    d, _, info = dg.distances(P, Q, precision="mixed")
    assert rel_err(d.cpu().numpy(), ref).max() <= TOL["mixed"]
    assert all(i["status"] == 0 for i in info)
