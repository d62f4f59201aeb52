"""GPU checks of the mixed-precision stagnation guard: on a long weighted
path FP32 cannot solve the refinement's inner problems (conditioning ~n^2
times FP32's unit roundoff is far above 1, and the FP32 weights differ from
the FP64 ones), so the outer residual stalls; the pairs must be handed to
the FP64 solver (info flag) and still meet the 1e-6 bound against the
closed form (effective resistance of a path: the sum of 1/w over the
edges between the two nodes).  On a well-conditioned graph the guard must
stay quiet."""
import numpy as np
import pytest

import oracle
from nvdgen import barabasi_albert, path_graph
from oracle import closed_forms as cf

from gpu_helpers import say, dev_graph, rel_err

pytestmark = pytest.mark.gpu


def test_long_weighted_path_mixed():
    """A 1e5-node path with weights uniform[1, 2) (not representable in FP32):
    conditioning ~n^2, so FP32 CG needs far more iterations than n and its
    corrections are poor; the mixed solve must still meet 1e-6 against the
    closed form, whether it finishes in FP32 refinement or hands over to
    FP64."""
    n = 100_000
    rng = np.random.default_rng(81)
    g = path_graph(n)
    ew = rng.uniform(1.0, 2.0, g.num_edges)       # edge e joins nodes e, e+1
    order = np.argsort(np.minimum(g.eu, g.ev))
    assert np.array_equal(np.minimum(g.eu, g.ev)[order], np.arange(n - 1))
    w_by_left = ew[order]                         # weight of edge (i, i+1)
    g = g.with_weights(ew)
    pairs = [(1000, 99000), (20000, 20500), (50000, 70000)]
    P = np.zeros((n, len(pairs)))
    Q = np.zeros((n, len(pairs)))
    for j, (a, b) in enumerate(pairs):
        P[a, j] = 1.0
        Q[b, j] = 1.0
    want = np.array([cf.tree_path(w_by_left[a:b]) for a, b in pairs])
    say("long weighted path, mixed", n)
    dg = dev_graph(g)
    d, _, info = dg.distances(P, Q, precision="mixed", rtol=1e-8, max_iter=400_000)
    dsq = d.cpu().numpy() ** 2
    assert rel_err(dsq, want).max() <= 1e-6, (dsq, want, info)
    assert all(i["status"] == 0 for i in info), info


@pytest.mark.parametrize("components", [1, 3])
def test_stalled_pairs_are_finished_in_fp64(monkeypatch, components):
    """The hand-over forced from the host (NVD_REFINE_STALL_RATIO2=0 makes
    every outer step count as stalled): after two outer steps every open pair
    is finished by the FP64 solver from its current x, is flagged, and meets
    the FP64 bound against the dense oracle."""
    rng = np.random.default_rng(83)
    parts = [barabasi_albert(1200, 3, rng) for _ in range(components)]
    offs = np.cumsum([0] + [p.n for p in parts])
    from nvdgen import Graph
    g = Graph(int(offs[-1]), np.concatenate([p.eu + o for p, o in zip(parts, offs[:-1])]),
              np.concatenate([p.ev + o for p, o in zip(parts, offs[:-1])]))
    g = g.with_weights(rng.lognormal(0, 1, g.num_edges))
    P, Q = rng.random((g.n, 6)), rng.random((g.n, 6))
    Q[:, 5] = P[:, 5]                            # d = 0: never opened
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    say("forced stall", components)
    dg = dev_graph(g)
    monkeypatch.setenv("NVD_REFINE_STALL_RATIO2", "0")
    d, X, info = dg.distances(P, Q, precision="mixed", rtol=1e-10, inner_rtol=1e-2,
                              return_x=True)
    d = d.cpu().numpy()
    assert rel_err(d[:5], ref[:5]).max() <= 1e-8, (d, ref, info)
    assert d[5] == 0.0 and info[5]["flags"] == 0
    assert all(i["flags"] & 1 and i["status"] == 0 for i in info[:5]), info
    assert all(i["rel_res"] <= 1e-10 for i in info[:5]), info
    monkeypatch.delenv("NVD_REFINE_STALL_RATIO2")
    d2, _, info2 = dg.distances(P, Q, precision="mixed", rtol=1e-10, inner_rtol=1e-2)
    assert all(i["flags"] == 0 for i in info2)
    assert rel_err(d2.cpu().numpy()[:5], ref[:5]).max() <= 1e-6


def test_guard_quiet_on_well_conditioned_graph():
    rng = np.random.default_rng(82)
    g = barabasi_albert(3000, 3, rng)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    P, Q = rng.random((g.n, 8)), rng.random((g.n, 8))
    say("guard quiet")
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)["d"]
    dg = dev_graph(g)
    d, _, info = dg.distances(P, Q, precision="mixed", rtol=1e-10)
    assert rel_err(d.cpu().numpy(), ref).max() <= 1e-6
    assert all(i["flags"] == 0 and i["status"] == 0 for i in info)
