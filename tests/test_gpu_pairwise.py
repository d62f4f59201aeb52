"""GPU parity of the all-pairs distance matrix (one solve with m right-hand
sides plus the residual-corrected Gram contraction) against the CPU
oracle's pairwise routes, and against pairs solved one by one."""
import numpy as np
import pytest

import oracle
from nvdgen import barabasi_albert, ws_connected, Graph, workload

from gpu_helpers import say, dev_graph, rel_err

pytestmark = pytest.mark.gpu


def _hub_graph(seed=0, n=2000, hub_deg=1500):
    """BA graph plus a hub joined to hub_deg nodes (split rows) plus three
    isolated nodes: four components."""
    rng = np.random.default_rng(seed)
    g = barabasi_albert(n, 3, rng)
    nb = rng.choice(n, hub_deg, replace=False)
    eu = np.concatenate([g.eu, nb])
    ev = np.concatenate([g.ev, np.full(hub_deg, n)])
    return Graph(n + 4, np.minimum(eu, ev), np.maximum(eu, ev))


def _check(D, ref, tol):
    """Relative error on d where the reference is clearly nonzero, absolute
    error (scaled by the largest distance) elsewhere; exact symmetry and a
    zero diagonal."""
    assert np.array_equal(D, D.T)
    assert np.all(np.diag(D) == 0.0)
    scale = ref.max()
    big = ref > 1e-3 * scale
    assert rel_err(D[big], ref[big]).max() <= tol, rel_err(D[big], ref[big]).max()
    assert np.abs(D[~big] - ref[~big]).max() <= 10 * tol * scale


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("m", [2, 5, 64, 100])
def test_pairwise_matches_dense_oracle(m, precision, tol):
    rng = np.random.default_rng(m)
    g = barabasi_albert(900, 3, rng)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    V = np.where(rng.random((g.n, m)) < 0.2, rng.random((g.n, m)), 0.0)
    say("pairwise dense", m, precision)
    dg = dev_graph(g)
    D, G, info = dg.pairwise(V, precision=precision, rtol=1e-10 if precision == "fp64" else 1e-8,
                             return_gram=True)
    D = D.cpu().numpy()
    ref = oracle.pairwise_dense(g.n, g.row_ptr, g.col_idx, g.w, V)
    _check(D, ref, tol)
    assert all(i["status"] == 0 for i in info)
    # Gram matrix in the L^+ inner product of the projected vectors
    Vb = V - V.mean(axis=0)
    x = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, V, np.zeros_like(V))["x"]
    Gref = Vb.T @ x
    Gm = G.cpu().numpy()
    assert np.abs(Gm - Gref).max() <= 100 * tol * np.abs(Gref).max()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_pairwise_disconnected_split_rows_and_repeats(precision, tol):
    """Four components (per-component projection), a split-row hub, a vector
    repeated and one shifted by a constant (distance 0)."""
    g = _hub_graph(1)
    rng = np.random.default_rng(2)
    V = rng.random((g.n, 7))
    V = np.column_stack([V, V[:, 2], V[:, 4] + 2.5])
    say("pairwise disconnected", precision)
    dg = dev_graph(g)
    assert dg.stats()["n_comp"] == 4
    D, _, _ = dg.pairwise(V, precision=precision, rtol=1e-10 if precision == "fp64" else 1e-8)
    D = D.cpu().numpy()
    ref = oracle.pairwise_dense(g.n, g.row_ptr, g.col_idx, None, V)
    _check(D, ref, tol)
    assert D[2, 7] <= 1e-6 * D.max() and D[4, 8] <= 1e-6 * D.max()


def test_pairwise_agrees_with_pair_solves():
    """D_ij from the Gram route against nvd_distances on (v_i, v_j)."""
    rng = np.random.default_rng(9)
    g = ws_connected(5000, 6, 0.1, np.random.SeedSequence(9))
    m = 12
    V = rng.standard_normal((g.n, m))
    say("pairwise vs pairs")
    dg = dev_graph(g)
    D, _, _ = dg.pairwise(V, precision="fp64", rtol=1e-10)
    D = D.cpu().numpy()
    iu, ju = np.triu_indices(m, 1)
    d, _, _ = dg.distances(V[:, iu], V[:, ju], precision="fp64", rtol=1e-10)
    assert rel_err(D[iu, ju], d.cpu().numpy()).max() <= 1e-8


def test_pairwise_ba_2e5_sampled_pairs():
    """The 2e5-node lognormal-weighted BA graph, 32 vectors (496 distances)
    in mixed precision; 24 sampled pairs against the oracle's PCG route."""
    w = workload(4)
    g = w.graphs[0]
    V = w.P[0]
    m = V.shape[1]
    say("pairwise c4", g.n, m)
    dg = dev_graph(g)
    D, _, info = dg.pairwise(V, precision="mixed", rtol=1e-8)
    D = D.cpu().numpy()
    assert all(i["status"] == 0 for i in info)
    rng = np.random.default_rng(4)
    iu, ju = np.triu_indices(m, 1)
    pick = rng.choice(iu.size, 24, replace=False)
    r = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, V[:, iu[pick]], V[:, ju[pick]])
    assert rel_err(D[iu[pick], ju[pick]], r["d"]).max() <= 1e-6
    assert np.array_equal(D, D.T)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_pairwise_near_duplicate_columns(precision, tol):
    """Columns 4..7 are columns 0..3 plus a 1e-4 perturbation: the pair
    distances among them are ~1e-4 of the vectors' own L^+ norms, so the
    Gram-difference form G_ii + G_jj - G_ij - G_ji cancels ~8 digits.  Every
    pair, close or not, must meet the relative bound."""
    rng = np.random.default_rng(77)
    g = barabasi_albert(900, 3, rng)
    g = g.with_weights(rng.uniform(0.5, 2.0, g.num_edges))
    base = np.where(rng.random((g.n, 4)) < 0.2, rng.random((g.n, 4)), 0.0)
    V = np.concatenate([base, base + 1e-4 * rng.standard_normal((g.n, 4))], axis=1)
    say("pairwise near duplicates", precision)
    dg = dev_graph(g)
    D, _, info = dg.pairwise(V, precision=precision, rtol=1e-10 if precision == "fp64" else 1e-8)
    D = D.cpu().numpy()
    ref = oracle.pairwise_dense(g.n, g.row_ptr, g.col_idx, g.w, V)
    off = ~np.eye(V.shape[1], dtype=bool)
    assert np.array_equal(D, D.T)
    assert ref[off].min() > 0
    e = rel_err(D[off], ref[off])
    assert e.max() <= tol, e.max()
    # the close pairs (i, i + 4) are far below the others
    assert max(ref[i, i + 4] for i in range(4)) < 1e-2 * ref[0, 1]
