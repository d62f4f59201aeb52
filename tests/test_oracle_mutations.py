"""Planted mistakes: each test copies the oracle package, plants one plausible
mistake in its source (a dropped term, a wrong sign, a wrong index, an
off-by-one in the null space), imports the copy under another name and checks
that the pin suite below catches it.  Mistakes are planted in the CPU oracle
only."""
import importlib
import itertools
import os
import shutil
import sys

import numpy as np
import pytest

from nvdgen import (path_graph, cycle_graph, random_tree, barabasi_albert,
                    Graph)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load_mutant(tmp_path, fname, old, new, tag):
    dst = tmp_path / f"oracle_mut_{tag}"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst)
    path = dst / fname
    src = path.read_text()
    assert src.count(old) >= 1, f"mutation anchor not found in {fname}: {old!r}"
    path.write_text(src.replace(old, new, 1))
    sys.path.insert(0, str(tmp_path))
    try:
        mod = importlib.import_module(dst.name)
    finally:
        sys.path.pop(0)
    return mod


def _unit(n, pairs):
    P = np.zeros((n, len(pairs)))
    Q = np.zeros((n, len(pairs)))
    for j, (a, b) in enumerate(pairs):
        P[a, j] = 1.0
        Q[b, j] = 1.0
    return P, Q


def pin_suite(o):
    """Returns the list of pins that FAIL for oracle module o."""
    failed = []

    def check(name, ok):
        if not ok:
            failed.append(name)

    def close(a, b, rtol=1e-9):
        a = np.asarray(a, dtype=float)
        b = np.asarray(b, dtype=float)
        return a.shape == b.shape and np.all(np.isfinite(a)) and \
            np.allclose(a, b, rtol=rtol, atol=1e-12)

    from oracle import closed_forms as cf   # the unmutated textbook values
    # path, all routes
    g = path_graph(9)
    pairs = list(itertools.combinations(range(9), 2))
    P, Q = _unit(9, pairs)
    want = [cf.path(i, j) for i, j in pairs]
    for route in ("ge_dense", "ge_grounded", "ge_pcg", "ge_tree"):
        try:
            r = getattr(o, route)(g.n, g.row_ptr, g.col_idx, None, P, Q)["dsq"]
            check("path-" + route, close(r, want))
        except Exception:
            failed.append("path-" + route + "-raised")
    # weighted tree, with random (not unit) vectors against the dense route
    rng = np.random.default_rng(1)
    tw = rng.uniform(0.3, 3.0, 29)
    t = random_tree(30, rng, tw)
    A, B = rng.random((30, 2)), rng.random((30, 2))
    try:
        ref = o.ge_dense(t.n, t.row_ptr, t.col_idx, t.w, A, B)
        tr = o.ge_tree(t.n, t.row_ptr, t.col_idx, t.w, A, B)
        check("tree-vs-dense", close(tr["d"], ref["d"]))
        check("tree-x", close(tr["x"], ref["x"], 1e-8))
    except Exception:
        failed.append("tree-raised")
    # series law on the weighted tree (closed form), dense route
    P1, Q1 = _unit(30, [(0, 29)])
    try:
        r0 = o.ge_dense(t.n, t.row_ptr, t.col_idx, t.w, P1, Q1)["dsq"][0]
        tt = o.ge_tree(t.n, t.row_ptr, t.col_idx, t.w, P1, Q1)
        par = tt["parent"]
        anc0 = set()
        u = 0
        while u >= 0:
            anc0.add(u)
            u = par[u]
        # walk 29 up to the common ancestor with 0, then 0 up to it
        w_of = {}
        for e, (a, b) in enumerate(zip(t.eu, t.ev)):
            w_of[(a, b)] = tw[e]
        def up(v, stop):
            out = []
            while v not in stop:
                p = par[v]
                out.append(w_of[(min(v, p), max(v, p))])
                v = p
            return out, v
        acc, lca = up(29, anc0)
        acc2, _ = up(0, {lca})
        check("tree-series", close(r0, cf.tree_path(acc + acc2)))
    except Exception:
        failed.append("tree-series-raised")
    # cycle FFT route against the closed form
    n = 13
    P, Q = _unit(n, [(0, j) for j in range(1, n)])
    try:
        check("cycle-fft", close(o.ge_cycle(n, P, Q, w=1.5)["dsq"],
                                 [cf.cycle(n, 0, j, 1.5) for j in range(1, n)]))
    except Exception:
        failed.append("cycle-raised")
    # disconnected graph: sum over components, all routes agree with it
    g1 = barabasi_albert(25, 2, np.random.default_rng(3))
    g2 = cycle_graph(n)
    N = g1.n + n + 2
    gd = Graph(N, np.concatenate([g1.eu, g2.eu + g1.n]), np.concatenate([g1.ev, g2.ev + g1.n]))
    A, B = np.random.default_rng(4).random((N, 2)), np.random.default_rng(5).random((N, 2))
    try:
        part = o.ge_dense(g1.n, g1.row_ptr, g1.col_idx, None, A[:25], B[:25])["dsq"] + \
            o.ge_cycle(n, A[25:25 + n], B[25:25 + n])["dsq"]
        for route in ("ge_dense", "ge_grounded", "ge_pcg"):
            r = getattr(o, route)(N, gd.row_ptr, gd.col_idx, None, A, B)["dsq"]
            check("disconnected-" + route, close(r, part))
    except Exception:
        failed.append("disconnected-raised")
    # Foster's theorem on a weighted BA graph
    gb = barabasi_albert(30, 2, np.random.default_rng(6))
    ew = np.random.default_rng(7).lognormal(0, 1, gb.num_edges)
    gw = gb.with_weights(ew)
    P, Q = _unit(gb.n, list(zip(gb.eu, gb.ev)))
    try:
        R = o.ge_dense(gb.n, gw.row_ptr, gw.col_idx, gw.w, P, Q)["dsq"]
        check("foster", abs(np.sum(ew * R) - (gb.n - 1)) < 1e-9)
    except Exception:
        failed.append("foster-raised")
    # gradient against central finite differences of the dense route
    try:
        A, B = np.random.default_rng(8).random((gb.n, 1)), np.random.default_rng(9).random((gb.n, 1))
        gr = o.grad_dense(gb.n, gw.row_ptr, gw.col_idx, gw.w, A, B)
        ge = np.zeros(gb.num_edges)
        np.add.at(ge, gw.csr_edge, gr["grad_w_csr"])
        ok = True
        for e in (0, 11, 40):
            h = 1e-5 * ew[e]
            wp, wm = ew.copy(), ew.copy()
            wp[e] += h
            wm[e] -= h
            fp = o.ge_dense(gb.n, gw.row_ptr, gw.col_idx, wp[gw.csr_edge], A, B)["dsq"][0]
            fm = o.ge_dense(gb.n, gw.row_ptr, gw.col_idx, wm[gw.csr_edge], A, B)["dsq"][0]
            ok &= abs((fp - fm) / (2 * h) - ge[e]) < 1e-6 * max(1, abs(ge[e]))
        h = 1e-6
        Ap, Am = A.copy(), A.copy()
        Ap[3] += h
        Am[3] -= h
        fd = (o.ge_dense(gb.n, gw.row_ptr, gw.col_idx, gw.w, Ap, B)["dsq"][0] -
              o.ge_dense(gb.n, gw.row_ptr, gw.col_idx, gw.w, Am, B)["dsq"][0]) / (2 * h)
        ok &= abs(fd - gr["grad_p"][3, 0]) < 1e-6
        check("grad-fd", ok)
    except Exception:
        failed.append("grad-raised")
    # all pairwise distances: path closed form (both routes), a disconnected
    # graph against the per-pair grounded route, and the metric invariants
    try:
        gp = path_graph(9)
        want = np.sqrt(np.abs(np.subtract.outer(np.arange(9), np.arange(9))).astype(float))
        for route in ("pairwise_dense", "pairwise_pcg"):
            D = getattr(o, route)(gp.n, gp.row_ptr, gp.col_idx, None, np.eye(9))
            check("pairwise-path-" + route, close(D, want))
        Vd = np.random.default_rng(10).random((N, 5))
        D = o.pairwise_dense(N, gd.row_ptr, gd.col_idx, None, Vd)
        iu, ju = np.triu_indices(5, 1)
        ref = o.ge_grounded(N, gd.row_ptr, gd.col_idx, None, Vd[:, iu], Vd[:, ju])["d"]
        check("pairwise-disconnected", close(D[iu, ju], ref) and close(D, D.T) and
              np.all(np.diag(D) == 0.0))
        ok = True
        for i, j, k in itertools.permutations(range(5), 3):
            ok &= D[i, j] <= D[i, k] + D[k, j] + 1e-12
        check("pairwise-triangle", ok)
    except Exception:
        failed.append("pairwise-raised")
    return failed


def test_unmutated_oracle_passes_suite():
    import oracle
    assert pin_suite(oracle) == []


MUTATIONS = [
    # (file, anchor, replacement)
    ("laplacian.py", "    return D - A\n", "    return D + A\n"),            # wrong sign of A
    ("laplacian.py", "    return D - A\n", "    return -A\n"),               # dropped degree term
    ("laplacian.py", "    off = row != col\n", "    off = row >= 0\n"),     # keeps self-loops: none in the pin graphs
    ("laplacian.py", "        out[:, j] -= (s / size)[labels]\n",
     "        out[:, j] -= s.sum() / size.sum()\n"),                          # global instead of per-component mean
    ("dense.py", "    coef = U[:, c:].T @ delta", "    coef = U[:, c - 0:].T @ delta[::-1]"),  # reversed operand
    ("dense.py", "    dsq = np.sum(coef * coef / lam[c:, None], axis=0)",
     "    dsq = np.sum(coef * coef / lam[c:, None] ** 2, axis=0)"),       # L^+2 instead of L^+
    ("dense.py", "    c = int(lab.max()) + 1 if n else 0", "    c = int(lab.max()) + 2 if n else 0"),  # off-by-one null space
    ("grounded.py", "        rest = nodes[1:]", "        rest = nodes[:-1]"),   # (still valid) -> neutral
    ("grounded.py", "    dbar = project(P - Q, lab)", "    dbar = P - Q"),         # projection dropped
    ("pcg.py", "        beta = rho_new / rho[cols]", "        beta = rho[cols] / rho_new"),
    ("pcg.py", "        r[:, cols] -= alpha * q", "        r[:, cols] += alpha * q"),
    ("pcg.py", "    J = np.sum(dbar * x, axis=0) + np.sum(x * r, axis=0)",
     "    J = np.sum(dbar * x, axis=0) - np.sum(x * r, axis=0) + 1e-6"),
    ("tree.py", "        x[lev] = x[parent[lev]] + f[lev] / pw[lev, None]",
     "        x[lev] = x[parent[lev]] - f[lev] / pw[lev, None]"),
    ("tree.py", "    dsq = np.sum(f[nonroot] ** 2 / pw[nonroot, None], axis=0)",
     "    dsq = np.sum(f[nonroot] ** 2 * pw[nonroot, None], axis=0)"),
    ("cycle.py", "    lam = 4.0 * w * np.sin(np.pi * kk / n) ** 2",
     "    lam = 4.0 * w * np.sin(2.0 * np.pi * kk / n) ** 2"),
    ("cycle.py", "    dsq = np.sum(np.abs(dh[1:]) ** 2 / lam[:, None], axis=0) / n",
     "    dsq = np.sum(np.abs(dh[1:]) ** 2 / lam[:, None], axis=0) / (n - 1)"),
    ("grad.py", "    gw = -0.5 * np.sum(g[None, :] * diff * diff, axis=1)",
     "    gw = 0.5 * np.sum(g[None, :] * diff * diff, axis=1)"),
    ("grad.py", "    gw = -0.5 * np.sum(g[None, :] * diff * diff, axis=1)",
     "    gw = -1.0 * np.sum(g[None, :] * diff * diff, axis=1)"),
    ("grad.py", "    return 2.0 * x * g[None, :], gw", "    return x * g[None, :], gw"),
    ("pairwise.py", "            diff = coef[:, i] - coef[:, j]", "            diff = coef[:, i] + coef[:, j]"),
    ("pairwise.py", "            dsq = max(float(np.sum(diff * diff / lam[c:])), 0.0)",
     "            dsq = max(float(np.sum(diff * diff * lam[c:])), 0.0)"),
    ("pairwise.py", "    c = int(components(n, row_ptr, col_idx).max()) + 1",
     "    c = int(components(n, row_ptr, col_idx).max())"),                 # keeps a null eigenpair
    ("pairwise.py", "    r = ge_pcg(n, row_ptr, col_idx, w, V[:, iu], V[:, ju], rtol=rtol)",
     "    r = ge_pcg(n, row_ptr, col_idx, w, V[:, iu], V[:, iu + 1], rtol=rtol)"),   # wrong partner
    ("pairwise.py", "            D[i, j] = D[j, i] = np.sqrt(dsq)", "            D[i, j] = np.sqrt(dsq)"),
]

# Mutations that do not change the mathematics (self-loops are absent from the
# pin graphs; grounding any node of a component is equally valid) must NOT be
# caught: they document that the suite is not merely sensitive to any edit.
EQUIVALENT = {2, 7}


@pytest.mark.parametrize("idx", range(len(MUTATIONS)))
def test_mutation_is_caught(tmp_path, idx):
    fname, old, new = MUTATIONS[idx]
    mod = _load_mutant(tmp_path, fname, old, new, idx)
    failed = pin_suite(mod)
    if idx in EQUIVALENT:
        assert failed == [], failed
    else:
        assert failed, f"planted mistake in {fname} not caught: {new.strip()}"
