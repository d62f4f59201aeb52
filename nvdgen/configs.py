"""The five synthetic workloads, built deterministically from fixed seeds.

RNG: NumPy ``Generator(PCG64)``; workload c (1..5) seeds from
``SeedSequence([2310, 11222, c])``.  Its children: 0 -> graph(s), 1 -> vector
pairs, 2 -> edge weights.  Batched workloads spawn one grandchild per graph
from each child (plus, for the graph child, one extra leading grandchild that
draws the graph sizes).

The paper's own graphs (Voteview congress networks, SNAP/Netzschleuder
networks, section 4.1.3) are not available; these synthetic stand-ins follow
the BA / WS shapes of its size sweep (section 4.2) and, for the largest one,
the size and mean degree of its largest real networks (Table 2).

``scale`` shrinks n (and n ranges) for quick tests; scale=1 is the full size.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .graphs import (Graph, barabasi_albert, watts_strogatz, is_connected,
                     configuration_model_powerlaw, giant_component, erdos_renyi, sbm_sparse)
from .vectors import (sparse_support_pairs, uniform_weights, lognormal_weights)

__all__ = ["Workload", "workload", "ws_connected", "seeds", "density_graph", "DENSITY_MODELS",
           "DENSITY_DEGREES", "DENSITY_N"]


def seeds(c):
    return np.random.SeedSequence([2310, 11222, int(c)]).spawn(3)


@dataclass
class Workload:
    name: str
    graphs: List[Graph]
    P: List[np.ndarray]          # per graph, (n_g, k_g) float64
    Q: List[np.ndarray]
    rtol: float
    precision: str               # "fp64" or "mixed"
    notes: dict = field(default_factory=dict)

    @property
    def k_total(self):
        return int(sum(p.shape[1] for p in self.P))


def ws_connected(n, k, beta, ss: np.random.SeedSequence, max_tries=64):
    """Watts-Strogatz draw that is regenerated from the next spawned seed
    until connected."""
    for child in ss.spawn(max_tries):
        g = watts_strogatz(n, k, beta, np.random.Generator(np.random.PCG64(child)))
        if is_connected(g.n, g.eu, g.ev):
            return g
    raise RuntimeError("no connected WS draw")


def _rng(ss):
    return np.random.Generator(np.random.PCG64(ss))


def workload(c: int, scale: float = 1.0, k: Optional[int] = None,
             num_graphs: Optional[int] = None) -> Workload:
    """Build workload c in 1..5 (see module docstring)."""
    sg, sp, sw = seeds(c)
    if c == 1:
        n = max(8, int(round(1000 * scale)))
        g = barabasi_albert(n, 3, _rng(sg))
        kk = 1 if k is None else k
        P, Q = sparse_support_pairs(g.n, kk, 0.10, _rng(sp))
        return Workload("ba_n1e3_m3_unit_k1", [g], [P], [Q], 1e-10, "fp64")
    if c == 2:
        n = max(8, int(round(1_000_000 * scale)))
        g = barabasi_albert(n, 3, _rng(sg))
        kk = 64 if k is None else k
        P, Q = sparse_support_pairs(g.n, kk, 0.05, _rng(sp))
        return Workload("ba_n1e6_m3_unit_k64", [g], [P], [Q], 1e-8, "mixed")
    if c == 3:
        G = 512 if num_graphs is None else num_graphs
        kk = 8 if k is None else k
        gch = sg.spawn(G + 1)
        pch = sp.spawn(G)
        wch = sw.spawn(G)
        lo, hi = np.log(1e3 * scale), np.log(1e5 * scale)
        sizes = np.exp(lo + (hi - lo) * _rng(gch[0]).random(G))
        sizes = np.maximum(16, np.round(sizes).astype(np.int64))
        graphs, Ps, Qs = [], [], []
        for gi in range(G):
            if gi % 2 == 0:
                g = ws_connected(int(sizes[gi]), 6, 0.1, gch[gi + 1])
            else:
                g = barabasi_albert(int(sizes[gi]), 4, _rng(gch[gi + 1]))
            g = g.with_weights(uniform_weights(g.num_edges, 0.5, 2.0, _rng(wch[gi])))
            P, Q = sparse_support_pairs(g.n, kk, 0.20, _rng(pch[gi]), dist="normal")
            graphs.append(g)
            Ps.append(P)
            Qs.append(Q)
        return Workload("batch512_ws_k6_ba_m4_k8", graphs, Ps, Qs, 1e-8, "mixed")
    if c == 4:
        n = max(8, int(round(200_000 * scale)))
        g = barabasi_albert(n, 5, _rng(sg))
        g = g.with_weights(lognormal_weights(g.num_edges, _rng(sw)))
        kk = 32 if k is None else k
        P, Q = sparse_support_pairs(g.n, kk, 0.10, _rng(sp))
        return Workload("ba_n2e5_m5_lognormal_k32", [g], [P], [Q], 1e-10, "fp64")
    if c == 5:
        n0 = max(64, int(round(10_000_000 * scale)))
        kmax = int(np.floor(n0 ** (1.0 / 1.5)))
        g = configuration_model_powerlaw(n0, 2.5, 3, kmax, _rng(sg))
        g = giant_component(g)
        kk = 16 if k is None else k
        P, Q = sparse_support_pairs(g.n, kk, 0.01, _rng(sp))
        return Workload("cm_pl2.5_n1e7_k16", [g], [P], [Q], 1e-8, "mixed",
                        notes={"n_before_gc": n0, "kmax": kmax})
    raise ValueError(c)


# ---------------------------------------------------------------------------
# Density sweep (section 4.2, "Runtimes (Density)"): |V| = 10,000 and the
# average degree from 1 to 64 on the four models of section 4.1.2, with
# roughly the same number of edges across models at each degree.
# ---------------------------------------------------------------------------
DENSITY_N = 10_000
DENSITY_MODELS = ("er", "ba", "ws", "sbm")
DENSITY_DEGREES = (1, 2, 4, 8, 16, 32, 64)


def density_graph(model: str, avg_degree: int, n: int = DENSITY_N, k: int = 8):
    """One graph of the density sweep and k vector pairs on it.

    * er:  G(n, m) with m = n * d / 2 edges (disconnected at low d).
    * ba:  each new node attaches to max(1, round(d / 2)) earlier nodes
           (average degree ~2 at d = 1: the model cannot go lower).
    * ws:  ring with k' = max(2, 2 round(d / 2)) neighbours, rewiring 0.1.
    * sbm: 10 equal groups, p_out = p_in / 10, p_in set for expected degree d.
    Vectors: uniform[0, 1) on independent 10% supports.  Seeds:
    SeedSequence([2310, 11222, 42, model index, d]) children 0 (graph) and 1
    (pairs)."""
    mi = DENSITY_MODELS.index(model)
    sg, sp = np.random.SeedSequence([2310, 11222, 42, mi, int(avg_degree)]).spawn(2)
    rg = _rng(sg)
    d = float(avg_degree)
    if model == "er":
        g = erdos_renyi(n, int(round(n * d / 2)), rg)
    elif model == "ba":
        g = barabasi_albert(n, max(1, int(round(d / 2))), rg)
    elif model == "ws":
        g = watts_strogatz(n, max(2, 2 * int(round(d / 2))), 0.1, rg)
    else:
        groups = 10
        s = n // groups
        p_in = d / ((s - 1) + 0.1 * (n - s))
        g = sbm_sparse([s] * groups, p_in, p_in / 10.0, rg)
    P, Q = sparse_support_pairs(g.n, k, 0.10, _rng(sp))
    return g, P, Q
