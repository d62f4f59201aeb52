"""Seeded synthetic graph generators (host side, NumPy).

These build the inputs only: undirected simple edge lists and the symmetric CSR
that carries them.  Nothing here computes a Laplacian, a degree matrix, a
projection or a distance -- that arithmetic lives separately in the CPU oracle
and in the HIP library, which share no code with each other.

Models follow the synthetic-data list of the paper (section 4.1.2):
Barabasi-Albert growth with preferential attachment, Watts-Strogatz ring
rewiring, Erdos-Renyi G(n, m) with uniformly drawn node-id pairs and the
stochastic block model; a configuration model with power-law degrees is added
for the large workload.  Exact generator conventions (seed graph, rewiring
rule, duplicate handling) are not fixed by the paper and are stated in each
docstring.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

__all__ = [
    "Graph", "to_csr", "barabasi_albert", "watts_strogatz", "erdos_renyi",
    "stochastic_block_model", "sbm_sparse", "configuration_model_powerlaw", "giant_component",
    "path_graph", "cycle_graph", "complete_graph", "star_graph",
    "complete_bipartite", "random_tree", "grid_graph", "is_connected",
]


class Graph:
    """Undirected simple graph as a symmetric CSR (both directions stored).

    row_ptr : int64 [n+1]; col_idx : int32 [nnz], sorted within each row;
    w : float64 [nnz] edge weights (equal in both directions) or None for unit
    weights.  ``eu, ev, ew`` keep the undirected edge list (eu < ev) the CSR
    was built from, in edge order; ``csr_edge`` maps each CSR entry to its
    undirected edge id.
    """

    def __init__(self, n, eu, ev, ew=None):
        self.n = int(n)
        self.eu = np.asarray(eu, dtype=np.int64)
        self.ev = np.asarray(ev, dtype=np.int64)
        self.ew = None if ew is None else np.asarray(ew, dtype=np.float64)
        self.row_ptr, self.col_idx, self.w, self.csr_edge = to_csr(
            self.n, self.eu, self.ev, self.ew)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def num_edges(self) -> int:
        return int(self.eu.shape[0])

    def with_weights(self, ew):
        return Graph(self.n, self.eu, self.ev, ew)


def to_csr(n, eu, ev, ew=None):
    """Symmetric CSR of an undirected edge list (both directions stored).

    Rows are sorted by column.  Returns (row_ptr int64, col_idx int32,
    w float64 or None, csr_edge int64) where csr_edge[k] is the undirected edge
    that CSR entry k came from.
    """
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    m = eu.shape[0]
    rows = np.concatenate([eu, ev])
    cols = np.concatenate([ev, eu])
    eid = np.concatenate([np.arange(m, dtype=np.int64)] * 2)
    order = np.lexsort((cols, rows))
    rows, cols, eid = rows[order], cols[order], eid[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    w = None if ew is None else np.asarray(ew, dtype=np.float64)[eid]
    return row_ptr, cols.astype(np.int32), w, eid


def _edge_keys(u, v, n):
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    return a * np.int64(n) + b


def is_connected(n, eu, ev) -> bool:
    if n <= 1:
        return True
    a = csr_matrix((np.ones(len(eu)), (eu, ev)), shape=(n, n))
    nc, _ = connected_components(a, directed=False)
    return nc == 1


# ---------------------------------------------------------------------------
# Barabasi-Albert
# ---------------------------------------------------------------------------
def barabasi_albert(n, m, rng, max_rounds=10_000):
    """Barabasi-Albert graph (paper section 4.1.2, BA bullet).

    Seed: a star on nodes 0..m with centre 0 (m edges).  Every later node t
    attaches to m *distinct* earlier nodes drawn with probability proportional
    to degree, by sampling uniform positions of the endpoint list of all edges
    that exist before t arrives (edge e occupies positions 2e, 2e+1).
    Result: m(n-m) edges, connected, simple.

    Vectorised: all positions are drawn first and resolved by pointer jumping
    (an odd position of a non-seed edge points at another draw).  Nodes whose m
    targets repeat redraw the later duplicates; since later draws may resolve
    through redrawn ones, resolution is repeated until no node has duplicates.
    """
    n = int(n)
    m = int(m)
    if m < 1 or n <= m:
        raise ValueError("need n > m >= 1")
    E = m * (n - m)
    src = np.empty(E, dtype=np.int64)
    dst = np.empty(E, dtype=np.int64)
    src[:m] = 0
    dst[:m] = np.arange(1, m + 1)
    if E == m:
        return Graph(n, src, dst)
    e = np.arange(m, E, dtype=np.int64)
    t = m + 1 + (e - m) // m
    src[m:] = t
    lim = 2 * (m + (t - m - 1) * m)  # endpoint-list length before node t
    r = np.floor(rng.random(E - m) * lim).astype(np.int64)
    np.minimum(r, lim - 1, out=r)

    def resolve():
        pos = r.copy()
        out = np.empty(E - m, dtype=np.int64)
        todo = np.arange(E - m)
        while todo.size:
            p = pos[todo]
            eidx = p >> 1
            odd = (p & 1).astype(bool)
            even_sel = ~odd
            out[todo[even_sel]] = src[eidx[even_sel]]
            seed_sel = odd & (eidx < m)
            out[todo[seed_sel]] = dst[eidx[seed_sel]]
            jump = odd & (eidx >= m)
            nxt = todo[jump]
            pos[nxt] = r[eidx[jump] - m]
            todo = nxt
        return out

    for _ in range(max_rounds):
        tgt = resolve().reshape(-1, m)
        srt = np.sort(tgt, axis=1)
        dupnode = np.any(srt[:, 1:] == srt[:, :-1], axis=1)
        if not dupnode.any():
            break
        # within each duplicated node, redraw every entry equal to an earlier one
        rows = np.nonzero(dupnode)[0]
        sub = tgt[rows]
        redraw = np.zeros_like(sub, dtype=bool)
        for j in range(1, m):
            redraw[:, j] = np.any(sub[:, :j] == sub[:, j:j + 1], axis=1)
        flat = (rows[:, None] * m + np.arange(m)[None, :])[redraw]
        r[flat] = np.minimum(
            np.floor(rng.random(flat.size) * lim[flat]).astype(np.int64),
            lim[flat] - 1)
    else:  # pragma: no cover
        raise RuntimeError("BA duplicate resolution did not converge")
    dst[m:] = tgt.reshape(-1)
    return Graph(n, np.minimum(src, dst), np.maximum(src, dst))


# ---------------------------------------------------------------------------
# Watts-Strogatz
# ---------------------------------------------------------------------------
def watts_strogatz(n, k, beta, rng, max_rounds=10_000):
    """Watts-Strogatz graph (paper section 4.1.2, WS bullet).

    Start from the ring where each node links to its k/2 nearest neighbours on
    each side; every edge (u, u+j) is selected for rewiring with probability
    beta, and a selected edge keeps u and gets a uniformly drawn far endpoint.
    Draws that make a self-loop or repeat an edge already present are redrawn
    (rewired edges are checked in edge order) until the graph is simple.
    The caller decides what to do with a disconnected result.
    """
    n = int(n)
    half = int(k) // 2
    if half < 1 or n <= 2 * half:
        raise ValueError("need n > k >= 2")
    u = np.repeat(np.arange(n, dtype=np.int64), half)
    v = (u + np.tile(np.arange(1, half + 1, dtype=np.int64), n)) % n
    sel = np.nonzero(rng.random(u.size) < beta)[0]
    v = v.copy()
    v[sel] = rng.integers(0, n, size=sel.size)
    pending = sel
    for _ in range(max_rounds):
        keys = _edge_keys(u, v, n)
        # an edge is bad if it is a self-loop or its key already appeared
        # earlier in the edge order (original ring edges keep priority by
        # being checked as "earlier" when not rewired)
        rewired = np.zeros(u.size, dtype=bool)
        rewired[sel] = True
        order = np.lexsort((np.arange(u.size), rewired, keys))
        ks = keys[order]
        dup_sorted = np.zeros(u.size, dtype=bool)
        dup_sorted[1:] = ks[1:] == ks[:-1]
        dup = np.zeros(u.size, dtype=bool)
        dup[order] = dup_sorted
        bad = (dup | (u == v)) & rewired
        pending = np.nonzero(bad)[0]
        if pending.size == 0:
            break
        v[pending] = rng.integers(0, n, size=pending.size)
    else:  # pragma: no cover
        raise RuntimeError("WS rewiring did not converge")
    return Graph(n, np.minimum(u, v), np.maximum(u, v))


# ---------------------------------------------------------------------------
# Erdos-Renyi G(n, m) and stochastic block model
# ---------------------------------------------------------------------------
def erdos_renyi(n, m, rng):
    """G(n, m): m distinct edges from uniformly drawn node-id pairs (section
    4.1.2, ER bullet); self-loops and repeats are redrawn."""
    n = int(n)
    m = int(m)
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        a = rng.integers(0, n, size=2 * need + 16)
        b = rng.integers(0, n, size=2 * need + 16)
        ok = a != b
        new = _edge_keys(a[ok], b[ok], n)
        allk = np.concatenate([keys, new])
        _, first = np.unique(allk, return_index=True)
        keep = np.sort(first)
        keys = allk[keep][:m]
    return Graph(n, keys // n, keys % n)


def stochastic_block_model(sizes, p_in, p_out, rng):
    """SBM (section 4.1.2, SBM bullet): every pair inside a block is an edge
    with probability p_in, across blocks with p_out (dense Bernoulli draws,
    meant for small n)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    n = int(sizes.sum())
    block = np.repeat(np.arange(sizes.size), sizes)
    iu, iv = np.triu_indices(n, 1)
    prob = np.where(block[iu] == block[iv], p_in, p_out)
    keep = rng.random(iu.size) < prob
    return Graph(n, iu[keep], iv[keep])


def sbm_sparse(sizes, p_in, p_out, rng):
    """SBM with the same distribution as ``stochastic_block_model`` (every
    pair an independent Bernoulli draw) for larger n: per block pair, the edge
    count is drawn from the binomial and that many distinct pairs uniformly."""
    sizes = np.asarray(sizes, dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    eu, ev = [], []
    for a in range(sizes.size):
        for b in range(a, sizes.size):
            if a == b:
                s = int(sizes[a])
                npairs = s * (s - 1) // 2
                cnt = rng.binomial(npairs, p_in)
                pick = rng.choice(npairs, cnt, replace=False)
                iu, iv = np.triu_indices(s, 1)
                eu.append(iu[pick] + offs[a])
                ev.append(iv[pick] + offs[a])
            else:
                sa, sb = int(sizes[a]), int(sizes[b])
                cnt = rng.binomial(sa * sb, p_out)
                pick = rng.choice(sa * sb, cnt, replace=False)
                eu.append(pick // sb + offs[a])
                ev.append(pick % sb + offs[b])
    return Graph(int(offs[-1]), np.concatenate(eu), np.concatenate(ev))


# ---------------------------------------------------------------------------
# Configuration model with power-law degrees
# ---------------------------------------------------------------------------
def configuration_model_powerlaw(n, gamma, kmin, kmax, rng):
    """Configuration model: iid degrees with P(k) proportional to k^-gamma on
    [kmin, kmax]; if the degree sum is odd, one uniformly drawn node gets one
    more stub; stubs are matched by a uniform shuffle; self-loops and repeated
    edges are erased (not redrawn).  Returns the full graph (may be
    disconnected); see :func:`giant_component`."""
    n = int(n)
    ks = np.arange(kmin, kmax + 1, dtype=np.float64)
    cdf = np.cumsum(ks ** (-float(gamma)))
    cdf /= cdf[-1]
    deg = kmin + np.searchsorted(cdf, rng.random(n), side="right")
    deg = np.minimum(deg, kmax).astype(np.int64)
    if deg.sum() % 2:
        deg[rng.integers(0, n)] += 1
    stubs = np.repeat(np.arange(n, dtype=np.int64), deg)
    rng.shuffle(stubs)
    a = stubs[0::2]
    b = stubs[1::2]
    del stubs
    ok = a != b
    keys = np.unique(_edge_keys(a[ok], b[ok], n))
    return Graph(n, keys // n, keys % n)


def giant_component(g: Graph, ew=None):
    """Restrict to the largest connected component, relabelled in increasing
    original id order.  Ties between equal-size components go to the one
    holding the smallest node id."""
    a = csr_matrix((np.ones(g.num_edges), (g.eu, g.ev)), shape=(g.n, g.n))
    nc, lab = connected_components(a, directed=False)
    if nc == 1:
        return g if ew is None else g.with_weights(ew)
    sizes = np.bincount(lab, minlength=nc)
    best = int(np.argmax(sizes))
    keep = lab == best
    newid = np.full(g.n, -1, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    emask = keep[g.eu]
    w = None if ew is None else np.asarray(ew)[emask]
    return Graph(int(keep.sum()), newid[g.eu[emask]], newid[g.ev[emask]], w)


# ---------------------------------------------------------------------------
# Small closed-form families (pins)
# ---------------------------------------------------------------------------
def path_graph(n, w=None):
    u = np.arange(n - 1)
    return Graph(n, u, u + 1, w)


def cycle_graph(n, w=None):
    u = np.arange(n)
    v = (u + 1) % n
    return Graph(n, np.minimum(u, v), np.maximum(u, v), w)


def complete_graph(n, w=None):
    iu, iv = np.triu_indices(n, 1)
    return Graph(n, iu, iv, w)


def star_graph(n_leaves, w=None):
    leaves = np.arange(1, n_leaves + 1)
    return Graph(n_leaves + 1, np.zeros_like(leaves), leaves, w)


def complete_bipartite(a, b, w=None):
    iu = np.repeat(np.arange(a), b)
    iv = a + np.tile(np.arange(b), a)
    return Graph(a + b, iu, iv, w)


def random_tree(n, rng, w=None):
    """Random recursive tree: node i > 0 hangs under a uniform earlier node."""
    par = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    ch = np.arange(1, n)
    return Graph(n, np.minimum(par, ch), np.maximum(par, ch), w)


def grid_graph(rows, cols, w=None):
    idx = np.arange(rows * cols).reshape(rows, cols)
    h = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()])
    v = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()])
    e = np.concatenate([h, v], axis=1)
    return Graph(rows * cols, e[0], e[1], w)
