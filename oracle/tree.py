"""Route O4: exact GE distance on a tree (or forest) in O(n).

TEST INFRASTRUCTURE ONLY (see the package docstring).

On a tree, L x = delta_bar has a unique flow: the current through the edge
between node v and its parent equals the total of delta_bar over the subtree
below v, f_v = sum_{u in sub(v)} delta_bar_u, and f_v = w_v (x_v - x_parent).
Hence x_v = x_parent + f_v / w_v, and
d^2 = delta_bar^T x = sum_v f_v^2 / w_v  (the electrical energy of the flow,
Thomson's principle).  Each tree of a forest is rooted at its smallest node.
The breadth-first levels are processed one at a time (vectorised per level).
"""
from __future__ import annotations

import numpy as np

from .laplacian import components, project

__all__ = ["ge_tree"]


def ge_tree(n, row_ptr, col_idx, w, P, Q):
    P = np.asarray(P, dtype=np.float64).reshape(n, -1)
    Q = np.asarray(Q, dtype=np.float64).reshape(n, -1)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col_idx, dtype=np.int64)
    wv = np.ones(col.size) if w is None else np.asarray(w, dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    lab = components(n, row_ptr, col_idx)
    ncomp = int(lab.max()) + 1 if n else 0
    if int(np.sum(col != rows)) // 2 != n - ncomp:
        raise ValueError("not a forest")
    dbar = project(P - Q, lab)

    parent = np.full(n, -1, dtype=np.int64)
    pw = np.zeros(n)
    seen = np.zeros(n, dtype=bool)
    roots = np.unique(lab, return_index=True)[1]
    seen[roots] = True
    levels = [roots]
    frontier = roots
    while frontier.size:
        cnt = row_ptr[frontier + 1] - row_ptr[frontier]
        src = np.repeat(frontier, cnt)
        eidx = np.repeat(row_ptr[frontier], cnt) + (
            np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt))
        dst = col[eidx]
        new = ~seen[dst]
        # in a forest every unseen neighbour is reached from exactly one node
        src, dst, ew = src[new], dst[new], wv[eidx[new]]
        seen[dst] = True
        parent[dst] = src
        pw[dst] = ew
        frontier = dst
        if frontier.size:
            levels.append(frontier)

    f = dbar.copy()
    for lev in levels[:0:-1]:                      # deepest level first
        np.add.at(f, parent[lev], f[lev])
    x = np.zeros_like(dbar)
    for lev in levels[1:]:
        x[lev] = x[parent[lev]] + f[lev] / pw[lev, None]
    nonroot = parent >= 0
    dsq = np.sum(f[nonroot] ** 2 / pw[nonroot, None], axis=0)
    return {"d": np.sqrt(dsq), "dsq": dsq, "x": project(x, lab),
            "flow": f, "parent": parent}
