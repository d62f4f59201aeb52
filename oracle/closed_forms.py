"""Textbook effective resistances R_ij = d(e_i, e_j)^2 (route O6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

With a = e_i and b = e_j the GE distance squared is (e_i - e_j)^T L^+
(e_i - e_j), the effective resistance between i and j when every edge is a
resistor of conductance w.  These classical values pin the oracle routes.
"""
from __future__ import annotations

__all__ = ["path", "cycle", "complete", "star_center_leaf", "star_leaf_leaf",
           "bipartite_same_side", "bipartite_across", "tree_path"]


def path(i, j, w=1.0):
    """Path graph: series resistors, R = |i - j| / w."""
    return abs(i - j) / w


def cycle(n, i, j, w=1.0):
    """Cycle C_n: two parallel series arcs of lengths s and n-s,
    R = s (n - s) / (n w)."""
    s = abs(i - j) % n
    return s * (n - s) / (n * w)


def complete(n, w=1.0):
    """Complete graph K_n, any i != j: R = 2 / (n w)."""
    return 2.0 / (n * w)


def star_center_leaf(w=1.0):
    return 1.0 / w


def star_leaf_leaf(w=1.0):
    return 2.0 / w


def bipartite_same_side(a, b):
    """K_{a,b}, two nodes on the side of size a (unit weights): 2 / b."""
    return 2.0 / b


def bipartite_across(a, b):
    """K_{a,b}, one node per side (unit weights): (a + b - 1) / (a b)."""
    return (a + b - 1.0) / (a * b)


def tree_path(weights_on_path):
    """Weighted tree: series sum of 1/w over the unique i-j path."""
    return float(sum(1.0 / w for w in weights_on_path))
