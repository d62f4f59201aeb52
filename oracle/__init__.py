"""CPU FP64 oracle for the Generalized Euclidean (GE) node-vector distance.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.  The
GPU library never calls it, and it calls nothing of the GPU library: it shares
no code with it (inputs come from the separate ``nvdgen`` generators).

What it computes (paper, section 3.1): for an undirected graph with edge
weights w > 0, L = D - A with D the (weighted) degree matrix, and node vectors
a, b, the distance  d = sqrt((a-b)^T L^+ (a-b))  with L^+ the Moore-Penrose
pseudoinverse.  The paper replaces the pseudoinverse by a Laplacian solve
(section 3.2); the oracle instead writes the definition out:

* ``dense``      -- L^+ through the full eigendecomposition of L (the paper's
                    exact baseline, section 3.1: SVD of a symmetric PSD matrix
                    is its eigendecomposition).  Primary route, n <= ~5e3.
* ``grounded``   -- a second exact route: per component, delete the row/column
                    of one node and Cholesky-solve the SPD remainder.
* ``pcg``        -- textbook Jacobi-preconditioned CG in FP64 to a relative
                    residual of 1e-13, for sizes the dense routes cannot reach;
                    pinned by agreement with the exact routes.
* ``tree``       -- exact O(n) flow formula on trees (any size).
* ``cycle``      -- exact circulant (FFT) formula on cycles (any size).
* ``closed_forms`` -- textbook effective resistances (path, cycle, complete,
                    star, complete bipartite, weighted tree).
* ``grad``       -- gradients of d^2 with respect to a, b and the edge weights.
* ``pairwise``   -- all pairwise distances among m node vectors (dense and
                    per-pair PCG routes).

Parity status: every function here is pinned by tests against closed forms,
special cases, invariants or an independent route; none is "parity unpinned".
"""
from .laplacian import laplacian_dense, laplacian_sparse, components, project
from .dense import ge_dense
from .grounded import ge_grounded
from .pcg import ge_pcg
from .tree import ge_tree
from .cycle import ge_cycle
from . import closed_forms
from .grad import grad_dense
from .pairwise import pairwise_dense, pairwise_pcg

__all__ = ["laplacian_dense", "laplacian_sparse", "components", "project",
           "ge_dense", "ge_grounded", "ge_pcg", "ge_tree", "ge_cycle",
           "closed_forms", "grad_dense", "pairwise_dense", "pairwise_pcg"]

