"""The density sweep of section 4.2 ("Runtimes (Density)"): |V| = 10^4,
average degree 1 .. 64 on ER, BA, WS and SBM graphs, 8 pairs each, FP64 and
mixed precision against the oracle (the exact grounded route at average
degree <= 2, where CG is weakest and disconnected graphs with thousands of
components occur, the FP64 PCG route above)."""
import numpy as np
import pytest

import oracle
from nvdgen import density_graph, DENSITY_MODELS, DENSITY_DEGREES

from gpu_helpers import say, dev_graph, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("model", DENSITY_MODELS)
def test_density_sweep_matches_oracle(model):
    for d in DENSITY_DEGREES:
        g, P, Q = density_graph(model, d)
        if d <= 2:
            ref = oracle.ge_grounded(g.n, g.row_ptr, g.col_idx, None, P, Q, sparse=True)["d"]
        else:
            ref = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, None, P, Q)["d"]
        say("density", model, d, g.nnz)
        dg = dev_graph(g)
        for prec, rtol, tol in (("fp64", 1e-10, 1e-8), ("mixed", 1e-8, 1e-6)):
            dd, _, info = dg.distances(P, Q, precision=prec, rtol=rtol)
            e = rel_err(dd.cpu().numpy(), ref).max()
            assert e <= tol, (model, d, prec, e)
            assert all(i["status"] == 0 for i in info), (model, d, prec)
        dg.close()
