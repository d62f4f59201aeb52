"""Writes the stored expected distances for the full-size workloads.

Calls only the CPU oracle (``oracle``) on inputs from the seeded generators
(``nvdgen``); nothing here touches the GPU library.  Usage:

    python tests/golden/make_golden.py c2      # BA n=1e6, m=3, 64 pairs
    python tests/golden/make_golden.py c4      # BA n=2e5, m=5, lognormal, 32 pairs
    python tests/golden/make_golden.py c5      # configuration model n=1e7, 16 pairs
    python tests/golden/make_golden.py c3      # 512 WS/BA graphs, 8 pairs each

Each output file records the workload recipe, the oracle route, its final
true relative residual per pair and the distances (repr of float64).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from nvdgen import workload  # noqa: E402

CFG = {"c2": 2, "c4": 4, "c5": 5}


def batch_main():
    """512-graph workload: dense route for n <= 4000, FP64 PCG route above."""
    t0 = time.time()
    w = workload(3)
    t1 = time.time()
    ds, relres, routes = [], [], []
    for g, P, Q in zip(w.graphs, w.P, w.Q):
        if g.n <= 4000:
            r = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
            relres += [0.0] * P.shape[1]
            routes.append("dense")
        else:
            r = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q, rtol=1e-13)
            relres += [float(v) for v in r["relres"]]
            routes.append("pcg")
        ds += [repr(float(v)) for v in r["d"]]
    t2 = time.time()
    out = {"workload": w.name, "config_index": 3, "graphs": len(w.graphs),
           "n_total": int(sum(g.n for g in w.graphs)),
           "nnz_total": int(sum(g.nnz for g in w.graphs)),
           "pairs": int(sum(P.shape[1] for P in w.P)),
           "oracle": "ge_dense (n <= 4000) / ge_pcg to 1e-13 (n > 4000), per graph",
           "routes": routes, "relres": relres, "d": ds,
           "seconds_generate": t1 - t0, "seconds_oracle": t2 - t1}
    path = os.path.join(HERE, "c3_expected.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: oracle {t2 - t1:.1f}s")


def main(name):
    c = CFG[name]
    t0 = time.time()
    w = workload(c)
    g = w.graphs[0]
    t1 = time.time()
    r = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, w.P[0], w.Q[0], rtol=1e-13)
    t2 = time.time()
    out = {
        "workload": w.name,
        "config_index": c,
        "n": g.n,
        "nnz": g.nnz,
        "pairs": int(w.P[0].shape[1]),
        "oracle": "ge_pcg (FP64 Jacobi-PCG, true relative residual <= 1e-13 or stagnation)",
        "relres": [float(v) for v in r["relres"]],
        "iters": [int(v) for v in r["iters"]],
        "d": [repr(float(v)) for v in r["d"]],
        "seconds_generate": t1 - t0,
        "seconds_oracle": t2 - t1,
    }
    path = os.path.join(HERE, f"{name}_expected.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: max relres {max(out['relres']):.2e}, oracle {t2 - t1:.1f}s")


if __name__ == "__main__":
    for a in sys.argv[1:]:
        if a == "c3":
            batch_main()
        else:
            main(a)
