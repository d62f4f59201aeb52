"""Throughput benchmark: Generalized Euclidean node-vector distances per second.

Headline workload (one GPU): configuration-model graph with power-law degrees
(P(k) ~ k^-2.5, k in [3, 46415]), n0 = 10^7 restricted to its giant
component (n = 10^7, 7.57e7 CSR entries), unit weights; 16 vector pairs, each
p and q uniform[0,1) on an independent random 1% of the nodes; FP32 CG with
FP64 iterative refinement to a true relative residual of 1e-8 (the mixed
path, every distance within 1e-6 of the FP64 oracle), and the plain FP64 CG
solver to the same residual beside it.  One step = one nvd_distances call
over all 16 pairs (projection, CG, refinement, quadratic form), inputs
resident in HBM.

Prints one JSON line.  Also reported: the FP32 SpMM's algorithmic bytes per
launch over its event-timed duration (roofline; the events run on a repeat
of the timed steps, since recording them around every launch slows the steps
by a few per cent), the oracle's CPU rate on one pair of the same workload,
the distances' largest relative error against the stored oracle values
(tests/golden/c5_expected.json), and the other workloads as legs: the
1e3-node latency case, the 2e5-node forward + adjoint case, the 1e6-node
64-pair case (with all pairwise distances among its 64 vectors), the
512-graph batch, the density sweep, a 1e6-node tree and the reference
Laplacian applies on the 1e7-node graph.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _profile_fields(path):
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    return fields


# The sources that define the SpMM kernel's device code: the kernel, its
# device helpers and the device-side types (host-only declarations live
# elsewhere and do not change the kernel).
KERNEL_SOURCES = ("paper_2310_11222_amd/csrc/spmm.hip", "paper_2310_11222_amd/csrc/device_common.hpp",
                  "paper_2310_11222_amd/csrc/device_types.hpp")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for src in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def load_traffic(tile, workload="cm1e7_k16"):
    """HBM bytes per launch of the FP32 SpMM from the committed counter
    profile, if it was taken on the current kernel source at this tile."""
    p = os.path.join(ROOT, "profiles", f"k_spmm_f32_{workload}_T{tile}_traffic.md")
    if not os.path.exists(p):
        return None
    fields = _profile_fields(p)
    if fields.get("kernel_source_sha256") != kernel_source_sha():
        return None
    if f"k_spmm<float, {tile}," not in fields.get("kernel", ""):
        return None
    return float(fields["traffic_bytes_per_launch"])


def load_golden_file(name):
    p = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        g = json.load(f)
    import numpy as np
    return np.array([float(v) for v in g["d"]])


def bench_batched(steps, warmup):
    """512 connected graphs of uneven size (n log-uniform in [1e3, 1e5], half
    Watts-Strogatz k=6 beta=0.1, half Barabasi-Albert m=4, weights
    uniform[0.5, 2)), 8 pairs each, FP32 CG + FP64 refinement to 1e-8, all
    4096 distances per call: the sweep solver (value), the single persistent
    launch replayed from a hipGraph, and the plain FP64 solver called one
    graph at a time."""
    import numpy as np
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import workload
    t0 = time.perf_counter()
    w = workload(3)
    log(f"batched workload: {len(w.graphs)} graphs, n_total={sum(g.n for g in w.graphs)}, "
        f"gen {time.perf_counter() - t0:.1f}s")
    dgs = [nvd.Graph(g.row_ptr, g.col_idx, g.w) for g in w.graphs]
    batch = nvd.Batch(dgs)
    packed = batch.pack(w.P, w.Q)
    K = int(packed[0].sum())
    out = torch.empty(K, dtype=torch.float64, device="cuda")
    def timed(persistent):
        for _ in range(warmup):
            batch.distances(None, None, packed=packed, out=out, rtol=w.rtol, persistent=persistent)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            d, _, info = batch.distances(None, None, packed=packed, out=out, rtol=w.rtol,
                                         persistent=persistent)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return d.cpu().numpy(), info, t1 - t0

    dp, _, tp = timed(True)
    d, info, tsw = timed(False)
    value = K * steps / tsw
    # plain FP64 solver, one graph at a time, same GPU
    t2 = time.perf_counter()
    d64 = []
    for dg, P, Q in zip(dgs, w.P, w.Q):
        dd, _, _ = dg.distances(P, Q, precision="fp64", rtol=w.rtol)
        d64.append(dd)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    d64 = torch.cat(d64).cpu().numpy()
    gold = load_golden_file("c3_expected.json")
    res = {"workload": "batch512_ws_k6_ba_m4_k8", "solver": "sweep", "value": round(value, 1),
           "unit": "distances/s", "ms_per_step": round(tsw * 1e3 / steps, 3), "pairs": K,
           "persistent": {"value": round(K * steps / tp, 1), "unit": "distances/s",
                          "ms_per_step": round(tp * 1e3 / steps, 3), "graph_launch": batch.query(),
                          "max_rel_err": None},
           "iters_mean": float(np.mean([i["iters"] for i in info])),
           "fp64_one_graph_at_a_time": {"value": round(K / (t3 - t2), 1), "unit": "distances/s"},
           "max_rel_err": None, "max_rel_err_fp64": None}
    if gold is not None and gold.size == K:
        res["max_rel_err"] = float(np.max(np.abs(d - gold) / gold))
        res["persistent"]["max_rel_err"] = float(np.max(np.abs(dp - gold) / gold))
        res["max_rel_err_fp64"] = float(np.max(np.abs(d64 - gold) / gold))
    log(f"batched: {res}")
    batch.close()
    for dg in dgs:
        dg.close()
    return res


def bench_density():
    """Section 4.2 density sweep: |V| = 10^4, average degree 1..64 on ER, BA,
    WS and SBM, 8 pairs per graph, mixed precision to 1e-8 (the time of one
    call after a warm-up call, and the largest CG iteration count), with the
    Jacobi diagonal, the spanning-tree preconditioner and the
    approximate-Cholesky factor (section 3.2; the forest and the factor are
    built by the warm-up call, whose time is not counted)."""
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import density_graph, DENSITY_MODELS, DENSITY_DEGREES
    out = {}
    for model in DENSITY_MODELS:
        rows = []
        for d in DENSITY_DEGREES:
            g, P, Q = density_graph(model, d)
            dg = nvd.Graph(g.row_ptr, g.col_idx, None)
            Pd = torch.as_tensor(P).cuda()
            Qd = torch.as_tensor(Q).cuda()
            row = {"avg_degree": d, "components": dg.stats()["n_comp"]}
            for pre, key in (("jacobi", ""), ("tree", "tree_"), ("achol", "achol_")):
                dg.distances(Pd, Qd, precision="mixed", rtol=1e-8, precond=pre)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, info = dg.distances(Pd, Qd, precision="mixed", rtol=1e-8, precond=pre)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                row[key + "ms_per_8"] = round(t * 1e3, 3)
                row[key + "converged"] = all(i["status"] == 0 for i in info)
                row[key + "iters"] = max(i["iters"] for i in info)
            st = dg.stats()
            row["achol_rounds"] = st["achol_rounds"]
            row["achol_remainder"] = st["achol_remainder"]
            rows.append(row)
            dg.close()
        out[model] = rows
    log("density sweep (ms per 8 distances, jacobi / tree / achol): " +
        json.dumps({m: [(r["ms_per_8"], r["tree_ms_per_8"], r["achol_ms_per_8"]) for r in v]
                    for m, v in out.items()}))
    return {"workload": "density_sweep_n1e4_deg1_to_64", "models": out}


def bench_tree_large():
    """A 10^6-node tree-like graph (Barabasi-Albert with one link per new
    node: a tree), 16 pairs on 5% supports, mixed precision to 1e-8: the
    Jacobi diagonal against the spanning-forest preconditioner (the time of
    one call after a warm-up call, which also builds the forest)."""
    import numpy as np
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import barabasi_albert, sparse_support_pairs
    rng = np.random.default_rng(np.random.SeedSequence([2310, 11222, 77]))
    g = barabasi_albert(1_000_000, 1, rng)
    P, Q = sparse_support_pairs(g.n, 16, 0.05, rng)
    dg = nvd.Graph(g.row_ptr, g.col_idx, None)
    Pd = torch.as_tensor(P).cuda()
    Qd = torch.as_tensor(Q).cuda()
    res = {"workload": "ba_tree_n1e6_m1_k16", "n": g.n, "nnz": g.nnz, "pairs": 16}
    ds = {}
    for pre in ("jacobi", "tree"):
        dg.distances(Pd, Qd, precision="mixed", rtol=1e-8, precond=pre)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, _, info = dg.distances(Pd, Qd, precision="mixed", rtol=1e-8, precond=pre)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ds[pre] = d.cpu().numpy()
        res[pre] = {"ms_per_call": round(t * 1e3, 3), "distances_per_s": round(16 / t, 1),
                    "iters": max(i["iters"] for i in info),
                    "converged": all(i["status"] == 0 for i in info)}
    res["max_rel_diff_tree_vs_jacobi"] = float(np.max(np.abs(ds["tree"] - ds["jacobi"]) / ds["jacobi"]))
    dg.close()
    log("tree-like graph: " + json.dumps(res))
    return res


def bench_spmv(calib_copy=False, g=None):
    """The reference SpMV loads for the HBM claim: Y = L X on the 10^7-node
    power-law configuration-model graph (unit weights), k = 1 and 16 columns,
    FP32 and FP64, 100 back-to-back launches each (time per launch from HIP
    events around the 100).  Algorithmic bytes: 4 nnz + 4 (n+1) + 2 k s n.
    k = 1 runs the apply by column slices (the default at this size) and,
    for comparison, the row-wise apply (NVD_SLICE=0)."""
    import numpy as np
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import workload
    if g is None:
        t0 = time.perf_counter()
        g = workload(5).graphs[0]
        log(f"spmv graph: n={g.n} nnz={g.nnz} gen {time.perf_counter() - t0:.1f}s")
    dg = nvd.Graph(g.row_ptr, g.col_idx, None)
    if calib_copy:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    rows = []
    for k, dt, name, path in ((1, torch.float32, "f32", "sliced"), (1, torch.float64, "f64", "sliced"),
                              (1, torch.float32, "f32", "row-wise"), (1, torch.float64, "f64", "row-wise"),
                              (16, torch.float32, "f32", "row-wise"), (16, torch.float64, "f64", "row-wise")):
        if k == 1 and path == "row-wise":
            os.environ["NVD_SLICE"] = "0"
        X = torch.rand(g.n, k, dtype=dt, device="cuda", generator=gen)
        Y = torch.empty_like(X)
        for _ in range(5):
            dg.laplacian_apply(X, out=Y)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(100):
            dg.laplacian_apply(X, out=Y)
        b.record()
        b.synchronize()
        us = a.elapsed_time(b) / 100 * 1e3
        alg = 4.0 * g.nnz + 4.0 * (g.n + 1) + 2.0 * k * X.element_size() * g.n
        os.environ.pop("NVD_SLICE", None)
        rows.append({"k": k, "dtype": name, "path": path, "us_per_launch": round(us, 1),
                     "algorithmic_bytes": alg, "achieved_gbs": round(alg / us / 1e3, 1),
                     "frac": round(alg / us / 1e3 / HBM_PEAK_GBS, 4)})
        del X, Y
    dg.close()
    res = {"workload": "config_model_n1e7_unit_laplacian_apply", "n": g.n, "nnz": g.nnz,
           "launches": rows, "traffic_k1_f32": load_spmv_traffic(),
           "traffic_k1_f32_sliced": load_slice_traffic()}
    log("spmv: " + json.dumps(res))
    return res


def bench_single_pair(dg, P, Q, rtol, golden, reps=3):
    """One distance at a time on the 10^7-node graph (the paper's per-distance
    setting, Table 2): pair 0 of the headline, mixed precision, tile of one
    column, with the apply by column slices (default at this size) and with
    the row-wise apply (NVD_SLICE=0).  The first sliced call builds the
    slices (its time is reported apart)."""
    import numpy as np
    import torch
    p, q = P[:, :1].contiguous(), Q[:, :1].contiguous()
    res = {"workload": "cm_pl2.5_n1e7_pair0", "precision": "mixed", "tile": 1}
    for path in ("sliced", "row-wise"):
        if path == "row-wise":
            os.environ["NVD_SLICE"] = "0"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, _, info = dg.distances(p, q, precision="mixed", rtol=rtol, tile_k=1)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(reps):
            d, _, info = dg.distances(p, q, precision="mixed", rtol=rtol, tile_k=1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        os.environ.pop("NVD_SLICE", None)
        err = None if golden is None else float(abs(d.cpu().numpy()[0] - golden[0]) / golden[0])
        res[path] = {"ms_per_distance": round(ms, 2), "first_call_ms": round(first * 1e3, 1),
                     "iters": info[0]["iters"], "rel_err_vs_oracle": err}
    log("single pair: " + json.dumps(res))
    return res


SLICE_SOURCES = ("paper_2310_11222_amd/csrc/slice.hip", "paper_2310_11222_amd/csrc/device_common.hpp",
                 "paper_2310_11222_amd/csrc/device_types.hpp")


def slice_source_sha():
    import hashlib
    h = hashlib.sha256()
    for src in SLICE_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def load_slice_traffic():
    """Counter bytes per k = 1 FP32 apply by column slices (slice pass plus
    combine) on the 10^7-node graph, from the committed profile, if taken on
    the current source."""
    p = os.path.join(ROOT, "profiles", "k_slice_f32_configmodel1e7_k1_traffic.md")
    if not os.path.exists(p):
        return None
    fields = _profile_fields(p)
    if fields.get("kernel_source_sha256") != slice_source_sha():
        return None
    return float(fields["traffic_bytes_per_launch"])


def load_spmv_traffic():
    """Counter bytes per launch of the k = 1 FP32 apply on the 10^7-node
    graph, from the committed profile, if taken on the current source."""
    p = os.path.join(ROOT, "profiles", "k_spmm_f32_configmodel1e7_k1_traffic.md")
    if not os.path.exists(p):
        return None
    fields = _profile_fields(p)
    if fields.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return float(fields["traffic_bytes_per_launch"])


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count()}


def cpu_baseline(w, pairs, iters=10):
    """The oracle's FP64 Jacobi-PCG route (unmodified) on the first `pairs`
    pairs of the same workload, with every thread pool held to one thread
    (SciPy's sparse product is single-threaded anyway), bounded in time: its
    set-up (components, projection, sparse Laplacian) runs in full and its
    PCG runs `iters` iterations (the routine's own max_iter); the time per
    distance is the set-up plus the PCG time scaled to the iteration count
    the oracle needs on these pairs to reach its 1e-13 true relative
    residual, as recorded in the stored oracle run."""
    import numpy as np
    import oracle
    from oracle.pcg import pcg_solve
    from threadpoolctl import threadpool_limits
    g = w.graphs[0]
    P = np.ascontiguousarray(w.P[0][:, :pairs])
    Q = np.ascontiguousarray(w.Q[0][:, :pairs])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        lab = oracle.components(g.n, g.row_ptr, g.col_idx)
        dbar = oracle.project(P - Q, lab)
        L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.w)
        deg = L.diagonal()
        t1 = time.perf_counter()
        pcg_solve(L, deg, dbar, max_iter=iters)
        t2 = time.perf_counter()
    gold = os.path.join(ROOT, "tests", "golden", "c5_expected.json")
    full = int(max(json.load(open(gold))["iters"][:pairs]))
    t_pairs = (t1 - t0) + (t2 - t1) * full / iters
    return {"rate": pairs / t_pairs, "setup_s": t1 - t0, "pcg_s": t2 - t1, "iters_run": iters,
            "iters_full": full, "seconds_measured": t2 - t0}


def bench_c1(reps=50):
    """Latency on the 1e3-node BA graph (m = 3, unit weights), one pair, FP64
    CG to 1e-10 (and the mixed path beside it): median wall time of a call
    over `reps` calls after warm-up, against the dense oracle."""
    import numpy as np
    import torch
    import oracle
    import paper_2310_11222_amd as nvd
    from nvdgen import workload
    w = workload(1)
    g = w.graphs[0]
    ref = oracle.ge_dense(g.n, g.row_ptr, g.col_idx, g.w, w.P[0], w.Q[0])["d"]
    dg = nvd.Graph(g.row_ptr, g.col_idx, g.w)
    P = torch.as_tensor(w.P[0]).cuda()
    Q = torch.as_tensor(w.Q[0]).cuda()
    res = {"workload": "ba_n1e3_m3_unit_k1", "n": g.n, "nnz": g.nnz, "pairs": 1}
    for prec, rtol in (("fp64", 1e-10), ("mixed", 1e-10)):
        for _ in range(5):
            dg.distances(P, Q, precision=prec, rtol=rtol)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            d, _, info = dg.distances(P, Q, precision=prec, rtol=rtol)
            ts.append(time.perf_counter() - t0)
        med = float(np.median(ts))
        res[prec] = {"us_per_call_median": round(med * 1e6, 1),
                     "us_per_call_mean": round(float(np.mean(ts)) * 1e6, 1),
                     "distances_per_s": round(1.0 / med, 1), "iters": info[0]["iters"],
                     "rel_err_vs_dense_oracle": float(abs(d.cpu().numpy()[0] - ref[0]) / ref[0])}
    dg.close()
    log("c1 latency: " + json.dumps(res))
    return res


def bench_c4(steps=3):
    """Forward + adjoint on the 2e5-node BA graph (m = 5, lognormal(0, 1)
    weights), 32 pairs, FP64 CG to 1e-10: loss = sum of d^2, gradients with
    respect to P, Q and every edge weight (the per-edge weights are gathered
    into CSR order, so autograd adds the two stored directions).  Time per
    step (forward, backward), distances against the stored oracle values."""
    import numpy as np
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import workload
    w = workload(4)
    g = w.graphs[0]
    ew = np.zeros(g.num_edges)
    ew[g.csr_edge] = g.w
    dg = nvd.Graph(g.row_ptr, g.col_idx, g.w)
    idx = torch.as_tensor(g.csr_edge, device="cuda")
    P0 = torch.as_tensor(w.P[0]).cuda()
    Q0 = torch.as_tensor(w.Q[0]).cuda()
    W0 = torch.as_tensor(ew).cuda()

    def step():
        P = P0.clone().requires_grad_(True)
        Q = Q0.clone().requires_grad_(True)
        W = W0.clone().requires_grad_(True)
        t0 = time.perf_counter()
        dsq = nvd.distance_sq(P, Q, dg, W[idx], precision="fp64", rtol=w.rtol)
        loss = dsq.sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return dsq.detach(), t1 - t0, t2 - t1

    step()
    tf, tb = [], []
    for _ in range(steps):
        dsq, a, b = step()
        tf.append(a)
        tb.append(b)
    gold = load_golden_file("c4_expected.json")
    d = np.sqrt(dsq.cpu().numpy())
    res = {"workload": "ba_n2e5_m5_lognormal_k32", "n": g.n, "nnz": g.nnz, "pairs": 32,
           "forward_ms": round(float(np.median(tf)) * 1e3, 3),
           "backward_ms": round(float(np.median(tb)) * 1e3, 3),
           "step_ms": round(float(np.median(np.add(tf, tb))) * 1e3, 3),
           "distances_per_s_with_gradients": round(32 / float(np.median(np.add(tf, tb))), 1),
           "max_rel_err": None}
    if gold is not None and gold.size == d.size:
        res["max_rel_err"] = float(np.max(np.abs(d - gold) / gold))
    dg.close()
    log("c4 forward+adjoint: " + json.dumps(res))
    return res


def bench_c2(steps, inner_rtol, no_pairwise):
    """The 1e6-node BA graph (m = 3, unit weights), 64 pairs on 5% supports,
    mixed and FP64 to 1e-8, and all 2,016 pairwise distances among the 64
    vectors P_j from one 64-column solve."""
    import numpy as np
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import workload
    w = workload(2)
    g = w.graphs[0]
    dg = nvd.Graph(g.row_ptr, g.col_idx, g.w)
    P = torch.as_tensor(w.P[0]).cuda()
    Q = torch.as_tensor(w.Q[0]).cuda()
    K = P.shape[1]
    gold = load_golden_file("c2_expected.json")
    res = {"workload": "ba_n1e6_m3_unit_k64", "n": g.n, "nnz": g.nnz, "pairs": K}
    for prec, nsteps in (("mixed", steps), ("fp64", max(1, steps // 2))):
        dg.distances(P, Q, precision=prec, rtol=w.rtol, inner_rtol=inner_rtol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            d, _, info = dg.distances(P, Q, precision=prec, rtol=w.rtol, inner_rtol=inner_rtol)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / nsteps
        dn = d.cpu().numpy()
        res[prec] = {"value": round(K / t, 1), "unit": "distances/s", "ms_per_step": round(t * 1e3, 3),
                     "iters_mean": float(np.mean([i["iters"] for i in info])),
                     "max_rel_err": float(np.max(np.abs(dn - gold) / gold)) if gold is not None else None}
    res["tile"] = dg.tuning(K, "mixed")[0]
    # the approximate-Cholesky preconditioner on the same graph and pairs
    t0 = time.perf_counter()
    dg.distances(P[:, :1], Q[:, :1], precision="mixed", rtol=w.rtol, precond="achol")
    torch.cuda.synchronize()
    t_fac = time.perf_counter() - t0
    t0 = time.perf_counter()
    d, _, info = dg.distances(P, Q, precision="mixed", rtol=w.rtol, precond="achol")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st = dg.stats()
    dn = d.cpu().numpy()
    res["mixed_achol"] = {"value": round(K / t, 1), "unit": "distances/s", "ms_per_step": round(t * 1e3, 3),
                          "iters_mean": float(np.mean([i["iters"] for i in info])),
                          "factor_and_first_call_s": round(t_fac, 3), "rounds": st["achol_rounds"],
                          "factor_nnz": st["achol_factor_nnz"], "remainder": st["achol_remainder"],
                          "max_rel_err": float(np.max(np.abs(dn - gold) / gold)) if gold is not None else None}
    if not no_pairwise:
        m = K
        npairs = m * (m - 1) // 2
        dg.pairwise(P, precision="mixed", rtol=w.rtol)
        torch.cuda.synchronize()
        reps = max(1, min(steps, 3))
        t0 = time.perf_counter()
        for _ in range(reps):
            D, _, _ = dg.pairwise(P, precision="mixed", rtol=w.rtol)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / reps
        # 8 sampled entries against pairs solved one by one (FP64)
        iu, ju = np.triu_indices(m, 1)
        pick = np.random.default_rng(0).choice(npairs, 8, replace=False)
        ii = torch.as_tensor(iu[pick], device="cuda")
        jj = torch.as_tensor(ju[pick], device="cuda")
        dpair, _, _ = dg.distances(P[:, ii].contiguous(), P[:, jj].contiguous(), precision="fp64",
                                   rtol=1e-10)
        Dn = D.cpu().numpy()
        diff = float(np.max(np.abs(Dn[iu[pick], ju[pick]] - dpair.cpu().numpy()) / dpair.cpu().numpy()))
        res["all_pairs"] = {"vectors": m, "pairs": npairs, "value": round(npairs / tp, 1),
                            "unit": "distances/s", "ms_per_call": round(tp * 1e3, 3),
                            "precision": "mixed", "max_rel_diff_vs_pair_solves": diff}
    dg.close()
    log("c2: " + json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-pairs", type=int, default=1,
                    help="pairs of the headline workload the CPU oracle solves (0: none)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--inner-rtol", type=float, default=1e-5)
    ap.add_argument("--no-legs", action="store_true",
                    help="headline only (for profiling): skip every other workload")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 1e3-node latency and the 2e5-node adjoint legs")
    ap.add_argument("--no-c2", action="store_true", help="skip the 1e6-node 64-pair leg")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-pairwise", action="store_true")
    ap.add_argument("--no-density", action="store_true",
                    help="skip the density sweep and the 1e6-node tree-like graph")
    ap.add_argument("--no-spmv", action="store_true",
                    help="skip the reference SpMV loads on the 1e7-node graph")
    ap.add_argument("--spmv-only", action="store_true",
                    help="run only the reference SpMV loads (for profiling) and print them")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 512 MiB device copy first (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "a layout across GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import workload

    torch.cuda.set_device(0)
    if args.spmv_only:
        print(json.dumps(bench_spmv(args.calib_copy)), flush=True)
        return
    if args.calib_copy:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 536870912 bytes read, 536870912 bytes written")
    log("generating the headline workload")
    t0 = time.perf_counter()
    w = workload(5)
    g = w.graphs[0]
    log(f"n={g.n} nnz={g.nnz} gen {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    dg = nvd.Graph(g.row_ptr, g.col_idx, g.w)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    P = torch.as_tensor(w.P[0]).cuda()
    Q = torch.as_tensor(w.Q[0]).cuda()
    K = P.shape[1]
    rtol = w.rtol
    golden = load_golden_file("c5_expected.json")

    def step(prec):
        return dg.distances(P, Q, precision=prec, rtol=rtol, inner_rtol=args.inner_rtol,
                            tile_k=args.tile)

    # ---- mixed precision (headline).  The timed steps run without per-kernel
    # events; the kernel durations for the roofline come from the same steps
    # repeated with them.
    t0 = time.perf_counter()
    tile_used = args.tile or dg.tuning(K, "mixed")[0]
    tune_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        d, _, info = step("mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d, _, info = step("mixed")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"mixed: {(t1 - t0) * 1e3 / args.steps:.2f} ms/step")
    nvd.prof_enable(True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step("mixed")
    torch.cuda.synchronize()
    prof = nvd.prof_read()
    nvd.prof_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = K * args.steps / (t1 - t0)
    d_mixed = d.cpu().numpy()
    iters_mixed = [i["iters"] for i in info]
    refine = [i["refine_steps"] for i in info]
    log(f"mixed: {ms_step:.2f} ms/step, {value:.1f} distances/s, iters {np.mean(iters_mixed):.1f}, "
        f"refine {np.mean(refine):.2f}")

    # ---- plain FP64 solver on the same GPU
    d64, _, info64 = step("fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.fp64_steps):
        d64, _, info64 = step("fp64")
    torch.cuda.synchronize()
    t64 = (time.perf_counter() - t0) / args.fp64_steps
    value64 = K / t64
    d64 = d64.cpu().numpy()
    log(f"fp64: {t64 * 1e3:.2f} ms/step, {value64:.1f} distances/s")

    # ---- accuracy vs stored oracle values
    acc = {"max_rel_err_mixed": None, "max_rel_err_fp64": None, "within_1e-6": None}
    if golden is not None and golden.size == K:
        acc["max_rel_err_mixed"] = float(np.max(np.abs(d_mixed - golden) / golden))
        acc["max_rel_err_fp64"] = float(np.max(np.abs(d64 - golden) / golden))
        acc["within_1e-6"] = bool(acc["max_rel_err_mixed"] <= 1e-6)
    log(f"accuracy {acc}")

    # ---- roofline of the dominant kernel (SpMM, FP32 in the inner solves)
    def kern(name):
        p = prof[name]
        if p["launches"] == 0:
            return None
        avg_ms = p["ms"] / p["launches"]
        bytes_per = p["bytes"] / p["launches"]
        return {"avg_us": avg_ms * 1e3, "bytes_per_launch": bytes_per,
                "gbs": bytes_per / (avg_ms * 1e-3) / 1e9, "launches": p["launches"],
                "ms_total": p["ms"]}

    kinds = {k: kern(k) for k in prof}
    dom = max((k for k in kinds if kinds[k]), key=lambda k: kinds[k]["ms_total"])
    sp = kinds["spmm_f32"]
    roof = {"kernel": f"k_spmm<float, {tile_used}> (EPI_CG: q = L p and p^T q)", "bound": "hbm",
            "achieved": round(sp["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(sp["gbs"] / HBM_PEAK_GBS, 4), "traffic": load_traffic(tile_used),
            "bytes_per_launch": sp["bytes_per_launch"], "avg_launch_us": round(sp["avg_us"], 2),
            "bytes_formula": "4 nnz + 4 (n + 1) + 2 T 4 n (CSR once, p read once, q written once)",
            "timing": "HIP events on the launch stream around every launch, over a repeat of the timed "
                      "steps (value is timed without them)"}
    log(f"kernels: " + json.dumps({k: (round(v['gbs'], 1), round(v['ms_total'], 2)) for k, v in kinds.items() if v}))

    # ---- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu and args.cpu_pairs > 0:
        cb = cpu_baseline(w, args.cpu_pairs)
        cpu = {"value": round(cb["rate"], 5), "unit": "distances/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {args.cpu_pairs} of the 16 pairs of the same workload through "
                         f"the oracle's FP64 Jacobi-PCG route on one thread: set-up (components, "
                         f"projection, sparse Laplacian) {cb['setup_s']:.1f} s in full, then "
                         f"{cb['iters_run']} PCG iterations in {cb['pcg_s']:.1f} s, scaled to the "
                         f"{cb['iters_full']} iterations the oracle takes to its 1e-13 residual on "
                         f"these pairs (stored oracle run)",
               "host": host_info(), "threads": 1,
               "seconds_measured": round(cb["seconds_measured"], 1)}
        log(f"cpu oracle {cb['rate']:.5f} distances/s ({cb['seconds_measured']:.1f}s measured)")

    single = None if (args.no_legs or args.no_spmv) else bench_single_pair(dg, P, Q, rtol, golden)
    small = None if (args.no_legs or args.no_small) else {"c1_latency": bench_c1(),
                                                          "c4_forward_adjoint": bench_c4()}
    spmv = None
    if not (args.no_legs or args.no_spmv):
        torch.cuda.empty_cache()
        spmv = bench_spmv(g=g)
    dg.close()
    del P, Q
    torch.cuda.empty_cache()
    c2 = None if (args.no_legs or args.no_c2) else bench_c2(args.steps, args.inner_rtol, args.no_pairwise)
    density = None if (args.no_legs or args.no_density) else bench_density()
    tree_large = None if (args.no_legs or args.no_density) else bench_tree_large()
    batched = None
    if not (args.no_legs or args.no_batched):
        torch.cuda.empty_cache()
        batched = bench_batched(max(2, args.steps // 2), 1)

    out = {
        "metric": "NVD distances/sec at rel err <=1e-6 vs FP64 oracle; SpMV HBM GB/s % of peak",
        "value": round(value, 2),
        "unit": "distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "cm_pl2.5_n1e7_k16", "n": g.n, "nnz": g.nnz, "pairs": K,
                   "rtol": rtol, "precision": "mixed (FP32 CG + FP64 refinement)",
                   "inner_rtol": args.inner_rtol, "tile": tile_used,
                   "tile_chosen_by": "option" if args.tile else "autotuner"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_path": {"value": round(value64, 2), "unit": "distances/s",
                      "ms_per_step": round(t64 * 1e3, 3)},
        "accuracy": acc,
        "legs": {"small": small, "c2": c2, "batched": batched, "density_sweep": density,
                 "tree_like_1e6": tree_large, "spmv_reference": spmv, "single_pair_1e7": single},
        "iters_mean": float(np.mean(iters_mixed)),
        "refine_mean": float(np.mean(refine)),
        "setup_s": round(setup_s, 3),
        "tune_s": round(tune_s, 3),
        "kernels": {k: v for k, v in kinds.items() if v},
        "dominant_kernel": dom,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
