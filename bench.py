"""Throughput benchmark: Generalized Euclidean node-vector distances per second.

Workload (one GPU): Barabasi-Albert graph, n = 1,000,000, m = 3, unit
weights; 64 vector pairs, each p and q uniform[0,1) on an independent random
5% of the nodes; FP32 CG with FP64 iterative refinement to a true relative
residual of 1e-8 (the headline path), and the plain FP64 CG solver to the
same residual beside it.  One step = one nvd_distances call over all 64
pairs (projection, CG, refinement, quadratic form), inputs resident in HBM.

Prints one JSON line.  Also reported: the SpMM kernel's algorithmic bytes
per launch over its event-timed duration (roofline; the events run on a
repeat of the timed steps, since recording them around every launch slows
the steps by ~7%), the oracle's CPU rate
on a bounded sample, and the distances' largest relative error against the
stored oracle values (tests/golden/c2_expected.json).
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


def load_golden():
    p = os.path.join(ROOT, "tests", "golden", "c2_expected.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        g = json.load(f)
    import numpy as np
    return np.array([float(v) for v in g["d"]])


def load_traffic(tile):
    """HBM bytes per launch of the FP32 SpMM from the committed counter
    profile, if it was taken on the current kernel source at this tile."""
    import hashlib
    p = os.path.join(ROOT, "profiles", f"k_spmm_f32_ba1e6_k64_T{tile}_traffic.md")
    if not os.path.exists(p):
        return None
    fields = {}
    for line in open(p):
        if ":" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in ("paper_2310_11222_amd/csrc/spmm.hip", "paper_2310_11222_amd/csrc/device_common.hpp",
                "paper_2310_11222_amd/csrc/nvd_internal.hpp"):
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    if f"k_spmm<float, {tile}," not in fields.get("kernel", ""):
        return None
    return float(fields["traffic_bytes_per_launch"])


def load_golden_batch():
    p = os.path.join(ROOT, "tests", "golden", "c3_expected.json")
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
    gold = load_golden_batch()
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
    Jacobi diagonal and with the spanning-tree preconditioner (section 3.2;
    the forest is built by the warm-up call)."""
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
            for pre, key in (("jacobi", ""), ("tree", "tree_")):
                dg.distances(Pd, Qd, precision="mixed", rtol=1e-8, precond=pre)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, info = dg.distances(Pd, Qd, precision="mixed", rtol=1e-8, precond=pre)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                row[key + "ms_per_8"] = round(t * 1e3, 3)
                row[key + "converged"] = all(i["status"] == 0 for i in info)
                row[key + "iters"] = max(i["iters"] for i in info)
            rows.append(row)
            dg.close()
        out[model] = rows
    log("density sweep (ms per 8 distances, jacobi / tree): " +
        json.dumps({m: [(r["ms_per_8"], r["tree_ms_per_8"]) for r in v] for m, v in out.items()}))
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


def bench_spmv(calib_copy=False):
    """The reference SpMV loads for the HBM claim: Y = L X on the 10^7-node
    power-law configuration-model graph (unit weights), k = 1 and 16 columns,
    FP32 and FP64, 100 back-to-back launches each (time per launch from HIP
    events around the 100).  Algorithmic bytes: 4 nnz + 4 (n+1) + 2 k s n."""
    import numpy as np
    import torch
    import paper_2310_11222_amd as nvd
    from nvdgen import workload
    t0 = time.perf_counter()
    w = workload(5)
    g = w.graphs[0]
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
    for k, dt, name in ((1, torch.float32, "f32"), (1, torch.float64, "f64"),
                        (16, torch.float32, "f32"), (16, torch.float64, "f64")):
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
        rows.append({"k": k, "dtype": name, "us_per_launch": round(us, 1),
                     "algorithmic_bytes": alg, "achieved_gbs": round(alg / us / 1e3, 1),
                     "frac": round(alg / us / 1e3 / HBM_PEAK_GBS, 4)})
        del X, Y
    dg.close()
    res = {"workload": "config_model_n1e7_unit_laplacian_apply", "n": g.n, "nnz": g.nnz,
           "launches": rows, "traffic_k1_f32": load_spmv_traffic()}
    log("spmv: " + json.dumps(res))
    return res


def load_spmv_traffic():
    """Counter bytes per launch of the k = 1 FP32 apply on the 10^7-node
    graph, from the committed profile, if taken on the current source."""
    import hashlib
    p = os.path.join(ROOT, "profiles", "k_spmm_f32_configmodel1e7_k1_traffic.md")
    if not os.path.exists(p):
        return None
    fields = {}
    for line in open(p):
        if ":" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in ("paper_2310_11222_amd/csrc/spmm.hip", "paper_2310_11222_amd/csrc/device_common.hpp",
                "paper_2310_11222_amd/csrc/nvd_internal.hpp"):
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(w, pairs):
    """The oracle (FP64 Jacobi-PCG route, unmodified defaults) on `pairs`
    pairs of the same workload, single-threaded."""
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_limits
    g = w.graphs[0]
    P = np.ascontiguousarray(w.P[0][:, :pairs])
    Q = np.ascontiguousarray(w.Q[0][:, :pairs])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = oracle.ge_pcg(g.n, g.row_ptr, g.col_idx, g.w, P, Q)
        t1 = time.perf_counter()
    return pairs / (t1 - t0), t1 - t0, r["d"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-pairs", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--inner-rtol", type=float, default=1e-5)
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
    log("generating workload")
    t0 = time.perf_counter()
    w = workload(2)
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
    golden = load_golden()

    def step(prec):
        return dg.distances(P, Q, precision=prec, rtol=rtol, inner_rtol=args.inner_rtol,
                            tile_k=args.tile)

    # ---- mixed precision (headline).  The timed steps run without per-kernel
    # events (recording two events around every launch costs ~7%); the kernel
    # durations for the roofline come from the same steps repeated with them.
    for _ in range(args.warmup):
        d, _, info = step("mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d, _, info = step("mixed")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
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
    log(f"mixed: {ms_step:.2f} ms/step, {value:.1f} distances/s, iters {np.mean(iters_mixed):.1f}, refine {np.mean(refine):.2f}")

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
    acc = {}
    if golden is not None and golden.size == K:
        acc["max_rel_err_mixed"] = float(np.max(np.abs(d_mixed - golden) / golden))
        acc["max_rel_err_fp64"] = float(np.max(np.abs(d64 - golden) / golden))
    else:
        acc["max_rel_err_mixed"] = None
        acc["max_rel_err_fp64"] = None
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

    tile_used = args.tile or dg.tuning(K, "mixed")[0]
    kinds = {k: kern(k) for k in prof}
    dom = max((k for k in kinds if kinds[k]), key=lambda k: kinds[k]["ms_total"])
    sp = kinds["spmm_f32"]
    roof = {"kernel": f"k_spmm<float, {tile_used}> (EPI_CG: q = L p and p^T q)", "bound": "hbm",
            "achieved": round(sp["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(sp["gbs"] / HBM_PEAK_GBS, 4), "traffic": load_traffic(tile_used),
            "bytes_per_launch": sp["bytes_per_launch"], "avg_launch_us": round(sp["avg_us"], 2),
            "timing": "HIP events on the launch stream around every launch, over a repeat of the timed "
                      "steps (value is timed without them)"}
    log(f"kernels: " + json.dumps({k: (round(v['gbs'], 1), round(v['ms_total'], 2)) for k, v in kinds.items() if v}))

    # ---- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu and args.cpu_pairs > 0:
        rate, secs, dref = cpu_baseline(w, args.cpu_pairs)
        cpu = {"value": round(rate, 4), "unit": "distances/s", "cores": 1, "kind": "oracle",
               "sample": f"first {args.cpu_pairs} of the 64 pairs, FP64 Jacobi-PCG oracle route "
                         f"(true rel. residual 1e-13), {secs:.1f} s single-threaded"}
        log(f"cpu oracle {rate:.3f} distances/s ({secs:.1f}s)")

    # ---- all pairwise distances among the 64 vectors P_j (one 64-column solve)
    all_pairs = None
    if not args.no_pairwise:
        m = P.shape[1]
        npairs = m * (m - 1) // 2
        dg.pairwise(P, precision="mixed", rtol=rtol)
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(reps):
            D, _, _ = dg.pairwise(P, precision="mixed", rtol=rtol)
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
        all_pairs = {"workload": "ba_n1e6_m3_unit_64_vectors_all_pairs", "vectors": m,
                     "pairs": npairs, "value": round(npairs / tp, 1), "unit": "distances/s",
                     "ms_per_call": round(tp * 1e3, 3), "precision": "mixed",
                     "max_rel_diff_vs_pair_solves": diff}
        log(f"all pairs: {all_pairs}")

    density = None if args.no_density else bench_density()
    tree_large = None if args.no_density else bench_tree_large()

    batched = None
    if not args.no_batched:
        dg.close()
        torch.cuda.empty_cache()
        batched = bench_batched(max(2, args.steps // 2), 1)

    spmv = None
    if not args.no_spmv:
        torch.cuda.empty_cache()
        spmv = bench_spmv()

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
        "config": {"workload": "ba_n1e6_m3_unit_k64", "n": g.n, "nnz": g.nnz, "pairs": K,
                   "rtol": rtol, "precision": "mixed (FP32 CG + FP64 refinement)",
                   "inner_rtol": args.inner_rtol, "tile": tile_used,
                   "tile_chosen_by": "option" if args.tile else "autotuner"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_path": {"value": round(value64, 2), "unit": "distances/s",
                      "ms_per_step": round(t64 * 1e3, 3)},
        "accuracy": acc,
        "batched": batched,
        "all_pairs": all_pairs,
        "density_sweep": density,
        "tree_like_1e6": tree_large,
        "spmv_reference": spmv,
        "iters_mean": float(np.mean(iters_mixed)),
        "refine_mean": float(np.mean(refine)),
        "setup_s": round(setup_s, 3),
        "kernels": {k: v for k, v in kinds.items() if v},
        "dominant_kernel": dom,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
