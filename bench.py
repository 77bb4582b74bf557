"""Benchmark: MM iterations/s of accelerated-MM non-rigid registration on one
MI355X, FP32 + FP64 refinement against the plain FP64 path, on the seeded
200,000-point workload (spherical-harmonic surface, l <= 16, articulated
warp, 15% outliers, 30% overlap cut; 4,000 nodes, k = 6, 10-NN edges;
50 MM iterations, Anderson m = 6).  Optionally the 64-pair batched workload
(pairs/s).  Prints one JSON line.

A "step" is one MM iteration of Alg. 2 over the whole hot path: surrogate
assembly, linear solve, Anderson mixing, energy evaluation of the candidate
(warp, closest points, Welsch terms) and the fallback re-evaluation.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the main kernels from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch averaged over a run of this
# benchmark), each divided by what the same counter reads for a plain copy of
# known size (profiles/sh200k_hbm_traffic_counters.txt).  Valid only for the
# kernel sources they were taken on: a change to those files voids them.
MEASURED_TRAFFIC = {
    "cg_step": {"fetch_kib": 4627.2, "fetch_per_byte": 131084.5 / 262144.0,
                "write_kib": 1133.8, "write_per_byte": 262144.0 / 262144.0,
                "sources": {
                            "paper_2206_03410_amd/csrc/amm_cg.hip": "c69d68b12abd3476",
                            "paper_2206_03410_amd/csrc/amm_device.h": "b6148a4b3f8d8557",
                            "paper_2206_03410_amd/csrc/amm_kernels.h": "945f9b0d5634d7c5",
                            "paper_2206_03410_amd/csrc/amm_internal.h": "fb7f5fb9b59d8276"}},
    "eval_points": {"fetch_kib": 10145.1, "fetch_per_byte": 131084.5 / 262144.0,
                    "write_kib": 8553.1, "write_per_byte": 262144.0 / 262144.0,
                    "sources": {
                            "paper_2206_03410_amd/csrc/amm_kernels.hip": "a4b5686b059d13a6",
                            "paper_2206_03410_amd/csrc/amm_nn.h": "541627b309bd02f0",
                            "paper_2206_03410_amd/csrc/amm_device.h": "b6148a4b3f8d8557",
                            "paper_2206_03410_amd/csrc/amm_kernels.h": "945f9b0d5634d7c5",
                            "paper_2206_03410_amd/csrc/amm_internal.h": "fb7f5fb9b59d8276"}},
    "assemble": {"fetch_kib": 16789.7, "fetch_per_byte": 131084.5 / 262144.0,
                 "write_kib": 6402.2, "write_per_byte": 262144.0 / 262144.0,
                 "sources": {
                            "paper_2206_03410_amd/csrc/amm_kernels.hip": "a4b5686b059d13a6",
                            "paper_2206_03410_amd/csrc/amm_device.h": "b6148a4b3f8d8557",
                            "paper_2206_03410_amd/csrc/amm_kernels.h": "945f9b0d5634d7c5",
                            "paper_2206_03410_amd/csrc/amm_internal.h": "fb7f5fb9b59d8276"}},
}


def measured_traffic(group):
    """Bytes per launch from the counters, or None if the kernel changed."""
    import hashlib
    m = MEASURED_TRAFFIC.get(group)
    if m is None:
        return None
    for path, h in m["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != h:
                return None
    return 1024.0 * (m["fetch_kib"] / m["fetch_per_byte"] + m["write_kib"] / m["write_per_byte"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(pair, T):
    """Bytes each kernel group must move per launch (inputs read once,
    outputs written once), for element size T."""
    N, M, n, k = pair.n_src, pair.n_tgt, pair.n_nodes, pair.k
    nadj = 2 * pair.n_edges
    nnzb = pair.nnzb
    return {
        # v, infl (idx+w), previous rho, accepted v_hat; writes v_hat, rho, d2, (e, w_a); targets once
        "eval_points": N * (3 * T + k * (4 + T) + 4 + 3 * T + 3 * T + 4 + T + 4 * T) + 3 * T * M,
        # node pairs, r, X of both ends; writes w_r, D
        "eval_edges": nadj * (8 + T + 2 * 12 * T + T + 4 * T),
        "eval_nodes": n * (9 * T + 9 * T),
        # points once (v, e, w_a, influences), X, w_r, D, R; writes K, B, r, D^-1
        "assemble": N * (3 * T + 4 * T + k * (4 + T)) + 12 * T * n + nadj * 5 * T + 9 * T * n
                    + 16 * T * nnzb + 4 * nnzb + 4 * (n + 1) + 12 * T * n * 2 + 16 * T * n,
        # one CG step as the method needs it: the blocks of K once and about eight
        # vectors of 3 right-hand sides (64 nnzb + 8 x 48 n in float32)
        "cg_step": 16 * T * nnzb + 8 * 12 * T * n,
        "residual64": 16 * T * nnzb + 4 * nnzb + 12 * 8 * n + 12 * T * n * 3,
    }


def cg_step_impl_bytes(pair, T):
    """What this build's fused CG step reads and writes per launch: K with
    its column indices and row pointers, r u w s p x and D^-1 of the rows
    read, p x and the next r u w s written (the Chronopoulos-Gear form keeps
    more vectors than plain CG)."""
    n, nnzb = pair.n_nodes, pair.nnzb
    return 16 * T * nnzb + 4 * nnzb + 4 * (n + 1) + 12 * T * n * 6 + 16 * T * n + 12 * T * n * 6


def load_pair(name):
    from paper_2206_03410_amd import synth
    t = time.time()
    pair = synth.make_workload(name)
    log(f"[bench] generated {name}: N={pair.n_src} M={pair.n_tgt} n={pair.n_nodes} "
        f"k={pair.k} edges={pair.n_edges} in {time.time() - t:.1f}s")
    return pair


def gpu_problem(amm, torch, pair, dtype=None):
    dev = "cuda:0"
    dtype = dtype or torch.float64
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    return amm.make_problem(t(pair.src, dtype), t(pair.tgt, dtype),
                            t(pair.node_idx, torch.int32), t(pair.infl_idx, torch.int32),
                            t(pair.infl_w, dtype), t(pair.edges, torch.int32),
                            pair.mean_edge_len)


def run_solve(amm, torch, h, pair, prec, iters, aa_m, timing=None):
    """One solve from X = I with a budget of `iters` MM iterations."""
    dt = torch.float32 if prec == amm.AMM_FP32_REFINE else torch.float64
    X = torch.empty(pair.n_nodes, 4, 3, dtype=dt, device="cuda:0")
    v = torch.empty(pair.n_src, 3, dtype=dt, device="cuda:0")
    prm = amm.amm_params_default(aa_m=aa_m, max_total_iters=iters, precision=prec)
    if timing is not None:
        amm.amm_enable_timing(h, True, timing or None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = amm.amm_solve(h, prm, X, v)[0]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = amm.amm_kernel_times(h) if timing is not None else {}
    if timing is not None:
        amm.amm_enable_timing(h, False)
    return st, wall, v.cpu().numpy().astype(np.float64), kt


def replayed_precision_error(amm, torch, h, pair, steps, aa_m, v64, st64):
    """Error of the FP32 + refinement path against the plain FP64 path along
    the same trajectory: the FP32 solve replays the FP64 run's Anderson
    accept/reject decisions and stage ends (free runs of the two part at the
    first decision either takes differently, and Anderson mixing then
    amplifies the difference), so what remains is the precision's own error.
    Deformed points as RMS over the bounding-box diagonal, energy relative."""
    log64 = amm.amm_iter_log(h)
    fa = [bool(r["accepted"]) if r["aa_used"] else None for r in log64]
    fs = [1 if (b is None or b["stage"] != a["stage"]) else 0 for a, b in zip(log64, log64[1:] + [None])]
    X = torch.empty(pair.n_nodes, 4, 3, dtype=torch.float32, device="cuda:0")
    v = torch.empty(pair.n_src, 3, dtype=torch.float32, device="cuda:0")
    prm = amm.amm_params_default(aa_m=aa_m, max_total_iters=steps, precision=amm.AMM_FP32_REFINE)
    st = amm.amm_solve(h, prm, X, v, force_accept=fa, force_stage_end=fs)[0]
    torch.cuda.synchronize()
    v32 = v.cpu().numpy().astype(np.float64)
    diag = float(np.linalg.norm(pair.tgt.max(0) - pair.tgt.min(0)))
    return {"iters": st["iters"], "iters_fp64": st64["iters"],
            "vhat_rms_over_diag": math.sqrt(((v32 - v64) ** 2).sum(1).mean()) / diag,
            "energy_rel": abs(st["energy"] - st64["energy"]) / abs(st64["energy"]),
            "solves_above_rtol": st["solves_above_rtol"]}


def timed_steps(amm, torch, h, pair, prec, steps, aa_m, repeats):
    """Exactly `steps` MM iterations per timed region: solves from X = I run
    back to back (a solve that converges early is followed by another, the
    last one capped at the remaining budget), bracketed by device
    synchronizations.  Returns the per-region wall times, the first solve's
    stats and the CG/refinement totals of one region."""
    dt = torch.float32 if prec == amm.AMM_FP32_REFINE else torch.float64
    X = torch.empty(pair.n_nodes, 4, 3, dtype=dt, device="cuda:0")
    walls, first, totals = [], None, None
    for r in range(repeats):
        done, cg, refine, solves = 0, 0, 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done < steps:
            prm = amm.amm_params_default(aa_m=aa_m, max_total_iters=steps - done, precision=prec)
            st = amm.amm_solve(h, prm, X, None)[0]
            first = first or st
            done += st["iters"]
            cg += st["cg_iters"]
            refine += st["refine_steps"]
            solves += 1
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        totals = {"cg_iters": cg, "refine_steps": refine, "solves": solves}
    return walls, first, totals


def cpu_baseline(pair, sample=40000):
    """The FP64 oracle on the same workload, one MM iteration: warp, Welsch
    terms, rotations, sparse-LU surrogate solve and Anderson mixing timed in
    full; brute-force closest points timed on `sample` queries and scaled to
    all N."""
    from oracle import amm_oracle as O
    threads = min(16, len(os.sched_getaffinity(0)))
    prob = O.from_pair(pair)
    X = O.identity(prob.n_nodes)
    p = O.Params(aa_m=6)
    t = time.perf_counter()
    vh = O.warp(prob, X)
    t_warp = time.perf_counter() - t
    rng = np.random.default_rng(0)
    idx = rng.choice(prob.n_src, sample, replace=False)
    t = time.perf_counter()
    rho_s, d2_s, _ = O.nearest(vh[idx], prob.tgt, threads=threads)
    t_nn = (time.perf_counter() - t) * prob.n_src / sample
    # closest points of all queries for the rest of the iteration by scipy's
    # exact k-d tree, timed as a second CPU reference for this stage
    from scipy.spatial import cKDTree
    t = time.perf_counter()
    dd, ii = cKDTree(prob.tgt).query(vh, 2, workers=threads)
    t_kd = time.perf_counter() - t
    t = time.perf_counter()
    D = O.reg_residuals(prob, X)
    R, er = O.proj_rotation(X[:, :3, :].transpose(0, 2, 1))
    ev0 = O.Eval(X, vh, ii[:, 0], dd[:, 0] ** 2, dd[:, 1] ** 2, D, R, er, 0, 0, 0, 0)
    nu_a, nu_min, nu_r = O.initial_nu(prob, p, ev0.d2)
    alpha, beta = O.term_weights(prob, p, nu_a, nu_r)
    ev = O.rescore(prob, ev0, nu_a, nu_r, alpha, beta)
    t_terms = time.perf_counter() - t
    t = time.perf_counter()
    Xn, _, _ = O.mm_update(prob, ev, nu_a, nu_r, alpha, beta)
    t_solve = time.perf_counter() - t
    t = time.perf_counter()
    hG = [X.reshape(-1) + 0.0, Xn.reshape(-1)]
    hF = [np.zeros(X.size), (Xn - X).reshape(-1)]
    O.anderson(hG, hF, 6)
    t_aa = time.perf_counter() - t
    per_iter = t_warp + t_nn + t_terms + t_solve + t_aa
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas")
    except Exception:
        pass
    return {
        "value": 1.0 / per_iter, "unit": "MM iterations/s", "cores": threads, "kind": "oracle",
        "blas_threads": blas,
        "sample": (f"one FP64 oracle MM iteration on the same 200k workload: warp, Welsch terms, "
                   f"rotations, sparse-LU surrogate solve and Anderson step in full; brute-force "
                   f"closest points on {sample} of {prob.n_src} queries, scaled x{prob.n_src // sample}"),
        "stage_s": {"warp": t_warp, "closest_points_scaled": t_nn, "terms": t_terms,
                    "surrogate_solve": t_solve, "anderson": t_aa},
        "closest_points_kdtree_s": t_kd,
        "cpu_model": cpu, "host": platform.node(),
    }


def batched_run(amm, torch, n_pairs, aa_m):
    """The 64-pair batch (FP32 + refinement, Alg. 2's own termination per
    pair): one handle for all pairs, timed with and without its set-up
    (amm_set_problems: validation, ordering, pattern of K and the search
    structures); and a plain per-pair loop (a set-up and a solve per pair,
    one after the other) beside it, with each pair's registration error
    (Eq. 25 against the generator's ground truth) compared between the
    two."""
    from paper_2206_03410_amd import synth
    t = time.time()
    pairs = synth.batch_pairs(n_pairs=n_pairs)
    log(f"[bench] generated {n_pairs} pairs ({sum(p.n_src for p in pairs)} points) in "
        f"{time.time() - t:.1f}s")
    rmse = lambda v, p: math.sqrt(((v - p.gt) ** 2).sum(1).mean())
    prm = lambda: amm.amm_params_default(aa_m=aa_m, precision=amm.AMM_FP32_REFINE)
    tot_nodes = sum(p.n_nodes for p in pairs)
    tot_pts = sum(p.n_src for p in pairs)
    h = amm.amm_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        probs = [gpu_problem(amm, torch, p) for p in pairs]
        torch.cuda.synchronize()
        t = time.perf_counter()
        leaf, _ = amm.amm_autotune(h, probs)
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t
        # device graph construction (Alg. 1) of every pair: one call per pair,
        # and all pairs in one call
        srcs = [torch.tensor(p.src, device="cuda:0") for p in pairs]
        amm.amm_build_graphs(h, srcs, 4)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for sp in srcs:
            amm.amm_build_graph(h, sp, 4)
        torch.cuda.synchronize()
        t_graph = time.perf_counter() - t
        t = time.perf_counter()
        g_nodes = sum(i["n_nodes"] for i in amm.amm_build_graphs(h, srcs, 4))
        torch.cuda.synchronize()
        t_graphs = time.perf_counter() - t
        X = torch.empty(tot_nodes, 4, 3, dtype=torch.float32, device="cuda:0")
        v = torch.empty(tot_pts, 3, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        t = time.perf_counter()
        amm.amm_set_problems(h, probs)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t
        t = time.perf_counter()
        st = amm.amm_solve(h, prm(), X, v, n_pairs=n_pairs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        vb = v.cpu().numpy().astype(np.float64)
        # the plain per-pair loop: set-up and solve of each pair alone
        loop_ms, loop_rmse = [], []
        for p, pr in zip(pairs, probs):
            Xp = torch.empty(p.n_nodes, 4, 3, dtype=torch.float32, device="cuda:0")
            vp = torch.empty(p.n_src, 3, dtype=torch.float32, device="cuda:0")
            torch.cuda.synchronize()
            t = time.perf_counter()
            amm.amm_set_problems(h, [pr])
            amm.amm_solve(h, prm(), Xp, vp)
            torch.cuda.synchronize()
            loop_ms.append(1e3 * (time.perf_counter() - t))
            loop_rmse.append(rmse(vp.cpu().numpy().astype(np.float64), p))
    finally:
        amm.amm_destroy(h)
    off, batch_rmse = 0, []
    for p in pairs:
        batch_rmse.append(rmse(vb[off:off + p.n_src], p))
        off += p.n_src
    eq = [abs(a - b) <= max(1e-4, 0.01 * b) for a, b in zip(batch_rmse, loop_rmse)]
    per = np.array([s["time_ms"] for s in st])
    loop_s = 1e-3 * sum(loop_ms)
    return {"pairs": n_pairs, "points": int(tot_pts),
            "pairs_per_s": n_pairs / (wall + t_setup), "pairs_per_s_solve_only": n_pairs / wall,
            "wall_s": wall, "setup_s": t_setup,
            "per_pair_loop_pairs_per_s": n_pairs / loop_s, "per_pair_loop_s": loop_s,
            "per_pair_loop_p50_ms": float(np.percentile(loop_ms, 50)),
            "per_pair_loop_p99_ms": float(np.percentile(loop_ms, 99)),
            "speedup_vs_loop": loop_s / (wall + t_setup),
            "equal_error_per_pair": bool(all(eq)), "pairs_equal_error": int(sum(eq)),
            "rmse_gt_batch_median": float(np.median(batch_rmse)),
            "autotuned_leaf": leaf, "autotune_s": t_tune,
            "graph_build_per_pair_calls_s": t_graph, "graph_build_one_call_s": t_graphs,
            "graph_build_nodes": g_nodes,
            "p50_pair_ms": float(np.percentile(per, 50)), "p99_pair_ms": float(np.percentile(per, 99)),
            "iters_total": int(sum(s["iters"] for s in st)),
            "converged": int(sum(s["converged"] for s in st)),
            "solves_above_rtol": int(sum(s["solves_above_rtol"] for s in st)),
            "definition": "pairs_per_s = pairs / (set-up + solve of the whole batch); per-pair p50/p99 = "
                          "each pair's time inside the batched solve; the loop sets up and solves one pair "
                          "at a time; equal error = every pair's RMSE to ground truth within max(1e-4, 1%) of "
                          "the loop's"}


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Attainable HBM bandwidth of a plain device-to-device copy (read +
    write bytes per second), median of `reps` copies of `nbytes`."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    return 2 * nbytes / float(np.median(ts)) / 1e9


def nn_search_report(amm, torch, h, pair, aa_m, steps, kt):
    """Work of the exact closest-point search over one FP32 solve (counted in
    a separate, untimed solve) against the measured time of the point
    evaluation per evaluation: the budgeted searches (eval_points), the
    deferred ones (eval_far) and the tile sums (eval_sums), from HIP events
    on their dispatches.  Headline candidate traffic per launch = queries x
    (12 B warped query + 8 B outputs) + target points examined x 16 B (one
    float4 each).  The search structure's own reads (nine 4-byte run starts
    per octree cell expansion read from memory) are reported apart: they
    are mostly cache hits, not HBM traffic; cell lower-bound tests read
    nothing (the cell's box follows from its coordinates)."""
    amm.amm_count_nn_work(h, True)
    try:
        run_solve(amm, torch, h, pair, amm.AMM_FP32_REFINE, steps, aa_m)
        w = amm.amm_nn_work(h)
    finally:
        amm.amm_count_nn_work(h, False)
    launches = max(1, round(w["queries"] / pair.n_src))
    q, bx, de, cl = (w[k] / launches for k in ("queries", "box_tests", "distance_evals", "cell_lookups"))
    n_eval = kt["eval_points"][1]
    part_us = {g: 1e3 * kt[g][0] / n_eval for g in ("eval_points", "eval_far", "eval_sums") if g in kt}
    t = sum(part_us.values()) * 1e-6
    cand = q * (12 + 8) + de * 16
    struct = cl * 36
    comp = pair.n_src * (12 + 4 + 4) + 12 * pair.n_tgt
    flops = 8 * de + 14 * bx
    return {"kernel": "eval_points + eval_far + eval_sums", "avg_launch_us": t * 1e6,
            "per_kernel_us": part_us, "search_step_budget": amm.amm_get_search_budget(h),
            "queries_per_launch": q,
            "cell_bound_tests_per_query": bx / q, "cell_expansions_from_memory_per_query": cl / q,
            "distance_evals_per_query": de / q,
            "compulsory_GBps": comp / t / 1e9,
            "compulsory_frac": comp / t / 1e9 / HBM_PEAK_GBS,
            "candidate_traffic_GBps": cand / t / 1e9,
            "candidate_traffic_frac": cand / t / 1e9 / HBM_PEAK_GBS,
            "structure_reads_GBps_cache": struct / t / 1e9,
            "distance_evals_per_s": de / t,
            "search_flops_frac_fp32_valu": flops / t / 157.3e12,
            "definition": "candidate traffic = queries x (12 B warped point + 8 B closest index and "
                          "squared distance) + target points examined x 16 B, per launch, over the "
                          "kernel's average launch time; structure reads (octree cell expansions read "
                          "from memory x 36 B; the upper four levels are in LDS) are cache traffic, "
                          "reported apart; flops: 8 per distance evaluation, 14 per cell bound test"}


def graph_build_report(amm, torch, h, pair, k, with_cpu):
    """Device construction of the deformation graph (Alg. 1, R = 5 l) on the
    workload's source points, with Euclidean and with geodesic distance:
    wall time of amm_build_graph (it synchronizes internally), median of 3
    after one untimed build; with the CPU leg, the oracle's sequential
    Euclidean pass on the same points."""
    src = torch.tensor(pair.src, device="cuda:0")
    amm.amm_build_graph(h, src, k)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = amm.amm_build_graph(h, src, k)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    out = {"gpu_ms": 1e3 * float(np.median(ts)), "k": k, **info}
    # the same build with the geodesic distance over the 6-NN edge graph
    amm.amm_build_graph(h, src, k, geodesic=True)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ginfo = amm.amm_build_graph(h, src, k, geodesic=True)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    out["geodesic"] = {"gpu_ms": 1e3 * float(np.median(ts)), **ginfo}
    if with_cpu:
        from oracle import graph_oracle as G
        t = time.perf_counter()
        lbar = G.mean_edge_length(pair.src)
        g = G.build_graph(pair.src, 5.0 * lbar, k)
        out["cpu_oracle_s"] = time.perf_counter() - t
        out["cpu_oracle_nodes_equal"] = len(g["node_idx"]) == info["n_nodes"]
    return out


def sequence_run(amm, torch, n_frames):
    """Template tracking (the frame i -> i + 2 sequences of Sec. 4): one
    50,000-point template registered to target frames 2, 4, ..., each solve
    run to Alg. 2's own termination in FP32 + refinement; the targets of the
    set-up pair are swapped between frames (amm_set_targets, inside each
    frame's time).  Warm: each frame starts from the previous frame's
    transforms; cold: from X = I."""
    from paper_2206_03410_amd import synth
    t0 = time.time()
    seq = synth.sh_sequence(6000, 50000, n_frames=n_frames, n_nodes=1000, k=4, e=8)
    log(f"[bench] generated the tracking sequence ({n_frames} frames) in {time.time() - t0:.1f}s")
    tpl = seq.template
    out = {"workload": f"{tpl.n_src} template points, {tpl.n_nodes} nodes, k=4, target frames "
                       f"{seq.frame_ids}, FP32 + refinement, Anderson m=5, Alg. 2 termination per frame"}
    h = amm.amm_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        amm.amm_set_problems(h, [gpu_problem(amm, torch, tpl)])
        for mode in ("warm", "cold", "warm"):
            X = torch.empty(tpl.n_nodes, 4, 3, dtype=torch.float32, device="cuda:0")
            v = torch.empty(tpl.n_src, 3, dtype=torch.float32, device="cuda:0")
            rows = []
            for f, tgt in enumerate(seq.frames):
                tgt_d = torch.tensor(tgt, device="cuda:0")
                prm = amm.amm_params_default(aa_m=5, precision=amm.AMM_FP32_REFINE,
                                             init_identity=1 if (mode == "cold" or f == 0) else 0)
                torch.cuda.synchronize()
                t = time.perf_counter()
                amm.amm_set_targets(h, 0, tgt_d)
                st = amm.amm_solve(h, prm, X, v)[0]
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                rm = math.sqrt(((v.cpu().numpy().astype(np.float64) - seq.gts[f]) ** 2).sum(1).mean())
                rows.append({"iters": st["iters"], "ms": 1e3 * dt, "rmse_gt": rm, "converged": st["converged"]})
            out[mode] = {"frames_per_s": len(rows) / (sum(r["ms"] for r in rows) * 1e-3),
                         "total_iters": sum(r["iters"] for r in rows),
                         "ms_per_frame": [round(r["ms"], 2) for r in rows],
                         "iters_per_frame": [r["iters"] for r in rows],
                         "rmse_gt": [r["rmse_gt"] for r in rows],
                         "all_converged": all(r["converged"] == 1 for r in rows)}
    finally:
        amm.amm_destroy(h)
    w, c = out["warm"], out["cold"]
    out["equal_error"] = all(abs(a - b) <= max(1e-4, 0.01 * b) for a, b in zip(w["rmse_gt"], c["rmse_gt"]))
    out["speedup_warm"] = w["frames_per_s"] / c["frames_per_s"]
    log(f"[bench] tracking: warm {w['frames_per_s']:.1f} frames/s ({w['total_iters']} MM iterations), "
        f"cold {c['frames_per_s']:.1f} frames/s ({c['total_iters']}), equal error {out['equal_error']}")
    return out


def variants_run(amm, torch, h, pair, steps, aa_m):
    """The Sec. 4.1 variants on the workload: each solve from X = I for
    `steps` MM iterations (FP32 + refinement), its rate and its registration
    error against the ground truth (Eq. 25, scaled units)."""
    runs = {"welsch": (amm.AMM_ROBUST_WELSCH, amm.AMM_NU_DYNAMIC), "l2": (amm.AMM_ROBUST_L2, amm.AMM_NU_DYNAMIC),
            "l2r": (amm.AMM_ROBUST_L2_TRUNC, amm.AMM_NU_DYNAMIC),
            "welsch_fmax": (amm.AMM_ROBUST_WELSCH, amm.AMM_NU_FIXED_MAX),
            "welsch_fmin": (amm.AMM_ROBUST_WELSCH, amm.AMM_NU_FIXED_MIN),
            "welsch_fmed": (amm.AMM_ROBUST_WELSCH, amm.AMM_NU_FIXED_MED)}
    out = {}
    X = torch.empty(pair.n_nodes, 4, 3, dtype=torch.float32, device="cuda:0")
    v = torch.empty(pair.n_src, 3, dtype=torch.float32, device="cuda:0")
    for name, (rb, nm) in runs.items():
        prm = amm.amm_params_default(aa_m=aa_m, max_total_iters=steps, precision=amm.AMM_FP32_REFINE,
                                     robust=rb, nu_mode=nm)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = amm.amm_solve(h, prm, X, v)[0]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        rm = math.sqrt(((v.cpu().numpy().astype(np.float64) - pair.gt) ** 2).sum(1).mean())
        out[name] = {"iters": st["iters"], "iters_per_s": st["iters"] / dt, "rmse_gt": rm,
                     "stages": st["stages"], "energy": st["energy"]}
    log("[bench] variants: " + ", ".join(f"{k} {v['iters_per_s']:.0f} it/s rmse {v['rmse_gt']:.4f}"
                                        for k, v in out.items()))
    return out


def torus_end_to_end(amm, torch, with_cpu):
    """The 2,000-point torus workload, plain FP64 (30 MM iterations,
    Anderson m = 5): whole-solve wall time on the GPU (median of 5, the
    problem already uploaded), and with the CPU leg the oracle's own solve
    of the same workload, with both final energies."""
    from paper_2206_03410_amd import synth
    pair = synth.make_workload("torus2k")
    h = amm.amm_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        amm.amm_set_problems(h, [gpu_problem(amm, torch, pair)])
        X = torch.empty(pair.n_nodes, 4, 3, dtype=torch.float64, device="cuda:0")
        prm = amm.amm_params_default(aa_m=5, max_total_iters=30, precision=amm.AMM_FP64_PLAIN)
        amm.amm_solve(h, prm, X)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = amm.amm_solve(h, prm, X)[0]
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
    finally:
        amm.amm_destroy(h)
    out = {"workload": "torus2k: 2,000 source / 2,100 target points, 80 nodes, k=4, 30 MM iterations, m=5, FP64",
           "gpu_s": float(np.median(ts)), "gpu_iters": st["iters"], "gpu_energy": st["energy"]}
    if with_cpu:
        from oracle import amm_oracle as O
        t = time.perf_counter()
        res = O.solve(O.from_pair(pair), O.Params(aa_m=5, max_total_iters=30))
        out["cpu_oracle_s"] = time.perf_counter() - t
        out["cpu_oracle_iters"] = res["total"]
        out["cpu_oracle_energy"] = res["E"]
    return out


def gradient_timing(amm, torch, with_cpu):
    """The 100,000-point gradient workload (2,000 nodes, k = 4): energy and
    adjoint with respect to X and the source points at X = I + delta, per
    call on the GPU (FP32 and FP64, median of 10); with the CPU leg the
    oracle's analytic gradient at the same point, its closest points from
    scipy's exact k-d tree."""
    from paper_2206_03410_amd import synth
    from scipy.spatial import cKDTree
    pair = synth.make_workload("grad100k")
    Xn = synth.perturbed_transforms(pair.n_nodes, 5005, 0.01, 0.001)
    out = {"workload": "grad100k: 100,000 points, 2,000 nodes, k=4, gradient w.r.t. X (12 per node) and "
                       "the source points, Sec. 3.3.3 start values of nu and Eq. 26 weights"}
    tree = cKDTree(pair.tgt)

    def nn(q, _tgt):
        d, i = tree.query(q, k=2)
        return i[:, 0].astype(np.int64), d[:, 0] ** 2, d[:, 1] ** 2
    # the scalars are the solver's start values, computed here with scipy's
    # exact closest points (the same definitions the solver applies)
    d0 = nn(pair.src, None)[1]
    l = pair.mean_edge_len
    nu_a = max(float(np.sqrt(np.median(d0))), l / np.sqrt(3.0))
    nu_r = 3.0 * l
    prm = amm.amm_params_default()
    alpha = prm.k_alpha * pair.n_src / pair.n_edges * (nu_r / nu_a) ** 2      # Eq. 26
    beta = prm.k_beta * pair.n_src / pair.n_nodes / (2.0 * nu_a * nu_a)
    for dt, name in ((torch.float32, "gpu_fp32_ms"), (torch.float64, "gpu_fp64_ms")):
        h = amm.amm_create(0, torch.cuda.current_stream().cuda_stream)
        try:
            amm.amm_set_problems(h, [gpu_problem(amm, torch, pair, dt)])
            X = torch.as_tensor(Xn, dtype=dt, device="cuda:0")
            V = torch.as_tensor(pair.src, dtype=dt, device="cuda:0")
            gX, gV = torch.empty_like(X), torch.empty_like(V)
            amm.amm_energy_grad(h, X, V, nu_a, nu_r, alpha, beta, gX, gV)
            ts = []
            for _ in range(10):
                torch.cuda.synchronize()
                t = time.perf_counter()
                amm.amm_energy_grad(h, X, V, nu_a, nu_r, alpha, beta, gX, gV)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            out[name] = 1e3 * float(np.median(ts))
        finally:
            amm.amm_destroy(h)
    if with_cpu:
        from oracle import amm_oracle as O
        prob = O.from_pair(pair)
        t = time.perf_counter()
        O.energy_grad(prob, Xn, nu_a, nu_r, alpha, beta, ev=O.evaluate(prob, Xn, nu_a, nu_r, alpha, beta, nn=nn))
        out["cpu_oracle_ms"] = 1e3 * (time.perf_counter() - t)
    return out


def copy_calibration():
    """A plain device copy of known size, for scaling the HBM traffic
    counters (FETCH_SIZE, WRITE_SIZE) of a profiled run: each of the 5
    copies reads and writes 256 MiB."""
    import torch
    n = 256 * 1024 * 1024 // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda:0").uniform_()
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "copies": 5}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="MM iterations in the timed solve")
    ap.add_argument("--warmup", type=int, default=5, help="MM iterations in the untimed warm-up solve")
    ap.add_argument("--workload", default="sh200k")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batched", type=int, default=64, help="pairs of the batched run (0 = skip)")
    ap.add_argument("--sequence", type=int, default=8,
                    help="target frames of the tracking run (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain-copy kernel that scales the traffic counters")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the registration "
              "hot path runs on a single device)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_03410_amd import amm, synth

    pair = load_pair(args.workload)
    aa_m = synth.WORKLOADS[args.workload]["aa_m"]
    repeats = 5
    h = amm.amm_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        prob = gpu_problem(amm, torch, pair)
        leaf, leaf_ms = amm.amm_autotune(h, [prob])
        budget = amm.amm_get_search_budget(h)
        log(f"[bench] autotuned closest-point leaf size {leaf}, search step budget {budget} "
            f"(warm evaluation {leaf_ms:.3f} ms)")
        pair.nnzb = amm.amm_k_nnzb(h)
        # first use of every kernel (code objects load lazily), untimed
        for prec in (amm.AMM_FP32_REFINE, amm.AMM_FP64_PLAIN):
            run_solve(amm, torch, h, pair, prec, 2, aa_m)
        # warm-up: every kernel group timed (per-stage breakdown, dominant kernel)
        st_w, wall_w, _, kt_w = run_solve(amm, torch, h, pair, amm.AMM_FP32_REFINE, args.warmup, aa_m,
                                          timing="")
        run_solve(amm, torch, h, pair, amm.AMM_FP64_PLAIN, args.warmup, aa_m)
        dom = max(kt_w, key=lambda k: kt_w[k][0])
        log(f"[bench] warm-up {args.warmup} iters {wall_w * 1e3:.1f} ms; kernel groups: "
            + ", ".join(f"{k} {v[0]:.2f}ms/{v[1]}" for k, v in sorted(kt_w.items(), key=lambda x: -x[1][0])))
        # timed: exactly `steps` MM iterations per region, median of `repeats` regions
        w32, st32, tot32 = timed_steps(amm, torch, h, pair, amm.AMM_FP32_REFINE, args.steps, aa_m, repeats)
        wall32 = float(np.median(w32))
        log(f"[bench] fp32+refine: {args.steps} iters, median {wall32:.4f}s of {['%.4f' % w for w in w32]}; "
            f"{tot32['solves']} solve(s), cg {tot32['cg_iters']} refine {tot32['refine_steps']}")
        # the dominant kernel's own duration (events on its dispatches) and the
        # deformed points for the error comparison, one more (untimed) solve
        st_d, _, v32, kt32 = run_solve(amm, torch, h, pair, amm.AMM_FP32_REFINE, args.steps, aa_m, timing=dom)
        plain = None
        if not args.no_plain:
            w64, st64, tot64 = timed_steps(amm, torch, h, pair, amm.AMM_FP64_PLAIN, args.steps, aa_m, repeats)
            st64d, _, v64, _ = run_solve(amm, torch, h, pair, amm.AMM_FP64_PLAIN, args.steps, aa_m)
            rep = replayed_precision_error(amm, torch, h, pair, args.steps, aa_m, v64, st64d)
            wall64 = float(np.median(w64))
            log(f"[bench] fp64 plain: {args.steps} iters, median {wall64:.4f}s; {tot64['solves']} solve(s), "
                f"cg {tot64['cg_iters']}")
            diag = float(np.linalg.norm(pair.tgt.max(0) - pair.tgt.min(0)))
            rm32 = math.sqrt(((v32 - pair.gt) ** 2).sum(1).mean())
            rm64 = math.sqrt(((v64 - pair.gt) ** 2).sum(1).mean())
            plain = {"iters_per_s": args.steps / wall64, "ms_per_iter": 1e3 * wall64 / args.steps,
                     "region_s": w64, "solves": tot64["solves"], "cg_iters": tot64["cg_iters"],
                     "first_solve_iters": st64["iters"],
                     "rmse_gt_fp32": rm32, "rmse_gt_fp64": rm64,
                     "equal_error": abs(rm32 - rm64) <= max(1e-4, 0.01 * rm64),
                     "speedup_fp32_refine": wall64 / wall32,
                     # free runs (each path takes its own Anderson decisions): the FP32 result against the FP64 one after the same
                     # number of MM iterations: deformed points (RMS over the target bounding-box
                     # diagonal) and the final energy
                     "free_run_vhat_rms_fp32_vs_fp64_over_diag": math.sqrt(((v32 - v64) ** 2).sum(1).mean()) / diag,
                     "free_run_energy_rel_diff_fp32_vs_fp64": abs(st_d["energy"] - st64d["energy"]) / abs(st64d["energy"]),
                     "solves_above_rtol": [st_d["solves_above_rtol"], st64d["solves_above_rtol"]],
                     "fp32_replayed_vs_fp64": rep}
        # the search's average launch time over the same solve that is counted
        _, _, _, kt_e = run_solve(amm, torch, h, pair, amm.AMM_FP32_REFINE, args.steps, aa_m, timing="")
        nn = nn_search_report(amm, torch, h, pair, aa_m, args.steps, kt_e)
        log(f"[bench] closest points: {nn['avg_launch_us']:.1f} us per evaluation ("
            + ", ".join(f"{k} {v:.1f}" for k, v in nn["per_kernel_us"].items()) + f"); "
            f"{nn['cell_bound_tests_per_query']:.1f} cell bound tests, "
            f"{nn['cell_expansions_from_memory_per_query']:.1f} cell expansions from memory and "
            f"{nn['distance_evals_per_query']:.1f} distance evaluations per query; candidate traffic "
            f"{nn['candidate_traffic_GBps']:.0f} GB/s")
        copy_gbs = copy_bandwidth(torch)
        log(f"[bench] plain device copy {copy_gbs:.0f} GB/s")
        variants = variants_run(amm, torch, h, pair, args.steps, aa_m)
        graph = graph_build_report(amm, torch, h, pair, pair.k, not args.no_cpu)
        log(f"[bench] graph build (Alg. 1): {graph['gpu_ms']:.1f} ms on the GPU, {graph['n_nodes']} nodes, "
            f"{graph['rounds']} rounds; geodesic {graph['geodesic']['gpu_ms']:.1f} ms, "
            f"{graph['geodesic']['n_nodes']} nodes"
            + (f"; oracle {graph['cpu_oracle_s']:.1f} s" if 'cpu_oracle_s' in graph else ""))
    finally:
        amm.amm_destroy(h)

    T = 4
    ab = algorithmic_bytes(pair, T)
    ms_tot, nl = kt32[dom]
    avg_s = ms_tot / nl * 1e-3
    # CG steps queued past convergence return at once and move no data: the
    # algorithmic bytes are those of the working steps (the solve's CG
    # iteration count), spread over every launch's time
    working = min(nl, int(st_d["cg_iters"])) if dom == "cg_step" else nl
    achieved = ab[dom] * working / nl / avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                "bytes_per_launch": ab[dom], "avg_launch_us": avg_s * 1e6, "launches": nl,
                "working_launches": working, "attainable_copy_GBps": copy_gbs}
    abw = ab
    stages = {}
    for k, v in kt_w.items():
        t_launch = v[0] / v[1] * 1e-3
        mt = measured_traffic(k)
        stages[k] = {"ms_per_iter": v[0] / max(st_w["iters"], 1), "launches": v[1],
                     "GBps": (abw[k] / t_launch / 1e9) if k in abw else None,
                     "measured_GBps": (mt / t_launch / 1e9) if mt else None}
    out = {
        "metric": "MM iterations/s at 200k points, FP32+refine vs plain; batched pairs/s at equal err",
        "value": args.steps / wall32, "unit": "MM iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall32 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {pair.n_src} source / {pair.n_tgt} target points, "
                               f"{pair.n_nodes} nodes, k={pair.k}, {pair.n_edges} node edges, "
                               f"{args.steps} MM iterations per timed region (solves from X = I back to "
                               f"back), Anderson m={aa_m}, FP32 + FP64 refinement to relative residual 1e-10, "
                               f"median of {repeats} regions",
                   "n_src": pair.n_src, "n_tgt": pair.n_tgt, "n_nodes": pair.n_nodes, "k": pair.k,
                   "n_edges": pair.n_edges, "nnzb": pair.nnzb},
        "roofline": roofline,
        "autotuned_leaf": leaf,
        "plain_fp64": plain,
        "stages_warmup": stages,
        "closest_points": nn,
        "graph_build": graph,
        "variants": variants,
        "timed_regions_s": w32,
        "solve": {"first_solve_iters": st32["iters"], "solves_per_region": tot32["solves"],
                  "cg_iters_per_region": tot32["cg_iters"], "refine_steps_per_region": tot32["refine_steps"],
                  "aa_accepted": st32["aa_accepted"], "aa_rejected": st32["aa_rejected"],
                  "energy": st32["energy"], "max_rel_residual": st32["max_rel_residual"]},
    }
    if args.batched:
        out["batched"] = batched_run(amm, torch, args.batched, 5)
    if args.sequence:
        out["tracking"] = sequence_run(amm, torch, args.sequence)
    out["torus_end_to_end"] = torus_end_to_end(amm, torch, not args.no_cpu)
    out["gradient"] = gradient_timing(amm, torch, not args.no_cpu)
    log(f"[bench] torus2k FP64 end to end {out['torus_end_to_end']['gpu_s'] * 1e3:.1f} ms on the GPU; "
        f"gradient at 100k points {out['gradient']['gpu_fp32_ms']:.2f} ms FP32, "
        f"{out['gradient']['gpu_fp64_ms']:.2f} ms FP64")
    if not args.no_cpu:
        t = time.time()
        out["cpu_baseline"] = cpu_baseline(pair)
        log(f"[bench] cpu baseline in {time.time() - t:.1f}s")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
