"""Benchmark: fast directional BEM matvec throughput and GMRES time to 1e-5
on the 81,920-triangle rigid sphere at kD = 100 (icosphere subdivided 6
times, radius 0.5, unit plane wave along +z, Burton-Miller coupling i/k for
the fluid-side normal, eps = 1e-4).

One step = one FDA matvec (near field, S2M, M2M, M2L, L2L, L2T) of a seeded
complex-normal vector, inputs resident in HBM.  The same run also reports
the plan build time, GMRES(50) time to a relative residual of 1e-5 (plain
and block-Jacobi), a per-stage timing, the roofline of the dominant kernel
and the FP64 CPU oracle timed on a bounded row sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(V, T, k, x, y_gpu, rows_sample, seconds_target=20.0):
    """The FP64 oracle (dense definition, OpenMP C) timed on the host cores
    for a bounded sample of rows, scaled to a full matvec; its output doubles
    as a sampled-row error check of the GPU product."""
    import oracle as O

    n = len(T)
    rng = np.random.default_rng(123)
    # calibrate on a few rows, then size the sample to about seconds_target
    r0 = np.sort(rng.choice(n, size=128, replace=False))
    t0 = time.perf_counter()
    O.matvec(V, T, k, x, row_idx=r0)
    per_row = (time.perf_counter() - t0) / 128
    m = int(max(16, min(rows_sample, seconds_target / max(per_row, 1e-9))))
    rows = np.sort(rng.choice(n, size=m, replace=False))
    t0 = time.perf_counter()
    yr = O.matvec(V, T, k, x, row_idx=rows)
    dt = time.perf_counter() - t0
    full = dt * n / m
    err = float(np.linalg.norm(y_gpu[rows] - yr) / np.linalg.norm(yr))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the same oracle on one thread over a few rows, extrapolated to a full
    # matvec (to set beside a one-core figure); the thread count is restored
    one = None
    try:
        import ctypes

        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        r1 = rows[: max(8, min(len(rows), int(2.0 / max(per_row * threads, 1e-9))))]
        t0 = time.perf_counter()
        O.matvec(V, T, k, x, row_idx=r1)
        one = dict(seconds_per_matvec=round((time.perf_counter() - t0) * n / len(r1), 1),
                   sample=f"{len(r1)} rows on 1 thread, extrapolated to N")
        gomp.omp_set_num_threads(threads)
    except OSError:
        pass
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=1.0 / full, unit="matvecs/s", cores=threads, kind="oracle", cpu_model=model,
                nproc=os.cpu_count(),
                sample=f"{m} of {n} rows of one FP64 dense matvec ({dt:.1f} s), scaled by N/{m}",
                seconds_per_matvec=full, one_thread_extrapolated=one), err, rows, yr


def mlp_held_out(weights_path):
    """The network's training size and held-out evaluation, as stored beside
    its weights by the training driver (its report), or None."""
    rep = os.path.splitext(weights_path)[0] + ".json"
    if not os.path.exists(rep):
        return None
    with open(rep) as f:
        sm = json.load(f).get("summary", {})
    tr, ev = sm.get("train", {}), sm.get("eval", {})
    if not ev:
        return None
    return dict(train_solves=tr.get("train_solves"), eval_solves=ev.get("eval_solves"),
                mean_iterations=ev.get("mean_iterations"), judge_rejected=ev.get("judge_rejected"),
                fewer_iterations_than_block_jacobi=ev.get("mlp_fewer_iterations_than_bj"),
                beats_block_jacobi=bool(ev["mean_iterations"]["mlp"] < ev["mean_iterations"]["block_jacobi"]))


def uneven_batch_leg(nmesh, steps, log, tune=True):
    """The seeded uneven batch (spheres and ellipsoids, N 5,120-81,920,
    kD 20-100): every plan's product run one after another on one stream,
    against all of them in one captured graph (fda_batch)."""
    import torch

    import workloads as W
    from paper_1403_4747_amd import Batch, FDAError, Plan

    plans, xs, ys, skipped, nel = [], [], [], [], 0
    t0 = time.perf_counter()
    for i, (V, T, k, info) in enumerate(W.uneven_batch(nmesh)):
        try:
            p = Plan(V, T, k, 1e-4)
        except FDAError as e:  # e.g. leaves that would need directional (high-frequency) handling
            skipped.append(dict(info, error=str(e)[:120]))
            continue
        plans.append(p)
        log(f"[bench] batch mesh {i}: N={len(T)} kD={info['kD']:.1f} built ({time.perf_counter() - t0:.1f} s)")
        xs.append(torch.from_numpy(W.complex_normal(len(T), 1, seed=100 + i)).to("cuda"))
        ys.append(torch.empty_like(xs[-1]))
        nel += len(T)
    build_s = time.perf_counter() - t0
    # the M2L launch autotuner per mesh (before the graph is captured)
    tuned = dict(changed=0, m2l_ms_before=0.0, m2l_ms_after=0.0, seconds=0.0)
    if tune:
        t0 = time.perf_counter()
        for p in plans:
            r = p.autotune(reps=10)
            tuned["changed"] += int(r["best"] != dict(variant=0, xcd_order=1,
                                                       width={l: 32 for l in r["best"]["width"]}))
            tuned["m2l_ms_before"] += r["ms_before"]
            tuned["m2l_ms_after"] += r["ms_after"]
        tuned = {q: (round(v, 3) if isinstance(v, float) else v) for q, v in tuned.items()}
        tuned["seconds"] = round(time.perf_counter() - t0, 2)
    for p, x, y in zip(plans, xs, ys):
        p.matvec(x, out=y)
    torch.cuda.synchronize()
    reps = max(3, steps // 10)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        for p, x, y in zip(plans, xs, ys):
            p.matvec(x, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1) / reps
    want = [y.clone() for y in ys]
    b = Batch(plans, xs, ys)
    b.launch()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        b.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    gr_ms = e0.elapsed_time(e1) / reps
    same = all(torch.equal(a, c) for a, c in zip(want, ys))
    b.close()
    for p in plans:
        p.close()
    out = dict(meshes=len(plans), skipped=len(skipped), elements=nel, build_seconds=round(build_s, 2),
               sequential_ms=round(seq_ms, 3), graph_ms=round(gr_ms, 3),
               batches_per_s=round(1000.0 / gr_ms, 3), graph_equals_sequential=bool(same),
               m2l_autotune=tuned if tune else None, skipped_cases=skipped[:4])
    log(f"[bench] uneven batch: {out}")
    return out


def large_case(args, log):
    """The large one-GPU case: rigid prolate spheroid with semi-axes
    (2.5, 0.5, 0.5) (D = 5) at kD = 1000, meshed uniformly with about 4 M
    triangles (edges of about 0.0025, 12.6 per wavelength), unit plane wave at
    30 degrees to the long axis, eps = 1e-4, leaves at least 2 longest edges
    wide (depth 9: at most 46 elements per leaf).  Plain FP64 FDA against
    the FP32 arm (FP64 self terms and Arnoldi) with block Jacobi and the
    learned preconditioner; matvec rate, GMRES time to 1e-5, build time,
    peak HBM and the error on oracle rows."""
    import torch

    import workloads as W
    from paper_1403_4747_amd import Plan

    V, T = W.spheroid_rings(0.0025)
    n, kD = len(T), 1000.0
    k = kD / 5.0
    th = math.radians(30.0)
    d = (math.cos(th), math.sin(th), 0.0)
    log(f"[bench] large case: spheroid N={n} kD={kD}")
    x = torch.from_numpy(W.complex_normal(n, 1, seed=0)).to("cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    free0 = torch.cuda.mem_get_info()[0]
    arms, ys = {}, {}
    for prec in ("fp64", "fp32"):
        t0 = time.perf_counter()
        p = Plan(V, T, k, 1e-4, prec=prec, leaf_min_h=2.0)
        torch.cuda.synchronize()
        arm = dict(build_seconds=round(time.perf_counter() - t0, 2))
        st = p.stats()
        arm.update(depth=st["depth"], leaves=st["nleaf"], max_leaf=st["max_leaf_count"], near_nnz=st["near_nnz"],
                   plan_gib=round((free0 - torch.cuda.mem_get_info()[0]) / 2**30, 2))
        if not args.no_tune:
            arm["m2l_autotune"] = p.autotune(reps=5)["best"]
        y = p.matvec(x)
        for _ in range(2):
            p.matvec(x, out=y)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            p.matvec(x, out=y)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        prof = p.profile(x, reps=3)
        arm.update(ms_per_matvec=round(ms, 3), matvecs_per_s=round(1000.0 / ms, 3),
                   stages_ms={q: round(v, 3) for q, v in prof.items() if q != "m2l_gemm"})
        if prof["m2l_lowrank"] > 0:
            a = st["m2l_flops"] / (prof["m2l_lowrank"] * 1e-3) / 1e12
            peak = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS
            arm["m2l_roofline"] = dict(achieved=round(a, 3), peak=peak, unit="TFLOP/s", frac=round(a / peak, 4),
                                       flops_per_launch=st["m2l_flops"])
        ys[prec] = y.cpu().numpy()
        if not args.no_solve:
            b = p.rhs_planewave(d)
            pcs = ["none", "block_jacobi"]
            if prec == "fp32" and os.path.exists(args.mlp_weights):
                from paper_1403_4747_amd import train_mlp

                p.set_mlp(train_mlp.load(args.mlp_weights))
                pcs.append("mlp")
            for pc in pcs:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = p.solve(b, tol=1e-5, restart=50, maxit=1000, precond=pc)
                torch.cuda.synchronize()
                arm["solve_" + pc] = dict(seconds=round(time.perf_counter() - t0, 3), iterations=info["iterations"],
                                          converged=info["converged"], rel_residual=info["rel_residual"])
                if pc == "mlp":
                    arm["solve_mlp"].update(mlp_rejected=info["mlp_rejected"], mlp_fallbacks=info["mlp_fallbacks"])
            p.set_mlp(None)
        arm["peak_hbm_gib"] = round((free0 - torch.cuda.mem_get_info()[0]) / 2**30, 2)
        log(f"[bench] large {prec}: {arm}")
        arms[prec] = arm
        p.close()
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        cpu, err, rows, yr = cpu_baseline(V, T, k, W.complex_normal(n, 1, seed=0), ys["fp64"], 4096, args.cpu_seconds / 2)
        arms["fp64"]["matvec_rel_err_vs_oracle_sampled"] = err
        arms["fp32"]["matvec_rel_err_vs_oracle_sampled"] = float(np.linalg.norm(ys["fp32"][rows] - yr) / np.linalg.norm(yr))
        log(f"[bench] large cpu baseline {cpu}")
    f64 = arms["fp64"]
    return {
        "metric": "FDA matvecs/s + GMRES time-to-1e-5, large case (prolate spheroid 2.5 x 0.5 x 0.5, N~4M, kD=1000)",
        "value": f64["matvecs_per_s"],
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 2,
        "ms_per_step": f64["ms_per_matvec"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"spheroid{n}_kD1000", "N": n, "k": k, "kD": kD, "eps": 1e-4, "leaf_min_h": 2.0,
                   "direction_deg_to_axis": 30.0, "arm": "plain FP64"},
        "time_to_1e-5_s": f64.get("solve_none", {}).get("seconds"),
        "arms": arms,
        "cpu_baseline": cpu,
    }


def adaptive_case(args, log):
    """Adaptive trees on a graded mesh: an icosphere of 20,480 triangles whose
    cap above z = 0.3 r is refined once and above z = 0.7 r twice more
    (79,106 triangles, 4.8:1 in edge length), radius 0.5, kD = 100, eps =
    1e-4, plane wave along +z.  A uniform tree refuses the mesh (a leaf of
    more than 256 elements); the adaptive tree puts leaves on three levels
    and evaluates W and X pairs directly.  Arms: adaptive FP64, adaptive
    FP32, and a uniform tree with leaves only 1.5 largest edges wide (the
    widest setting that builds: near-singular pairs then reach the far
    field).  Matvec rate, stage times, GMRES to 1e-5 and the error on oracle
    rows of each arm."""
    import torch

    import workloads as W
    from paper_1403_4747_amd import FDAError, Plan, inspect

    V, T = W.graded_sphere(5)
    n, k = len(T), 100.0
    log(f"[bench] adaptive case: graded sphere N={n} kD={k:g}")
    x = torch.from_numpy(W.complex_normal(n, 1, seed=0)).to("cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    try:
        inspect(V, T, k, 1e-4)
        uniform_refusal = None
    except FDAError as e:
        uniform_refusal = str(e)
    arms, ys = {}, {}
    for name, kw in (("adaptive_fp64", dict(adaptive=1)), ("adaptive_fp32", dict(adaptive=1, prec="fp32")),
                     ("uniform_leaf1.5h_fp64", dict(leaf_min_h=1.5))):
        t0 = time.perf_counter()
        p = Plan(V, T, k, 1e-4, **kw)
        torch.cuda.synchronize()
        arm = dict(build_seconds=round(time.perf_counter() - t0, 2))
        st = p.stats()
        arm.update(depth=st["depth"], leaves_per_level=st["leaves"], leaves=st["nleaf"], max_leaf=st["max_leaf_count"],
                   near_nnz=st["near_nnz"], near_from_w_x=st["wx_elem_pairs"], u_pairs=st["u_pairs"],
                   w_pairs=st["w_pairs"], x_pairs=st["x_pairs"], m2l_flops=st["m2l_flops"])
        if not args.no_tune:
            arm["m2l_autotune"] = p.autotune(reps=5)["best"]
        y = p.matvec(x)
        for _ in range(2):
            p.matvec(x, out=y)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            p.matvec(x, out=y)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        prof = p.profile(x, reps=3)
        arm.update(ms_per_matvec=round(ms, 4), matvecs_per_s=round(1000.0 / ms, 2),
                   stages_ms={q: round(v, 4) for q, v in prof.items() if q != "m2l_gemm"})
        ys[name] = y.cpu().numpy()
        if not args.no_solve:
            b = p.rhs_planewave((0.0, 0.0, 1.0))
            for pc in ("none", "block_jacobi"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = p.solve(b, tol=1e-5, restart=50, maxit=1000, precond=pc)
                torch.cuda.synchronize()
                arm["solve_" + pc] = dict(seconds=round(time.perf_counter() - t0, 3), iterations=info["iterations"],
                                          converged=info["converged"], rel_residual=info["rel_residual"])
        log(f"[bench] adaptive case {name}: {arm}")
        arms[name] = arm
        p.close()
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        cpu, err, rows, yr = cpu_baseline(V, T, k, W.complex_normal(n, 1, seed=0), ys["adaptive_fp64"], 4096,
                                          args.cpu_seconds / 2)
        for name in arms:
            arms[name]["matvec_rel_err_vs_oracle_sampled"] = float(np.linalg.norm(ys[name][rows] - yr) /
                                                                   np.linalg.norm(yr))
        log(f"[bench] adaptive case cpu baseline {cpu}")
    a64 = arms["adaptive_fp64"]
    return {
        "metric": "FDA matvecs/s, adaptive tree on a graded sphere (N=79,106, kD=100)",
        "value": a64["matvecs_per_s"],
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 2,
        "ms_per_step": a64["ms_per_matvec"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"graded_sphere{n}_kD100", "N": n, "k": k, "kD": k, "eps": 1e-4,
                   "refinement": "icosphere s=5, +1 level above z=0.3r, +2 above z=0.7r", "arm": "adaptive FP64"},
        "uniform_tree_refusal": uniform_refusal,
        "arms": arms,
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere81920_kD100")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fast", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the M2L launch autotuner (fda_autotune) after the build")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (calibrates HBM counters)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--nrhs-multi", type=int, default=64, help="also time products of this many columns (0: skip)")
    ap.add_argument("--batch", type=int, default=32,
                    help="also time the uneven multi-mesh batch of this many meshes in one graph (0: skip)")
    ap.add_argument("--mlp-weights", default=os.path.join(ROOT, "paper_1403_4747_amd", "weights",
                                                          "mlp_ellipsoid_s5_h256.npz"),
                    help="trained learned-preconditioner weights for the fast arm's solve")
    ap.add_argument("--large", action="store_true",
                    help="run only the large case (prolate spheroid, about 4 M triangles, kD = 1000) and print its line")
    ap.add_argument("--adaptive", action="store_true",
                    help="run only the adaptive-tree case (graded sphere, 79,106 triangles, kD = 100) and print its line")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "m2l_lowrank_sphere81920_kD100_traffic.json"),
                    help="measured HBM traffic of the M2L kernel (written from rocprofv3 counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_1403_4747_amd import Plan

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    if args.large:
        print(json.dumps(large_case(args, log)), flush=True)
        return
    if args.adaptive:
        print(json.dumps(adaptive_case(args, log)), flush=True)
        return
    V, T, prm = W.workload(args.workload)
    n, k = len(T), prm["k"]
    log(f"[bench] workload {args.workload}: N={n} k={k}")
    t0 = time.perf_counter()
    popt = prm.get("plan", {})  # build options of the workload's configuration
    plan = Plan(V, T, k, prm["eps"], **popt)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    st = plan.stats()
    log(f"[bench] build phases (s): {[round(v, 3) for v in st['build_phase_seconds'][:7]]} "
        "(tree, G factors, translations, low-rank M2L, leaf operators, upload, near field)")
    log(f"[bench] build {build_s:.2f} s; depth {st['depth']} top {st['top_level']} pairs {st['m2l_pairs']} "
        f"ranks {st['rank_up']} p {st['p']} m2l low-rank max {st['m2l_rank_max']} mean "
        f"{[round(v, 1) for v in st['m2l_rank_mean']]} level flops {[round(v / 1e9, 3) for v in st['m2l_level_flops']]} GF")

    # the M2L launch autotuner (setup, outside the timed region)
    tune = None
    if not args.no_tune:
        t0 = time.perf_counter()
        tune = plan.autotune(reps=20)
        tune["seconds"] = round(time.perf_counter() - t0, 3)
        log(f"[bench] M2L autotune: {tune}")

    x = torch.from_numpy(W.complex_normal(n, 1, seed=0)).to("cuda")
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        plan.matvec(x, out=y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        plan.matvec(x, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / args.steps
    log(f"[bench] matvec {ms:.3f} ms ({args.steps} steps, wall {wall:.3f} s)")

    # many right-hand sides: 64 columns per product (plane-wave directions
    # become GEMM columns of every stage), reported as columns per second
    multi = {}
    if args.nrhs_multi > 1:
        xm = torch.from_numpy(np.ascontiguousarray(W.complex_normal(n, args.nrhs_multi, seed=1).T)).to("cuda")
        ym = torch.empty_like(xm)
        plan.matvec(xm, out=ym)
        torch.cuda.synchronize()
        reps = max(3, args.steps // 10)
        e0.record(stream)
        for _ in range(reps):
            plan.matvec(xm, out=ym)
        e1.record(stream)
        torch.cuda.synchronize()
        msm = e0.elapsed_time(e1) / reps
        # column 0 against the single-column product of the same vector
        y0 = plan.matvec(xm[0].contiguous())
        multi = dict(nrhs=args.nrhs_multi, ms_per_matvec=round(msm, 4),
                     columns_per_s=round(args.nrhs_multi * 1000.0 / msm, 2),
                     col0_rel_diff_vs_single=float(torch.linalg.norm(ym[0] - y0) / torch.linalg.norm(y0)))
        # per-stage times of the same product (every stage alone on one
        # stream) and the matrix-core rate of its M2L, M2M and L2L stages:
        # algorithmic flops of one column times the column count
        pm = plan.profile(xm, reps=2, out=ym)
        multi["stages_ms"] = {q: round(pm[q], 3) for q in ("near", "s2m", "m2m", "m2l", "l2l", "l2t", "perm", "total")}
        m2l_fl = args.nrhs_multi * sum(float(f) for f in st["m2l_level_flops"])
        rate = {"m2l": m2l_fl, "m2m": args.nrhs_multi * float(st["m2m_flops"]),
                "l2l": args.nrhs_multi * float(st["l2l_flops"])}
        multi["mfma_rate"] = {q: dict(tflops=round(f / (pm[q] * 1e-3) / 1e12, 2),
                                      frac_of_fp64_peak=round(f / (pm[q] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4))
                              for q, f in rate.items() if pm[q] > 0}
        log(f"[bench] nrhs={args.nrhs_multi}: {multi}")
        del xm, ym
        if not args.no_solve:
            # plane waves from nrhs_multi directions on a Fibonacci sphere,
            # solved together (one product of all unconverged columns per
            # GMRES step; each column stops on its own residual)
            dirs = W.fibonacci_directions(args.nrhs_multi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bm = plan.rhs_planewave(dirs)
            um, info = plan.solve(bm, tol=1e-5, restart=50, maxit=2000)
            torch.cuda.synchronize()
            multi["solve"] = dict(directions=args.nrhs_multi, seconds=round(time.perf_counter() - t0, 4),
                                  products=info["iterations"], converged=info["converged"],
                                  rel_residual_max=info["rel_residual"],
                                  column_iterations_max=max(info["col_iterations"]),
                                  column_iterations_mean=round(float(np.mean(info["col_iterations"])), 2))
            log(f"[bench] {args.nrhs_multi}-direction solve: {multi['solve']}")
            del bm, um
            torch.cuda.empty_cache()

    if args.calib_copy_mb > 0:
        # one elementwise kernel that reads and writes calib_copy_mb MiB each
        src = torch.empty(args.calib_copy_mb * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mb} MiB done")
        del src, dst

    prof = plan.profile(x, reps=max(3, min(20, args.steps)), out=y)
    log(f"[bench] stages (ms): {prof}")
    log(f"[bench] near nnz {st['near_nnz']} ({st['near_nnz'] * 16 / (prof['near'] * 1e-3) / 1e9:.0f} GB/s of FP64 entries); "
        f"M2M {st['m2m_flops'] / 1e9:.3f} GF -> {st['m2m_flops'] / (prof['m2m'] * 1e-3) / 1e12:.2f} TF/s; "
        f"L2L {st['l2l_flops'] / 1e9:.3f} GF -> {st['l2l_flops'] / (prof['l2l'] * 1e-3) / 1e12:.2f} TF/s")
    y_np = y.cpu().numpy()

    # roofline of the dominant kernel: the M2L product kernel.  Every
    # low-rank level runs in one launch of k_m2l_lowrank; levels whose
    # translations stay full rank (none at this size) run k_ggemm.
    # Algorithmic flops = 8 real flops per complex multiply-add of the
    # SVD-reduced translations (unpadded ranks), summed over the levels,
    # divided by the HIP-event duration of the launch(es) on the plan's stream.
    full = [l for l in range(st["depth"] + 1) if st["m2l_level_flops"][l] > 0 and st["m2l_rank_max"][l] == 0]
    lowr = [l for l in range(st["depth"] + 1) if st["m2l_level_flops"][l] > 0 and st["m2l_rank_max"][l] > 0]
    lr_flops = sum(float(st["m2l_level_flops"][l]) for l in lowr)
    lr_ms = prof["m2l_lowrank"]
    if lowr and lr_ms > 0:
        achieved = lr_flops / (lr_ms * 1e-3) / 1e12
        roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=round(achieved / FP64_PEAK_TFLOPS, 4), traffic=None,
                        kernel=f"k_m2l_lowrank<double2> (M2L, levels {lowr} in one launch)", launches_per_matvec=1,
                        flops_per_launch=lr_flops, avg_launch_ms=round(lr_ms, 5),
                        full_rank_levels=full,
                        # every distinct factor once, every outgoing state
                        # read once, every incoming state written once
                        algorithmic_bytes=int(st["m2l_factor_bytes"] + st["m2l_state_bytes"]))
    else:
        ms_f = sum(prof["m2l_gemm"][l] for l in full)
        fl_f = sum(float(st["m2l_level_flops"][l]) for l in full)
        achieved = fl_f / (ms_f * 1e-3) / 1e12 if ms_f > 0 else 0.0
        roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=round(achieved / FP64_PEAK_TFLOPS, 4), traffic=None,
                        kernel=f"k_ggemm<double2> (M2L, levels {full})", launches_per_matvec=len(full),
                        flops_per_launch=fl_f / max(1, len(full)), avg_launch_ms=round(ms_f / max(1, len(full)), 5))
    if args.traffic_json and os.path.exists(args.traffic_json):
        # HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes,
        # scaled by the same counters' reading for a plain copy of known size;
        # only valid while the kernel source is the one that was measured
        import hashlib

        tj = json.load(open(args.traffic_json))
        src = os.path.join(ROOT, tj.get("source", ""))
        if os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == tj.get("source_sha256"):
            roofline["traffic"] = tj.get("bytes_per_launch")

    solve = {}
    if not args.no_solve:
        b = plan.rhs_planewave(prm["direction"])
        torch.cuda.synchronize()
        for pc in ("none", "block_jacobi"):
            t0 = time.perf_counter()
            u, info = plan.solve(b, tol=1e-5, restart=50, maxit=2000, precond=pc)
            torch.cuda.synchronize()
            solve[pc] = dict(seconds=round(time.perf_counter() - t0, 4), iterations=info["iterations"],
                             rel_residual=info["rel_residual"], converged=info["converged"])
            log(f"[bench] solve {pc}: {solve[pc]}")

    # fast arm: FP32 storage and FP32 matrix cores, FP64 self terms and Arnoldi
    fast = {}
    if not args.no_fast:
        plan32 = Plan(V, T, k, prm["eps"], prec="fp32", **popt)
        tune32 = None if args.no_tune else plan32.autotune(reps=20)
        y32 = torch.empty_like(x)
        for _ in range(args.warmup):
            plan32.matvec(x, out=y32)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            plan32.matvec(x, out=y32)
        e1.record(stream)
        torch.cuda.synchronize()
        ms32 = e0.elapsed_time(e1) / args.steps
        prof32 = plan32.profile(x, reps=max(3, min(20, args.steps)), out=y32)
        fast = dict(matvecs_per_s=round(1000.0 / ms32, 3), ms_per_matvec=round(ms32, 4),
                    stages_ms={q: round(v, 4) for q, v in prof32.items() if q != "m2l_gemm"}, m2l_autotune=tune32)
        if prof32["m2l_lowrank"] > 0:
            a32 = lr_flops / (prof32["m2l_lowrank"] * 1e-3) / 1e12
            fast["m2l_roofline"] = dict(achieved=round(a32, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                                        frac=round(a32 / FP32_PEAK_TFLOPS, 4),
                                        kernel="k_m2l_lowrank<float2> (one launch)")
        if not args.no_solve:
            b32 = plan32.rhs_planewave(prm["direction"])
            pcs = ["none", "block_jacobi"]
            if os.path.exists(args.mlp_weights):
                from paper_1403_4747_amd import train_mlp

                net = train_mlp.load(args.mlp_weights)
                plan32.set_mlp(net)
                pcs.append("mlp")
            for pc in pcs:
                t0 = time.perf_counter()
                u32, info = plan32.solve(b32, tol=1e-5, restart=50, maxit=2000, precond=pc)
                torch.cuda.synchronize()
                fast["solve_" + pc] = dict(seconds=round(time.perf_counter() - t0, 4), iterations=info["iterations"],
                                           rel_residual=info["rel_residual"], converged=info["converged"])
                if pc == "mlp":
                    fast["solve_mlp"].update(mlp_rejected=info["mlp_rejected"], mlp_fallbacks=info["mlp_fallbacks"],
                                             weights=os.path.relpath(args.mlp_weights, ROOT),
                                             held_out=mlp_held_out(args.mlp_weights))
            # difference of the two arms' solutions (surface field)
            u64, _ = plan.solve(b, tol=1e-5, restart=50, maxit=2000)
            fast["solution_rel_diff_vs_fp64_arm"] = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
        if args.nrhs_multi > 1:
            # the same many-column product on the FP32 plan
            xm = torch.from_numpy(np.ascontiguousarray(W.complex_normal(n, args.nrhs_multi, seed=1).T)).to("cuda")
            ym = torch.empty_like(xm)
            plan32.matvec(xm, out=ym)
            torch.cuda.synchronize()
            reps = max(3, args.steps // 10)
            e0.record(stream)
            for _ in range(reps):
                plan32.matvec(xm, out=ym)
            e1.record(stream)
            torch.cuda.synchronize()
            msm = e0.elapsed_time(e1) / reps
            fast["multi_rhs"] = dict(nrhs=args.nrhs_multi, ms_per_matvec=round(msm, 4),
                                     columns_per_s=round(args.nrhs_multi * 1000.0 / msm, 2))
            del xm, ym
        fast["y32"] = y32.cpu().numpy()
        plan32.close()
        log("[bench] fast arm: " + str({q: v for q, v in fast.items() if q != 'y32'}))

    batch = {}
    if args.batch > 0:
        batch = uneven_batch_leg(args.batch, args.steps, log, tune=not args.no_tune)

    cpu, err = (None, None)
    if not args.no_cpu:
        cpu, err, rows, yr = cpu_baseline(V, T, k, W.complex_normal(n, 1, seed=0), y_np, 32768, args.cpu_seconds)
        log(f"[bench] cpu baseline {cpu}, sampled-row rel err {err:.3e}")
        if "y32" in fast:
            fast["matvec_rel_err_vs_oracle_sampled"] = float(np.linalg.norm(fast["y32"][rows] - yr) / np.linalg.norm(yr))
    fast.pop("y32", None)

    out = {
        "metric": "FDA matvecs/s (N=81,920, kD=100); GMRES time-to-1e-5 reported alongside",
        "value": round(1000.0 / ms, 3),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": n, "k": k, "kD": k * 2 * prm["radius"],
                   "eps": prm["eps"], "svd_eps": popt.get("svd_eps", prm["eps"] / 10),
                   "nrhs": 1, "arm": "plain FP64"},
        "build_seconds": round(build_s, 3),
        "m2l_autotune": tune,
        "build_phase_seconds": [round(v, 3) for v in st["build_phase_seconds"][:7]],
        "stages_ms": {q: round(v, 4) for q, v in prof.items() if q != "m2l_gemm"},
        "m2l_lowrank_ms": round(prof["m2l_lowrank"], 4),
        "m2l_flops_per_matvec": st["m2l_flops"],
        "time_to_1e-5_s": solve.get("none", {}).get("seconds"),
        "build_plus_solve_s": round(build_s + solve["none"]["seconds"], 3) if "none" in solve else None,
        "multi_rhs": multi or None,
        "uneven_batch": batch or None,
        "solve": solve,
        "matvec_rel_err_vs_oracle_sampled": err,
        "fast_arm_fp32": fast or None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
