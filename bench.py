#!/usr/bin/env python
"""Benchmark: V-cycle-preconditioned FGMRES solves of the H(div)-DG Brinkman problem.

Default workload (C5, the largest configuration): 2048 x 2048 quads, 11 levels,
RT_2 x dQ_2, Brinkman mu = 1e-2, 85 log-normal permeability layers with channels,
16 smooth random right-hand sides, right-hand sides already in HBM.  One step = one
complete solve of the 16 right-hand sides (FP64 flexible GMRES per column to a 1e-10
relative residual, the variable V-cycle of Section 3.2 as preconditioner in FP32 with
bfloat16-stored patch inverses: level operators, colour-ordered vertex-patch
smoother, transfers, coarse solve).

Prints one JSON line: right-hand sides solved per second (whole job), DoF*iterations/s,
the plain FP64 V-cycle beside it, the roofline of the finest-level colour step (HIP
events around its launches), a measured device copy and the CPU oracle timed on a
bounded sample.  --workload C2 runs the 256^2 RT_1 configuration (FP64, FP32 and
bfloat16 V-cycles, standard cycle, 16-column batch).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "precond. solves/sec & DoF·iters/s to 1e-10 rel resid; mixed vs FP64, HBM %"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernels_sha16():
    """First 16 hex digits of the sha256 of the 2-D kernel sources (kernels.hip, then the
    colour-step bodies it includes): the version of the kernels a stored counter reading
    belongs to."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "colour_body.inc", "colour_kernel.inc", "colour_mr_kernel.inc"):
        with open(os.path.join(ROOT, "paper_1602_04858_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(profile):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary in
    profiles/ (KiB per dispatch, each scaled by what the counter reads for a plain copy
    of known size), or None if the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    for line in open(path):
        line = line.strip()
        if line.startswith("counters:"):
            kv = dict(t.split("=") for t in line.split()[1:])
            if kv.get("kernels_sha16") != kernels_sha16():
                return None
            return (float(kv["fetch_kib"]) * float(kv["fetch_factor"]) +
                    float(kv["write_kib"]) * float(kv["write_factor"])) * 1024.0
    return None


def timed_solves(torch, s, b, steps, warmup, rtol):
    x = s.zeros()
    info = None
    for _ in range(warmup):
        x, info = s.solve(b, rtol=rtol, maxit=1000, x=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(steps):
        x, info = s.solve(b, rtol=rtol, maxit=1000, x=x)
        its.append(max(i.iterations for i in info) if isinstance(info, list) else info.iterations)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return x, info, dt, its


def cpu_baseline(w, iterations_full, sample_its, colouring=0):
    """The oracle (plain FP64 CPU) on the same workload and smoother colouring: setup
    untimed, then the first `sample_its` FGMRES iterations timed and scaled to a full
    solve."""
    from oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    o = Oracle(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.kappa, w.cycle, w.m_fine, colouring)
    b = o.rhs(w.source)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, its, _, _ = o.fgmres(b, rtol=1e-10, maxit=sample_its, restart=100)
    dt = time.perf_counter() - t0
    per_it = dt / abs(its)
    solve_s = per_it * iterations_full
    out = {"value": 1.0 / solve_s, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"first {abs(its)} FGMRES iterations of the same solve ({dt:.1f} s, setup {t_setup:.1f} s "
                     f"untimed), scaled to the {iterations_full} iterations of the full solve",
           "seconds_per_iteration": per_it, "host": host_info()}
    omp_set = getattr(oracle_lib(), "omp_set_num_threads", None)
    if omp_set is not None:
        omp_set(1)
        t0 = time.perf_counter()
        _, its1, _, _ = o.fgmres(b, rtol=1e-10, maxit=2, restart=100)
        dt1 = time.perf_counter() - t0
        omp_set(threads)
        out["single_thread"] = {"value": 1.0 / (dt1 / abs(its1) * iterations_full), "unit": "solves/s",
                                "cores": 1, "sample": f"first {abs(its1)} iterations ({dt1:.1f} s)",
                                "seconds_per_iteration": dt1 / abs(its1)}
    return out


def bench_c4(args, torch, bmg, inputs):
    """C4: a batch of independent problems (N in {128, 256, 384, 512}, mu log-uniform
    in [1e-4, 1], per-problem kappa contrast), FP32 V-cycle inside FP64 FGMRES, solved
    together over several worker streams.  One step = one solve of every problem."""
    ws = [inputs.workload("C4", i) for i in range(args.problems)]
    dense = 4000
    params = [bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, bmg.P_FP32, 40, dense)
              for w in ws]
    t0 = time.perf_counter()
    batch = bmg.Batch(params, [w.kappa for w in ws], nstreams=args.streams)
    setup = time.perf_counter() - t0
    bs = [torch.as_tensor(bmg.assemble_rhs(p, w.source), dtype=torch.float64, device="cuda")
          for p, w in zip(params, ws)]
    ndofs = [batch.ndof(i) for i in range(len(ws))]
    log(f"bench: C4 {len(ws)} problems, {sum(ndofs)} dofs, setup {setup:.1f} s, {args.streams} streams")
    xs = None
    for _ in range(args.warmup):
        xs, infos, st = batch.solve(bs, rtol=args.rtol, maxit=1000, xs=xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xs, infos, st = batch.solve(bs, rtol=args.rtol, maxit=1000, xs=xs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    its = [i.iterations for i in infos]
    worst = max(i.rel_residual_true for i in infos)
    value = args.steps * len(ws) / dt
    log(f"bench: C4 {value:.2f} problems/s, iterations {min(its)}..{max(its)}, worst true residual {worst:.2e}")
    out = {"metric": "C4 batch: problems solved/s to 1e-10 rel resid (FP32 V-cycle in FP64 FGMRES)",
           "value": value, "unit": "problems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 preconditioner, f64 Krylov", "data": "synthetic",
           "config": {"workload": f"C4: {len(ws)} problems, N in {{128,256,384,512}}, RT_1, mu log-uniform "
                                  "[1e-4,1], seeded kappa contrast 1e4-1e6 + channels, smooth random f; "
                                  f"batch over {args.streams} streams, dense coarse <= {dense} dofs",
                      "problems": len(ws), "streams": args.streams, "rtol": args.rtol},
           "total_dofs": sum(ndofs), "iterations_min": min(its), "iterations_max": max(its),
           "dof_iters_per_s": sum(n * i for n, i in zip(ndofs, its)) * args.steps / dt,
           "worst_true_rel_residual": worst, "setup_s": setup, "status": st}
    print(json.dumps(out), flush=True)


def c5_cpu_baseline(nfull, its_full, n_sample=128, sample_its=10, single_its=2):
    """The oracle (plain FP64 CPU) on the C5 generator (RT_2, layered kappa, smooth
    source) at n_sample^2, one right-hand side: setup untimed, the first sample_its FGMRES
    iterations timed; the time per iteration and unknown is scaled to one right-hand side
    of the full workload at its iteration count (the full 2048^2 hierarchy does not fit
    the oracle's host memory)."""
    from oracle import Oracle
    from paper_1602_04858_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    w = inputs.scaled_workload("C5", n_sample)
    t0 = time.perf_counter()
    o = Oracle.from_workload(w)
    b = o.rhs(w.source)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, its, _, _ = o.fgmres(b, rtol=1e-10, maxit=sample_its, restart=8)
    dt = time.perf_counter() - t0
    per_it_dof = dt / abs(its) / o.ndof()
    solve_s = per_it_dof * nfull * its_full
    out = {"value": 1.0 / solve_s, "unit": "right-hand sides solved/s", "cores": threads, "kind": "oracle",
           "sample": f"C5 generator at {n_sample}x{n_sample} ({o.ndof()} unknowns), first {abs(its)} FGMRES(8) "
                     f"iterations ({dt:.1f} s; setup {t_setup:.1f} s untimed), time per iteration and unknown "
                     f"scaled to {nfull} unknowns x {its_full} iterations",
           "seconds_per_iteration_per_unknown": per_it_dof, "host": host_info()}
    # the same sample on one thread (the oracle's OpenMP runtime, set through its library)
    omp_set = getattr(oracle_lib(), "omp_set_num_threads", None)
    if omp_set is not None and single_its > 0:
        omp_set(1)
        t0 = time.perf_counter()
        _, its1, _, _ = o.fgmres(b, rtol=1e-10, maxit=single_its, restart=8)
        dt1 = time.perf_counter() - t0
        omp_set(threads)
        per1 = dt1 / abs(its1) / o.ndof()
        out["single_thread"] = {"value": 1.0 / (per1 * nfull * its_full), "unit": "right-hand sides solved/s",
                                "cores": 1, "sample": f"first {abs(its1)} iterations ({dt1:.1f} s)",
                                "seconds_per_iteration_per_unknown": per1}
    return out


def oracle_lib():
    from oracle import lib
    return lib()


def host_info():
    """nproc, CPU model and memory of the host the CPU baseline ran on."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    info["mem_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def bench_c5(args, torch, bmg, inputs):
    """C5 (the largest configuration): 2048^2 quads, 11 levels, RT_2 x dQ_2, Brinkman
    mu = 1e-2, 85 log-normal layers + channels, 16 smooth random right-hand sides solved
    together (FP64 FGMRES per column, lockstep), variable V-cycle with FP32 arithmetic
    and bfloat16-stored patch inverses; the patch products of the interior patches are
    MFMA tiles.  One step = one solve of all 16 right-hand sides to 1e-10.  Beside it:
    the plain FP64 V-cycle on one right-hand side (a 16-column FP64 Krylov basis does not
    fit in HBM at this size), the finest-level colour step's roofline, a device copy and
    the CPU oracle on a bounded sample."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    n, R = args.n, args.rhs
    w = inputs.workload("C5") if n == 2048 else inputs.scaled_workload("C5", n)
    restart = args.restart
    log(f"bench: C5 at {w.n}^2, k=2, {R} right-hand sides, FGMRES({restart}), bf16 inverses, fp32 V-cycle")
    p = bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, bmg.P_BF16, restart,
                        args.dense_coarse_max, R)
    srcs = [inputs.smooth_source(5100 + c) for c in range(R)]
    with ThreadPoolExecutor(min(16, R)) as ex:
        cols = list(ex.map(lambda f: bmg.assemble_rhs(p, f), srcs))
    B = torch.as_tensor(np.stack(cols), dtype=torch.float64, device="cuda")
    del cols
    t0 = time.perf_counter()
    s = bmg.Solver(p, w.kappa)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    ndof = s.ndof()
    log(f"bench: setup {setup:.1f} s, {ndof} unknowns per right-hand side")
    x = s.zeros()
    for i in range(args.warmup):
        x, infos = s.solve(B, rtol=args.rtol, maxit=200, x=x)
        log(f"bench: warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_all = []
    for i in range(args.steps):
        x, infos = s.solve(B, rtol=args.rtol, maxit=200, x=x)
        its_all.append([inf.iterations for inf in infos])
        log(f"bench: step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    its = its_all[-1]
    worst = max(inf.rel_residual_true for inf in infos)
    conv = all(inf.converged == 1 for inf in infos)
    value = args.steps * R / dt
    log(f"bench: mixed {value:.3f} right-hand sides/s ({dt / args.steps:.2f} s per step), iterations "
        f"{min(its)}..{max(its)}, worst true residual {worst:.2e}")
    # roofline of the finest-level colour step: HIP events around its launches (one V-cycle)
    J = w.levels
    s.kernel_timing(J, 34 * 4)
    s.vcycle(B)
    nl, ms, by = s.kernel_timing_read()
    s.kernel_timing(-1, 0)
    avg_s = ms * 1e-3 / nl
    achieved = by / nl / avg_s / 1e9
    traffic = stored_traffic("colour_step_c5_counters.md") if w.n == 2048 and R == 16 else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_colour_mr<2> (interior patches, MFMA) + k_colour boundary list, finest-level colour step",
            "launches": nl, "avg_us": avg_s * 1e6, "bytes_per_launch": by / nl}
    if traffic is not None:
        roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["traffic_over_algorithmic"] = traffic / (by / nl)
        roof["traffic_source"] = "profiles/colour_step_c5_counters.md"
    log(f"bench: finest colour step {achieved:.0f} GB/s, {avg_s * 1e6:.0f} us per step")
    x0 = x[0].clone()
    s.close()
    del s, x
    torch.cuda.empty_cache()
    # a STREAM-style device copy (2 GiB read + 2 GiB written, HIP events)
    src = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roof["measured_copy_gbs"] = copy_gbs
    roof["frac_of_measured_copy"] = achieved / copy_gbs
    out = {"metric": METRIC, "value": value, "unit": "right-hand sides solved/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 V-cycle with bf16-stored patch inverses (bf16 MFMA, f32 accumulate), f64 FGMRES",
           "data": "synthetic",
           "config": {"workload": f"C5: {w.n}x{w.n} quads, {w.levels + 1} levels (2x2 coarsest), RT_2 x dQ_2 "
                                  "H(div)-DG Brinkman mu=0.01, 85 log-normal kappa layers (log10 in [-6,1]) + "
                                  f"meandering channels, {R} smooth random right-hand sides solved together, "
                                  "no-slip left/right, open top/bottom; variable V-cycle m=2, multiplicative "
                                  f"vertex-patch smoother, FP64 FGMRES({restart}) per right-hand side, rtol "
                                  f"{args.rtol:g}",
                      "N": w.n, "levels": w.levels + 1, "k": w.k, "mu": w.mu, "n_rhs": R, "restart": restart,
                      "rtol": args.rtol},
           "ndof_per_rhs": ndof, "iterations_min": min(its), "iterations_max": max(its),
           "dof_iters_per_s": ndof * sum(sum(i) for i in its_all) / dt, "worst_true_rel_residual": worst,
           "converged": conv, "setup_s": setup}
    # the plain FP64 path beside it: FP64 V-cycle (FP64 rotated inverses), one right-hand side
    if not args.no_mixed:
        p64 = bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, bmg.P_FP64, restart,
                              args.dense_coarse_max, 1)
        t0 = time.perf_counter()
        s64 = bmg.Solver(p64, w.kappa)
        torch.cuda.synchronize()
        setup64 = time.perf_counter() - t0
        b0 = B[0].contiguous()
        t0 = time.perf_counter()
        x64, i64 = s64.solve(b0, rtol=args.rtol, maxit=200)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        diff = (torch.linalg.norm(x0 - x64) / torch.linalg.norm(x64)).item()
        out["fp64"] = {"value": 1.0 / dt64, "unit": "right-hand sides solved/s", "n_rhs": 1,
                       "precond": "fp64 V-cycle, fp64 rotated patch inverses", "iterations": i64.iterations,
                       "true_rel_residual": i64.rel_residual_true, "setup_s": setup64}
        out["speedup_mixed_vs_fp64"] = value * dt64
        out["rel_diff_mixed_vs_fp64_column0"] = diff
        log(f"bench: FP64 {1.0 / dt64:.3f} right-hand sides/s ({i64.iterations} iterations, setup {setup64:.1f} s), "
            f"mixed/fp64 {value * dt64:.2f}x, column 0 difference {diff:.1e}")
        s64.close()
        del s64, x64
    out["roofline"] = roof
    if not args.no_cpu_baseline:
        log("bench: CPU oracle sample")
        out["cpu_baseline"] = c5_cpu_baseline(ndof, max(its))
        out["cpu_baseline"]["note"] = "per right-hand side; the GPU value counts all 16 solved together"
    print(json.dumps(out), flush=True)


def bench_d3(args, torch, bmg, inputs):
    """3-D Brinkman / Darcy (Section 4, SPE10-like layered kappa stand-in): RT_k x dQ_k
    (--k3: 1, or 0 for the lowest order the paper's 128^3 SPE10 run uses) on an n^3
    hexahedral mesh, mu = --mu3, g = (1, 0, 0) on the Dirichlet sides (--bc3 marks open
    ones), f = 0, FP64 V-cycle in FP64 FGMRES to --rtol."""
    import numpy as np
    n = args.n3
    # the coarsest mesh, inverted densely: 8^3 for RT_0 (2240 unknowns), 4^3 for RT_1
    # (2240 unknowns; its 8^3 would be 17152)
    n0 = args.coarse3 or (8 if args.k3 == 0 else 4)
    levels = int(round(math.log2(n // n0))) + 1  # coarsest mesh n0^3, solved densely
    kap = inputs.kappa_layered3(n, 6000)
    k3, mu3 = args.k3, args.mu3
    bc3 = tuple(int(v) for v in args.bc3.split(","))
    sig3 = (k3 + 1) * (k3 + 2)
    p = bmg.make_params3(n0, levels, mu3, sigma=sig3, restart=50, k=k3, bc=bc3)
    t0 = time.perf_counter()
    s = bmg.Solver3(p, kap)
    setup = time.perf_counter() - t0
    b = torch.as_tensor(bmg.assemble_rhs3(p, kap, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0)), device="cuda")
    ndof = s.ndof()
    log(f"bench: 3-D N={n} levels={levels} ndof {ndof}, setup {setup:.1f} s")
    for _ in range(args.warmup):
        x, info = s.solve(b, rtol=args.rtol, maxit=500)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(args.steps):
        x, info = s.solve(b, rtol=args.rtol, maxit=500)
        its.append(info.iterations)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = torch.empty_like(b)
    # one V-cycle timed alone (HIP events on the solver's stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    for _ in range(3):
        r = s.vcycle(b)
    ev1.record(s.stream)
    ev1.synchronize()
    vc_ms = ev0.elapsed_time(ev1) / 3
    log(f"bench: 3-D {args.steps / dt:.3f} solves/s, iterations {its}, true residual "
        f"{info.rel_residual_true:.2e}, V-cycle {vc_ms:.2f} ms")
    x64 = x.clone()
    s.close()
    # FP32-stored patch pseudo-inverses (FP64 arithmetic): half the bytes of the
    # bandwidth-bound fine-level colour steps
    mixed = None
    if not args.no_mixed:
        p32 = bmg.make_params3(n0, levels, mu3, sigma=sig3, restart=50, prec=bmg.P_FP32, k=k3, bc=bc3)
        t0 = time.perf_counter()
        s32 = bmg.Solver3(p32, kap)
        setup32 = time.perf_counter() - t0
        for _ in range(args.warmup):
            x32, i32 = s32.solve(b, rtol=args.rtol, maxit=500)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its32 = []
        for _ in range(args.steps):
            x32, i32 = s32.solve(b, rtol=args.rtol, maxit=500)
            its32.append(i32.iterations)
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t0
        err = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
        mixed = {"value": args.steps / dt32, "unit": "solves/s", "precond": "fp32-stored patch inverses, fp64 "
                 "arithmetic", "iterations": its32[-1], "true_rel_residual": i32.rel_residual_true,
                 "rel_diff_vs_fp64": err, "speedup_vs_fp64": (args.steps / dt32) / (args.steps / dt),
                 "setup_s": setup32}
        log(f"bench: 3-D fp32 inverses {args.steps / dt32:.3f} solves/s, iterations {its32}, diff {err:.1e}")
        s32.close()
    # standard V-cycle (m = 2 smoothing steps on every level) beside the paper's variable
    # one: the coarse levels (latency-bound launches) then smooth 4x / 2x less
    std = None
    if not args.no_mixed:
        ps = bmg.make_params3(n0, levels, mu3, sigma=sig3, restart=50, cycle=bmg.CYCLE_STANDARD, k=k3, bc=bc3)
        ss = bmg.Solver3(ps, kap)
        for _ in range(args.warmup):
            xs, infs = ss.solve(b, rtol=args.rtol, maxit=500)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        itss = []
        for _ in range(args.steps):
            xs, infs = ss.solve(b, rtol=args.rtol, maxit=500)
            itss.append(infs.iterations)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0
        std = {"value": args.steps / dts, "unit": "solves/s", "cycle": "standard, m=2 on every level",
               "iterations": itss[-1], "true_rel_residual": infs.rel_residual_true,
               "rel_diff_vs_variable": (torch.linalg.norm(xs - x64) / torch.linalg.norm(x64)).item()}
        log(f"bench: 3-D standard V-cycle {args.steps / dts:.3f} solves/s, iterations {itss}")
        ss.close()
    model = "Darcy" if mu3 == 0 else "Brinkman"
    sides = "all sides Dirichlet" if not any(bc3) else f"sides (x0,x1,y0,y1,z0,z1) {args.bc3} (1 = open)"
    out = {"metric": f"3-D {model} solves/s to {args.rtol:g} rel resid", "value": args.steps / dt,
           "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"3-D {model} {n}^3 hexahedra, RT_{k3} x dQ_{k3}, mu={mu3:g}, g=(1,0,0), "
                                  f"{sides}, f=0, 85-layer log-normal kappa (SPE10 stand-in), coarsest mesh {n0}^3, "
                                  "variable V-cycle m=2, FP64 FGMRES(50)", "N": n, "levels": levels, "k": k3,
                      "mu": mu3, "bc": list(bc3), "rtol": args.rtol},
           "ndof": ndof, "iterations": its[-1], "dof_iters_per_s": ndof * sum(its) / dt,
           "true_rel_residual": info.rel_residual_true, "setup_s": setup, "vcycle_ms": vc_ms}
    if mixed:
        out["mixed"] = mixed
    if std:
        out["standard_vcycle"] = std
    print(json.dumps(out), flush=True)


def bench_sweep(args, torch, bmg, inputs):
    """Robustness study standing in for the paper's Tables 1-2 (Section 4, characteristic
    permeability fields): GMRES iterations to a 1e-6 reduction of the residual for
    two-phase fields (foam walls, disjoint inclusions, connected inclusions; seeded
    128 x 128 images) with kappa = 1 / 10^-e (e = 4, 5, 6) in case (a) and the phases
    reversed in case (b), Darcy (mu = 0) and Brinkman (mu = 1e-2), h = 1/128, 1/256,
    1/512 (the image resolved by 1, 4, 16 cells per pixel).  RT_1 x dQ_1, variable V-cycle
    (m_J = 2), FP64 FGMRES(100), f = (1, 0), no-slip left / right, open top / bottom."""
    import numpy as np
    sizes = [int(v) for v in args.sweep_sizes.split(",")]
    rows = []
    t0 = time.perf_counter()
    for ki, kind in enumerate(inputs.PHASE_KINDS):
        for case in ("a", "b"):
            for model, mu in (("darcy", 0.0), ("brinkman", 1e-2)):
                for e in (4, 5, 6):
                    its = {}
                    for n in sizes:
                        kap = inputs.kappa_two_phase(kind, 7100 + ki, n, e, reverse=(case == "b"))
                        levels = int(round(math.log2(n // 2)))
                        p = bmg.make_params(2, levels, 1, mu, 6.0, (0, 0, 1, 1), 1, 2, bmg.P_FP64, 100, 16384)
                        s = bmg.Solver(p, kap)
                        b = torch.as_tensor(bmg.assemble_rhs(p, inputs.constant_source(1.0, 0.0)), device="cuda")
                        _, info = s.solve(b, rtol=1e-6, maxit=400)
                        its[n] = info.iterations if info.converged else -info.iterations
                        s.close()
                        del s
                    rows.append({"field": kind, "case": case, "model": model, "contrast": f"1e{e}",
                                 "iterations": {str(n): its[n] for n in sizes}})
                    log(f"bench: sweep {kind:10s} ({case}) {model:8s} 1e{e}: " +
                        " ".join(f"h=1/{n}: {its[n]}" for n in sizes) + f"  [{time.perf_counter() - t0:.0f} s]")
    out = {"metric": "GMRES iterations to 1e-6 residual reduction (robustness in h and contrast)",
           "unit": "iterations", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "two-phase kappa stand-ins for the foam / inclusion / connected-inclusion "
                                  "fields, RT_1, variable V-cycle m=2, FP64 FGMRES(100), rtol 1e-6",
                      "sizes": sizes},
           "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-sample-its", type=int, default=10)
    ap.add_argument("--oracle-check", action="store_true",
                    help="C2: also solve the workload with the oracle (about a minute on the host) and report "
                         "every leg's relative difference from its solution")
    ap.add_argument("--workload", default="C5", choices=["C2", "C3", "C3darcy", "C4", "C5", "D3", "sweep"],
                    help="C5 (default: 2048^2 RT_2, 16 right-hand sides, the largest configuration), C2 (256^2 "
                         "RT_1), the 1024^2 precision study, the 48-problem batch, the 3-D solver, or the "
                         "robustness sweep over two-phase fields (iteration counts)")
    ap.add_argument("--sweep-sizes", default="128,256,512", help="sweep: cells per side")
    ap.add_argument("--streams", type=int, default=4, help="C4: worker streams of the batch")
    ap.add_argument("--problems", type=int, default=48, help="C4: problems in the batch")
    ap.add_argument("--n", type=int, default=2048, help="C5: cells per side (the 2048^2 generator at this size)")
    ap.add_argument("--restart", type=int, default=7,
                    help="C5: FGMRES restart (16 FP64 basis columns of 113 M unknowns: 7 fits in HBM)")
    ap.add_argument("--rhs", type=int, default=16, help="C5: right-hand sides solved together")
    ap.add_argument("--n3", type=int, default=32, help="D3: cells per side of the 3-D mesh (a power of two)")
    ap.add_argument("--k3", type=int, default=1, choices=[0, 1], help="D3: Raviart-Thomas degree")
    ap.add_argument("--coarse3", type=int, default=0, choices=[0, 2, 4, 8],
                    help="D3: cells per side of the coarsest mesh, solved densely (0: 8 for RT_0, 4 for RT_1)")
    ap.add_argument("--mu3", type=float, default=1e-2, help="D3: viscosity (0: Darcy)")
    ap.add_argument("--bc3", default="0,0,0,0,0,0", help="D3: per side x0,x1,y0,y1,z0,z1: 0 Dirichlet, 1 open")
    ap.add_argument("--dense-coarse-max", type=int, default=16384,
                    help="levels up to this many dofs are applied as one precomputed dense matrix (0 = off)")
    ap.add_argument("--colouring", default="auto", choices=["S9", "L8", "auto"],
                    help="vertex colouring of the smoother (S9: 9 colours, 17 colour steps per smoothing "
                         "step; L8: 8 colours, 15; auto: the faster one per precision, timed by bmg_autotune "
                         "before the timed region)")
    ap.add_argument("--smoother", default="multiplicative", choices=["multiplicative", "additive"],
                    help="the paper's symmetric multiplicative smoother, or the additive variant over the same "
                         "patches (damping --omega)")
    ap.add_argument("--omega", type=float, default=0.25)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-MiB device buffer three times (a plain copy kernel of known "
                         "size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}); "
              "splitting problems, right-hand sides or the mesh across GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1602_04858_amd import bmg, inputs

    if args.copy_calibration > 0:
        n = args.copy_calibration << 17  # float64 elements in MIB MiB
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration, 3 copies of {args.copy_calibration} MiB")
        del src, dst

    if args.workload == "C4":
        return bench_c4(args, torch, bmg, inputs)
    if args.workload == "C5":
        return bench_c5(args, torch, bmg, inputs)
    if args.workload == "D3":
        return bench_d3(args, torch, bmg, inputs)
    if args.workload == "sweep":
        return bench_sweep(args, torch, bmg, inputs)

    w = inputs.workload(args.workload)
    log(f"bench: workload {w.name} N={w.n} levels={w.levels + 1} k={w.k} mu={w.mu}")
    colouring = bmg.COLOURING_L8 if args.colouring == "L8" else bmg.COLOURING_S9
    tuned = {}

    def choose(p, key):
        if args.colouring != "auto":
            return p
        best, ms = bmg.autotune(p, w.kappa)
        tuned[key] = {"chosen": "L8" if best.colouring == bmg.COLOURING_L8 else "S9", "ms_per_vcycle": ms}
        log(f"bench: autotune {key}: S9 {ms['S9']:.3f} ms, L8 {ms['L8']:.3f} ms per V-cycle -> "
            f"{tuned[key]['chosen']}")
        return best

    smoother = bmg.SMOOTHER_ADDITIVE if args.smoother == "additive" else bmg.SMOOTHER_MULTIPLICATIVE
    p64 = choose(bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, bmg.P_FP64, 100,
                                 args.dense_coarse_max, 1, colouring, smoother, args.omega), "fp64")
    t0 = time.perf_counter()
    s64 = bmg.Solver(p64, w.kappa)
    setup64 = time.perf_counter() - t0
    b = torch.as_tensor(bmg.assemble_rhs(p64, w.source), dtype=torch.float64, device="cuda")
    ndof = s64.ndof()
    log(f"bench: FP64 setup {setup64:.2f} s, ndof {ndof}")

    x64, info64, dt64, its64 = timed_solves(torch, s64, b, args.steps, args.warmup, args.rtol)
    value = args.steps / dt64
    log(f"bench: FP64 {value:.3f} solves/s, iterations {its64}, true residual {info64.rel_residual_true:.2e}")

    # roofline of the finest-level smoother kernel: events around its launches
    J = w.levels
    s64.kernel_timing(J, 34 * (max(its64) + 4))  # at least the launches of the finest smoother in one solve
    s64.solve(b, rtol=args.rtol, maxit=1000)
    nl, ms, by = s64.kernel_timing_read()
    s64.kernel_timing(-1, 0)
    avg_s = ms * 1e-3 / nl
    achieved = by / nl / avg_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_colour<double,double,1,1> (finest-level colour step)",
            "launches": nl, "avg_us": avg_s * 1e6, "bytes_per_launch": by / nl}
    log(f"bench: finest smoother {achieved:.0f} GB/s over {nl} launches, avg {avg_s * 1e6:.1f} us")
    # a STREAM-style copy on this GPU (2 GiB read + 2 GiB written per copy, HIP events)
    # as the attainable HBM rate beside the published peak
    src = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roof["measured_copy_gbs"] = copy_gbs
    roof["frac_of_measured_copy"] = achieved / copy_gbs
    log(f"bench: device copy {copy_gbs:.0f} GB/s; finest smoother at {achieved / copy_gbs:.2f} of it")

    std_cycle = None
    if args.workload == "C2" and not args.no_mixed:
        # the standard V-cycle (m_J = 2 smoothing steps on every level) beside the paper's
        # variable one (m_j = m_J 2^(J-j)): far fewer coarse-level launches, more iterations
        ps = bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, bmg.CYCLE_STANDARD, w.m_fine, bmg.P_FP64, 100,
                             args.dense_coarse_max, 1, p64.colouring, smoother, args.omega)
        ss = bmg.Solver(ps, w.kappa)
        xs, infs, dts, itss = timed_solves(torch, ss, b, args.steps, args.warmup, args.rtol)
        std_cycle = {"value": args.steps / dts, "unit": "solves/s", "precond": "fp64, standard V-cycle m=2",
                     "iterations": itss[-1], "true_rel_residual": infs.rel_residual_true,
                     "rel_diff_vs_variable": (torch.linalg.norm(xs - x64) / torch.linalg.norm(x64)).item()}
        log(f"bench: FP64 standard V-cycle {args.steps / dts:.3f} solves/s, iterations {itss}")
        ss.close()
        del ss

    col64 = "L8" if p64.colouring == bmg.COLOURING_L8 else "S9"
    out = {"metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt64 / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.n}x{w.n} quads, {w.levels + 1} levels (2x2 coarsest), RT_1 x dQ_1 "
                                  f"H(div)-DG {'Darcy' if w.mu == 0 else 'Brinkman'} mu={w.mu:g}, seeded log-normal "
                                  "kappa (log10 ~ N(-3,1.5) in [-6,0]) + 20 channels, f=(1,0), no-slip left/right, "
                                  "open top/bottom; variable V-cycle m=2, FP64 V-cycle inside FP64 FGMRES(100), "
                                  f"rtol 1e-10, {col64} colouring, {args.smoother} smoother",
                      "N": w.n, "levels": w.levels + 1, "k": w.k, "mu": w.mu, "rtol": args.rtol,
                      "colouring": col64, "smoother": args.smoother},
           "ndof": ndof, "iterations": its64[-1], "dof_iters_per_s": ndof * sum(its64) / dt64,
           "true_rel_residual": info64.rel_residual_true, "setup_s": setup64}

    sols = {"fp64": x64}  # the solutions compared with the oracle's (--oracle-check)
    if not args.no_mixed:
        for key, prec in (("mixed", bmg.P_FP32), ("mixed_bf16", bmg.P_BF16)):
            p32 = choose(bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, prec, 100,
                                         args.dense_coarse_max, 1, colouring, smoother, args.omega), key)
            s32 = bmg.Solver(p32, w.kappa)
            x32, info32, dt32, its32 = timed_solves(torch, s32, b, args.steps, args.warmup, args.rtol)
            s32.kernel_timing(J, 34 * (max(its32) + 4))
            s32.solve(b, rtol=args.rtol, maxit=1000)
            nl32, ms32, by32 = s32.kernel_timing_read()
            s32.kernel_timing(-1, 0)
            err = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
            out[key] = {"value": args.steps / dt32, "unit": "solves/s",
                        "precond": "fp32" if prec == bmg.P_FP32 else "fp32 arithmetic, bf16 patch inverses",
                        "iterations": its32[-1], "true_rel_residual": info32.rel_residual_true,
                        "rel_diff_vs_fp64": err, "speedup_vs_fp64": (args.steps / dt32) / value,
                        "dof_iters_per_s": ndof * sum(its32) / dt32,
                        "finest_smoother_gbs": by32 / (ms32 * 1e-3), "finest_smoother_avg_us": ms32 * 1e3 / nl32}
            log(f"bench: {key} {args.steps / dt32:.3f} solves/s, iterations {its32}, diff {err:.1e}, "
                f"finest smoother {by32 / (ms32 * 1e-3) / 1e9:.0f} GB/s")
            s32.close()
            del s32
            sols[key] = x32

    if not args.no_mixed and args.workload == "C2":
        # batched: 16 right-hand sides of the same problem solved together with the FP32
        # V-cycle (each column its own FGMRES; one V-cycle launch serves all columns).
        # C2 only: at 1024^2 sixteen FGMRES(100) bases would not fit in HBM
        R = 16
        pb = bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, bmg.P_FP32, 100,
                             args.dense_coarse_max, R, p64.colouring, smoother, args.omega)
        sb = bmg.Solver(pb, w.kappa)
        B = torch.stack([b] + [torch.as_tensor(bmg.assemble_rhs(pb, inputs.smooth_source(700 + c)), device="cuda")
                               for c in range(R - 1)]).contiguous()
        xb, infb, dtb, _ = timed_solves(torch, sb, B, args.steps, args.warmup, args.rtol)
        itsb = [i.iterations for i in infb]
        errb = (torch.linalg.norm(xb[0] - x64) / torch.linalg.norm(x64)).item()
        sols["mixed_batched_column0"] = xb[0].clone()
        sb.close()
        del sb
        # the same 16 columns with the FP64 V-cycle: the like-for-like FP64 rate
        pb64 = bmg.make_params(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.cycle, w.m_fine, bmg.P_FP64, 100,
                               args.dense_coarse_max, R, p64.colouring, smoother, args.omega)
        sb64 = bmg.Solver(pb64, w.kappa)
        xb64, infb64, dtb64, _ = timed_solves(torch, sb64, B, args.steps, args.warmup, args.rtol)
        sb64.close()
        del sb64
        errb64 = max((torch.linalg.norm(xb[c] - xb64[c]) / torch.linalg.norm(xb64[c])).item() for c in range(R))
        out["mixed_batched"] = {"value": args.steps * R / dtb, "unit": "right-hand sides solved/s", "n_rhs": R,
                                "precond": "fp32", "iterations_min": min(itsb), "iterations_max": max(itsb),
                                "worst_true_rel_residual": max(i.rel_residual_true for i in infb),
                                "rel_diff_vs_fp64_column0": errb,
                                "fp64_batched": {"value": args.steps * R / dtb64, "unit": "right-hand sides solved/s",
                                                 "iterations_max": max(i.iterations for i in infb64)},
                                "speedup_vs_fp64_batched": dtb64 / dtb,
                                "worst_rel_diff_vs_fp64_batched": errb64,
                                "speedup_vs_fp64_single": (args.steps * R / dtb) / value}
        log(f"bench: mixed batched ({R} right-hand sides) {args.steps * R / dtb:.2f} solves/s, iterations "
            f"{min(itsb)}..{max(itsb)}; FP64 batched {args.steps * R / dtb64:.2f} ({dtb64 / dtb:.2f}x)")
        xb, xb64 = None, None
    if std_cycle:
        out["standard_vcycle"] = std_cycle
    if tuned:
        out["autotune"] = tuned
    out["roofline"] = roof
    if not args.no_cpu_baseline and args.workload == "C2":
        log("bench: CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(w, its64[-1], args.cpu_sample_its, p64.colouring)
        if args.oracle_check:
            # every path's solution against a tightly converged oracle solve of the same workload
            from oracle import Oracle
            o = Oracle(w.n0, w.levels, w.k, w.mu, w.sigma, w.bc, w.kappa, w.cycle, w.m_fine, p64.colouring)
            xo, _, _, _ = o.fgmres(o.rhs(w.source), rtol=1e-13, maxit=400, restart=100)
            xo = torch.as_tensor(xo, device="cuda")
            out["rel_diff_vs_oracle"] = {k: (torch.linalg.norm(v - xo) / torch.linalg.norm(xo)).item()
                                         for k, v in sols.items()}
            log(f"bench: solutions vs oracle {out['rel_diff_vs_oracle']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
