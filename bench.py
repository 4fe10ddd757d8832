"""Benchmark: one step = one complete ieti_solve (load vector, d = B K~^{-1} f,
outer CG on F lambda = d to ||r|| <= 1e-8 ||r_0||, recovery of u, FP64
global residual) on the deformed square with 16x16 patches of uneven size and
degree (elements per patch column/row from {32,48,64,96}, degree from {2,3,4};
817,899 torn dofs), inexact local solves by flexible CG with FP64 multigrid
V-cycles (the p-robust tensor smoother of Sec. 4 on the finest level, Chebyshev
below) inside the FP64 outer CG.  Setup (planning, assembly, multigrid
hierarchy, primal basis, coarse factorisation) happens before the timed region;
f at the quadrature points is resident in HBM when timing starts.

Prints one JSON line: MDoF/s (torn dofs per second of solve time); the
roofline of the dominant kernel (with the tensor smoother the fused coarse part
of the V-cycles, with Chebyshev the finest-level sweep) and of the whole F
apply (every kernel of q = F p), from HIP events on the solver's stream over
the same number of steps run right after the timed ones (events around every
launch serialise the launches); the error of each measured solution against
the stored oracle samples (tests/golden); beside the headline the FP32 form,
the Chebyshev smoother, the plain FP64 exact-local form (speedups), the 4x4x4
cube and the 8x8 workload in their configurations' form (with the tensor
smoother and the plain form beside them); and the CPU oracle timed on all host
cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden_error(name, u):
    """Relative l2 over the stored oracle samples (64 per patch + 2000 global) and the largest sampled
    deviation over the oracle's max norm; u is the torn result on the host."""
    import numpy as np
    path = os.path.join(GOLDEN, f"full_{name}.json")
    try:
        g = json.load(open(path))
    except OSError:
        return None
    if "torn_positions" not in g:
        return None
    idx = np.asarray(g["torn_positions"])
    ref = np.asarray(g["values"])
    got = u[idx]
    return {"rel_l2_sampled": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "max_rel_sampled": float(np.abs(got - ref).max() / g["max_abs"]),
            "samples": int(len(idx))}


def measure(wl, golden_name, steps, warmup, profile=True, **opt):
    """Setup, warm-up, `steps` timed solves, then (profile) the same number of solves with kernel events."""
    import torch

    from paper_1705_04531_amd import Solver, _abi, options_for

    t0 = time.perf_counter()
    solver = Solver(wl.patches, options_for(wl, **opt))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    x = solver.quadrature(device=False)
    f = torch.from_numpy(wl.f(x)).to("cuda")
    u = torch.empty(solver.ndof_torn, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        solver.solve(f, u)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = solver.solve(f, u)
        stats.append(st)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    out = {"ms_per_step": ms, "setup_s": setup_s, "stats": stats[-1], "u": u.cpu().numpy()}
    if profile:
        solver.profile(True)
        t1 = time.perf_counter()
        for _ in range(steps):
            solver.solve(f, u)
        torch.cuda.synchronize()
        out["ms_per_step_with_events"] = (time.perf_counter() - t1) / steps * 1e3
        out["prof"] = {k: solver.profile_query(k) for k in range(_abi.IETI_KPROF_COUNT)}
        solver.profile(False)
    solver.close()
    out["error_vs_oracle"] = golden_error(golden_name, out["u"])
    return out


def rate(entry):
    """Algorithmic bytes over event-timed kernel time of a profiled class, against the HBM peak."""
    if not entry or entry["ms"] <= 0 or entry["launches"] == 0:
        return None
    gbs = entry["bytes"] / (entry["ms"] * 1e-3) / 1e9
    return {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "launches": entry["launches"], "avg_us": round(entry["ms"] / entry["launches"] * 1e3, 3),
            "bytes_per_launch": round(entry["bytes"] / entry["launches"])}


def summary(m, wl):
    st = m["stats"]
    out = {"ms_per_step": round(m["ms_per_step"], 3),
           "MDoF_per_s": round(wl.ndof_torn / (m["ms_per_step"] * 1e-3) / 1e6, 3),
           "setup_s": round(m["setup_s"], 3), "outer_iterations": st["outer_iterations"],
           "inner_iterations_mean": round(st["inner_iterations_mean"], 2),
           "global_residual": st["global_residual"], "error_vs_oracle": m["error_vs_oracle"]}
    if "prof" in m:
        from paper_1705_04531_amd import _abi
        out["f_apply"] = rate(m["prof"][_abi.IETI_KPROF_FAPPLY])
        out["finest_sweep"] = rate(m["prof"][_abi.IETI_KPROF_SMOOTH_FINE])
        out["coarse_part"] = rate(m["prof"][_abi.IETI_KPROF_COARSE])
    return out


# ---------------------------------------------------------------- CPU oracle on all host cores
def _oracle_worker(args):
    """One worker process: builds its blocks' oracle solvers, waits for the others, solves them."""
    blocks, barrier, q = args
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import ietidp

    with threadpool_limits(limits=1):
        full = W.deformed_16x16_mixed()
        solvers = []
        for (o0, o1) in blocks:
            sub = W.sub_block(full, (o0, o1), (4, 4))
            solvers.append((sub.ndof_torn, ietidp.IetiDP(sub)))
        barrier.wait()
        t0 = time.perf_counter()
        ndof, its = 0, []
        for n, ie in solvers:
            _, _, info = ie.solve(tol=1e-8)
            ndof += n
            its.append(info["iterations"])
        q.put((ndof, time.perf_counter() - t0, its))


def cpu_baseline():
    """The oracle (exact-local IETI-DP, FP64, SciPy/SuperLU) on the headline workload cut into its 16
    blocks of 4x4 patches (each block an independent multipatch problem with the same patches, geometry
    and f), the blocks spread over one worker process per host core (BLAS threads 1).  Each worker
    factorises its blocks, all start solving together; value = all blocks' torn dofs / wall time from the
    common start until the last worker finishes (d, CG to 1e-8, recovery; factorisation not included)."""
    import multiprocessing as mp

    cores = min(len(os.sched_getaffinity(0)), 16)
    blocks = [(i, j) for j in range(0, 16, 4) for i in range(0, 16, 4)]
    ctx = mp.get_context("fork")
    barrier = ctx.Barrier(cores + 1)
    q = ctx.Queue()
    per = [blocks[w::cores] for w in range(cores)]
    procs = [ctx.Process(target=_oracle_worker, args=((per[w], barrier, q),)) for w in range(cores)]
    t_setup = time.perf_counter()
    for p in procs:
        p.start()
    barrier.wait()
    t0 = time.perf_counter()
    res = [q.get() for _ in range(cores)]
    wall = time.perf_counter() - t0
    for p in procs:
        p.join()
    ndof = sum(r[0] for r in res)
    its = sorted(i for r in res for i in r[2])
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": ndof / wall / 1e6,
        "unit": "MDoF/s",
        "cores": cores,
        "host_cpu": f"{cpu}, {len(os.sched_getaffinity(0))} threads available",
        "kind": "oracle",
        "sample": (f"the 16x16 mixed workload cut into 16 independent 4x4-patch blocks ({ndof} torn dofs in "
                   f"total), {cores} worker processes with one BLAS thread each; exact local solves (SuperLU), "
                   f"CG to 1e-8 in {its[0]}-{its[-1]} iterations per block; value = dofs / wall time of the "
                   f"solves ({wall:.2f} s); factorisation setup ({t0 - t_setup:.1f} s wall) not included"),
    }


# ---------------------------------------------------------------- serving
def serve(args):
    """Serving stream: requests of mixed size (2D deformed square, grid {2,4,8}^2, p {2,3,4},
    n_el {16,...,128}, sine-series f) through the request loop.  Pass 1 submits all at once
    (saturated throughput X); pass 2 replays the stream's Poisson arrivals at 0.8 X and reports
    latency percentiles; the baseline solves the same requests one after another with FP64
    exact local solves."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1705_04531_amd import Server, _abi, options_for, quadrature_points

    reqs = W.serving_stream(seed=0, n_requests=args.requests)
    inputs = []
    for r in reqs:
        x = quadrature_points(r.workload.patches)
        inputs.append((r.workload, r.workload.f(x)))
    ndof = sum(wl.ndof_torn for wl, _ in inputs)
    opt = options_for(inputs[0][0])

    def run(rate_, slots, options):
        srv = Server(options, slots=slots)
        tick = []
        t0 = time.perf_counter()
        for i, (wl, f) in enumerate(inputs):
            if rate_:
                delay = t0 + reqs[i].arrival_unit / rate_ - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tick.append(srv.submit(wl.patches, f))
        lat, bad = [], 0
        for i, t in enumerate(tick):
            rc, u, st, times = srv.poll(t, wait=True)
            bad += rc != 0
            lat.append(times[2] - times[0])
            if (i + 1) % 64 == 0:
                print(f"[serve] {i + 1}/{len(tick)} done, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
        span = time.perf_counter() - t0
        srv.close()
        return span, np.array(lat), bad

    torch.cuda.synchronize()
    span_sat, lat_sat, bad = run(0.0, args.slots, opt)
    X = len(inputs) / span_sat
    span, lat, bad2 = run(0.8 * X, args.slots, opt)
    base_span, base_lat, bad3 = run(0.0, 1, options_for(inputs[0][0], local_solver=_abi.IETI_LOCAL_EXACT,
                                                         mg_precision=64, batch_dofs=0))
    out = {
        "metric": "serving solves/s and p50/p99 latency (Poisson arrivals at 0.8x saturated throughput)",
        "value": round(len(inputs) / span, 3),
        "unit": "solves/s",
        "higher_is_better": True,
        "n_gpus": 1,
        "dtype": "f64 outer / f32 MG",
        "data": "synthetic",
        "config": {"workload": f"serving stream, {len(inputs)} requests (seed 0), {ndof} torn dofs in total",
                   "slots": args.slots, "arrival_rate_per_s": round(0.8 * X, 3)},
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "saturated_solves_per_s": round(X, 3),
        "saturated_p50_ms": round(float(np.percentile(lat_sat, 50)), 2),
        "sequential_fp64_exact": {"solves_per_s": round(len(inputs) / base_span, 3),
                                  "p50_ms": round(float(np.percentile(base_lat, 50)), 2)},
        "speedup_vs_sequential": round(base_span / span_sat, 3),
        "failed": int(bad + bad2 + bad3),
    }
    print(json.dumps(out), flush=True)


WORKLOADS = {
    # name: (builder, golden file stem, MG precision of the configuration)
    "deformed16x16": ("deformed_16x16_mixed", "deformed16x16_mixed", 32),
    "deformed8x8": ("deformed_8x8", "deformed8x8_p3_n64", 64),
    "cube4": ("cube_4x4x4", "cube4x4x4_p2_n24", 32),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline (no FP32 form, plain form, other workloads)")
    ap.add_argument("--variants", action="store_true",
                    help="also time D-MG, MG-MG-S and the tensor smoother on the headline workload")
    ap.add_argument("--serve", action="store_true", help="serving benchmark instead of the solve benchmark")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--local-solver", choices=["mg", "exact_mg", "mg_saddle", "exact"], default="mg",
                    help="variant of the headline solver: mg (MG-MG, default), exact_mg (D-MG), mg_saddle (MG-MG-S), "
                         "exact (the plain FP64 exact-local form D-D, for profiling its kernels)")
    ap.add_argument("--smoother", choices=["chebyshev", "tensor"], default="tensor",
                    help="finest-level smoother of the headline: tensor (the p-robust smoother of Sec. 4, default) or "
                         "chebyshev")
    ap.add_argument("--precision", type=int, choices=[32, 64], default=64,
                    help="multigrid precision of the headline solver (the outer CG is always FP64)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="deformed16x16")
    ap.add_argument("--cheb-coarse", type=int, default=0,
                    help="Chebyshev degree on the coarser multigrid levels (0: the library's table)")
    ap.add_argument("--coarse-degree", type=int, choices=[0, 1], default=0,
                    help="1: degree-1 coarse levels with L2-projection transfers (Sec. 4)")
    ap.add_argument("--coarse-level", type=int, default=0,
                    help="first multigrid level of the fused per-patch coarse kernel (0: the library's choice, "
                         "-1: every level by batched launches)")
    ap.add_argument("--coarse-dofs", type=int, default=0,
                    help="largest multigrid level solved by its dense inverse (0: the library's default)")
    ap.add_argument("--prec-vcycles", type=int, default=0,
                    help="V-cycles per Dirichlet solve in the preconditioner (0: the library's default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 512 MiB FP64 tensor 3 times (scale for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the solver shards by patches across GPUs only in design, see the documentation)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve(args)
        return
    if args.calibrate_copy:
        import torch
        a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": a.numel() * 8}), flush=True)
        return

    # the CPU oracle runs first, in worker processes forked before this process loads the HIP library
    cpu = None
    if not args.no_cpu_baseline and args.workload == "deformed16x16":
        print("[bench] CPU oracle on all host cores", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    import workloads as W
    from paper_1705_04531_amd import _abi

    build_name, gname, cfg_prec = WORKLOADS[args.workload]
    wl = getattr(W, build_name)()
    tensor = args.smoother == "tensor"
    variant = {"mg": _abi.IETI_LOCAL_MG, "exact_mg": _abi.IETI_LOCAL_EXACT_MG,
               "mg_saddle": _abi.IETI_LOCAL_MG_SADDLE, "exact": _abi.IETI_LOCAL_EXACT}[args.local_solver]
    extra_opt = {"smoother": _abi.IETI_SMOOTHER_TENSOR} if tensor else {}
    print(f"[bench] headline {wl.name}, MG precision {args.precision}, {args.local_solver}", file=sys.stderr,
          flush=True)
    if args.coarse_level:
        extra_opt["coarse_level"] = args.coarse_level
    if args.coarse_degree:
        extra_opt["coarse_degree"] = args.coarse_degree
    if args.cheb_coarse:
        extra_opt["cheb_degree_coarse"] = args.cheb_coarse
    if args.coarse_dofs:
        extra_opt["coarse_dofs"] = args.coarse_dofs
    if args.prec_vcycles:
        extra_opt["prec_vcycles"] = args.prec_vcycles
    m = measure(wl, gname, args.steps, args.warmup, local_solver=variant, mg_precision=args.precision, **extra_opt)
    ms_per_step = m["ms_per_step"]
    value = wl.ndof_torn / (ms_per_step * 1e-3) / 1e6
    st = m["stats"]
    prof = m["prof"]
    mgt = "double" if args.precision == 64 else "float"
    # the kernel with the most time in the rocprofv3 trace of this command: with the tensor smoother the fused
    # coarse part of the V-cycles (k_vcoarse), with Chebyshev the finest-level sweep
    dom = prof[_abi.IETI_KPROF_COARSE if tensor else _abi.IETI_KPROF_SMOOTH_FINE]
    kr = rate(dom) or {"achieved": 0.0, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": 0.0}
    roofline = {
        "bound": "hbm",
        "kernel": (f"k_vcoarse<{mgt},false,{1 if wl.patches[0].dim == 3 else 0}> (fused coarse levels of every patch, one work-group per patch; "
                   f"events on the preconditioner's cycles, which run every patch)" if tensor else
                   f"k_stencil<{mgt},{mgt},{mgt},EPI_CHEB,FINE> (finest-level Chebyshev sweep, all degree "
                   f"classes in one launch)"),
        **kr,
        "traffic": None,
        "traffic_note": "counter traffic per launch is in profiles/ (rocprofv3 --pmc runs of this command)",
        "ms_per_step_with_events": round(m["ms_per_step_with_events"], 3),
        "f_apply": rate(prof[_abi.IETI_KPROF_FAPPLY]),
        "preconditioner": rate(prof[_abi.IETI_KPROF_PREC]),
        "apply64": rate(prof[_abi.IETI_KPROF_APPLY64]),
        "finest_residual_sweep": rate(prof[_abi.IETI_KPROF_RESID_FINE]),
        "finest_chebyshev_sweep": rate(prof[_abi.IETI_KPROF_SMOOTH_FINE]),
    }
    out = {
        "metric": "dual-PCG solve time & MDoF/s at rel. res 1e-8; solves/s + p50/p99 latency",
        "value": round(value, 3),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f64 outer / f32 MG",
        "data": "synthetic",
        "config": {
            "workload": wl.description + f", inexact local solves ({args.local_solver}) by FP{args.precision} "
                        f"multigrid, FP64 outer CG to 1e-8",
            "ndof_torn": wl.ndof_torn,
            "ndof_global": wl.ndof_global,
            "global_MDoF_per_s": round(wl.ndof_global / (ms_per_step * 1e-3) / 1e6, 3),
            "n_lambda": st["n_lambda"],
            "n_primal": st["n_primal"],
            "outer_iterations": st["outer_iterations"],
            "inner_iterations_mean": round(st["inner_iterations_mean"], 2),
            "inner_iterations_max": st["inner_iterations_max"],
            "global_residual": st["global_residual"],
            "time_pcg_ms": round(st["time_pcg_ms"], 3),
            "time_rhs_ms": round(st["time_rhs_ms"], 3),
            "time_recovery_ms": round(st["time_recovery_ms"], 3),
            "setup_s": round(m["setup_s"], 3),
            "local_solver": args.local_solver,
            "mg_precision": args.precision,
            "smoother": {"finest": args.smoother, "cheb_degree": st["cheb_degree"],
                         "cheb_degree_coarse": st["cheb_degree_coarse"],
                         "fine_tile_staged": st["fine_tile_staged"]},
            "error_vs_oracle": m["error_vs_oracle"],
        },
        "roofline": roofline,
    }
    if not args.no_extras and args.local_solver == "mg":
        extras = {}
        TENSOR = {"smoother": _abi.IETI_SMOOTHER_TENSOR}
        # the same workload: the other precision with the headline's smoother, the other smoother at the headline's
        # precision (each against the same oracle samples)
        other = 32 if args.precision == 64 else 64
        print(f"[bench] {wl.name} FP{other} multigrid", file=sys.stderr, flush=True)
        m2 = measure(wl, gname, min(args.steps, 3), 1, mg_precision=other, **extra_opt)
        extras[f"{args.smoother}_mg{other}"] = summary(m2, wl)
        alt = "chebyshev" if tensor else "tensor"
        print(f"[bench] {wl.name} {alt} smoother FP{args.precision}", file=sys.stderr, flush=True)
        m3 = measure(wl, gname, min(args.steps, 3), 1, mg_precision=args.precision, **({} if tensor else TENSOR))
        extras[f"{alt}_mg{args.precision}"] = summary(m3, wl)
        # the headline form with the inner iterations replayed as captured HIP graphs (same launches)
        print(f"[bench] {wl.name} graph replay", file=sys.stderr, flush=True)
        mg_ = measure(wl, gname, min(args.steps, 3), 1, profile=False, local_solver=variant,
                      mg_precision=args.precision, use_graph=1, **extra_opt)
        extras["graph_replay"] = {"ms_per_step": round(mg_["ms_per_step"], 3),
                                  "ms_per_step_direct": round(ms_per_step, 3),
                                  "bitwise_equal_to_direct": bool((mg_["u"] == m["u"]).all())}
        # the plain FP64 exact-local form (D-D; 2D: host band factors, 3D: device block-band factors)
        print(f"[bench] {wl.name} plain FP64 exact-local form", file=sys.stderr, flush=True)
        mp_ = measure(wl, gname, min(args.steps, 3), 1, profile=False, local_solver=_abi.IETI_LOCAL_EXACT,
                      mg_precision=64)
        plain = summary(mp_, wl)
        plain["speedup_inexact_headline_over_plain"] = round(mp_["ms_per_step"] / ms_per_step, 3)
        plain[f"speedup_inexact_{args.smoother}_mg{other}_over_plain"] = round(mp_["ms_per_step"] / m2["ms_per_step"], 3)
        extras["plain_fp64_exact_local"] = plain
        # the other full-size workloads in their configurations' form (Chebyshev smoother, the named precision),
        # with the tensor smoother and the plain form beside them
        for wname in sorted(WORKLOADS):
            if wname == args.workload:
                continue
            bname, gn, prec = WORKLOADS[wname]
            w2 = getattr(W, bname)()
            print(f"[bench] {w2.name} FP{prec} multigrid", file=sys.stderr, flush=True)
            mw = measure(w2, gn, min(args.steps, 3), 1, mg_precision=prec)
            e = dict(summary(mw, w2), mg_precision=prec, ndof_torn=w2.ndof_torn)
            mt = measure(w2, gn, min(args.steps, 3), 1, profile=False, mg_precision=prec, **TENSOR)
            e["tensor_smoother"] = summary(mt, w2)
            print(f"[bench] {w2.name} plain FP64 exact-local form", file=sys.stderr, flush=True)
            mpw = measure(w2, gn, min(args.steps, 3), 1, profile=False, local_solver=_abi.IETI_LOCAL_EXACT,
                          mg_precision=64)
            e["plain_fp64_exact_local"] = summary(mpw, w2)
            e["speedup_inexact_over_plain"] = round(mpw["ms_per_step"] / mw["ms_per_step"], 3)
            e["speedup_inexact_tensor_over_plain"] = round(mpw["ms_per_step"] / mt["ms_per_step"], 3)
            mgw = measure(w2, gn, min(args.steps, 3), 1, profile=False, mg_precision=prec, use_graph=1)
            e["graph_replay"] = {"ms_per_step": round(mgw["ms_per_step"], 3),
                                 "ms_per_step_direct": round(mw["ms_per_step"], 3),
                                 "bitwise_equal_to_direct": bool((mgw["u"] == mw["u"]).all())}
            extras[wname] = e
        if args.variants:
            for label, o in (("exact_mg64", {"local_solver": _abi.IETI_LOCAL_EXACT_MG, "mg_precision": 64}),
                             ("exact_mg32", {"local_solver": _abi.IETI_LOCAL_EXACT_MG, "mg_precision": 32}),
                             ("saddle_mg64", {"local_solver": _abi.IETI_LOCAL_MG_SADDLE, "mg_precision": 64}),
                             ("saddle_mg32", {"local_solver": _abi.IETI_LOCAL_MG_SADDLE, "mg_precision": 32}),
                             ("tensor_saddle_mg32", {"smoother": _abi.IETI_SMOOTHER_TENSOR, "mg_precision": 32,
                                                     "local_solver": _abi.IETI_LOCAL_MG_SADDLE}),
                             ("tensor_degree1_coarse_mg64", {"smoother": _abi.IETI_SMOOTHER_TENSOR,
                                                             "mg_precision": 64, "coarse_degree": 1})):
                print(f"[bench] {wl.name} {label}", file=sys.stderr, flush=True)
                extras[label] = summary(measure(wl, gname, min(args.steps, 3), 1, profile=False, **o), wl)
        out["extras"] = extras
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
