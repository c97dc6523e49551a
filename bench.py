"""Newton-step benchmark of the nested block solver on one MI355X.

Workload (default): the synthetic contraction-expansion tube, ~4e6 nodes /
~1.6e7 DOFs (inlet r = 0.6, 20-degree cone to a throat r = 0.2 of length 4,
sudden expansion to r = 0.6 for length 12; throat Reynolds number 3500,
outlet resistance R = 1e5, dt = 5e-4).  One step = the forward hot path of
one Newton iteration: VMS tangent + residual assembly, per-step
preconditioner set-up, FP32-inner nested FGMRES solve to rtol 1e-8 and the
Newton update.  After the timed steps: the same tangent solved in the
all-FP64 form, the adjoint (transposed nested) solve, the streaming ceiling
of the device, and the CPU oracle on a bounded sample.

Prints one JSON line; `value` is the FP32-inner Newton-step solve time
(per-step set-up + Krylov iterations, median over the timed steps) in ms.

    python bench.py [--steps K --warmup W --config NAME --pc-A jacobi|amg]
    python bench.py --kernels --config NAME   # finest-level kernels alone, for counter runs
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Newton-step solve time @rtol 1e-8, FP32-inner vs FP64; BSR SpMV HBM GB/s"
HBM_PEAK_GBS = 8000.0
STREAM_BYTES = 2 << 30  # 2 GiB: far beyond the 256 MB last-level cache
KT_PERIOD = 4  # kernel classes timed on every 4th launch during the timed steps
LLC_BYTES = 256e6  # MI355X last-level (Infinity) cache


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def describe(case, nnzb):
    kinds = {"conexp": "contraction-expansion tube (r 0.6 -> 20-degree cone -> throat r 0.2, L 4 -> sudden "
                       "expansion to r 0.6, L 12), throat Re 3500, R = 1e5, dt 5e-4",
             "pipe": "straight pipe r 0.3, L 3, R = 1e3, dt 1e-3",
             "ybif": "Y-bifurcation, R = (1.5e3, 3e3), dt 1e-3"}
    k = next((v for key, v in kinds.items() if case.name.startswith(key)), case.name)
    return (f"{case.name}: {k}; {case.n_nodes} nodes, {4 * case.n_nodes} DOFs, {case.n_elems} tets, "
            f"nnzb {nnzb}; one Newton step (assembly + set-up + FP32-inner nested solve + update)")


def cpu_baseline(sample: str, solve_opts: dict):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the same
    recipe: assembly, then the per-step set-up and the nested solve with the
    benchmark's solver options; torch (the assembly's forward-mode AD) runs
    on every host core of the process, scipy's sparse products on one."""
    import torch

    from ns_inputs import build
    from oracle import amg, krylov
    from oracle import discretization as dz

    cores = len(os.sched_getaffinity(0))
    nthr = torch.get_num_threads()
    torch.set_num_threads(cores)
    try:
        case = build(sample)
        t0 = time.perf_counter()
        S = dz.assemble(case)
        t1 = time.perf_counter()
        ns = krylov.NestedSolver(S, amg.node_adjacency(case.n_nodes, case.tets), krylov.SolveOpts(**solve_opts))
        x, info = ns.solve(S.rhs)
        t2 = time.perf_counter()
    finally:
        torch.set_num_threads(nthr)
    return case, {
        "value": round(1e3 * (t2 - t1), 1),
        "unit": "ms",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{sample}: the same contraction-expansion recipe at {case.n_nodes} nodes "
                   f"({case.n_elems} tets); value = oracle (numpy/scipy, FP64) set-up + nested FGMRES solve to "
                   f"rtol 1e-8 with the benchmark's options ({info['outer']} outer iterations, true relative "
                   f"residual {info['true_rel_res']:.2e}); not extrapolated to the full mesh"),
        "assembly_ms": round(1e3 * (t1 - t0), 1),
        "threads": {"torch_assembly": cores, "scipy_sparse_solve": 1,
                    "omp_num_threads": os.environ.get("OMP_NUM_THREADS")},
    }


def kernel_source_sha():
    import hashlib
    src = open(os.path.join(ROOT, "paper_1911_10814_amd", "csrc", "kernels_la.hip"), "rb").read()
    return hashlib.sha256(src).hexdigest()[:16]


def measured_traffic(kernel_class: str, config: str):
    """HBM bytes per launch of a kernel class from the committed counter record
    (profiles/), or None when the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel_class}_{config}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_la_sha256_16") != kernel_source_sha():
        return None
    return rec["traffic_bytes_per_launch"]


def stream_ceiling(dev):
    """Hand-written streaming kernels (ns_stream_bench): read-only and copy
    GB/s over 2 GiB buffers."""
    import torch

    from paper_1911_10814_amd import stream_bench
    a = torch.ones(STREAM_BYTES, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    out = {"read_GBps": STREAM_BYTES / (stream_bench(0, a, b, 10) * 1e-3) / 1e9,
           "copy_GBps": 2 * STREAM_BYTES / (stream_bench(1, a, b, 10) * 1e-3) / 1e9,
           "bytes": STREAM_BYTES}
    del a, b
    torch.cuda.empty_cache()
    return {k: round(v, 1) if isinstance(v, float) else v for k, v in out.items()}


def layout_note(lay):
    """How the bound context stores the finest-level FP32 planes and column indices."""
    rows = f"fixed-width rows of {lay['ell']} blocks" if lay["ell_bound"] else "the node graph's rows"
    cols = "16-bit column offsets" if lay["col16_bound"] else "32-bit column indices"
    return f"FP32 tangent planes in {rows}; {cols}"


def kernels_mode(args):
    """Finest-level kernels launched on their own (the A operator SpMV, one
    AMG V-cycle of A, one V-cycle of S_hat with its factored finest level, one
    point-Jacobi GMRES A-solve for the CGS2 kernels) and a device copy of known
    size that calibrates the FETCH_SIZE / WRITE_SIZE counters; prints the
    algorithmic bytes per launch of the A operator."""
    import numpy as np
    import torch

    from ns_inputs import build
    from paper_1911_10814_amd import NsContext, SolveOptions, stream_bench

    case = build(args.config)
    log(f"kernels: {args.config}: {case.n_nodes} nodes built")
    ctx = NsContext(case).bind()
    ctx.assemble(case.v, case.p, case.vdot, rho=case.rho, mu=case.mu, dt=case.dt, rho_inf=case.rho_inf, R=case.R)
    log("kernels: bound and assembled")
    o = SolveOptions(precision=args.precision)
    x3 = torch.as_tensor(np.random.default_rng(0).standard_normal(3 * case.n_nodes), device="cuda")
    x1 = torch.as_tensor(np.random.default_rng(1).standard_normal(case.n_nodes), device="cuda")
    ctx.kernel_timing(("spmv_A",))
    ctx.kernel_timing_read("spmv_A")
    for _ in range(args.reps):
        ctx.apply("A", x3, o)
    torch.cuda.synchronize()
    a_launches, _, a_bytes = ctx.kernel_timing_read("spmv_A")
    ctx.kernel_timing(())
    for _ in range(args.reps):
        ctx.apply("vcycle_A", x3, o)
    for _ in range(args.reps):
        ctx.apply("vcycle_S", x1, o)
    # one GMRES A-solve with point Jacobi: the CGS2 kernels at short bases
    ctx.apply("solve_A", x3, SolveOptions(precision=args.precision, pc_A="jacobi", rtol_A=1e-3))
    log("kernels: operators done")
    copy_bytes = 512 << 20
    a = torch.ones(copy_bytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    ms = stream_bench(1, a, b, args.reps)
    N, nnzb = case.n_nodes, ctx.nnzb
    print(json.dumps({
        "config": args.config, "N": N, "nnzb": nnzb, "precision": args.precision, "reps": args.reps,
        "spmv_A_bytes": a_bytes / max(a_launches, 1),
        "copy_bytes_read": copy_bytes, "copy_bytes_written": copy_bytes, "copy_launches": args.reps + 1,
        "copy_GBps": 2 * copy_bytes / (ms * 1e-3) / 1e9, "kernels_la_sha256_16": kernel_source_sha(),
    }), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="conexp_4m")
    ap.add_argument("--pc-A", default="jacobi", choices=("jacobi", "amg"),
                    help="P_A of every A-solve (the paper's two options)")
    ap.add_argument("--fp64-reps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="conexp_60k")
    ap.add_argument("--kernels", action="store_true", help="launch the finest-level kernels alone (counter runs)")
    ap.add_argument("--precision", default="fp32_inner")
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the solver runs on a single "
              "MI355X and its multi-GPU decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)
    if args.kernels:
        kernels_mode(args)
        return

    import numpy as np
    import torch

    from ns_inputs import build
    from paper_1911_10814_amd import NsContext, SolveOptions, gen_alpha

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    case = build(args.config)
    ctx = NsContext(case, device=dev).bind()
    log(f"{args.config}: N={case.n_nodes} E={case.n_elems} nnzb={ctx.nnzb} built + symbolic + bound in "
        f"{time.perf_counter() - t0:.1f}s, workspace {ctx.workspace_bytes / 1e9:.1f} GB")
    am, af, gam = gen_alpha(case.rho_inf)
    v = torch.as_tensor(case.v, device=dev)
    p = torch.as_tensor(case.p, device=dev)
    vd = torch.as_tensor(case.vdot, device=dev)
    y0 = torch.cat([v.reshape(-1), p])
    yd0 = torch.cat([vd.reshape(-1), torch.zeros_like(p)])
    solver_kw = dict(pc_A=args.pc_A)
    o32 = SolveOptions(precision="fp32_inner", **solver_kw)
    o64 = SolveOptions(precision="fp64", **solver_kw)
    classes = ("spmv_A", "cheb_A0", "spmv_full", "sfact", "cgs2", "cheb_S1")

    def assemble():
        return ctx.assemble(v, p, vd, rho=case.rho, mu=case.mu, dt=case.dt, rho_inf=case.rho_inf, R=case.R)

    def step():
        ts = {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        rhs = assemble()
        torch.cuda.synchronize()
        ts["assembly_ms"] = 1e3 * (time.perf_counter() - t)
        t = time.perf_counter()
        x, info = ctx.solve(rhs, o32)
        ts["solve_ms"] = 1e3 * (time.perf_counter() - t)
        y, yd = y0.clone(), yd0.clone()
        t = time.perf_counter()
        ctx.newton_update(gam * case.dt, x, y, yd)
        torch.cuda.synchronize()
        ts["update_ms"] = 1e3 * (time.perf_counter() - t)
        return ts, info, rhs, x

    # the kernel classes are timed with HIP events on the solver's stream
    # throughout (the launches record the events themselves), every
    # KT_PERIOD-th launch of each class, so that the events' own cost stays a
    # small part of the timed steps; the warm-up steps create the event pool,
    # the timed steps' samples are read after
    ctx.kernel_timing(classes, period=KT_PERIOD)
    for k in range(args.warmup):
        ts, info, _, _ = step()
        log(f"warm-up {k}: solve {ts['solve_ms']:.0f} ms, outer {info['outer_iters']} A {info['a_iters']} "
            f"S {info['s_iters']} inner {info['inner_iters']}")
    for k in classes:
        ctx.kernel_timing_read(k)
    torch.cuda.synchronize()
    times = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts, info, rhs, x32 = step()
        times.append(ts)
        log(f"step {k}: {ts} outer {info['outer_iters']} A-its {info['a_iters']} S-its {info['s_iters']} "
            f"inner-its {info['inner_iters']} res {info['true_rel_res']:.2e}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    kt = {k: ctx.kernel_timing_read(k) for k in classes}
    ctx.kernel_timing(())

    # all-FP64 form on the same tangent (re-assembled, so its set-up is timed too)
    f64 = []
    for k in range(args.fp64_reps):
        r = assemble()
        torch.cuda.synchronize()
        t = time.perf_counter()
        x64, i64 = ctx.solve(r, o64)
        i64["wall_ms"] = 1e3 * (time.perf_counter() - t)
        f64.append(i64)
        log(f"fp64 solve {k}: {i64['wall_ms']:.0f} ms, outer {i64['outer_iters']} res {i64['true_rel_res']:.2e}")
    n3 = 3 * case.n_nodes
    xa, xb = x32.cpu().numpy(), x64.cpu().numpy()
    err_v = float(np.linalg.norm(xa[:n3] - xb[:n3]) / np.linalg.norm(xb[:n3]))
    err_p = float(np.linalg.norm(xa[n3:] - xb[n3:]) / np.linalg.norm(xb[n3:]))

    # adjoint solve for d(outlet flow)/dx, FP32-inner, and the gradient contraction
    a = ctx.outlet_vectors()
    g = torch.zeros(4 * case.n_nodes, dtype=torch.float64, device=dev)
    g[:n3] = gam * case.dt * a[0].reshape(-1)
    del a
    torch.cuda.synchronize()
    t = time.perf_counter()
    lam, ainfo = ctx.adjoint(g, o32)
    adj_ms = 1e3 * (time.perf_counter() - t)
    grad = ctx.resistance_gradient(lam, x64)
    log(f"adjoint: {adj_ms:.0f} ms, outer {ainfo['outer_iters']}, dQ/dR {grad}")
    del lam, g

    stream = stream_ceiling(dev)
    log(f"stream ceiling: {stream}")

    solve32 = statistics.median(t["solve_ms"] for t in times)
    solve64 = statistics.median(i["wall_ms"] for i in f64)
    dom = max(kt, key=lambda k: kt[k][1])
    n_l, ms_l, by_l = kt[dom]
    achieved = (by_l / (ms_l * 1e-3)) / 1e9 if ms_l > 0 else None
    kernels = {k: {"launches_timed": n, "avg_us": round(1e3 * ms / n, 2) if n else None,
                   "GBps": round((b / (ms * 1e-3)) / 1e9, 1) if ms > 0 else None,
                   "ms_per_step_est": round(KT_PERIOD * ms / args.steps, 2)}
               for k, (n, ms, b) in kt.items()}
    out = {
        "metric": METRIC,
        "value": round(solve32, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_total / args.steps, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (inside P_SCR) / f64 (outer FGMRES, residual, update)",
        "data": "synthetic",
        "config": {"workload": describe(case, ctx.nnzb), "rtol": 1e-8, "rtol_A": 1e-3, "rtol_S": 1e-3,
                   "rtol_I": 1e-3, "P_A": args.pc_A, "P_S": "AMG(S_hat) V-cycle"},
        "matrix_layout": layout_note(ctx.layout()),
        "fp64_solve_ms": round(solve64, 3),
        "speedup_fp32_inner_vs_fp64": round(solve64 / solve32, 3),
        "fp32_inner_vs_fp64_rel_err": {"v": err_v, "p": err_p},
        "stage_ms_median": {k: round(statistics.median(t[k] for t in times), 3) for k in times[0]},
        "iterations_fp32_inner": {k: info[k] for k in ("outer_iters", "a_solves", "a_iters", "s_solves", "s_iters",
                                                       "inner_solves", "inner_iters")},
        "iterations_fp64": {k: f64[-1][k] for k in ("outer_iters", "a_iters", "s_iters", "inner_iters")},
        "setup_ms": {"fp32_inner": round(info["setup_ms"], 3), "fp64": round(f64[-1]["setup_ms"], 3)},
        "true_rel_res": {"fp32_inner": info["true_rel_res"], "fp64": f64[-1]["true_rel_res"]},
        "adjoint_fp32_inner_ms": round(adj_ms, 1),
        "kernels": kernels,
        "kernel_timing": {"events": "HIP events recorded by the launches, timed steps only",
                          "sampled_every": KT_PERIOD},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": measured_traffic(dom, args.config),
                     "bytes_per_launch": round(by_l / n_l) if n_l else None, "launches_timed": n_l,
                     "measured_stream_GBps": stream, "frac_of_measured_read": (
                         round(achieved / stream["read_GBps"], 4) if achieved else None),
                     # a launch whose bytes fit the last-level cache is not an HBM figure
                     "fits_last_level_cache": bool(n_l and by_l / n_l < LLC_BYTES)},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        okw = {"pc_A": args.pc_A}
        scase, cb = cpu_baseline(args.cpu_sample, okw)
        sctx = NsContext(scase, device=dev).bind()
        sr = sctx.assemble(scase.v, scase.p, scase.vdot, rho=scase.rho, mu=scase.mu, dt=scase.dt,
                           rho_inf=scase.rho_inf, R=scase.R)
        same = {}
        for prec in ("fp64", "fp32_inner"):
            sctx.solve(sr, SolveOptions(precision=prec, **solver_kw))
            sr = sctx.assemble(scase.v, scase.p, scase.vdot, rho=scase.rho, mu=scase.mu, dt=scase.dt,
                               rho_inf=scase.rho_inf, R=scase.R)
            torch.cuda.synchronize()
            t = time.perf_counter()
            sctx.solve(sr, SolveOptions(precision=prec, **solver_kw))
            same[prec] = round(1e3 * (time.perf_counter() - t), 2)
        cb["gpu_same_sample_ms"] = same
        sctx.close()
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb['value']} ms on {cb['cores']} cores; gpu on the same sample {same}")
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
