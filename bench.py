"""Newton-step benchmark of the nested block solver on one MI355X.

One step = the whole hot path of one Newton iteration on the synthetic pipe
workload (circular pipe r = 0.3, L = 3, ~2e5 nodes / ~8e5 DOFs, outlet
resistance R = 1e3): VMS tangent + residual assembly, per-step preconditioner
set-up and FP32-inner nested FGMRES solve to rtol 1e-8, Newton update, and
the adjoint (transposed nested) solve for d(outlet flow)/dR.  After the timed
steps the same tangent is solved K times in the all-FP64 form for the
FP32-inner vs FP64 comparison.

Prints one JSON line.  `value` is the FP32-inner Newton-step solve time (per-
step set-up + Krylov iterations, median over the timed steps), in ms.
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


def cpu_baseline(sample: str, scale_to_nnzb: int):
    """The FP64 CPU oracle (single thread) on a bounded sample: assembly and
    nested solve of the same pipe recipe at a coarser resolution, wall time
    scaled to the benchmark mesh by the ratio of nonzero blocks."""
    import torch

    from ns_inputs import build
    from oracle import amg, krylov
    from oracle import discretization as dz

    nthr = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        case = build(sample)
        t0 = time.perf_counter()
        S = dz.assemble(case)
        t1 = time.perf_counter()
        ns = krylov.NestedSolver(S, amg.node_adjacency(case.n_nodes, case.tets), krylov.SolveOpts())
        x, info = ns.solve(S.rhs)
        t2 = time.perf_counter()
    finally:
        torch.set_num_threads(nthr)
    nnzb_s = S.A_F.nnz // 9
    ratio = scale_to_nnzb / nnzb_s
    return {
        "value": (t2 - t1) * 1e3 * ratio,
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle (numpy/scipy/torch CPU, FP64, 1 thread) on {sample} ({case.n_nodes} nodes, nnzb {nnzb_s}): "
                   f"set-up + nested solve {1e3 * (t2 - t1):.0f} ms ({info['outer']} outer its), "
                   f"assembly {1e3 * (t1 - t0):.0f} ms; solve time scaled x{ratio:.1f} by nnzb to the benchmark mesh"),
        "assembly_ms_scaled": (t1 - t0) * 1e3 * ratio,
        "host_cpus": len(os.sched_getaffinity(0)),
        "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
    }


def measured_traffic(kernel_class: str, config: str):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/), or None when the kernel source changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel_class}_{config}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1911_10814_amd", "csrc", "kernels_la.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("kernels_la_sha256_16"):
        return None
    return rec["traffic_bytes_per_launch"]


def hbm_case_rooflines():
    """Roofline fractions of the finest-level FP32 kernels on the meshes whose
    matrices stream from HBM (2e6-node pipe, 4e6-node contraction-expansion),
    as recorded by rocprofv3 in profiles/ (not re-measured by this run); only
    records taken against the current kernel source are reported."""
    import hashlib

    src = open(os.path.join(ROOT, "paper_1911_10814_amd", "csrc", "kernels_la.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()[:16]
    out = {}
    for cfg in ("pipe_2m", "conexp_4m"):
        path = os.path.join(ROOT, "profiles", f"finest_A_{cfg}_roofline.json")
        if not os.path.exists(path):
            continue
        rec = json.load(open(path))
        if any(r.get("kernels_la_sha256_16") != sha for r in rec.values()):
            continue
        out[cfg] = {cls: {"avg_us": r["avg_duration_us_rocprof"], "frac": r["frac_of_8000"],
                          "traffic_over_algorithmic": r["traffic_bytes_per_launch"] / r["algorithmic_bytes_per_launch"]}
                    for cls, r in rec.items()}
    return out or None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="pipe_200k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="pipe_40k")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the multi-GPU decomposition is a "
              "design only and is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from ns_inputs import build
    from paper_1911_10814_amd import NsContext, SolveOptions, gen_alpha

    dev = torch.device("cuda:0")
    case = build(args.config)
    t0 = time.perf_counter()
    ctx = NsContext(case, device=dev).bind()
    t_sym = time.perf_counter() - t0
    print(f"[bench] {args.config}: N={case.n_nodes} E={case.n_elems} nnzb={ctx.nnzb} "
          f"symbolic+bind {t_sym:.2f}s workspace {ctx.workspace_bytes / 1e9:.2f} GB", file=sys.stderr, flush=True)
    am, af, gam = gen_alpha(case.rho_inf)
    Q = ctx.outlet_flow(case.v)
    P_af = case.R * Q
    v = torch.as_tensor(case.v, device=dev)
    p = torch.as_tensor(case.p, device=dev)
    vd = torch.as_tensor(case.vdot, device=dev)
    y0 = torch.cat([v.reshape(-1), p])
    yd0 = torch.cat([vd.reshape(-1), torch.zeros_like(p)])
    a = ctx.outlet_vectors()  # [n_out, N, 3], Dirichlet entries zeroed
    g = torch.zeros(4 * case.n_nodes, dtype=torch.float64, device=dev)
    g[:3 * case.n_nodes] = gam * case.dt * a[0].reshape(-1)  # d(updated outlet flow)/dx
    o32 = SolveOptions(precision="fp32_inner")
    o64 = SolveOptions(precision="fp64")

    def step(timing=None):
        ts = {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        rhs = ctx.assemble(v, p, vd, rho=case.rho, mu=case.mu, dt=case.dt, rho_inf=case.rho_inf, m=case.R,
                           P_af=P_af)
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
        t = time.perf_counter()
        lam, ainfo = ctx.adjoint(g, o32)
        ts["adjoint_ms"] = 1e3 * (time.perf_counter() - t)
        return ts, info, ainfo, rhs, x

    for _ in range(args.warmup):
        step()
        print("[bench] warm-up step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts, info, ainfo, rhs, x32 = step()
        times.append(ts)
        print(f"[bench] step {k}: {ts} outer {info['outer_iters']} A-its {info['a_iters']} "
              f"S-its {info['s_iters']} inner-its {info['inner_iters']} res {info['true_rel_res']:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    # per-launch kernel durations with HIP events on the solver's stream: one
    # more step with the timed kernel classes bracketed by event pairs (such a
    # step runs its launches one by one instead of from captured graphs)
    ctx.kernel_timing(("spmv_A", "cheb_A0", "spmv_full"))
    step()
    ctx.kernel_timing(())
    kt = {k: ctx.kernel_timing_read(k) for k in ("spmv_A", "cheb_A0", "spmv_full")}

    def solve_fresh(opts):
        """Re-assemble (so the per-step set-up runs again) and solve; wall time of the solve call."""
        r = ctx.assemble(v, p, vd, rho=case.rho, mu=case.mu, dt=case.dt, rho_inf=case.rho_inf, m=case.R,
                         P_af=P_af)
        torch.cuda.synchronize()
        t = time.perf_counter()
        xx, ii = ctx.solve(r, opts)
        ii["wall_ms"] = 1e3 * (time.perf_counter() - t)
        return xx, ii

    # all-FP64 form on the same tangent
    f64 = []
    for k in range(args.steps):
        x64, i64 = solve_fresh(o64)
        f64.append(i64)
        print(f"[bench] fp64 solve {k}: setup {i64['setup_ms']:.1f} ms solve {i64['solve_ms']:.1f} ms outer "
              f"{i64['outer_iters']} res {i64['true_rel_res']:.2e}", file=sys.stderr, flush=True)
    n3 = 3 * case.n_nodes
    xa, xb = x32.cpu().numpy(), x64.cpu().numpy()
    err_v = float(np.linalg.norm(xa[:n3] - xb[:n3]) / np.linalg.norm(xb[:n3]))
    err_p = float(np.linalg.norm(xa[n3:] - xb[n3:]) / np.linalg.norm(xb[n3:]))
    # the paper's lighter P_A option (point Jacobi) in both precisions, other
    # smoother settings, and the SIMPLE outer preconditioner
    variants = {}
    for name, o in (("fp32_inner_jacobi", SolveOptions(precision="fp32_inner", pc_A="jacobi")),
                    ("fp64_jacobi", SolveOptions(precision="fp64", pc_A="jacobi")),
                    ("fp32_inner_cheb1", SolveOptions(precision="fp32_inner", cheb_degree=1)),
                    ("fp32_inner_cheb2_ratio30", SolveOptions(precision="fp32_inner", cheb_ratio=30.0)),
                    ("fp32_inner_cheb3", SolveOptions(precision="fp32_inner", cheb_degree=3)),
                    ("fp32_inner_cheb3_S", SolveOptions(precision="fp32_inner", cheb_degree_S=3)),
                    ("fp32_inner_simple", SolveOptions(precision="fp32_inner", pc="simple")),
                    ("fp32_inner_jacobi_inner", SolveOptions(precision="fp32_inner", pc_I="jacobi"))):
        runs = [solve_fresh(o)[1] for _ in range(args.steps)]
        variants[name] = {"solve_ms": round(statistics.median(r["wall_ms"] for r in runs), 3),
                          "outer_iters": runs[-1]["outer_iters"], "a_iters": runs[-1]["a_iters"],
                          "s_iters": runs[-1]["s_iters"], "inner_iters": runs[-1]["inner_iters"],
                          "true_rel_res": runs[-1]["true_rel_res"]}
        print(f"[bench] {name}: {variants[name]}", file=sys.stderr, flush=True)

    # one time step of the predictor multi-corrector (Sec. 2.5) from the state,
    # resistance outlet, tol_R = tol_A = 1e-6, FP32-inner solves
    model = {"Rp": case.R, "P": case.R * Q, "Q": Q}
    tsr = ctx.time_step(y0, yd0, rho=case.rho, mu=case.mu, dt=case.dt, rho_inf=case.rho_inf, model=model,
                        opts=o32)[2]
    tstep = {k: tsr[k] for k in ("iterations", "converged", "res_hist", "lin_outer", "lin_a", "lin_s", "lin_inner",
                                 "assemble_ms", "solve_ms", "total_ms")}
    print(f"[bench] time step: {tstep}", file=sys.stderr, flush=True)

    solve32 = statistics.median(t["solve_ms"] for t in times)
    solve64 = statistics.median(i["wall_ms"] for i in f64)
    # dominant kernel: largest total time among the timed classes
    dom = max(kt, key=lambda k: kt[k][1])
    n_l, ms_l, by_l = kt[dom]
    achieved = (by_l / (ms_l * 1e-3)) / 1e9 if ms_l > 0 else None
    traffic = measured_traffic(dom, args.config)
    kernels = {k: {"launches": n, "avg_us": 1e3 * ms / n if n else None,
                   "GBps": (b / (ms * 1e-3)) / 1e9 if ms > 0 else None, "total_ms": ms}
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
        "dtype": "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: straight pipe r=0.3 L=3, {case.n_nodes} nodes, "
                               f"{4 * case.n_nodes} DOFs, {case.n_elems} tets, nnzb {ctx.nnzb}, R=1e3, "
                               f"one Newton step (assembly + FP32-inner nested solve + update + adjoint)",
                   "rtol": 1e-8, "rtol_A": 1e-3, "rtol_S": 1e-3, "rtol_I": 1e-3, "pc_A": "amg"},
        "fp64_solve_ms": round(solve64, 3),
        "speedup_fp32_inner_vs_fp64": round(solve64 / solve32, 3),
        "fp32_inner_vs_fp64_rel_err": {"v": err_v, "p": err_p},
        "stage_ms_median": {k: round(statistics.median(t[k] for t in times), 3) for k in times[0]},
        "iterations_fp32_inner": {k: info[k] for k in ("outer_iters", "a_solves", "a_iters", "s_solves", "s_iters",
                                                       "inner_solves", "inner_iters")},
        "iterations_fp64": {k: f64[-1][k] for k in ("outer_iters", "a_iters", "s_iters", "inner_iters")},
        "setup_ms": {"fp32_inner": info["setup_ms"], "fp64": f64[-1]["setup_ms"]},
        "variants": variants,
        "time_step_fp32_inner": tstep,
        "true_rel_res": {"fp32_inner": info["true_rel_res"], "fp64": f64[-1]["true_rel_res"]},
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                     "bytes_per_launch": by_l / n_l if n_l else None},
        "roofline_hbm_cases_from_profiles": hbm_case_rooflines(),
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample, ctx.nnzb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
