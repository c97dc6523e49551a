"""Kernel probe for hardware-counter runs: launches the finest-level kernels of
the nested solve on their own (the A operator SpMV, one AMG V-cycle of A) and
a plain device copy of known size that calibrates the FETCH_SIZE / WRITE_SIZE
counters.  Prints the algorithmic bytes per launch of each probed kernel.

    python3 paper_1911_10814_amd/probe.py --config pipe_200k --reps 10
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="pipe_200k")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--precision", default="fp32_inner")
    ap.add_argument("--copy-mib", type=int, default=512)
    args = ap.parse_args()

    import numpy as np
    import torch

    from ns_inputs import build
    from paper_1911_10814_amd import NsContext, SolveOptions

    case = build(args.config)
    print(f"[probe] {args.config}: {case.n_nodes} nodes built", file=sys.stderr, flush=True)
    ctx = NsContext(case).bind()
    Q = ctx.outlet_flow(case.v)
    ctx.assemble(case.v, case.p, case.vdot, rho=case.rho, mu=case.mu, dt=case.dt, rho_inf=case.rho_inf,
                 m=case.R, P_af=case.R * Q)
    print("[probe] bound and assembled", file=sys.stderr, flush=True)
    o = SolveOptions(precision=args.precision)
    x3 = torch.as_tensor(np.random.default_rng(0).standard_normal(3 * case.n_nodes), device="cuda")
    for _ in range(args.reps):
        ctx.apply("A", x3, o)
    for _ in range(args.reps):
        ctx.apply("vcycle_A", x3, o)
    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    # measured streaming ceilings of the part (device copy and a read-only sum),
    # beside the nominal 8 TB/s
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * n * 4 * args.reps / (e0.elapsed_time(e1) * 1e6)
    t = src.sum()  # first call initialises the reduction
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.reps):
        t = src.sum()
    e1.record()
    torch.cuda.synchronize()
    read_gbs = n * 4 * args.reps / (e0.elapsed_time(e1) * 1e6)
    s = 4 if args.precision == "fp32_inner" else 8
    N, nnzb = case.n_nodes, ctx.nnzb
    print(json.dumps({
        "config": args.config, "N": N, "nnzb": nnzb, "precision": args.precision, "reps": args.reps,
        "spmv_A_bytes": nnzb * (9 * s + 4) + 4 * (N + 1) + 6 * s * N,
        "copy_bytes_read": n * 4, "copy_bytes_written": n * 4,
        "measured_copy_GBps": copy_gbs, "measured_read_GBps": read_gbs,
    }))


if __name__ == "__main__":
    main()
