"""Solver-settings studies of the paper (Sec. 4), on the synthetic inputs.

    python -m paper_1911_10814_amd.studies tolerances [--config conexp_150k] [--cr 0.5 2.0]
    python -m paper_1911_10814_amd.studies resistance [--config pipe_200k] [--cr 1.0]
    python -m paper_1911_10814_amd.studies pa         [--config pipe_200k]
    python -m paper_1911_10814_amd.studies outlets    [--config plate_784]

* ``tolerances`` -- the nozzle study: FGMRES at delta^r = 1e-8 with the nested
  preconditioner at delta_A = delta_S = delta_I in {1e-8, 1e-6, 1e-4, 1e-2}
  and with SIMPLE at delta_A = delta_S in {1e-8, 1e-2}, for two Courant
  numbers (the time step is set from the target Courant number, the largest
  node speed and the shortest edge).
* ``resistance`` -- the cylinder study: outlet resistance R in {1e2 .. 1e5},
  delta_A = delta_S = 1e-4, the nested preconditioner with delta_I in
  {1e-4 .. 1e-1} against SIMPLE.
* ``pa`` -- AMG against Jacobi for the A-solves: GMRES on A to delta_A = 1e-8
  with either preconditioner, and whole solves with the settings used for
  the patient-specific models (delta^r = 1e-2, delta_A = 1e-3,
  delta_S = delta_I = 1e-2, m_A = m_S = n^max_A = n^max_S = 20), also with
  AMG for the intermediate A-solves and Jacobi for the inner ones.
* ``outlets`` -- many reduced-model outlets (the perforated plate: 784
  outlets, as many as the pulmonary model's): the Newton-step solve with all
  rank-one terms, and time steps of the predictor multi-corrector algorithm
  with a three-element Windkessel on every outlet (Algorithm 1).

Every solve prints one JSON line as soon as it ends (iteration counts per
level, true relative residual, set-up and solve time of the best of
``--repeat`` runs), so a partial sweep is still usable.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from ns_inputs import build

from .solver import NsContext, SolveOptions


def courant(case) -> tuple[float, float, float]:
    """(largest node speed, shortest edge, Courant number at the case's dt)."""
    e = np.concatenate([case.tets[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    h = float(np.linalg.norm(case.xyz[e[:, 0]] - case.xyz[e[:, 1]], axis=1).min())
    vmax = float(np.linalg.norm(case.v, axis=1).max())
    return vmax, h, vmax * case.dt / h


class System:
    """One mesh and state on the GPU, re-assembled for each physical setting."""

    def __init__(self, config: str, cr: float | None, R: float | None):
        kw = {} if R is None else {"R": R}
        case = build(config, **kw)
        vmax, h, _ = courant(case)
        if cr is not None:
            case = build(config, dt=cr * h / vmax, **kw)
        self.case = case
        self.cr = vmax * case.dt / h
        self.ctx = NsContext(case).bind()
        self.assemble(case.R)

    def assemble(self, R):
        c = self.case
        R = np.broadcast_to(np.asarray(R, float), (c.n_outlets,)).copy()
        self.rhs = self.ctx.assemble(c.v, c.p, c.vdot, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, R=R)
        torch.cuda.synchronize()


def run(sysm: System, opts: SolveOptions, repeat: int, **label):
    best = None
    for _ in range(repeat):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = sysm.ctx.solve(sysm.rhs, opts)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        if best is None or wall < best[0]:
            best = (wall, info)
    wall, info = best
    rec = dict(label, config=sysm.case.name, n_nodes=sysm.case.n_nodes, cr=round(sysm.cr, 3),
               precision=opts.precision, pc=opts.pc, pc_A=opts.pc_A, rtol=opts.rtol, rtol_A=opts.rtol_A,
               rtol_S=opts.rtol_S, rtol_I=opts.rtol_I if opts.pc == "scr" else None, m_A=opts.m_A, m_S=opts.m_S,
               status=info["status"], outer=info["outer_iters"], a_iters=info["a_iters"], s_iters=info["s_iters"],
               inner_iters=info["inner_iters"], true_rel_res=info["true_rel_res"],
               setup_ms=round(info["setup_ms"], 3), solve_ms=round(info["solve_ms"], 3), wall_ms=round(wall, 3))
    print(json.dumps(rec), flush=True)
    return rec


def study_tolerances(a):
    for cr in a.cr or [0.5, 2.0]:
        s = System(a.config, cr, None)
        for pc_A in a.pc_A:
            for d in (1e-8, 1e-6, 1e-4, 1e-2):
                run(s, SolveOptions(precision=a.precision, pc_A=pc_A, rtol_A=d, rtol_S=d, rtol_I=d), a.repeat,
                    study="tolerances")
            for d in (1e-8, 1e-2):
                run(s, SolveOptions(precision=a.precision, pc="simple", pc_A=pc_A, rtol_A=d, rtol_S=d), a.repeat,
                    study="tolerances")


def study_resistance(a):
    s = System(a.config, (a.cr or [1.0])[0], None)
    for R in (1e2, 1e3, 1e4, 1e5):
        s.assemble(R)
        for pc_A in a.pc_A:
            for dI in (1e-4, 1e-3, 1e-2, 1e-1):
                run(s, SolveOptions(precision=a.precision, pc_A=pc_A, rtol_A=1e-4, rtol_S=1e-4, rtol_I=dI),
                    a.repeat, study="resistance", R=R)
            run(s, SolveOptions(precision=a.precision, pc="simple", pc_A=pc_A, rtol_A=1e-4, rtol_S=1e-4), a.repeat,
                study="resistance", R=R)


def study_pa(a):
    s = System(a.config, a.cr[0] if a.cr else None, None)
    ctx = s.ctx
    b = s.rhs[:3 * ctx.N].contiguous()
    for pc_A in ("amg", "jacobi"):
        o = SolveOptions(precision=a.precision, pc_A=pc_A, rtol_A=1e-8)
        best = None
        for _ in range(a.repeat):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sched = ctx.apply("solve_A", b, o)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            best = wall if best is None else min(best, wall)
        print(json.dumps(dict(study="pa_solve_A", config=s.case.name, n_nodes=s.case.n_nodes,
                              precision=a.precision, pc_A=pc_A, rtol_A=1e-8, iterations=int(sched[0]),
                              wall_ms_incl_setup=round(best, 3))), flush=True)
    # P_A for every A-solve, and AMG for the intermediate solves with Jacobi for the inner ones
    for pc_A, pc_I in (("jacobi", None), ("amg", None), ("amg", "jacobi")):
        run(s, SolveOptions(precision=a.precision, pc_A=pc_A, pc_I=pc_I, rtol=1e-2, rtol_A=1e-3, rtol_S=1e-2,
                            rtol_I=1e-2, m_A=20, m_S=20, nmax_A=20, nmax_S=20), a.repeat,
            study="pa_patient_settings", pc_I=pc_I)
        run(s, SolveOptions(precision=a.precision, pc_A=pc_A, pc_I=pc_I), a.repeat, study="pa_default_settings",
            pc_I=pc_I)


def study_outlets(a):
    s = System(a.config, a.cr[0] if a.cr else None, None)
    c, ctx = s.case, s.ctx
    for prec in ("fp32_inner", "fp64"):
        run(s, SolveOptions(precision=prec), a.repeat, study="outlets_solve", n_outlets=c.n_outlets)
    w = c.meta["rcr"]
    y = torch.as_tensor(np.concatenate([c.v.ravel(), c.p]), device="cuda")
    yd = torch.zeros_like(y)
    Q = ctx.outlet_flow(c.v)
    Pi = w["Rd"] * Q
    model = {"Rp": w["Rp"], "C": w["C"], "Rd": w["Rd"], "Pd": np.zeros(c.n_outlets), "Pi": Pi,
             "P": w["Rp"] * Q + Pi, "Q": Q, "n_ts": 100}
    for step in range(a.steps):
        y, yd, info, out = ctx.time_step(y, yd, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, model=model,
                                         opts=SolveOptions(precision=a.precision))
        model.update(Pi=out["Pi"], P=out["P"], Q=out["Q"])
        rec = {k: info[k] for k in ("iterations", "converged", "res_hist", "lin_outer", "lin_a", "lin_s",
                                    "lin_inner", "assemble_ms", "solve_ms", "total_ms")}
        print(json.dumps(dict(study="outlets_time_step", config=c.name, n_nodes=c.n_nodes, n_outlets=c.n_outlets,
                              step=step, precision=a.precision, P_mean=float(np.mean(out["P"])),
                              Q_sum=float(np.sum(out["Q"])), **rec)), flush=True)


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("study", choices=["tolerances", "resistance", "pa", "outlets"])
    p.add_argument("--config", default=None)
    p.add_argument("--cr", type=float, nargs="*", default=None, help="target Courant number(s)")
    p.add_argument("--precision", default="fp32_inner", choices=["fp64", "fp32_inner"])
    p.add_argument("--pc-A", dest="pc_A", nargs="+", default=["amg", "jacobi"], choices=["amg", "jacobi"])
    p.add_argument("--repeat", type=int, default=2)
    p.add_argument("--steps", type=int, default=3, help="time steps of the outlets study")
    a = p.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the studies run the HIP library and need a GPU")
    a.config = a.config or {"tolerances": "conexp_150k", "resistance": "pipe_200k", "pa": "pipe_200k",
                            "outlets": "plate_784"}[a.study]
    {"tolerances": study_tolerances, "resistance": study_resistance, "pa": study_pa,
     "outlets": study_outlets}[a.study](a)


if __name__ == "__main__":
    main()
