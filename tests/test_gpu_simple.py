"""GPU parity of the SIMPLE outer preconditioner (Sec. 3.2) against the oracle.

Same bars as the P_SCR path: FP64 in schedule-replay mode (same iteration
path) to 1e-10 relative, tolerance mode to the true-residual criterion,
FP32-inner to 1e-6 relative against the FP64 oracle solution.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from conftest import get_assembled, get_case
from gpu_helpers import rel
from oracle import adjoint as oadj
from oracle import amg
from oracle import discretization as dz
from oracle import krylov as kr
from test_gpu_parity import CASES, ctx_for, oracle_solver

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", CASES)
def test_simple_apply_matches_oracle(name):
    from paper_1911_10814_amd import SolveOptions
    ctx = ctx_for(name)
    ns = oracle_solver(name, pc="simple")
    s = np.random.default_rng(21).standard_normal(4 * ctx.N)
    sched = kr.Schedule()
    yo = ns.simple_apply(s, sched)
    assert len(sched.log) == 2
    y, _ = ctx.apply("psimple", s, SolveOptions(pc="simple", schedule=sched.log))
    y = y.cpu().numpy()
    n3 = 3 * ctx.N
    print(name, "P_SIMPLE^-1 err v", rel(y[:n3], yo[:n3]), "p", rel(y[n3:], yo[n3:]), flush=True)
    assert rel(y[:n3], yo[:n3]) <= 1e-10 and rel(y[n3:], yo[n3:]) <= 1e-10


@pytest.mark.parametrize("name", CASES)
def test_simple_solve_fp64_replay_and_tolerance(name):
    from paper_1911_10814_amd import SolveOptions
    ctx = ctx_for(name)
    S = get_assembled(name)
    ns = oracle_solver(name, pc="simple")
    xo, info = ns.solve(S.rhs)
    n3 = 3 * ctx.N
    xg, gi = ctx.solve(ctx._rhs, SolveOptions(pc="simple", schedule=info["schedule"]))
    xg = xg.cpu().numpy()
    ev, ep = rel(xg[:n3], xo[:n3]), rel(xg[n3:], xo[n3:])
    print(name, "SIMPLE replay err v", ev, "p", ep, "outer", gi["outer_iters"], flush=True)
    assert ev <= 1e-10 and ep <= 1e-10
    assert gi["inner_solves"] == 0 and gi["a_solves"] == gi["s_solves"] == gi["outer_iters"]
    xt, ti = ctx.solve(ctx._rhs, SolveOptions(pc="simple"))
    assert ti["converged"] and ti["true_rel_res"] <= 1e-8
    Ad = S.dense()
    assert np.linalg.norm(S.rhs - Ad @ xt.cpu().numpy()) <= 1e-8 * np.linalg.norm(S.rhs) * (1 + 1e-6)
    if ti["schedule"] == info["schedule"]:
        assert rel(xt.cpu().numpy(), xo) <= 1e-10


@pytest.mark.parametrize("name", CASES)
def test_simple_solve_fp32_inner(name):
    from paper_1911_10814_amd import SolveOptions
    ctx = ctx_for(name)
    S = get_assembled(name)
    xo, _ = oracle_solver(name, pc="simple").solve(S.rhs)
    x32, info = ctx.solve(ctx._rhs, SolveOptions(pc="simple", precision="fp32_inner"))
    print(name, "SIMPLE fp32-inner", info, flush=True)
    assert info["converged"] and info["true_rel_res"] <= 1e-8
    n3 = 3 * ctx.N
    x = x32.cpu().numpy()
    assert rel(x[:n3], xo[:n3]) <= 1e-6 and rel(x[n3:], xo[n3:]) <= 1e-6


@pytest.mark.parametrize("name", ["channel2", "pipe_tiny"])
def test_simple_adjoint_matches_oracle(name):
    from paper_1911_10814_amd import SolveOptions
    ctx = ctx_for(name)
    S = get_assembled(name)
    c = get_case(name)
    ph = dz.physics_of(c)
    _, _, g = ph.alphas
    gJ = oadj.mean_outlet_pressure_weights(S, 0, g * ph.dt)
    adj = amg.node_adjacency(c.n_nodes, c.tets)
    lo, info = oadj.adjoint_solve(S, adj, gJ, kr.SolveOpts(pc="simple"))
    lg, _ = ctx.adjoint(torch.as_tensor(gJ, device="cuda"), SolveOptions(pc="simple", schedule=info["schedule"]))
    assert rel(lg.cpu().numpy(), lo) <= 1e-10


def test_unknown_outer_preconditioner_is_rejected():
    from paper_1911_10814_amd import SolveOptions, _lib
    ctx = ctx_for("cube")
    o, keep, _ = SolveOptions().to_c()
    o.pc = 7
    x = torch.zeros(4 * ctx.N, dtype=torch.float64, device="cuda")
    st = _lib.NsStats()
    lib = _lib.load()
    rc = lib.ns_nested_solve(ctx.h, C.byref(o), C.c_void_p(ctx._rhs.data_ptr()), C.c_void_p(x.data_ptr()),
                             C.byref(st), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1 and b"outer preconditioner" in lib.ns_last_error(ctx.h)
