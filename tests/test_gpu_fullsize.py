"""Parity at full size on the benchmark pipe (2e5 nodes) and the larger
workloads (2e6-node pipe with an outlet-resistance sweep, 1e6-node
Y-bifurcation with the adjoint gradient, 4e6-node contraction-expansion),
on sampled outputs the oracle computes one by one: the oracle assembles only
the elements (and outlet faces) touching a seeded sample of nodes, so the
tangent rows, residual entries and tangent columns of those nodes are
complete, and they are compared with the GPU's entry by entry.  The solves are
checked through the sampled rows of r = rhs - [A B; C D] x (forward) and
g - [A B; C D]^T lam (adjoint) built from the oracle's rows and the GPU's
solution, and the FP32-inner solution against the FP64 one.
"""
import gc

import numpy as np
import pytest
import torch

from conftest import get_case
from ns_inputs.cases import Case
from oracle import discretization as dz

pytestmark = pytest.mark.gpu

FULL = ["pipe_200k", "pipe_2m", "ybif_1m", "conexp_4m", "plate_784"]


def sampled_nodes(case, k=48, seed=7):
    rng = np.random.default_rng(seed)
    N = case.n_nodes
    nodes = set(rng.choice(N, size=k, replace=False).tolist())
    fn = np.unique(case.faces)
    nodes |= set(rng.choice(fn, size=min(6, len(fn)), replace=False).tolist())   # outlet nodes
    wall = np.nonzero(case.mask[:, 0])[0]
    nodes |= set(rng.choice(wall, size=4, replace=False).tolist())                # Dirichlet nodes
    return np.array(sorted(nodes))


def full_outlet_vectors(case):
    """a^k over the whole outlet, zeroed at Dirichlet DOFs (the patch
    assembly only holds the faces touching the sampled nodes)."""
    a, _, _ = dz.outlet_vectors(case)
    dm = case.mask[:, :3].ravel().astype(bool)
    out = []
    for k in range(case.n_outlets):
        ak = a[k].ravel().copy()
        ak[dm] = 0.0
        out.append(ak)
    return out


def patch_oracle(case, nodes, R, P_af):
    """Oracle assembly over the elements / outlet faces touching `nodes`."""
    sel = np.isin(case.tets, nodes).any(axis=1)
    fsel = np.isin(case.faces, nodes).any(axis=1)
    optr = [0]
    faces = []
    for k in range(case.n_outlets):
        f = case.faces[case.outlet_ptr[k]:case.outlet_ptr[k + 1]]
        m = fsel[case.outlet_ptr[k]:case.outlet_ptr[k + 1]]
        faces.append(f[m])
        optr.append(optr[-1] + int(m.sum()))
    sub = Case(case.name, case.xyz, case.tets[sel], case.mask, np.array(optr, np.int32),
               np.concatenate(faces).astype(np.int32), case.v, case.p, case.vdot, case.rho, case.mu, case.dt,
               case.rho_inf, np.asarray(R, float), {})
    return dz.assemble(sub, P_af=np.asarray(P_af, float), R=np.asarray(R, float))


def rows_of(nodes, N):
    """Field-split DOF indices (u, v, w, p) of the given nodes: [k, 4]."""
    return np.stack([3 * nodes, 3 * nodes + 1, 3 * nodes + 2, 3 * N + nodes], axis=1)


class Full:
    """One workload: GPU context, oracle outlet data, sampled patch."""

    def __init__(self, name):
        from paper_1911_10814_amd import NsContext
        print(f"[full] building {name}", flush=True)
        self.case = c = get_case(name)
        self.ctx = NsContext(c).bind()
        self.nodes = sampled_nodes(c)
        self.a = full_outlet_vectors(c)
        a_raw, self.w, self.area = dz.outlet_vectors(c)
        self.Q = np.array([np.sum(a_raw[k] * c.v) for k in range(c.n_outlets)])
        self.set_R(c.R)
        print(f"[full] {name}: N={c.n_nodes} E={c.n_elems} nnzb={self.ctx.nnzb}", flush=True)

    def set_R(self, R):
        c = self.case
        self.R = np.asarray(R, float)
        self.rhs = self.ctx.assemble(c.v, c.p, c.vdot, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, R=self.R)
        self.S = patch_oracle(c, self.nodes, self.R, self.R * self.Q)

    def residual_rows(self, b, x, transposed=False):
        """Sampled rows of b - T x (T^T for the adjoint), T with the rank-one term."""
        S = self.S.transposed() if transposed else self.S
        N = self.case.n_nodes
        n3 = 3 * N
        Tx = np.concatenate([S.A_F @ x[:n3] + S.B @ x[n3:], S.C @ x[:n3] + S.D @ x[n3:]])
        for ak, ck in zip(self.a, self.S.c):
            Tx[:n3] += ck * ak * (ak @ x[:n3])
        d = rows_of(self.nodes, N).ravel()
        return (b - Tx)[d]

    def close(self):
        self.ctx = None
        gc.collect()
        torch.cuda.empty_cache()


@pytest.fixture(scope="module", params=FULL)
def full(request):
    f = Full(request.param)
    yield f
    f.close()


def test_outlet_flow(full):
    assert np.allclose(full.ctx.outlet_flow(full.case.v), full.Q, rtol=1e-12, atol=0)


def test_sampled_tangent_rows_and_residual(full):
    case, ctx, S, nodes = full.case, full.ctx, full.S, full.nodes
    N = case.n_nodes
    T = dz.sp.bmat([[S.A_F, S.B], [S.C, S.D]]).tocsr()
    rp, col = ctx.pattern()
    blocks = ctx.export_bsr().cpu().numpy()
    worst = 0.0
    for i in nodes:
        ks = np.arange(rp[i], rp[i + 1])
        cols = rows_of(col[ks], N)  # [nb, 4]
        for r, gr in enumerate(rows_of(np.array([i]), N)[0]):
            orow = T.getrow(gr).toarray().ravel()
            g = blocks[ks, r, :]
            o = orow[cols]
            scale = np.abs(o).max() or 1.0
            worst = max(worst, np.abs(g - o).max() / scale)
            orow[cols.ravel()] = 0.0
            assert not orow.any()          # no entries outside the node pattern
    print(case.name, "sampled rows: worst relative difference", worst, flush=True)
    assert worst <= 1e-12
    d = rows_of(nodes, N).ravel()
    rg = full.rhs.cpu().numpy()[d]
    assert np.abs(rg - S.rhs[d]).max() <= 1e-12 * max(np.abs(S.rhs[d]).max(), 1e-300)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32_inner", 1e-5)])
def test_sampled_operator_rows(full, prec, tol):
    """The operators of the path at full size, in the launch configuration the
    solves use (16-bit column offsets, rows without XCD ranges, the lane counts
    of the large meshes), against the oracle's complete rows at the sampled
    nodes: 4x4 outer operator with the rank-one term, A = F + K, B, C and D.
    Each sampled entry within tol of the sum of |T_ij x_j| over its row: FP64
    rounding, or in FP32 the rounding of values and input (2^-24 each) plus
    FP32 accumulation over at most ~250 products per row (worst case 1.5e-5,
    tol 1e-5; measured ~1e-7)."""
    from paper_1911_10814_amd import SolveOptions
    case, ctx, S = full.case, full.ctx, full.S
    N = case.n_nodes
    n3 = 3 * N
    x = np.random.default_rng(17).standard_normal(4 * N)
    o = SolveOptions(precision=prec)
    d3 = rows_of(full.nodes, N)[:, :3].ravel()
    dp = full.nodes
    rank_one = np.zeros(n3)
    for ak, ck in zip(full.a, S.c):
        rank_one += ck * ak * (ak @ x[:n3])
    absK = np.zeros(n3)
    for ak, ck in zip(full.a, S.c):
        absK += abs(ck) * np.abs(ak) * (np.abs(ak) @ np.abs(x[:n3]))
    aAF, aB, aC, aD = (abs(M) for M in (S.A_F, S.B, S.C, S.D))
    ax = np.abs(x)
    want = {
        "A": (S.A_F @ x[:n3] + rank_one, aAF @ ax[:n3] + absK, x[:n3], d3),
        "B": (S.B @ x[n3:], aB @ ax[n3:], x[n3:], d3),
        "C": (S.C @ x[:n3], aC @ ax[:n3], x[:n3], dp),
        "D": (S.D @ x[n3:], aD @ ax[n3:], x[n3:], dp),
    }
    worst = {}
    for op, (ref, scale, xin, rows) in want.items():
        y = ctx.apply(op, xin, o)[0].cpu().numpy()
        e = np.abs(y[rows] - ref[rows]) / np.maximum(scale[rows], 1e-300)
        worst[op] = float(e.max())
    yf = ctx.apply("full", x, o)[0].cpu().numpy()
    full_ref = np.concatenate([want["A"][0] + want["B"][0], want["C"][0] + want["D"][0]])
    full_scale = np.concatenate([want["A"][1] + want["B"][1], want["C"][1] + want["D"][1]])
    rows4 = rows_of(full.nodes, N).ravel()
    worst["full"] = float((np.abs(yf[rows4] - full_ref[rows4]) / np.maximum(full_scale[rows4], 1e-300)).max())
    print(case.name, prec, "sampled operator rows, worst error / row scale", worst, flush=True)
    assert max(worst.values()) <= tol


def _solve_and_check(full, opts, label, with_info=False):
    x, info = full.ctx.solve(full.rhs, opts)
    print(full.case.name, label, {k: info[k] for k in ("outer_iters", "a_iters", "s_iters", "inner_iters",
                                                        "true_rel_res", "solve_ms")}, flush=True)
    assert info["converged"] and info["true_rel_res"] <= opts.rtol
    xn = x.cpu().numpy()
    r = full.residual_rows(full.rhs.cpu().numpy(), xn)
    # the sampled rows of the true residual are bounded by its norm (plus the
    # rounding of the oracle's own row products)
    bn = float(torch.linalg.norm(full.rhs))
    assert np.abs(r).max() <= (1.01 * info["true_rel_res"] + 1e-12) * bn
    return (xn, info) if with_info else xn


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# Configurations where an FP64 solve stopped at rtol 1e-8 lands within 1e-7 of
# the tight reference, so rtol 1e-8 determines x to 1e-6 with a 10x margin
# (measured before these bounds were set): the FP32-inner 1e-6 target is
# asserted at rtol 1e-8 there.  Elsewhere rtol 1e-8 does not determine x to
# 1e-6 for either precision (conditioning), the rtol-1e-8 errors are reported,
# and the precision claim is asserted at rtol 1e-12.
ASSERT_AT_1E8 = {"pipe_200k", "pipe_2m", "ybif_1m"}
TIGHT = dict(rtol=1e-12, pc_A="jacobi")


def _errors(x, xr, n3):
    return _rel(x[:n3], xr[:n3]), _rel(x[n3:], xr[n3:])


def test_solves_fp64_and_fp32_inner(full):
    """FP64 and FP32-inner solves at rtol 1e-8 (default options) against an
    FP64 reference at rtol 1e-12: the FP32-inner error is <= 1e-6 where rtol
    1e-8 determines x to that accuracy (ASSERT_AT_1E8), reported elsewhere;
    the FP32-inner solve at rtol 1e-12 is within 1e-6 of the reference on
    every configuration."""
    from paper_1911_10814_amd import SolveOptions
    name = full.case.name
    n3 = 3 * full.case.n_nodes
    x64, i64 = _solve_and_check(full, SolveOptions(precision="fp64"), "fp64", with_info=True)
    x32, i32 = _solve_and_check(full, SolveOptions(precision="fp32_inner"), "fp32_inner", with_info=True)
    xr = _solve_and_check(full, SolveOptions(precision="fp64", **TIGHT), "fp64 reference rtol 1e-12")
    x32t = _solve_and_check(full, SolveOptions(precision="fp32_inner", **TIGHT), "fp32_inner rtol 1e-12")
    e64, e32, e32t = _errors(x64, xr, n3), _errors(x32, xr, n3), _errors(x32t, xr, n3)
    print(name, "error vs the rtol-1e-12 reference (v, p): fp64@1e-8 %.2e %.2e (res %.2e), fp32_inner@1e-8 %.2e %.2e "
          "(res %.2e), fp32_inner@1e-12 %.2e %.2e" % (*e64, i64["true_rel_res"], *e32, i32["true_rel_res"], *e32t),
          flush=True)
    if name in ASSERT_AT_1E8:
        assert max(e32) <= 1e-6
    elif max(e32) > 1e-6:
        print(name, "fp32_inner at rtol 1e-8 misses 1e-6 (conditioning: fp64 at rtol 1e-8 is %.2e off)" % max(e64),
              flush=True)
    assert max(e32t) <= 1e-6


def test_resistance_sweep(full):
    """Outlet resistance sweep on the 2e6-node pipe (the Schur complement
    stiffens with R), intermediate and Schur tolerances 1e-4, inner 1e-2.
    Errors against an FP64 reference at rtol 1e-12: the FP32-inner solve at
    rtol 1e-8 is within 1e-6 at R = 1e2 (where the FP64 solve at rtol 1e-8 is
    within 1e-7); at R = 1e4 and 1e6 rtol 1e-8 does not determine x to 1e-6
    and the errors are reported; at every R the FP32-inner solve at rtol 1e-12
    is within 1e-6 of the reference."""
    if full.case.name != "pipe_2m":
        pytest.skip("the resistance sweep runs on the 2e6-node pipe")
    from paper_1911_10814_amd import SolveOptions
    n3 = 3 * full.case.n_nodes
    base = full.R.copy()
    try:
        for R in (1e2, 1e4, 1e6):
            full.set_R([R])
            kw = dict(rtol_A=1e-4, rtol_S=1e-4, rtol_I=1e-2)
            xr = _solve_and_check(full, SolveOptions(precision="fp64", rtol=1e-12, **kw), f"R={R:g} fp64 reference")
            x64 = _solve_and_check(full, SolveOptions(precision="fp64", **kw), f"R={R:g} fp64")
            x32 = _solve_and_check(full, SolveOptions(precision="fp32_inner", **kw), f"R={R:g} fp32_inner")
            x32t = _solve_and_check(full, SolveOptions(precision="fp32_inner", rtol=1e-12, **kw),
                                    f"R={R:g} fp32_inner rtol 1e-12")
            e64, e32, e32t = _errors(x64, xr, n3), _errors(x32, xr, n3), _errors(x32t, xr, n3)
            print(f"R={R:g} error vs reference (v, p): fp64@1e-8 {e64[0]:.2e} {e64[1]:.2e}, fp32_inner@1e-8 "
                  f"{e32[0]:.2e} {e32[1]:.2e}, fp32_inner@1e-12 {e32t[0]:.2e} {e32t[1]:.2e}", flush=True)
            if R == 1e2:
                assert max(e32) <= 1e-6
            assert max(e32t) <= 1e-6
    finally:
        full.set_R(base)


def test_fp64_replay_matches_oracle_on_the_benchmark_pipe(full):
    """FP64 nested solve of the 2e5-node pipe on the oracle's iteration path
    (its per-call iteration counts, stored with its solution's norms and
    sampled entries by tests/golden/make_pipe_200k_replay.py): within 1e-10
    relative, velocity and pressure blocks separately."""
    if full.case.name != "pipe_200k":
        pytest.skip("the stored oracle solve is of the 2e5-node pipe")
    import json
    import os
    from paper_1911_10814_amd import SolveOptions
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pipe_200k_fp64_replay.json")))
    n3 = 3 * full.case.n_nodes
    assert abs(float(torch.linalg.norm(full.rhs)) - g["norm_rhs"]) <= 1e-13 * g["norm_rhs"]
    x, info = full.ctx.solve(full.rhs, SolveOptions(schedule=g["schedule"]))
    assert info["schedule"] == g["schedule"]
    x = x.cpu().numpy()
    idx = np.array(g["idx"])
    xo = np.array(g["x"])
    v, p = idx < n3, idx >= n3
    ev = np.linalg.norm(x[idx[v]] - xo[v]) / np.linalg.norm(xo[v])
    ep = np.linalg.norm(x[idx[p]] - xo[p]) / np.linalg.norm(xo[p])
    nv = abs(np.linalg.norm(x[:n3]) - g["norm_v"]) / g["norm_v"]
    np_ = abs(np.linalg.norm(x[n3:]) - g["norm_p"]) / g["norm_p"]
    print("pipe_200k fp64 replay: sampled error v %.2e p %.2e, norms %.2e %.2e" % (ev, ep, nv, np_), flush=True)
    assert max(ev, ep, nv, np_) <= 1e-10


def test_adjoint_sampled_rows(full):
    """Adjoint solve checked on sampled rows of g - [A B; C D]^T lam: column i
    of the tangent only receives contributions from elements and faces that
    contain node i, all of which the patch assembly holds."""
    from paper_1911_10814_amd import SolveOptions
    n3 = 3 * full.case.n_nodes
    g = torch.zeros(4 * full.case.n_nodes, dtype=torch.float64, device="cuda")
    g[:n3] = full.ctx.outlet_vectors()[0].reshape(-1)
    lam, info = full.ctx.adjoint(g, SolveOptions())
    print(full.case.name, "adjoint", {k: info[k] for k in ("outer_iters", "a_iters", "s_iters", "true_rel_res")},
          flush=True)
    assert info["converged"] and info["true_rel_res"] <= 1e-8
    r = full.residual_rows(g.cpu().numpy(), lam.cpu().numpy(), transposed=True)
    assert np.abs(r).max() <= (1.01 * info["true_rel_res"] + 1e-12) * float(torch.linalg.norm(g))


def test_bifurcation_gradient_matches_finite_differences(full):
    """d(mean outlet pressure)/d(R1, R2) on the 1e6-node Y-bifurcation:
    FP32-inner forward solve and the adjoint through the autograd function,
    against central differences (step 1e-6 R) of FP64 solves at rtol 1e-12."""
    if full.case.name != "ybif_1m":
        pytest.skip("the gradient check runs on the Y-bifurcation")
    from paper_1911_10814_amd import NestedSolveFn, SolveOptions
    from paper_1911_10814_amd.solver import gen_alpha
    c = full.case
    N = c.n_nodes
    am, af, gam = gen_alpha(c.rho_inf)
    # J = sum_k mean pressure of outlet k at n+1: (1/|G_k|) w_k . (p + gamma dt dp_dot)
    gJ = np.zeros(4 * N)
    for k in range(c.n_outlets):
        gJ[3 * N:] += gam * c.dt * full.w[k] / full.area[k]
    gJ = torch.as_tensor(gJ, device="cuda")
    P_n = c.R * full.Q
    fwd = SolveOptions(precision="fp32_inner", rtol=1e-12)
    tight = SolveOptions(rtol=1e-12, rtol_A=1e-8, rtol_S=1e-8, rtol_I=1e-8)
    try:
        R = torch.tensor(c.R, dtype=torch.float64, requires_grad=True)
        x = NestedSolveFn.apply(R, full.ctx, c, P_n, full.Q, fwd, SolveOptions(rtol=1e-10))
        (gJ * x).sum().backward()
        grad = R.grad.numpy()

        def loss(Rv):
            with torch.no_grad():
                xx = NestedSolveFn.apply(torch.tensor(Rv), full.ctx, c, P_n, full.Q, tight, None)
                return float((gJ * xx).sum())

        for k in range(c.n_outlets):
            h = 1e-6 * c.R[k]
            Rp, Rm = c.R.copy(), c.R.copy()
            Rp[k] += h
            Rm[k] -= h
            fd = (loss(Rp) - loss(Rm)) / (2 * h)
            print("ybif grad", k, grad[k], "fd", fd, flush=True)
            assert abs(grad[k] - fd) <= 1e-5 * abs(fd)
    finally:
        full.set_R(c.R)
