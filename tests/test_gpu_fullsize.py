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
        self.rhs = self.ctx.assemble(c.v, c.p, c.vdot, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, m=self.R,
                                     P_af=self.R * self.Q)
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


def test_solves_fp64_and_fp32_inner(full):
    """FP64 and FP32-inner solves at rtol 1e-8.  Their solutions agree to
    1e-6 when the tangent is well conditioned.  Otherwise the error of either
    solve is bounded only by its final true relative residual times the
    conditioning, so both are compared with an FP64 reference at rtol 1e-10
    per unit of their own final residual.  That ratio depends on the direction
    of the final residual (the FP64 solve's ratio is only a lower bound on the
    condition number, and FP32 rounding in the preconditioner turns the
    residual), so the FP32-inner error per unit residual must stay within 10x
    the FP64 solve's."""
    from paper_1911_10814_amd import SolveOptions
    n3 = 3 * full.case.n_nodes
    x64, i64 = _solve_and_check(full, SolveOptions(precision="fp64"), "fp64", with_info=True)
    x32, i32 = _solve_and_check(full, SolveOptions(precision="fp32_inner"), "fp32_inner", with_info=True)
    ev, ep = _rel(x32[:n3], x64[:n3]), _rel(x32[n3:], x64[n3:])
    print(full.case.name, "fp32_inner vs fp64: v %.2e p %.2e" % (ev, ep), flush=True)
    if ev <= 1e-6 and ep <= 1e-6:
        return
    xr = _solve_and_check(full, SolveOptions(precision="fp64", rtol=1e-10), "fp64 reference")
    r64, r32 = i64["true_rel_res"], i32["true_rel_res"]
    for part in (slice(0, n3), slice(n3, None)):
        e64, e32 = _rel(x64[part], xr[part]), _rel(x32[part], xr[part])
        print(full.case.name, f"error vs reference: fp64 {e64:.2e} (res {r64:.2e}) fp32_inner {e32:.2e} "
              f"(res {r32:.2e})", flush=True)
        assert e32 <= max(1e-6, 10 * (e64 / r64) * r32)


def test_resistance_sweep(full):
    """Outlet resistance sweep on the 2e6-node pipe (the Schur complement
    stiffens with R), intermediate and Schur tolerances 1e-4, inner 1e-2.
    The tangent's conditioning grows with R, so at rtol 1e-8 even the FP64
    solution is only as close to the exact one as its residual allows; both
    solves are compared with an FP64 reference at rtol 1e-12, and the
    FP32-inner error must stay within 1e-6 or within 10x the FP64 solve's."""
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
            for part in (slice(0, n3), slice(n3, None)):
                e64, e32 = _rel(x64[part], xr[part]), _rel(x32[part], xr[part])
                print(f"R={R:g} error vs reference: fp64 {e64:.2e} fp32_inner {e32:.2e}", flush=True)
                assert e32 <= max(1e-6, 10 * e64)
    finally:
        full.set_R(base)


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
