"""Parity at the benchmark workload (2e5-node pipe), in the launch
configuration bench.py times, on sampled outputs the oracle computes one by
one: the oracle assembles only the elements (and outlet faces) touching a
seeded sample of nodes, so the tangent rows and residual entries of those
nodes are complete, and compares them with the GPU's rows entry by entry.
The solves are checked through the sampled rows of the residual
r = rhs - [A B; C D] x built from the oracle's rows and the GPU's x, and the
FP32-inner solution against the FP64 one.
"""
import numpy as np
import pytest
import torch

from conftest import get_case
from ns_inputs.cases import Case
from oracle import discretization as dz

pytestmark = pytest.mark.gpu

NAME = "pipe_200k"
_STATE = {}


def sampled_nodes(case, k=48, seed=7):
    rng = np.random.default_rng(seed)
    N = case.n_nodes
    nodes = set(rng.choice(N, size=k, replace=False).tolist())
    fn = np.unique(case.faces)
    nodes |= set(rng.choice(fn, size=6, replace=False).tolist())        # outlet nodes
    wall = np.nonzero(case.mask[:, 0])[0]
    nodes |= set(rng.choice(wall, size=4, replace=False).tolist())      # Dirichlet nodes
    return np.array(sorted(nodes))


def patch_oracle(case, nodes):
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
               case.rho_inf, case.R, {})
    a, _, _ = dz.outlet_vectors(case)  # flow rates need the whole outlet
    Q = np.array([np.sum(a[k] * case.v) for k in range(case.n_outlets)])
    return dz.assemble(sub, P_af=case.R * Q, R=case.R), Q


def state():
    if not _STATE:
        from paper_1911_10814_amd import NsContext
        case = get_case(NAME)
        ctx = NsContext(case).bind()
        Q = ctx.outlet_flow(case.v)
        rhs = ctx.assemble(case.v, case.p, case.vdot, rho=case.rho, mu=case.mu, dt=case.dt, rho_inf=case.rho_inf,
                           m=case.R, P_af=case.R * Q)
        nodes = sampled_nodes(case)
        S, Qo = patch_oracle(case, nodes)
        _STATE.update(case=case, ctx=ctx, rhs=rhs, nodes=nodes, S=S, Q=Q, Qo=Qo)
    return _STATE


def rows_of(nodes, N):
    """Field-split DOF indices (u, v, w, p) of the given nodes: [k, 4]."""
    return np.stack([3 * nodes, 3 * nodes + 1, 3 * nodes + 2, 3 * N + nodes], axis=1)


def test_outlet_flow_full_size():
    st = state()
    assert np.allclose(st["Q"], st["Qo"], rtol=1e-12, atol=0)


def test_sampled_tangent_rows_and_residual():
    st = state()
    case, ctx, S, nodes = st["case"], st["ctx"], st["S"], st["nodes"]
    N = case.n_nodes
    T = dz.sp.bmat([[S.A_F, S.B], [S.C, S.D]]).tocsr()
    rp, col = ctx.pattern()
    blocks = ctx.export_bsr().cpu().numpy()
    worst = 0.0
    for i in nodes:
        ks = np.arange(rp[i], rp[i + 1])
        J = col[ks]
        cols = rows_of(J, N)  # [nb, 4]
        for r, gr in enumerate(rows_of(np.array([i]), N)[0]):
            orow = T.getrow(gr).toarray().ravel()
            g = blocks[ks, r, :]                 # [nb, 4]
            o = orow[cols]                       # [nb, 4]
            scale = np.abs(o).max() or 1.0
            worst = max(worst, np.abs(g - o).max() / scale)
            # the row has no entries outside the node pattern
            orow[cols.ravel()] = 0.0
            assert not orow.any()
    print("sampled rows: worst relative difference", worst, flush=True)
    assert worst <= 1e-12
    d = rows_of(nodes, N).ravel()
    rg = st["rhs"].cpu().numpy()[d]
    ro = S.rhs[d]
    assert np.abs(rg - ro).max() <= 1e-12 * max(np.abs(ro).max(), 1e-300)


def sampled_residual(st, x):
    case, S, nodes = st["case"], st["S"], st["nodes"]
    N = case.n_nodes
    d = rows_of(nodes, N).ravel()
    n3 = 3 * N
    Ax = np.concatenate([S.A_F @ x[:n3] + S.B @ x[n3:], S.C @ x[:n3] + S.D @ x[n3:]])
    for ak, ck in zip(full_outlet_vectors(case), S.c):
        Ax[:n3] += ck * ak * (ak @ x[:n3])
    return (st["rhs"].cpu().numpy() - Ax)[d]


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


@pytest.mark.parametrize("prec", ["fp64", "fp32_inner"])
def test_full_size_solve_sampled_residual(prec):
    from paper_1911_10814_amd import SolveOptions
    st = state()
    x, info = st["ctx"].solve(st["rhs"], SolveOptions(precision=prec))
    print(prec, {k: info[k] for k in ("outer_iters", "a_iters", "s_iters", "inner_iters", "true_rel_res")},
          flush=True)
    assert info["converged"] and info["true_rel_res"] <= 1e-8
    r = sampled_residual(st, x.cpu().numpy())
    bn = float(torch.linalg.norm(st["rhs"]))
    assert np.abs(r).max() <= 1e-8 * bn
    st[prec] = x.cpu().numpy()
    if "fp64" in st and "fp32_inner" in st:
        n3 = 3 * st["case"].n_nodes
        a, b = st["fp32_inner"], st["fp64"]
        assert np.linalg.norm(a[:n3] - b[:n3]) <= 1e-6 * np.linalg.norm(b[:n3])
        assert np.linalg.norm(a[n3:] - b[n3:]) <= 1e-6 * np.linalg.norm(b[n3:])


def test_full_size_adjoint_sampled_rows():
    """Adjoint solve checked on sampled rows of g - [A B; C D]^T lam: column i
    of the tangent only receives contributions from elements and faces that
    contain node i, all of which the patch assembly holds, so the rows of the
    transposed system at the sampled nodes are complete there too."""
    from paper_1911_10814_amd import SolveOptions
    st = state()
    ctx, case, S, nodes = st["ctx"], st["case"], st["S"], st["nodes"]
    N = case.n_nodes
    n3 = 3 * N
    g = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
    g[:n3] = ctx.outlet_vectors()[0].reshape(-1)
    lam, info = ctx.adjoint(g, SolveOptions())
    print("adjoint", {k: info[k] for k in ("outer_iters", "a_iters", "s_iters", "true_rel_res")}, flush=True)
    assert info["converged"] and info["true_rel_res"] <= 1e-8
    St = S.transposed()
    y = lam.cpu().numpy()
    Ty = np.concatenate([St.A_F @ y[:n3] + St.B @ y[n3:], St.C @ y[:n3] + St.D @ y[n3:]])
    for ak, ck in zip(full_outlet_vectors(case), S.c):
        Ty[:n3] += ck * ak * (ak @ y[:n3])
    d = rows_of(nodes, N).ravel()
    r = (g.cpu().numpy() - Ty)[d]
    assert np.abs(r).max() <= 1e-8 * float(torch.linalg.norm(g))
