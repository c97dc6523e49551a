"""VMS residual and consistent tangent of one Newton step, FP64, plain CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Definitions followed:
* residual forms B_m (volume, outlet traction, backflow) and B_p, the fine
  scales v', p', tau_M, tau_C and the metric tensor G with the simplex matrix M
  -- Sec. 2.3 (VMS formulation, equations for B_m^vol, B_m^bc, B_m^bf, B_p,
  tau_M and G);
* the generalized-alpha parameters alpha_m, alpha_f, gamma -- Sec. 2.4.1;
* the tangent blocks F, K, B, C, D as alpha_m / (alpha_f gamma dt) weighted
  derivatives of the residual -- Sec. 2.5 (tangent-matrix equations), with
  K = alpha_f gamma dt sum_k m^k a^k a^k^T and m^k = R^k for a resistance
  outlet, a^k_{Ai} = int N_A n_i.

Readings where the paper is silent:
* quadrature: 4-point degree-2 Gauss rule on tetrahedra, 3-point interior rule
  on outlet triangles;
* tau_M and tau_C are frozen (evaluated at the current state) when the tangent
  is formed; the tangent is the exact Jacobian of that frozen-tau residual;
* d(x)_-/dx = 1 for x < 0 and 0 for x >= 0;
* Dirichlet degrees of freedom: their rows and columns are zeroed, the
  diagonal entry set to 1, the residual entry set to 0, and a^k zeroed there.

The tangent is obtained with forward-mode automatic differentiation of the
residual as written (16 directional derivatives per element), so it is the
derivative of exactly the residual evaluated here.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import torch

torch.set_default_dtype(torch.float64)

C_T = 4.0
C_I = 36.0
BETA_BF = 0.2
M_SIMPLEX = (2.0 ** (1.0 / 3.0) / 2.0) * np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]])

_QA = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
_QB = (5.0 - np.sqrt(5.0)) / 20.0
# barycentric coordinates (N_0..N_3) of the 4 tetrahedron quadrature points, weight V/4 each
TET_QUAD = np.array([[_QA, _QB, _QB, _QB], [_QB, _QA, _QB, _QB], [_QB, _QB, _QA, _QB], [_QB, _QB, _QB, _QA]])
# barycentric coordinates of the 3 triangle quadrature points, weight |f|/3 each
TRI_QUAD = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])


def gen_alpha(rho_inf: float):
    """alpha_m, alpha_f, gamma of the generalized-alpha method (Sec. 2.4.1)."""
    am = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf)
    af = 1.0 / (1.0 + rho_inf)
    return am, af, af


@dataclasses.dataclass
class Physics:
    rho: float
    mu: float
    dt: float
    rho_inf: float
    beta: float = BETA_BF
    c_t: float = C_T
    c_i: float = C_I

    @property
    def alphas(self):
        return gen_alpha(self.rho_inf)

    @property
    def c_m(self):
        return self.alphas[0]

    @property
    def c_f(self):
        _, af, g = self.alphas
        return af * g * self.dt


def physics_of(case) -> Physics:
    return Physics(case.rho, case.mu, case.dt, case.rho_inf)


# ----------------------------------------------------------------------------
# Element geometry
# ----------------------------------------------------------------------------


def tet_geometry(xyz: np.ndarray, tets: np.ndarray):
    """Volume, basis gradients dN_a/dx_i [E,4,3] and metric G [E,3,3].

    x = x_0 + sum_k xi_k (x_k - x_0); dxi_k/dx_i = (J^{-1})_{ki};
    G_ij = sum_kl dxi_k/dx_i M_kl dxi_l/dx_j (Sec. 2.3, definition of G).
    """
    p = xyz[tets]
    J = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    vol = det / 6.0
    Jinv = np.linalg.inv(J)  # [E,3(k),3(i)] = dxi_k/dx_i
    gN = np.empty((len(tets), 4, 3))
    gN[:, 1:, :] = Jinv
    gN[:, 0, :] = -Jinv.sum(axis=1)
    G = np.einsum("eki,kl,elj->eij", Jinv, M_SIMPLEX, Jinv)
    return vol, gN, G


def tau_mc(G: np.ndarray, vq: np.ndarray, ph: Physics):
    """tau_M and tau_C at quadrature points (Sec. 2.3).  vq: [E,Q,3]."""
    vGv = np.einsum("eqi,eij,eqj->eq", vq, G, vq)
    GG = np.einsum("eij,eij->e", G, G)[:, None]
    tauM = (1.0 / ph.rho) / np.sqrt(ph.c_t / ph.dt ** 2 + vGv + ph.c_i * (ph.mu / ph.rho) ** 2 * GG)
    trG = np.einsum("eii->e", G)[:, None]
    tauC = 1.0 / (tauM * trG)
    return tauM, tauC


# ----------------------------------------------------------------------------
# Element residual (torch so that the exact derivative is available)
# ----------------------------------------------------------------------------


def _volume_residual(ve, ae, pe, gN, vol, tauM, tauC, ph: Physics):
    """Momentum rows Rm [E,4,3] and continuity rows Rp [E,4] of B_m^vol, B_p.

    ve, ae: [E,4,3] nodal velocity at n+af and acceleration at n+am;
    pe: [E,4] nodal pressure at n+af; tauM, tauC: [E,Q] (held fixed here).
    Per quadrature point, with w = N_a e_i and q = N_a (Sec. 2.3):
      rho N_a (a_i + (v.grad)v_i) - d_iN_a p + mu sum_l d_lN_a (d_l v_i + d_i v_l)
      - rho v'_i (v.grad N_a) + rho N_a (v'.grad) v_i - rho v'_i (v'.grad N_a)
      - d_iN_a p'
    and  N_a div v - grad N_a . v',  with v' = -tau_M (rho a + rho (v.grad)v
    + grad p) (the viscous term of v' vanishes for linear elements, b = 0) and
    p' = -tau_C div v.
    """
    rho, mu = ph.rho, ph.mu
    Nq = torch.as_tensor(TET_QUAD)
    gradv = torch.einsum("eai,eaj->eij", ve, gN)  # d_j v_i
    gradp = torch.einsum("ea,eaj->ej", pe, gN)
    divv = gradv.diagonal(dim1=1, dim2=2).sum(-1)
    visc = mu * (torch.einsum("eal,eil->eai", gN, gradv) + torch.einsum("eal,eli->eai", gN, gradv))
    Rm = torch.zeros_like(ve)
    Rp = torch.zeros_like(pe)
    w = (vol / 4.0)[:, None]
    for q in range(4):
        N = Nq[q]
        vq = torch.einsum("a,eai->ei", N, ve)
        aq = torch.einsum("a,eai->ei", N, ae)
        pq = torch.einsum("a,ea->e", N, pe)
        conv = torch.einsum("eij,ej->ei", gradv, vq)
        rM = rho * (aq + conv) + gradp
        vp = -tauM[:, q, None] * rM
        pp = -tauC[:, q] * divv
        v_gN = torch.einsum("ei,eai->ea", vq, gN)
        vp_gN = torch.einsum("ei,eai->ea", vp, gN)
        vp_gv = torch.einsum("eij,ej->ei", gradv, vp)
        rq = (rho * N[None, :, None] * (aq + conv)[:, None, :]
              - gN * pq[:, None, None]
              + visc
              - rho * vp[:, None, :] * v_gN[:, :, None]
              + rho * N[None, :, None] * vp_gv[:, None, :]
              - rho * vp[:, None, :] * vp_gN[:, :, None]
              - gN * pp[:, None, None])
        Rm = Rm + w[:, :, None] * rq
        Rp = Rp + w * (N[None, :] * divv[:, None] - torch.einsum("eai,ei->ea", gN, vp))
    return Rm, Rp


def _backflow_residual(vf, nrm, area, ph: Physics):
    """Rows of B_m^bf on outlet triangles: -rho beta (v.n)_- N_a v_i (Sec. 2.3).

    vf: [F,3,3] nodal velocity; nrm: [F,3] unit outward normal; area: [F].
    """
    Nq = torch.as_tensor(TRI_QUAD)
    R = torch.zeros_like(vf)
    for q in range(3):
        N = Nq[q]
        vq = torch.einsum("a,fai->fi", N, vf)
        vn = (vq * nrm).sum(-1)
        neg = torch.where(vn < 0, vn, torch.zeros_like(vn))
        R = R + (area / 3.0)[:, None, None] * (-ph.rho * ph.beta) * neg[:, None, None] * N[None, :, None] * vq[:, None, :]
    return R


# ----------------------------------------------------------------------------
# Global assembly
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Assembled:
    """Eliminated linear system of one Newton step, field-split ordering
    x = [dv_dot (3N, node-interleaved); dp_dot (N)]."""
    A_F: sp.csr_matrix       # F block (3N x 3N), without the rank-one term
    B: sp.csr_matrix         # 3N x N
    C: sp.csr_matrix         # N x 3N
    D: sp.csr_matrix         # N x N
    a: list                  # a^k as dense 3N vectors (zeroed at Dirichlet DOFs)
    c: np.ndarray            # rank-one weights alpha_f gamma dt R^k
    rhs: np.ndarray          # -[R_m; R_p], zero at Dirichlet DOFs (4N)
    residual: np.ndarray     # [R_m; R_p] before elimination (4N)
    Q: np.ndarray            # outlet flow rates a^k . v (with Dirichlet entries kept)
    area: np.ndarray         # outlet areas
    w_p: list                # int_{Gamma^k} N_A (N vectors), for mean outlet pressures
    n_nodes: int

    def apply_A(self, x):
        y = self.A_F @ x
        for ak, ck in zip(self.a, self.c):
            y = y + ck * ak * (ak @ x)
        return y

    def apply(self, x):
        n3 = 3 * self.n_nodes
        xv, xp = x[:n3], x[n3:]
        return np.concatenate([self.apply_A(xv) + self.B @ xp, self.C @ xv + self.D @ xp])

    def dense(self):
        n3 = 3 * self.n_nodes
        A = self.A_F.toarray()
        for ak, ck in zip(self.a, self.c):
            A = A + ck * np.outer(ak, ak)
        return np.block([[A, self.B.toarray()], [self.C.toarray(), self.D.toarray()]])

    def diag_A(self):
        """diag(F) + sum_k c_k (a^k)^2 : the point diagonal of A = F + K."""
        d = self.A_F.diagonal().copy()
        for ak, ck in zip(self.a, self.c):
            d += ck * ak * ak
        return d

    def transposed(self):
        """Blocks of the transposed system [A^T C^T; B^T D^T]."""
        return dataclasses.replace(self, A_F=self.A_F.T.tocsr(), B=self.C.T.tocsr(),
                                   C=self.B.T.tocsr(), D=self.D.T.tocsr())


def outlet_vectors(case):
    """a^k_{Ai} = int_{Gamma^k} N_A n_i and w^k_A = int N_A over outlet k.

    For a linear basis on a flat triangle int N_A = |f|/3 exactly.
    Returns (a [n_out, N, 3], w [n_out, N], area [n_out])."""
    N = case.n_nodes
    n_out = case.n_outlets
    a = np.zeros((n_out, N, 3))
    w = np.zeros((n_out, N))
    area = np.zeros(n_out)
    for k in range(n_out):
        f = case.faces[case.outlet_ptr[k]:case.outlet_ptr[k + 1]]
        p = case.xyz[f]
        cr = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
        ar = 0.5 * np.linalg.norm(cr, axis=1)
        n = cr / (2.0 * ar[:, None])
        for c in range(3):
            np.add.at(a[k], f[:, c], (ar / 3.0)[:, None] * n)
            np.add.at(w[k], f[:, c], ar / 3.0)
        area[k] = ar.sum()
    return a, w, area


def assemble(case, P_af=None, R=None, ph: Physics | None = None, v=None, p=None, vdot=None,
             tau_off: bool = False, chunk: int = 200000) -> Assembled:
    """Residual and tangent of one Newton step (Sec. 2.5, steps 6 and 8).

    ``P_af`` -- outlet pressures P^k_{n+af} entering the traction term;
    ``R``    -- outlet resistances (the m^k of the rank-one term).
    Defaults: the case's R and P_af = R^k Q^k (state at rest in time, so
    P_n = P_{n+1} = R Q).  ``tau_off`` zeroes tau_M and tau_C (Galerkin form).
    """
    ph = ph or physics_of(case)
    am, af, gam = ph.alphas
    c_m, c_f = am, af * gam * ph.dt
    v = case.v if v is None else v
    p = case.p if p is None else p
    vdot = case.vdot if vdot is None else vdot
    R = case.R if R is None else np.asarray(R, float)
    N = case.n_nodes
    n3 = 3 * N
    a_vec, w_vec, area = outlet_vectors(case)
    Q = np.array([np.sum(a_vec[k] * v) for k in range(case.n_outlets)])
    if P_af is None:
        P_af = R * Q
    P_af = np.asarray(P_af, float)

    vol, gN, G = tet_geometry(case.xyz, case.tets)
    tets = case.tets
    E = len(tets)
    res = np.zeros(4 * N)
    rows_l, cols_l, vals_l = [], [], []
    # global DOF index of (node, comp): comp<3 -> 3*node+comp, comp==3 -> 3N+node
    for s in range(0, E, chunk):
        e = slice(s, min(E, s + chunk))
        te = tets[e]
        ve0 = torch.as_tensor(v[te])
        ae0 = torch.as_tensor(vdot[te])
        pe0 = torch.as_tensor(p[te])
        gNe = torch.as_tensor(gN[e])
        vole = torch.as_tensor(vol[e])
        vq = np.einsum("qa,eai->eqi", TET_QUAD, v[te])
        tM, tC = tau_mc(G[e], vq, ph)
        if tau_off:
            tM, tC = np.zeros_like(tM), np.zeros_like(tC)
        tM, tC = torch.as_tensor(tM), torch.as_tensor(tC)

        def f(dv, dpp):
            return _volume_residual(ve0 + c_f * dv, ae0 + c_m * dv, pe0 + c_f * dpp, gNe, vole, tM, tC, ph)

        z3 = torch.zeros_like(ve0)
        z1 = torch.zeros_like(pe0)
        Rm, Rp = f(z3, z1)
        ne = te.shape[0]
        rvals = np.concatenate([Rm.numpy(), Rp.numpy()[:, :, None]], axis=2)  # [e,4(a),4(i)]
        gidx = np.concatenate([3 * te[:, :, None] + np.arange(3)[None, None, :], (n3 + te)[:, :, None]], axis=2)
        np.add.at(res, gidx.ravel(), rvals.ravel())
        Jcols = np.empty((ne, 4, 4, 4, 4))  # [e, a, i, b, j]
        for b in range(4):
            for j in range(4):
                t3 = torch.zeros_like(ve0)
                t1 = torch.zeros_like(pe0)
                if j < 3:
                    t3[:, b, j] = 1.0
                else:
                    t1[:, b] = 1.0
                _, (dRm, dRp) = torch.func.jvp(f, (z3, z1), (t3, t1))
                Jcols[:, :, :3, b, j] = dRm.numpy()
                Jcols[:, :, 3, b, j] = dRp.numpy()
        rows = np.broadcast_to(gidx[:, :, :, None, None], Jcols.shape)
        cols = np.broadcast_to(gidx[:, None, None, :, :], Jcols.shape)
        rows_l.append(rows.ravel().copy())
        cols_l.append(cols.ravel().copy())
        vals_l.append(Jcols.ravel().copy())

    # outlet faces: traction term P_af a^k and backflow
    for k in range(case.n_outlets):
        res[:n3] += P_af[k] * a_vec[k].ravel()
        f = case.faces[case.outlet_ptr[k]:case.outlet_ptr[k + 1]]
        px = case.xyz[f]
        cr = np.cross(px[:, 1] - px[:, 0], px[:, 2] - px[:, 0])
        ar = 0.5 * np.linalg.norm(cr, axis=1)
        nrm = torch.as_tensor(cr / (2.0 * ar[:, None]))
        art = torch.as_tensor(ar)
        vf0 = torch.as_tensor(v[f])

        def g(dv):
            return _backflow_residual(vf0 + c_f * dv, nrm, art, ph)

        z = torch.zeros_like(vf0)
        Rb = g(z).numpy()
        gi = 3 * f[:, :, None] + np.arange(3)[None, None, :]
        np.add.at(res, gi.ravel(), Rb.ravel())
        Jb = np.empty((len(f), 3, 3, 3, 3))
        for b in range(3):
            for j in range(3):
                t = torch.zeros_like(vf0)
                t[:, b, j] = 1.0
                _, dR = torch.func.jvp(g, (z,), (t,))
                Jb[:, :, :, b, j] = dR.numpy()
        rows_l.append(np.broadcast_to(gi[:, :, :, None, None], Jb.shape).ravel().copy())
        cols_l.append(np.broadcast_to(gi[:, None, None, :, :], Jb.shape).ravel().copy())
        vals_l.append(Jb.ravel().copy())

    T = sp.coo_matrix((np.concatenate(vals_l), (np.concatenate(rows_l), np.concatenate(cols_l))),
                      shape=(4 * N, 4 * N)).tocsr()
    T.sum_duplicates()

    # Dirichlet / pin elimination
    dmask = np.concatenate([case.mask[:, :3].ravel(), case.mask[:, 3]]).astype(bool)
    keep = sp.diags((~dmask).astype(float))
    T = (keep @ T @ keep).tocsr() + sp.diags(dmask.astype(float))
    T = T.tocsr()
    T.sort_indices()
    rhs = -res.copy()
    rhs[dmask] = 0.0
    a_list = []
    for k in range(case.n_outlets):
        ak = a_vec[k].ravel().copy()
        ak[dmask[:n3]] = 0.0
        a_list.append(ak)
    return Assembled(A_F=T[:n3, :n3].tocsr(), B=T[:n3, n3:].tocsr(), C=T[n3:, :n3].tocsr(),
                     D=T[n3:, n3:].tocsr(), a=a_list, c=c_f * R.copy(), rhs=rhs, residual=res,
                     Q=Q, area=area, w_p=[w_vec[k] for k in range(case.n_outlets)], n_nodes=N)


def residual_only(case, v, p, vdot, P_af, ph: Physics | None = None, tau_fixed=None):
    """Residual [R_m; R_p] (4N, before elimination) at an arbitrary state.

    ``tau_fixed`` -- optional (tauM, tauC) arrays [E,Q] to hold the
    stabilisation parameters fixed (the frozen-tau residual whose exact
    derivative is the tangent)."""
    ph = ph or physics_of(case)
    N = case.n_nodes
    n3 = 3 * N
    vol, gN, G = tet_geometry(case.xyz, case.tets)
    te = case.tets
    if tau_fixed is None:
        vq = np.einsum("qa,eai->eqi", TET_QUAD, v[te])
        tM, tC = tau_mc(G, vq, ph)
    else:
        tM, tC = tau_fixed
    Rm, Rp = _volume_residual(torch.as_tensor(v[te]), torch.as_tensor(vdot[te]), torch.as_tensor(p[te]),
                              torch.as_tensor(gN), torch.as_tensor(vol), torch.as_tensor(tM),
                              torch.as_tensor(tC), ph)
    res = np.zeros(4 * N)
    np.add.at(res, (3 * te[:, :, None] + np.arange(3)).ravel(), Rm.numpy().ravel())
    np.add.at(res, (n3 + te).ravel(), Rp.numpy().ravel())
    a_vec, _, _ = outlet_vectors(case)
    for k in range(case.n_outlets):
        res[:n3] += P_af[k] * a_vec[k].ravel()
        f = case.faces[case.outlet_ptr[k]:case.outlet_ptr[k + 1]]
        px = case.xyz[f]
        cr = np.cross(px[:, 1] - px[:, 0], px[:, 2] - px[:, 0])
        ar = 0.5 * np.linalg.norm(cr, axis=1)
        Rb = _backflow_residual(torch.as_tensor(v[f]), torch.as_tensor(cr / (2 * ar[:, None])),
                                torch.as_tensor(ar), ph).numpy()
        np.add.at(res, (3 * f[:, :, None] + np.arange(3)).ravel(), Rb.ravel())
    return res


def frozen_tau(case, v, ph: Physics | None = None):
    ph = ph or physics_of(case)
    _, _, G = tet_geometry(case.xyz, case.tets)
    vq = np.einsum("qa,eai->eqi", TET_QUAD, v[case.tets])
    return tau_mc(G, vq, ph)
