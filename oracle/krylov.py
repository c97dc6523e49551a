"""Nested Krylov solver of one Newton step, FP64, plain CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``fgmres``      -- FGMRES(m) with right preconditioning, restarted every m
  steps, stopping on the relative residual delta^r (Sec. 3, outer solver);
  after each cycle the true residual is recomputed and the solver restarts
  from the current iterate while it is above the tolerance and fewer than
  n^max iterations were taken.
* ``gmres_left``  -- GMRES(m) with a left preconditioner (the paper states left
  preconditioning for S in Sec. 3.1 and is silent for A; left is used for
  both), stopping on the preconditioned relative residual.
* ``schur_apply`` -- Algorithm 2: D x - C A^{-1}(B x) with an inner GMRES on A.
* ``scr_apply``   -- Algorithm 3: the action of P_SCR^{-1}.
* ``simple_apply`` -- the action of P_SIMPLE^{-1} (Sec. 3.2): the inverse of
  the three factors  [I 0; C A^{-1} I] [A 0; 0 S_hat] [I diag(A)^{-1} B; 0 I]
  taken in turn, i.e. Algorithm 3 with its Schur solve on the sparse S_hat
  (no inner solver) and its second A-solve replaced by the diagonal update
  y_v = yhat_v - diag(A)^{-1} B y_p.  The intermediate solvers follow the
  P_SCR settings (delta_A, delta_S, m_A, m_S, P_A, P_S).

Readings where the paper is silent: all Krylov solves start from zero;
orthogonalisation is classical Gram-Schmidt applied twice; the Hessenberg
least-squares problem is solved with Givens rotations; a step is a
(happy) breakdown when the new basis norm is <= 1e-14 times the norm of the
vector before orthogonalisation.

Iteration schedule: every Krylov call reserves a slot in ``Schedule.log`` when
it starts (so calls are numbered in start order) and stores its iteration
count when it ends.  Given a ``replay`` list, each call runs exactly that many
iterations instead of testing its tolerance (used to make two
implementations follow the same iteration path).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import amg as amg_mod

BREAKDOWN = 1e-14


class Schedule:
    def __init__(self, replay=None):
        self.log = []
        self.replay = None if replay is None else list(replay)

    def begin(self):
        idx = len(self.log)
        self.log.append(None)
        forced = None
        if self.replay is not None:
            forced = int(self.replay[idx])
        return idx, forced

    def end(self, idx, count):
        self.log[idx] = int(count)


def _givens_column(H, cs, sn, g, j):
    """Apply the previous rotations to column j of H, create rotation j, update g."""
    for i in range(j):
        t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
        H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
        H[i, j] = t
    rho = np.hypot(H[j, j], H[j + 1, j])
    if rho == 0.0:
        cs[j], sn[j] = 1.0, 0.0
    else:
        cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
    H[j, j] = rho
    H[j + 1, j] = 0.0
    g[j + 1] = -sn[j] * g[j]
    g[j] = cs[j] * g[j]


def _cgs2(V, w):
    """Classical Gram-Schmidt, two passes.  V: [k, n]."""
    wpre = np.linalg.norm(w)
    h1 = V @ w
    w = w - V.T @ h1
    h2 = V @ w
    w = w - V.T @ h2
    return h1 + h2, w, wpre


def gmres_left(apply_M, apply_P, b, rtol, m, nmax, sched: Schedule, atol=1e-50):
    """Left-preconditioned GMRES(m) for M x = b from x0 = 0."""
    idx, forced = sched.begin()
    n = b.shape[0]
    x = np.zeros(n)
    r = apply_P(b)
    beta0 = np.linalg.norm(r)
    total = 0
    if beta0 == 0.0 or forced == 0:
        sched.end(idx, 0)
        return x, 0
    tol = max(rtol * beta0, atol)
    beta = beta0
    while True:
        V = np.zeros((m + 1, n))
        V[0] = r / beta
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        finished = False
        for j in range(m):
            w = apply_P(apply_M(V[j]))
            h, w, wpre = _cgs2(V[:j + 1], w)
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            breakdown = hn <= BREAKDOWN * wpre
            if not breakdown:
                V[j + 1] = w / hn
            _givens_column(H, cs, sn, g, j)
            total += 1
            k = j + 1
            if forced is not None:
                done = total >= forced
            else:
                done = abs(g[j + 1]) <= tol
            if done or breakdown or total >= nmax:
                finished = True
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + V[:k].T @ y
        if finished:
            break
        r = apply_P(b - apply_M(x))
        beta = np.linalg.norm(r)
        if beta == 0.0 or (forced is None and beta <= tol):
            break
    sched.end(idx, total)
    return x, total


def fgmres(apply_A, apply_Pinv, b, rtol, m, nmax, sched: Schedule, atol=1e-50):
    """Right-preconditioned flexible GMRES(m) for A x = b from x0 = 0.

    Returns (x, iterations, true relative residual, converged)."""
    idx, forced = sched.begin()
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0 or forced == 0:
        sched.end(idx, 0)
        return x, 0, 0.0, True
    tol = max(rtol * bnorm, atol)
    r = b.copy()
    beta = bnorm
    total = 0
    while True:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        V[0] = r / beta
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            Z[j] = apply_Pinv(V[j])
            w = apply_A(Z[j])
            h, w, wpre = _cgs2(V[:j + 1], w)
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            breakdown = hn <= BREAKDOWN * wpre
            if not breakdown:
                V[j + 1] = w / hn
            _givens_column(H, cs, sn, g, j)
            total += 1
            k = j + 1
            if forced is not None:
                done = total >= forced
            else:
                done = abs(g[j + 1]) <= tol
            if done or breakdown or total >= nmax:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + Z[:k].T @ y
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if forced is not None:
            if total >= forced or beta == 0.0:
                break
        elif beta <= tol or total >= nmax or beta == 0.0:
            break
    sched.end(idx, total)
    return x, total, beta / bnorm, beta <= tol


# ----------------------------------------------------------------------------
# Nested block preconditioner (Algorithms 2 and 3)
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class SolveOpts:
    rtol: float = 1e-8
    m: int = 200
    nmax: int = 200
    rtol_A: float = 1e-3
    rtol_S: float = 1e-3
    rtol_I: float = 1e-3
    m_A: int = 200
    m_S: int = 200
    nmax_A: int = 200
    nmax_S: int = 200
    pc_A: str = "amg"        # "amg" or "jacobi"
    pc_I: str | None = None  # P of the inner A-solves of Algorithm 2 (None: as pc_A)
    cheb_degree: int = 2
    cheb_degree_S: int = 0   # Chebyshev degree on the S_hat hierarchy (0: cheb_degree)
    cheb_ratio: float = 10.0
    cycles_S: int = 1        # V-cycle iterations per application of P_S
    cc_scale_A: float = 1.0  # coarse-grid correction scaling of the A hierarchy
    cc_scale_S: float = 1.0  # and of the S_hat hierarchy
    cycle_index_A: int = 1   # AMG cycle index below the finest level (1: V, 2: W), A hierarchy
    cycle_index_S: int = 1   # and S_hat hierarchy
    pc: str = "scr"          # outer preconditioner: "scr" (Algorithm 3) or "simple" (Sec. 3.2)
    coarse_nodes: int = 128
    coarse_matchings: int = 3   # greedy matchings composed per coarsening step below the finest
    max_levels: int = 16
    atol: float = 1e-50


class NestedSolver:
    """Holds the per-step preconditioner set-up for one assembled system."""

    def __init__(self, S, adj, opts: SolveOpts):
        self.S = S
        self.o = opts
        self.N = S.n_nodes
        self.aggs = amg_mod.build_aggregates(adj, opts.coarse_nodes, opts.max_levels, opts.coarse_matchings)
        dA = S.diag_A()
        self.dA = dA
        # lumped rank-one diagonal added to F for the A-hierarchy (diag(K))
        dK = np.zeros(3 * self.N)
        for ak, ck in zip(S.a, S.c):
            dK += ck * ak * ak
        self.amgA = amg_mod.AMG(S.A_F, 3, self.aggs, opts.cheb_degree, extra_diag=dK, cheb_ratio=opts.cheb_ratio,
                                cc_scale=opts.cc_scale_A, cycle_index=opts.cycle_index_A)
        # S_hat = D - C diag(A)^{-1} B  (Sec. 3.1)
        import scipy.sparse as sp
        self.Shat = (S.D - S.C @ sp.diags(1.0 / dA) @ S.B).tocsr()
        self.amgS = amg_mod.AMG(self.Shat, 1, self.aggs, opts.cheb_degree_S or opts.cheb_degree,
                                cheb_ratio=opts.cheb_ratio, cc_scale=opts.cc_scale_S,
                                cycle_index=opts.cycle_index_S)

    def pS(self, r):
        """P_S: ``cycles_S`` steps of the stationary V-cycle iteration on
        S_hat from zero, z <- z + V(r - S_hat z)."""
        z = self.amgS.vcycle(r)
        for _ in range(self.o.cycles_S - 1):
            z = z + self.amgS.vcycle(r - self.Shat @ z)
        return z

    def pA(self, r, pc=None):
        if (pc or self.o.pc_A) == "jacobi":
            return r / self.dA
        return self.amgA.vcycle(r)

    def solve_A(self, b, rtol, sched, inner=False):
        o = self.o
        pc = (o.pc_I or o.pc_A) if inner else o.pc_A
        x, _ = gmres_left(self.S.apply_A, lambda r: self.pA(r, pc), b, rtol, o.m_A, o.nmax_A, sched, o.atol)
        return x

    def schur_apply(self, xp, sched):
        """Algorithm 2."""
        S = self.S
        xhat = S.D @ xp
        xbar = S.B @ xp
        xt = self.solve_A(xbar, self.o.rtol_I, sched, inner=True)
        return xhat - S.C @ xt

    def scr_apply(self, s, sched):
        """Algorithm 3."""
        S, o = self.S, self.o
        n3 = 3 * self.N
        sv, sp_ = s[:n3], s[n3:]
        yv_hat = self.solve_A(sv, o.rtol_A, sched)
        tp = sp_ - S.C @ yv_hat
        yp, _ = gmres_left(lambda q: self.schur_apply(q, sched), self.pS, tp, o.rtol_S,
                           o.m_S, o.nmax_S, sched, o.atol)
        tv = sv - S.B @ yp
        yv = self.solve_A(tv, o.rtol_A, sched)
        return np.concatenate([yv, yp])

    def simple_apply(self, s, sched):
        """P_SIMPLE^{-1} s (Sec. 3.2): lower factor, block diagonal, upper factor."""
        S, o = self.S, self.o
        n3 = 3 * self.N
        sv, sp_ = s[:n3], s[n3:]
        yv_hat = self.solve_A(sv, o.rtol_A, sched)
        tp = sp_ - S.C @ yv_hat
        yp, _ = gmres_left(lambda q: self.Shat @ q, self.pS, tp, o.rtol_S, o.m_S, o.nmax_S, sched, o.atol)
        yv = yv_hat - (S.B @ yp) / self.dA
        return np.concatenate([yv, yp])

    def solve(self, rhs, replay=None):
        sched = Schedule(replay)
        o = self.o
        if o.pc not in ("scr", "simple"):
            raise ValueError(f"unknown outer preconditioner {o.pc!r}")
        apply_pc = self.scr_apply if o.pc == "scr" else self.simple_apply
        x, its, relres, conv = fgmres(self.S.apply, lambda v: apply_pc(v, sched), rhs, o.rtol,
                                      o.m, o.nmax, sched, o.atol)
        return x, dict(outer=its, true_rel_res=relres, converged=conv, schedule=sched.log)
