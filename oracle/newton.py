"""One time step by the predictor multi-corrector algorithm, FP64, plain CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``windkessel``  -- the reduced model of an outlet over one time step: the
  three-element Windkessel ODE for the distal pressure drop Pi (Sec. 2.3),
  integrated by the fourth-order Runge-Kutta scheme of Algorithm 1 (stages at
  the thirds of each sub-interval, weights 1/8, 3/8, 3/8, 1/8, the flow rate
  interpolated linearly in time); zero compliance is the resistance model.
* ``time_step``   -- the predictor multi-corrector stage of Sec. 2.5: predictor
  y = y_n, ydot = (gamma-1)/gamma ydot_n; each corrector computes the outlet
  flows of the current iterate, the outlet pressures at t_{n+1} from the
  reduced model and their derivatives m^k by a central difference quotient,
  the state at n+alpha_f / n+alpha_m, assembles, stops on the relative or
  absolute residual tolerance, else solves the tangent system with the nested
  solver and applies the update y += gamma dt dydot, ydot += dydot.

Readings: the residual norm is the l2 norm of the assembled residual with the
Dirichlet entries removed (the rhs of the linear system); ||R_(0)|| is the
first corrector's residual; the returned state is the last iterate (the one
whose residual met the tolerance); at most l_max systems are solved and the
residual of the returned iterate is always evaluated, also after the l_max-th
update (one more assembly), so the history ends with it.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import amg as amg_mod
from . import discretization as dz
from . import krylov as kr


def windkessel(Rp, C, Rd, Pd, Pi_n, Q_n, Q_np1, n_ts, dt):
    """P_{n+1} and Pi_{n+1} of one outlet over one time step (Algorithm 1)."""
    if C == 0.0:
        return (Rp + Rd) * Q_np1 + Pd, 0.0
    h = dt / n_ts

    def F(Pi, Q):
        return -Pi / (Rd * C) + Q / C

    def Qm(m):
        return (1.0 - m / n_ts) * Q_n + (m / n_ts) * Q_np1

    Pi = Pi_n
    for m in range(n_ts):
        q0, q1 = Qm(m), Qm(m + 1)
        k1 = F(Pi, q0)
        k2 = F(Pi + k1 * h / 3.0, 2.0 * q0 / 3.0 + q1 / 3.0)
        k3 = F(Pi - k1 * h / 3.0 + k2 * h, q0 / 3.0 + 2.0 * q1 / 3.0)
        k4 = F(Pi + k1 * h - k2 * h + k3 * h, q1)
        Pi = Pi + k1 * h / 8.0 + 3.0 * k2 * h / 8.0 + 3.0 * k3 * h / 8.0 + k4 * h / 8.0
    return Rp * Q_np1 + Pi + Pd, Pi


@dataclasses.dataclass
class OutletModel:
    Rp: np.ndarray
    C: np.ndarray
    Rd: np.ndarray
    Pd: np.ndarray          # distal pressure at t_{n+1}
    Pi: np.ndarray          # at t_n
    P: np.ndarray           # at t_n
    Q: np.ndarray           # at t_n
    n_ts: int = 100


@dataclasses.dataclass
class NewtonOpts:
    tol_R: float = 1e-6
    tol_A: float = 1e-6
    eps_abs: float = 1e-8
    eps_rel: float = 1e-5
    l_max: int = 20


def _flows(case, a_raw, y):
    N = case.n_nodes
    v = y[:3 * N].reshape(N, 3)
    return np.array([np.sum(a_raw[k] * v) for k in range(case.n_outlets)])


def time_step(case, y_n, ydot_n, model: OutletModel, nopt: NewtonOpts = NewtonOpts(),
              sopt: kr.SolveOpts = kr.SolveOpts(), linear_solve=None):
    """One time step.  ``linear_solve(S) -> dx`` replaces the nested solver
    (used by the dense check).  Returns (y, ydot, info, model at t_{n+1})."""
    ph = dz.physics_of(case)
    am, af, gam = ph.alphas
    dt = ph.dt
    N = case.n_nodes
    n3 = 3 * N
    a_raw, _, _ = dz.outlet_vectors(case)
    adj = amg_mod.node_adjacency(N, case.tets)
    y = y_n.copy()
    ydot = (gam - 1.0) / gam * ydot_n
    no = case.n_outlets

    def G(k, q):
        return windkessel(model.Rp[k], model.C[k], model.Rd[k], model.Pd[k], model.Pi[k], model.Q[k], q,
                          model.n_ts, dt)

    hist = []
    iterations = 0
    converged = False
    r0 = None
    for l in range(1, nopt.l_max + 2):
        Q = _flows(case, a_raw, y)
        m = np.zeros(no)
        Paf = np.zeros(no)
        for k in range(no):
            eps = max(nopt.eps_abs, nopt.eps_rel * abs(Q[k]))
            P = G(k, Q[k])[0]
            m[k] = (G(k, Q[k] + 0.5 * eps)[0] - G(k, Q[k] - 0.5 * eps)[0]) / eps
            Paf[k] = (1.0 - af) * model.P[k] + af * P
        yaf = y_n + af * (y - y_n)
        ydam = ydot_n + am * (ydot - ydot_n)
        S = dz.assemble(case, P_af=Paf, R=m, v=yaf[:n3].reshape(N, 3), p=yaf[n3:], vdot=ydam[:n3].reshape(N, 3))
        r = float(np.linalg.norm(S.rhs))
        hist.append(r)
        if r0 is None:
            r0 = r
        if r <= nopt.tol_R * r0 or r <= nopt.tol_A:
            converged = True
            break
        if l > nopt.l_max:
            break
        if linear_solve is None:
            dx, _ = kr.NestedSolver(S, adj, sopt).solve(S.rhs)
        else:
            dx = linear_solve(S)
        y = y + gam * dt * dx
        ydot = ydot + dx
        iterations = l
    Q = _flows(case, a_raw, y)
    out = dataclasses.replace(model, Pi=model.Pi.copy(), P=model.P.copy(), Q=Q.copy())
    for k in range(no):
        out.P[k], out.Pi[k] = G(k, Q[k])
    return y, ydot, dict(iterations=iterations, converged=converged, res_hist=hist, res0=r0), out
