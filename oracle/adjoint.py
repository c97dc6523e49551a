"""Adjoint of the Newton-step solve and outlet-resistance derivatives, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The transposed tangent is [A^T C^T; B^T D^T]; with B' = C^T, C' = B^T its
Schur complement is D^T - B^T A^{-T} C^T = S^T, so the nested method of
Algorithms 2-3 applies unchanged to the transposed blocks (rank-one K is
symmetric).

Differentiable map (state frozen): R -> x(R) = A(R)^{-1} r(R), where R enters
* the tangent through K = alpha_f gamma dt sum_k R^k a^k a^k^T (Sec. 2.5), and
* the residual through the traction pressure
  P^k_{n+af} = (1 - alpha_f) P^k_n + alpha_f R^k Q^k (resistance outlet,
  Sec. 2.2 and Sec. 2.5 step 5), with P^k_n held fixed.
So dA/dR_k = blockdiag(c_f a^k a^k^T, 0) with c_f = alpha_f gamma dt, and
dr/dR_k = -[alpha_f Q^k a^k; 0].  For a loss L(x) with lambda solving
A^T lambda = dL/dx:  dL/dR_k = lambda^T (dr/dR_k - (dA/dR_k) x).
"""
from __future__ import annotations

import numpy as np

from . import krylov


def adjoint_solve(S, adj, g, opts, replay=None):
    """Nested FGMRES on the transposed system."""
    ns = krylov.NestedSolver(S.transposed(), adj, opts)
    return ns.solve(g, replay=replay)


def grad_R(S, x, lam, alpha_f, c_f):
    """dL/dR_k = -(lambda_v . a^k) (alpha_f Q^k + c_f a^k . x_v)."""
    n3 = 3 * S.n_nodes
    lv, xv = lam[:n3], x[:n3]
    return np.array([-(lv @ ak) * (alpha_f * Qk + c_f * (ak @ xv)) for ak, Qk in zip(S.a, S.Q)])


def mean_outlet_pressure_weights(S, k, gamma_dt):
    """dJ_k/dx for J_k = (1/|Gamma^k|) sum_A w^k_A (p_A + gamma dt dp_dot_A)."""
    n3 = 3 * S.n_nodes
    g = np.zeros(4 * S.n_nodes)
    g[n3:] = gamma_dt * S.w_p[k] / S.area[k]
    return g
