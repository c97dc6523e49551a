"""Plain, slow, FP64 CPU oracle for one Newton step of the nested block solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product (the HIP library and its Python binding) never calls it
and shares no code with it; both take their inputs from ``ns_inputs``.

What it computes, and where it comes from (Liu, Yang, Dong, Marsden, "The
nested block preconditioning technique for the incompressible Navier-Stokes
equations with emphasis on hemodynamic simulations"):

* ``discretization`` -- the residual-based VMS residual (Sec. 2.3) at the
  generalized-alpha intermediate states (Sec. 2.4.1) and its consistent
  tangent blocks A = F + K, B, C, D (Sec. 2.5, tangent-matrix equations), with
  the resistance outlet entering as the rank-one term K (Sec. 2.5).
* ``amg``    -- the algebraic multigrid V-cycle used as P_A and P_S.  The paper
  uses BoomerAMG (Sec. 3.1, AMG settings table); this oracle follows the
  repository's own written AMG definition instead (aggregation by two greedy
  pairwise matchings, Chebyshev smoothing, dense coarsest solve).
* ``krylov`` -- FGMRES(m) outer solver (Sec. 3), GMRES(m_A)/GMRES(m_S)
  intermediate and inner solvers, the matrix-free Schur complement action
  (Algorithm 2) and the SCR preconditioner action (Algorithm 3).
* ``adjoint`` -- the transposed system and the derivative of an outlet
  quantity with respect to the outlet resistances.
"""
