/*
 * ns_api.h -- C ABI of the MI355X (gfx950) nested block solver for one
 * Newton-Raphson step of the VMS / generalized-alpha incompressible
 * Navier-Stokes discretisation (Liu, Yang, Dong, Marsden, "The nested block
 * preconditioning technique for the incompressible Navier-Stokes equations
 * with emphasis on hemodynamic simulations").
 *
 * The linear system of one Newton step is (Sec. 2.5, step 9 of the
 * predictor multi-corrector algorithm, and the block notation of Sec. 3)
 *
 *     [ A  B ] [ dv_dot ]     [ R_m ]
 *     [ C  D ] [ dp_dot ] = - [ R_p ] ,      A = F + K,
 *     K = alpha_f gamma dt sum_k m^k a^k a^k^T   (rank-one outlet terms),
 *
 * solved by FGMRES(m) (Sec. 3) right-preconditioned with the Schur
 * complement reduction P_SCR (Algorithm 3), whose Schur solve applies
 * S x = D x - C A^{-1} (B x) matrix-free (Algorithm 2) with an inner GMRES on
 * A, and whose A- and S-solves are GMRES(m_A), GMRES(m_S) preconditioned by
 * AMG V-cycles on A and on S_hat = D - C diag(A)^{-1} B (Sec. 3.1).
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Pointers named d_* are device pointers (HIP global memory of the device
 *   that was current at ns_ctx_bind); h_* are host pointers.  The caller owns
 *   all of them; the library keeps no reference to caller memory after a call
 *   returns, except the workspace given to ns_ctx_bind.
 * - Vectors over the 4N unknowns use the field-split layout
 *   [velocity (3N, node-interleaved: 3*node + component) ; pressure (N)].
 * - All device arithmetic of an entry point is enqueued on the given stream.
 *   ns_assemble_tangent returns without waiting; the solves wait for their
 *   stream (their stopping tests read one scalar per Krylov iteration).
 * - Negative status: the call failed, outputs are undefined, and
 *   ns_last_error(ctx) describes the failure.  NS_NOT_CONVERGED (> 0): the
 *   best iterate is in the output and the statistics are filled in.
 * - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef NS_API_H
#define NS_API_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_ctx ns_ctx; /* opaque, owned by the library */

typedef enum {
    NS_OK = 0,
    NS_NOT_CONVERGED = 1,   /* soft failure: tolerance not met within nmax */
    NS_ERR_ARG = -1,        /* invalid argument or inconsistent sizes */
    NS_ERR_HIP = -2,        /* a HIP runtime call failed */
    NS_ERR_NAN = -3,        /* a residual estimate became NaN or Inf */
    NS_ERR_BREAKDOWN = -4,  /* zero-norm preconditioned vector in the outer solver */
    NS_ERR_WORKSPACE = -5,  /* workspace missing or smaller than required */
    NS_ERR_STATE = -6       /* call order violated (e.g. solve before assembly) */
} ns_status;

/* Mesh: P1 tetrahedra (Sec. 2.3, linear basis), outlet surfaces Gamma_out^k
 * (Sec. 2.2) and the Dirichlet partition Gamma_g.  Host arrays, read during
 * ns_ctx_create and ns_ctx_bind only.
 *   h_xyz        [n_nodes][3] coordinates
 *   h_tets       [n_elems][4] vertex indices, positive orientation
 *   h_outlet_ptr [n_outlets + 1] CSR offsets of each outlet into h_faces
 *   h_faces      [h_outlet_ptr[n_outlets]][3] outlet triangles, right-hand
 *                normal pointing out of the domain; outlets must have
 *                disjoint node sets
 *   h_dirichlet  [n_nodes][4] 1 = Dirichlet (u, v, w) or pinned pressure   */
typedef struct {
    int32_t n_nodes, n_elems, n_outlets;
    const double* h_xyz;
    const int32_t* h_tets;
    const int32_t* h_outlet_ptr;
    const int32_t* h_faces;
    const uint8_t* h_dirichlet;
} ns_mesh;

/* Context options: sizes of the Krylov workspaces and the AMG hierarchy.
 * A field set to 0 takes the default in brackets. */
typedef struct {
    int32_t max_m;        /* largest outer restart length m      [200] */
    int32_t max_m_A;      /* largest m_A                          [200] */
    int32_t max_m_S;      /* largest m_S                          [200] */
    int32_t coarse_nodes; /* AMG coarsening stops at <= this many nodes [128] */
    int32_t max_levels;   /* AMG levels including the coarsest    [16]  */
    int32_t coarse_matchings; /* greedy pairwise matchings composed per
                           * coarsening step below the finest level, 2..4
                           * (aggregates of at most 2^k nodes); the finest
                           * step always uses two              [3]   */
} ns_ctx_opts;

/* Physics of one Newton step (Sec. 2.3, 2.4.1, 2.5).
 *   rho, mu    density and dynamic viscosity
 *   dt         time step size dt_n
 *   rho_inf    spectral radius of the generalized-alpha method
 *   beta_bf    backflow coefficient beta [0.2]
 *   c_t, c_i   C_T [4] and C_I [36] of tau_M
 * The outlets enter through m^k = dP^k_{n+af}/dQ^k (the rank-one weight) and
 * the traction pressure P^k_{n+af}, given in one of two ways:
 *   resistance outlets, h_R != NULL (Sec. 2.2, 2.5): P^k_{n+1} = R^k Q^k, so
 *     m^k = R^k and P^k_{n+af} = (1 - alpha_f) P^k_n + alpha_f R^k Q^k, formed
 *     by the library;
 *     h_R   [n_outlets] resistances R^k
 *     h_P_n [n_outlets] P^k_n at t_n, or NULL for P^k_n = R^k Q^k (a state at
 *           rest in time)
 *     h_Q   [n_outlets] flow rates Q^k = a^k . v of the current iterate, or
 *           NULL to take a^k . v from d_v_af on the device (the same at a
 *           frozen state, where y_{n+af} = y_{n+1})
 *     ns_resistance_gradient then differentiates the solve with respect to R;
 *   any reduced model, h_R == NULL: h_m [n_outlets] m^k and h_P_af
 *     [n_outlets] P^k_{n+af} as computed by the caller (ns_time_step fills them
 *     from the Windkessel model); h_P_n and h_Q are ignored.  */
typedef struct {
    double rho, mu, dt, rho_inf, beta_bf, c_t, c_i;
    const double* h_m;
    const double* h_P_af;
    const double* h_R;
    const double* h_P_n;
    const double* h_Q;
} ns_phys;

typedef enum { NS_PC_AMG = 0, NS_PC_JACOBI = 1 } ns_pc;
/* Outer (FGMRES) preconditioner.  NS_OUTER_SCR: the nested Schur complement
 * reduction of Algorithm 3, whose S-solve applies S = D - C A^-1 B
 * matrix-free (Algorithm 2).  NS_OUTER_SIMPLE: the SIMPLE preconditioner of
 * Sec. 3.2, the product [I 0; C A^-1 I][A 0; 0 S_hat][I diag(A)^-1 B; 0 I]
 * inverted factor by factor: one A-solve (rtol_A), one GMRES(m_S) solve on
 * the sparse S_hat = D - C diag(A)^-1 B (rtol_S, P_S), then
 * y_v = yhat_v - diag(A)^-1 B y_p; no inner solver (rtol_I unused). */
typedef enum { NS_OUTER_SCR = 0, NS_OUTER_SIMPLE = 1 } ns_outer_pc;
typedef enum { NS_FP64 = 0, NS_FP32_INNER = 1 } ns_precision;

/* Solver options (Sec. 3 and 3.1; paper defaults in brackets).  A field set
 * to 0 takes its default. */
typedef struct {
    double rtol;            /* delta^r of FGMRES                      [1e-8]  */
    double atol;            /* delta^a of every Krylov level          [1e-50] */
    double rtol_A;          /* delta^r_A, intermediate A-solves       [1e-3]  */
    double rtol_S;          /* delta^r_S, Schur solve                 [1e-3]  */
    double rtol_I;          /* delta^r_I, inner A-solve of Alg. 2     [1e-3]  */
    double cheb_ratio;      /* AMG smoother interval [lambda/cheb_ratio, lambda],
                             * lambda >= spectral radius of D^-1 M     [10]    */
    double cc_scale_A;      /* AMG coarse-grid correction x += c P e_c, c in
                             * (0, 2], on the A hierarchy              [1]     */
    double cc_scale_S;      /* the same on the S_hat hierarchy         [1]     */
    int32_t m, nmax;        /* FGMRES restart length / max iterations [200]   */
    int32_t m_A, nmax_A;    /* GMRES on A                             [200]   */
    int32_t m_S, nmax_S;    /* GMRES on S                             [200]   */
    int32_t pc_A;           /* ns_pc: P_A                             [AMG]   */
    int32_t precision;      /* ns_precision                           [FP64]  */
    int32_t cheb_degree;    /* AMG Chebyshev smoother degree, 1..8    [2]     */
    int32_t cycles_S;       /* V-cycle iterations per application of P_S
                             * (stationary iteration on S_hat from zero;
                             * may diverge when > 1)                   [1]    */
    int32_t pc;             /* ns_outer_pc: outer preconditioner      [SCR]   */
    int32_t cheb_degree_S;  /* Chebyshev degree on the S_hat hierarchy,
                             * 0..8; 0 = cheb_degree                  [0]     */
    int32_t pc_I;           /* P of the inner A-solves of Algorithm 2
                             * (Sec. 4 suggests a light one there):
                             * 0 = as pc_A, 1 = AMG, 2 = Jacobi       [0]     */
    int32_t cycle_index_A;  /* AMG cycle index on the A hierarchy: the coarse-
                             * grid correction and post-smoothing are repeated
                             * this many times on every level below the finest
                             * (1 = V-cycle, 2 = W-cycle), 1..3       [1]     */
    int32_t cycle_index_S;  /* the same on the S_hat hierarchy        [1]     */
    int32_t reserved;       /* must be 0 */
    /* Iteration schedule.  If h_sched != NULL, the i-th Krylov call (calls
     * numbered in the order they start: FGMRES, then each GMRES on A or S)
     * runs exactly h_sched[i] iterations instead of testing its tolerance.
     * If h_sched_out != NULL, the iteration count of each call is written to
     * h_sched_out[i] for i < sched_cap, and the number of calls to
     * ns_stats.n_calls. */
    const int32_t* h_sched;
    int32_t sched_len;
    int32_t sched_cap;
    int32_t* h_sched_out;
} ns_solve_opts;

typedef struct {
    int32_t outer_iters;    /* FGMRES iterations */
    int32_t a_solves, a_iters;         /* intermediate A-solves (Alg. 3 steps 1, 5;
                                        * SIMPLE: one per application) */
    int32_t s_solves, s_iters;         /* Schur solves (Alg. 3 step 3; SIMPLE:
                                        * the S_hat solve) */
    int32_t inner_solves, inner_iters; /* inner A-solves (Alg. 2 step 3) */
    int32_t n_calls;        /* Krylov calls (schedule entries) */
    int32_t amg_levels_A, amg_levels_S;
    double true_rel_res;    /* ||r - A x|| / ||r|| recomputed in FP64 */
    double setup_ms;        /* per-step preconditioner set-up */
    double solve_ms;        /* Krylov iterations */
} ns_stats;

/* ns_ctx_create: symbolic set-up on the host from the mesh alone (node
 * graph, 4x4-block BSR pattern, element colouring, element-to-block maps,
 * S_hat pattern, AMG aggregates and Galerkin maps).  No device work.
 * On success *out owns the context and *workspace_bytes is the size of the
 * device workspace ns_ctx_bind needs.  Errors: NS_ERR_ARG for inconsistent
 * sizes, indices out of range, or outlets that share nodes. */
ns_status ns_ctx_create(const ns_mesh* mesh, const ns_ctx_opts* opts, ns_ctx** out,
                        size_t* workspace_bytes);

/* ns_ctx_bind: lay out the caller-owned device workspace d_workspace
 * (>= workspace_bytes, 256-byte aligned) and upload the mesh, pattern and
 * maps on `stream`; computes the outlet vectors a^k_{Ai} = int N_A n_i
 * (Sec. 2.5).  The workspace must stay allocated until ns_ctx_destroy or
 * the next ns_ctx_bind (binding again moves the context to the new
 * workspace; a tangent must then be assembled again before a solve).
 * Meshes of up to 1024 nodes replay each Krylov step and set-up chain from
 * a HIP graph captured on first use; larger ones launch directly (the
 * environment variable NS_GRAPHS=0 or 1, read here, forces either form).
 * Five more kernel-path choices are made by size and can be forced here
 * the same way (each computes the same sums; used to test every path on small
 * meshes): NS_XCD_ROWS=0/1, block-SpMV rows mapped to one contiguous range
 * per XCD (default: when the gathered vector is <= 8 MB);
 * NS_PROLONG_PASS=0/1, the finest A level's coarse correction added by a
 * pass of its own instead of inside the first post-smoothing step (default:
 * from 5e5 rows); NS_ROW_UNROLL=2/4, the trip of the 4- and 8-lane row
 * walks of the sparse products, 16 or 32 entries per trip (default: 32 for
 * matrices whose mean row is longer than 16 entries); and NS_COL16=0, the
 * finest-level products reading the 32-bit column indices instead of 16-bit
 * offsets from the row (default: the offsets, whenever every node's
 * neighbours lie within 32767 of it in the numbering); and NS_ELL=0, the
 * FP32 tangent planes kept in the node graph's row layout instead of
 * fixed-width rows (default: fixed-width rows of the longest row's length,
 * padded with zero blocks, whenever the 16-bit offsets apply and no row is
 * longer than 16 blocks; the padding adds only exact zeros, so the results
 * are the same bit for bit).
 * Errors: NS_ERR_WORKSPACE, NS_ERR_HIP. */
ns_status ns_ctx_bind(ns_ctx* ctx, void* d_workspace, size_t bytes, hipStream_t stream);

void ns_ctx_destroy(ns_ctx* ctx);
const char* ns_last_error(const ns_ctx* ctx);

/* ns_outlet_flow: Q^k = int_{Gamma_out^k} v . n = a^k . v (Sec. 2.2 and
 * step 1 of the multi-corrector) for d_v [n_nodes][3]; writes h_Q
 * [n_outlets].  Waits for the stream. */
ns_status ns_outlet_flow(ns_ctx* ctx, const double* d_v, double* h_Q, hipStream_t stream);

/* ns_rank_one_dots: out[k] = a^k . x_v with the Dirichlet entries of a^k
 * zeroed (the vectors of the rank-one term K, Sec. 2.5) for d_xv
 * [n_nodes][3] (the velocity part of a field-split vector); writes h_out
 * [n_outlets].  Used to contract outlet-resistance derivatives.  Waits for
 * the stream. */
ns_status ns_rank_one_dots(ns_ctx* ctx, const double* d_xv, double* h_out, hipStream_t stream);

/* ns_resistance_gradient: derivative of a loss L(x) of the last solve's
 * solution with respect to the outlet resistances, for a tangent assembled
 * with resistance outlets (ns_phys.h_R).  x(R) = A(R)^{-1} r(R) at the frozen
 * state: R^k enters the tangent through K (dA/dR_k = blockdiag(c_f a^k a^k^T,
 * 0), c_f = alpha_f gamma dt, Sec. 2.5) and the right-hand side through the
 * traction pressure (dr/dR_k = -[alpha_f Q^k a^k; 0], P^k_n held fixed), so
 * with lambda solving A^T lambda = dL/dx (ns_adjoint_solve)
 *     dL/dR_k = lambda^T (dr/dR_k - (dA/dR_k) x)
 *             = -(a^k . lambda_v) (alpha_f Q^k + c_f a^k . x_v),
 * a^k with its Dirichlet entries zeroed.  The dots and the contraction run on
 * the device.
 *   d_lambda  [4 n_nodes] adjoint solution, d_x [4 n_nodes] the solve's x
 *   h_grad    [n_outlets] out: dL/dR_k
 * Waits for the stream.  Errors: NS_ERR_STATE when the last assembly did not
 * take resistance outlets. */
ns_status ns_resistance_gradient(ns_ctx* ctx, const double* d_lambda, const double* d_x, double* h_grad,
                                 hipStream_t stream);

/* ns_resistance_gradient_noalloc: for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): ns_resistance_gradient with its scratch (the two per-outlet dot
 * products) in a file-scope device array of the library instead of the
 * context's workspace, and its result written to device memory:
 *   d_grad  [n_outlets] out (device): dL/dR_k
 * Enqueues three kernels on `stream` and returns: no allocation, no copy, no
 * synchronisation.  At most 4096 outlets (the array holds 2 x 4096 doubles per
 * device, kept until the process ends).  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other
 * contexts, other host threads) race; calls on one stream are ordered.  The
 * context's device must be current.  Errors: NS_ERR_ARG (null pointers, more
 * than 4096 outlets), NS_ERR_STATE (as ns_resistance_gradient; another device
 * current), NS_ERR_HIP. */
ns_status ns_resistance_gradient_noalloc(ns_ctx* ctx, const double* d_lambda, const double* d_x, double* d_grad,
                                         hipStream_t stream);

/* ns_gen_alpha: the generalized-alpha parameters of Sec. 2.4.1 for the
 * spectral radius rho_inf in [0, 1]: h_out3 = {alpha_m, alpha_f, gamma},
 * alpha_m = (3 - rho_inf) / (2 (1 + rho_inf)), alpha_f = gamma = 1 / (1 + rho_inf).
 * Host-only.  Errors: NS_ERR_ARG for rho_inf outside [0, 1]. */
ns_status ns_gen_alpha(double rho_inf, double* h_out3);

/* ns_assemble_tangent: residual and consistent tangent of one Newton step
 * (Sec. 2.5, steps 6 and 8; forms of Sec. 2.3) at the intermediate states
 *   d_v_af    [n_nodes][3] velocity y_{n+af} (Dirichlet values imposed)
 *   d_p_af    [n_nodes]    pressure at n+af
 *   d_vdot_am [n_nodes][3] acceleration at n+am
 * Writes d_rhs [4 n_nodes] = -[R_m; R_p] (field-split), zero at Dirichlet
 * entries, and keeps the eliminated blocks A (without K), B, C, D in the
 * workspace.  Quadrature: 4-point rule on tetrahedra, 3-point rule on outlet
 * triangles; tau_M, tau_C held fixed in the derivative; Dirichlet rows and
 * columns replaced by the identity.  Colour-by-colour, no atomics.
 * Asynchronous on `stream`. */
ns_status ns_assemble_tangent(ns_ctx* ctx, const ns_phys* phys, const double* d_v_af,
                              const double* d_p_af, const double* d_vdot_am, double* d_rhs,
                              hipStream_t stream);

/* ns_nested_solve: solve [A B; C D] x = rhs for the last assembled tangent
 * with FGMRES + P_SCR (Algorithms 2 and 3).  d_rhs, d_x: [4 n_nodes] FP64.
 * The per-step set-up (diag(A), S_hat, AMG numeric) runs first when the
 * tangent changed since the previous solve.  In NS_FP32_INNER mode P_SCR runs
 * in FP32 (inner Krylov vectors, SpMV, V-cycles, dot products) while the
 * outer FGMRES, the Hessenberg least squares, the true residual and the AMG
 * coarsest solve stay in FP64.  h_stats may be NULL.
 * Errors: NS_ERR_STATE (no tangent assembled), NS_ERR_NAN, NS_ERR_BREAKDOWN,
 * NS_ERR_HIP, NS_ERR_ARG (options beyond the context's Krylov sizes). */
ns_status ns_nested_solve(ns_ctx* ctx, const ns_solve_opts* opts, const double* d_rhs,
                          double* d_x, ns_stats* h_stats, hipStream_t stream);

/* ns_adjoint_solve: solve the transposed system [A^T C^T; B^T D^T] lam = g
 * with the same nested method on the transposed blocks (B' = C^T,
 * C' = B^T, S_hat' = S_hat^T; K is symmetric).  Same conventions and errors
 * as ns_nested_solve. */
ns_status ns_adjoint_solve(ns_ctx* ctx, const ns_solve_opts* opts, const double* d_g,
                           double* d_lambda, ns_stats* h_stats, hipStream_t stream);

/* Reduced model of every outlet (Sec. 2.3): the three-element Windkessel
 *   dPi/dt = -Pi / (R_d C) + Q / C,   P = R_p Q + Pi + P_d,
 * integrated over (t_n, t_{n+1}) with n_ts steps of the fourth-order
 * Runge-Kutta scheme of Algorithm 1 (flow rate interpolated linearly between
 * Q_n and Q_{n+1}).  C = 0 selects the resistance model P = (R_p + R_d) Q + P_d.
 * Host arrays of n_outlets entries; h_Pi, h_P, h_Q are read as the values at
 * t_n and overwritten with those at t_{n+1} by ns_time_step. */
typedef struct {
    const double* h_Rp;     /* proximal resistance                        */
    const double* h_C;      /* compliance (0: resistance outlet)          */
    const double* h_Rd;     /* distal resistance                          */
    const double* h_Pd;     /* distal pressure at t_{n+1}                 */
    double* h_Pi;           /* Pi^k: in t_n, out t_{n+1}                  */
    double* h_P;            /* P^k:  in t_n, out t_{n+1}                  */
    double* h_Q;            /* Q^k:  in t_n, out t_{n+1}                  */
    int32_t n_ts;           /* Runge-Kutta steps per time step        [100] */
    int32_t reserved;
} ns_outlet_model;

/* Options of the predictor multi-corrector stage (Sec. 2.5).  0 = default. */
typedef struct {
    double tol_R;           /* relative residual tolerance            [1e-6] */
    double tol_A;           /* absolute residual tolerance            [1e-6] */
    double eps_abs;         /* difference-quotient step for m^k       [1e-8] */
    double eps_rel;         /*   eps = max(eps_abs, eps_rel |Q^k|)    [1e-5] */
    int32_t l_max;          /* maximum corrector iterations           [20]   */
    int32_t reserved;
} ns_newton_opts;

/* Per-time-step statistics. */
typedef struct {
    int32_t iterations;     /* corrector iterations that solved a linear system */
    int32_t converged;      /* 1 if a stopping criterion was met               */
    double res0;            /* ||R_(1)||, the first residual                   */
    double res;             /* ||R|| at the accepted iterate                   */
    double res_hist[32];    /* ||R_(l)|| for l = 1 .. min(iterations + 1, 32)  */
    int32_t lin_outer, lin_a, lin_s, lin_inner;  /* summed Krylov iterations  */
    double assemble_ms, solve_ms, total_ms;
} ns_step_stats;

/* ns_time_step: one time step t_n -> t_{n+1} by the predictor
 * multi-corrector algorithm of Sec. 2.5.  Predictor y = y_n,
 * ydot = (gamma - 1)/gamma ydot_n; then for l = 1 .. l_max: outlet flows
 * Q^k of the current iterate, P^k_{n+1} from the reduced model and m^k from
 * its central difference quotient; the state at n+af / n+am and
 * P^k_{n+af} = (1 - af) P^k_n + af P^k_{n+1}; assembly; stop when
 * ||R_(l)|| <= tol_R ||R_(1)|| or ||R_(l)|| <= tol_A (the l2 norm of the
 * assembled residual, Dirichlet entries excluded); else solve the tangent
 * system with ns_nested_solve options `solve` and apply the update of step 10.
 * At most l_max systems are solved; the residual of the returned iterate is
 * always assembled and tested (after the l_max-th update too), and
 * NS_NOT_CONVERGED is returned when it misses both tolerances.
 *   phys       rho, mu, dt, rho_inf, beta_bf, c_t, c_i (the outlet fields are
 *              unused: the reduced models give m^k and P^k_{n+af})
 *   d_y_n, d_ydot_n   [4 n_nodes] field-split state at t_n (Dirichlet values
 *                     imposed in d_y_n)
 *   d_y, d_ydot       [4 n_nodes] out: state at t_{n+1} (may not alias inputs)
 * The assembled tangent of the last corrector stays in the workspace.
 * Errors: as ns_assemble_tangent and ns_nested_solve; NS_NOT_CONVERGED when
 * l_max iterations did not meet a tolerance (outputs hold the last iterate). */
ns_status ns_time_step(ns_ctx* ctx, const ns_phys* phys, ns_outlet_model* model,
                       const ns_newton_opts* newton, const ns_solve_opts* solve,
                       const double* d_y_n, const double* d_ydot_n, double* d_y, double* d_ydot,
                       ns_step_stats* h_stats, hipStream_t stream);

/* ns_newton_update: the update of step 10 of the multi-corrector (Sec. 2.5):
 * y += gamma dt dy_dot, y_dot += dy_dot, on d_y, d_ydot [4 n_nodes]
 * (field-split) with d_dx [4 n_nodes]; FP64.  Asynchronous. */
ns_status ns_newton_update(ns_ctx* ctx, double gamma_dt, const double* d_dx, double* d_y,
                           double* d_ydot, hipStream_t stream);

/* ---- kernel timing ----------------------------------------------------------
 * Kernel classes that can be timed with HIP events on the solve's stream:
 *   NS_KT_SPMV_A    the finest-level 3x3 block SpMV of A: the A operator
 *                   (F x + rank-one epilogue) and the V-cycle residual
 *   NS_KT_CHEB_A0   the fused residual + Chebyshev step on the finest level of
 *                   the A hierarchy
 *   NS_KT_SPMV_FULL the 4x4 field-split SpMV of the outer FGMRES
 *   NS_KT_SFACT     the factored S_hat = D - C diag(A)^-1 B on the finest
 *                   S_hat level (two launches timed as one: the B pass and the
 *                   D, C pass with the smoothing or residual epilogue)
 *   NS_KT_CGS2      one CGS2 orthogonalisation step, any Krylov level (four
 *                   launches timed as one; bytes with k = j + 1 basis vectors
 *                   of length n: (4k + 8) n values, (3k + 7) n for k <= 16,
 *                   where the pass-1 update and pass-2 dots read V once)
 *   NS_KT_CHEB_S1   a Chebyshev step on level 1 of the S_hat hierarchy
 * ns_kernel_timing(ctx, mask) enables timing of the classes in `mask` (bit
 * 1 << class) for later solves (0 disables); every timed launch is bracketed
 * by two events from a pool of 65536 pairs per solve (launches beyond it are not
 * timed).  ns_kernel_timing_read(ctx, class, out3) returns and clears
 * out3 = {launches, total milliseconds, algorithmic bytes moved}; the bytes
 * count one read of the matrix values, column indices and row pointers, one
 * read of every input vector entry and one write of every output entry. */
typedef enum {
    NS_KT_SPMV_A = 0, NS_KT_CHEB_A0 = 1, NS_KT_SPMV_FULL = 2, NS_KT_SFACT = 3, NS_KT_CGS2 = 4, NS_KT_CHEB_S1 = 5,
    NS_KT_COUNT = 6
} ns_kernel_class;
ns_status ns_kernel_timing(ns_ctx* ctx, int32_t mask);
/* ns_kernel_timing_period(ctx, period): bracket only every period-th launch
 * of each timed class (1, the default: every launch), counting from this
 * call; the launches in between run without events, so a long solve is
 * timed on a sample with a period-th of the events' own cost.  The totals
 * read back are those of the sampled launches (their count, time and bytes).
 * Errors: NS_ERR_ARG for period < 1. */
ns_status ns_kernel_timing_period(ns_ctx* ctx, int32_t period);
ns_status ns_kernel_timing_read(ns_ctx* ctx, int32_t kclass, double* h_out3);

/* ns_stream_bench: the streaming ceiling of the device, for comparing the
 * solver's bandwidth-bound kernels with a measured peak beside the nominal
 * one.  mode 0 reads `bytes` from d_src (16-byte loads; the first 4 KiB of
 * d_dst may be written), mode 1 copies `bytes` from d_src to d_dst.  Both
 * buffers hold at least `bytes` (>= 4 KiB in mode 0), 16-byte aligned, and do
 * not overlap; bytes is a multiple of 16.  One untimed launch, then `reps`
 * launches timed with HIP events on a stream of its own; writes the average
 * milliseconds per launch to *h_ms.  Waits for completion; uses the current
 * device.  Errors: NS_ERR_ARG, NS_ERR_HIP. */
ns_status ns_stream_bench(int32_t mode, const void* d_src, void* d_dst, size_t bytes, int32_t reps, double* h_ms);

/* ---- inspection entry points (used by the tests) -------------------------- */

/* Sizes: [0] n_nodes, [1] nnzb, [2] nnz of S_hat, [3] colours, [4] outlet
 * nodes, [5] AMG levels (including the coarsest). */
ns_status ns_query(const ns_ctx* ctx, int64_t* h_sizes6);

/* Layout of the finest-level matrix data: [0] the width of the fixed-width
 * rows the FP32 planes may take (the longest row, when no row is longer than
 * 16 blocks and the 16-bit offsets apply; 0 otherwise), [1] 1 when every
 * column lies within 32767 of its row (16-bit offsets available); both known
 * from ns_ctx_create on.  [2] and [3]: 1 when the bound context uses the
 * fixed-width FP32 rows and the 16-bit offsets (ns_ctx_bind may switch either
 * off: NS_ELL=0, NS_COL16=0); 0 before the first bind.  Host only. */
ns_status ns_query_layout(const ns_ctx* ctx, int32_t* h_out4);

/* Node-graph pattern: h_row_ptr [n_nodes + 1], h_col [nnzb] (sorted). */
ns_status ns_export_pattern(const ns_ctx* ctx, int32_t* h_row_ptr, int32_t* h_col);

/* Column offsets of the fixed-width rows (width w = ns_query_layout()[0]):
 * h_dcol [n_nodes * w], slot l of row i at i*w + l holding col - i, 0 past
 * the row's end.  NS_ERR_ARG when the pattern has no fixed-width rows.
 * Host only. */
ns_status ns_export_fixed_width_offsets(const ns_ctx* ctx, int16_t* h_dcol);

/* Aggregate map of AMG level `level` (fine node -> coarse node), [nodes of
 * that level]. */
ns_status ns_export_aggregates(const ns_ctx* ctx, int32_t level, int32_t* h_agg);

/* Element colours h_color [n_elems]. */
ns_status ns_export_colors(const ns_ctx* ctx, int32_t* h_color);

/* Assembled blocks, d_dst [nnzb][4][4] row-major (rows: u, v, w, continuity;
 * columns: u, v, w, p) of the tangent (transposed = 0) or of its transpose
 * (transposed = 1, available after ns_adjoint_solve).  Synchronous. */
ns_status ns_export_bsr(ns_ctx* ctx, int32_t transposed, double* d_dst, hipStream_t stream);

/* S_hat values on its pattern: h_row_ptr [n+1], h_col [nnz], d_val [nnz]
 * (FP64, from the last set-up of the forward system).  Synchronous. */
ns_status ns_export_shat(ns_ctx* ctx, int32_t* h_row_ptr, int32_t* h_col, double* d_val,
                         hipStream_t stream);

/* Outlet vectors with the Dirichlet entries zeroed, d_a [n_outlets][n_nodes][3].
 * Synchronous. */
ns_status ns_export_outlet_vectors(ns_ctx* ctx, double* d_a, hipStream_t stream);

typedef enum {
    NS_OP_FULL = 0,   /* y = [A B; C D] x  (A = F + K), x, y: [4N]        */
    NS_OP_A = 1,      /* y = (F + K) x,                 x, y: [3N]        */
    NS_OP_B = 2,      /* y = B x,                       x: [N],  y: [3N]  */
    NS_OP_C = 3,      /* y = C x,                       x: [3N], y: [N]   */
    NS_OP_D = 4,      /* y = D x,                       x, y: [N]         */
    NS_OP_SHAT = 5,   /* y = S_hat x,                   x, y: [N]         */
    NS_OP_VCYCLE_A = 6, /* y = one AMG V-cycle of the A hierarchy on x [3N] */
    NS_OP_VCYCLE_S = 7, /* y = one AMG V-cycle of the S_hat hierarchy [N]  */
    NS_OP_SCHUR = 8,  /* y = Algorithm 2 applied to x [N] (inner rtol_I)  */
    NS_OP_PSCR = 9,   /* y = Algorithm 3 applied to x [4N]                */
    NS_OP_SOLVE_A = 10, /* y = GMRES(m_A) solution of A y = x to rtol_A   */
    NS_OP_PSIMPLE = 11  /* y = P_SIMPLE^-1 x (Sec. 3.2), x, y: [4N]        */
} ns_op;

/* ns_apply: one operator of the forward system, after the per-step set-up
 * (which it runs if needed).  d_x, d_y: FP64 device vectors; with precision
 * NS_FP32_INNER the operator runs in FP32 on rounded inputs.  opts may be
 * NULL for the plain operators (0-5).  Synchronous. */
ns_status ns_apply(ns_ctx* ctx, int32_t op, const ns_solve_opts* opts, const double* d_x,
                   double* d_y, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* NS_API_H */
