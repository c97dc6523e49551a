"""Aggregation AMG V-cycle used as P_A and P_S, FP64, plain CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper preconditions A and the sparse Schur approximation S_hat with AMG
V-cycles (Sec. 3.1, with BoomerAMG settings in the AMG settings table).  That
package choice is prior art here; this module follows the repository's own
written definition, which the GPU library implements independently:

* node graph: i ~ j when i and j share a tetrahedron edge;
* one coarsening level = composed greedy pairwise matchings: visit nodes in
  ascending order; an unmatched node is paired with its first (lowest index)
  unmatched neighbour, or left single; coarse ids are handed out in the order
  the pairs/singles are created; each further matching runs on the quotient
  graph of the previous one; two matchings from the finest level, three
  (``coarse_matchings``) on every coarser one (aggregates of at most 4, then
  8 nodes: fewer levels, each a latency-bound launch on the GPU, at the same
  or lower iteration counts); levels are added while the level has more than
  ``coarse_nodes`` nodes (and coarsening still reduces the count), up to
  ``max_levels`` levels;
* unsmoothed (piecewise-constant) prolongation, nodal for A (3x3 blocks, the
  three velocity components kept apart) and scalar for S_hat, with the same
  node aggregates; coarse operators are Galerkin products P^T M P;
* smoother: Chebyshev polynomial of degree ``cheb_degree`` (default 2; degree
  1 is damped point Jacobi with weight 1/theta) in D^{-1} M (D the point diagonal)
  on [lambda/cheb_ratio, lambda] (cheb_ratio default 10); lambda must bound the spectral radius of D^{-1} M
  from above, else the smoother amplifies the top modes.  It is the smaller of
  the Gershgorin bound max_i sum_j |M_ij / D_ii| (a guaranteed bound) and
  1.2 x the estimate from 20 power iterations on D^{-1} M from the start
  vector x_i = 0.5 + ((i * 2654435761) mod 2^32)/2^32 (power iteration
  approaches the spectral radius from below); one pre- and one
  post-smoothing application (zero initial guess before pre-smoothing);
* coarse-grid correction scaled by ``cc_scale`` (default 1): x += c P e_c at
  every level, where e_c is the coarse level's cycle applied to P^T r.  The
  piecewise-constant prolongation represents a smooth error only by its
  aggregate means, so the Galerkin correction (the M-orthogonal projection on
  range(P)) falls short of the smooth error; an over-correction c in (1, 2)
  compensates.  The cycle stays a fixed linear operator for any c;
* cycle index ``cycle_index`` (default 1, the V-cycle): on every level below
  the finest, the coarse-grid correction and the post-smoothing are applied
  that many times in turn (2: a W-cycle); the finest level takes one;
* coarsest level: dense LU solve in FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def node_adjacency(n: int, tets: np.ndarray):
    """Sorted neighbour lists (self excluded) of the P1 node graph."""
    e = np.concatenate([tets[:, [i, j]] for i in range(4) for j in range(4) if i != j])
    g = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    g.sum_duplicates()
    g.sort_indices()
    return [g.indices[g.indptr[i]:g.indptr[i + 1]].copy() for i in range(n)]


def greedy_matching(adj):
    """Pairwise matching in ascending node order (see module docstring)."""
    n = len(adj)
    agg = np.full(n, -1, dtype=np.int64)
    nc = 0
    for i in range(n):
        if agg[i] != -1:
            continue
        agg[i] = nc
        for j in adj[i]:
            if j != i and agg[j] == -1:
                agg[j] = nc
                break
        nc += 1
    return agg, nc


def quotient(adj, agg, nc):
    """Coarse adjacency: I ~ J (I != J) when some i in I, j in J are adjacent."""
    sets = [set() for _ in range(nc)]
    for i, nb in enumerate(adj):
        I = agg[i]
        for j in nb:
            J = agg[j]
            if J != I:
                sets[I].add(J)
    return [np.array(sorted(s), dtype=np.int64) for s in sets]


def build_aggregates(adj, coarse_nodes: int = 128, max_levels: int = 16, coarse_matchings: int = 3):
    """List of fine->coarse maps, one per coarsening level.  Each step
    composes greedy pairwise matchings (each on the quotient graph of the
    previous one): two on the finest level, ``coarse_matchings`` below it."""
    aggs = []
    cur = adj
    while len(cur) > coarse_nodes and len(aggs) + 1 < max_levels:
        k = 2 if not aggs else coarse_matchings
        agg = np.arange(len(cur))
        g = cur
        n2 = len(cur)
        for m in range(k):
            am, n2 = greedy_matching(g)
            agg = am[agg]
            if m + 1 < k:
                g = quotient(g, am, n2)
        if n2 >= len(cur):
            break
        aggs.append(agg)
        cur = quotient(cur, agg, n2)
    return aggs


def power_start(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.uint64)
    return 0.5 + ((i * np.uint64(2654435761)) % np.uint64(2 ** 32)).astype(np.float64) / 2.0 ** 32


def lambda_max(M: sp.csr_matrix, dinv: np.ndarray, iters: int = 10) -> float:
    """Largest eigenvalue magnitude estimate of D^{-1} M: 10 power iterations
    from the fixed start vector; returns ||D^{-1} M x|| of the last step."""
    x = power_start(M.shape[0])
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = dinv * (M @ x)
        lam = np.linalg.norm(y)
        x = y / lam
    return lam


def gershgorin_bound(M: sp.csr_matrix, dinv: np.ndarray) -> float:
    """max_i sum_j |dinv_i M_ij|: every eigenvalue of D^{-1} M lies in a
    Gershgorin disc of a row, so its modulus is at most this."""
    return float(np.max(np.abs(sp.diags(dinv) @ M).sum(axis=1)))


def smoother_bound(M: sp.csr_matrix, dinv: np.ndarray) -> float:
    """Upper end of the smoother interval (module docstring)."""
    return min(gershgorin_bound(M, dinv), 1.2 * lambda_max(M, dinv, 20))


def chebyshev(M, dinv, b, x, degree, lmin, lmax):
    """Chebyshev iteration of the given degree for M x = b, preconditioned by
    D^{-1}, with eigenvalue interval [lmin, lmax] of D^{-1} M."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b - M @ x if x is not None else b.copy()
    x = np.zeros_like(b) if x is None else x.copy()
    d = dinv * r / theta
    x = x + d
    for _ in range(1, degree):
        rho_new = 1.0 / (2.0 * sigma - rho)
        r = b - M @ x
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        x = x + d
        rho = rho_new
    return x


class AMG:
    """V-cycle for M (scipy CSR) with block size ``bs`` on the node aggregates."""

    def __init__(self, M, bs: int, aggs, cheb_degree: int = 2, extra_diag=None, cheb_ratio: float = 10.0,
                 cc_scale: float = 1.0, cycle_index: int = 1):
        self.bs = bs
        self.deg = cheb_degree
        self.ratio = cheb_ratio
        self.cc_scale = cc_scale
        self.gamma = cycle_index
        M = sp.csr_matrix(M, dtype=np.float64)
        if extra_diag is not None:
            M = (M + sp.diags(extra_diag)).tocsr()
        self.M = [M]
        self.P = []
        for agg in aggs:
            nf = len(agg)
            nc = int(agg.max()) + 1
            Pn = sp.csr_matrix((np.ones(nf), (np.arange(nf), agg)), shape=(nf, nc))
            P = sp.kron(Pn, sp.identity(bs), format="csr") if bs > 1 else Pn
            self.P.append(P)
            self.M.append((P.T @ self.M[-1] @ P).tocsr())
        self.dinv = [1.0 / Ml.diagonal() for Ml in self.M[:-1]]
        self.lmax = [smoother_bound(Ml, di) for Ml, di in zip(self.M[:-1], self.dinv)]
        self.lu = sla.lu_factor(self.M[-1].toarray())

    @property
    def n_levels(self):
        return len(self.M)

    def vcycle(self, b, level: int = 0):
        if level == len(self.M) - 1:
            return sla.lu_solve(self.lu, b)
        M, dinv, lmax = self.M[level], self.dinv[level], self.lmax[level]
        x = chebyshev(M, dinv, b, None, self.deg, lmax / self.ratio, lmax)
        P = self.P[level]
        for _ in range(self.gamma if level > 0 else 1):
            r = b - M @ x
            x = x + self.cc_scale * (P @ self.vcycle(P.T @ r, level + 1))
            x = chebyshev(M, dinv, b, x, self.deg, lmax / self.ratio, lmax)
        return x
