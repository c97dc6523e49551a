"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test targets one part of the oracle so that a plausible mistake in it
(a dropped term, a wrong sign or index, a transposed operand) fails here:
closed forms of special states, exact quadrature, invariance of the metric
tensor, finite differences, dense linear algebra and brute force.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import get_assembled, get_case
from ns_inputs import meshes
from ns_inputs.cases import Case
from oracle import adjoint as adj_mod
from oracle import amg
from oracle import discretization as dz
from oracle import krylov as kr

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _box_case(n=3, v=None, p=None, vdot=None, lx=1.0):
    xyz, tets = meshes.kuhn_box(n, n, n, lx, 1.0, 1.0)
    N = len(xyz)
    z3 = np.zeros((N, 3))
    return Case("box", xyz, tets, np.zeros((N, 4), np.uint8), np.zeros(1, np.int32), np.zeros((0, 3), np.int32),
                z3 if v is None else v(xyz), np.zeros(N) if p is None else p(xyz),
                z3 if vdot is None else vdot(xyz), 1.0, 0.04, 1e-3, 0.5, np.zeros(0), {})


def _interior(xyz, lx=1.0):
    t = 1e-12
    return ~np.any((xyz < t) | (xyz > np.array([lx, 1.0, 1.0]) - t), axis=1)


def _grads(X):
    """Basis gradients of the linear tetrahedron with vertices X [4,3]
    (columns of the inverse of [[1, x, y, z]])."""
    Minv = np.linalg.inv(np.hstack([np.ones((4, 1)), X]))
    return Minv[1:, :].T, abs(np.linalg.det(np.hstack([np.ones((4, 1)), X]))) / 6.0


def _res(case, ph, tau_off=True):
    E = case.n_elems
    tau = (np.zeros((E, 4)), np.zeros((E, 4))) if tau_off else None
    return dz.residual_only(case, case.v, case.p, case.vdot, np.zeros(0), ph, tau_fixed=tau)


def _mass_apply(case, f):
    """Consistent P1 mass matrix (int N_a N_b = V (1 + delta_ab) / 20) times nodal f [N,3]."""
    out = np.zeros_like(f)
    for t in case.tets:
        _, V = _grads(case.xyz[t])
        for a in range(4):
            for b in range(4):
                out[t[a]] += V * (2.0 if a == b else 1.0) / 20.0 * f[t[b]]
    return out


# --------------------------------------------------------------------------- constants


def test_gen_alpha_constants():
    assert dz.gen_alpha(0.5) == pytest.approx((5.0 / 6.0, 2.0 / 3.0, 2.0 / 3.0), abs=1e-15)
    # rho_inf = 1 reduces the scheme to the mid-point rule
    assert dz.gen_alpha(1.0) == pytest.approx((0.5, 0.5, 0.5), abs=1e-15)
    assert dz.gen_alpha(0.0) == pytest.approx((1.5, 1.0, 1.0), abs=1e-15)


def test_tet_quadrature_exact_degree2():
    rng = np.random.default_rng(3)
    X = rng.random((4, 3))
    _, V = _grads(X)
    for a, b in itertools.product(range(4), range(4)):
        q = sum(V / 4 * dz.TET_QUAD[k, a] * dz.TET_QUAD[k, b] for k in range(4))
        assert q == pytest.approx(V * (1 + (a == b)) / 20.0, rel=1e-13)
    assert dz.TET_QUAD.sum(axis=1) == pytest.approx(np.ones(4), abs=1e-15)


def test_metric_G_permutation_invariant_only_with_M():
    rng = np.random.default_rng(7)
    X = rng.random((4, 3))
    tets = np.array([[0, 1, 2, 3]])
    _, _, G0 = dz.tet_geometry(X, tets)
    for perm in itertools.permutations(range(4)):
        _, _, Gp = dz.tet_geometry(X[list(perm)], tets)
        assert np.abs(Gp - G0).max() <= 1e-12 * np.abs(G0).max()
    # without the simplex matrix M the tensor depends on the vertex numbering
    J = lambda Y: np.linalg.inv(np.stack([Y[1] - Y[0], Y[2] - Y[0], Y[3] - Y[0]], 1))
    Y = X[[1, 0, 2, 3]]
    assert np.abs(J(X).T @ J(X) - J(Y).T @ J(Y)).max() > 1e-3


def test_tau_M_small_dt_limit():
    rng = np.random.default_rng(1)
    X = rng.random((4, 3))
    _, _, G = dz.tet_geometry(X, np.array([[0, 1, 2, 3]]))
    for dt in [1e-6, 1e-8]:
        ph = dz.Physics(1.3, 0.04, dt, 0.5)
        tM, tC = dz.tau_mc(G, rng.random((1, 4, 3)), ph)
        assert tM == pytest.approx(np.full((1, 4), dt / (2 * 1.3)), rel=1e-6)
        assert tC == pytest.approx(1.0 / (tM * np.trace(G[0])), rel=1e-14)


# --------------------------------------------------------------------------- residual special cases


def test_convection_term_closed_form():
    """mu = 0, tau off, v = (z, x, 0): R_m = rho M [(v.grad)v] with
    (v.grad)v = (0, z, 0) (the transposed form would give (x, 0, z))."""
    c = _box_case(3, v=lambda X: np.stack([X[:, 2], X[:, 0], 0 * X[:, 0]], 1))
    ph = dz.Physics(1.7, 0.0, 1e-3, 0.5)
    R = _res(c, ph)
    N = c.n_nodes
    expect = 1.7 * _mass_apply(c, np.stack([0 * c.xyz[:, 0], c.xyz[:, 2], 0 * c.xyz[:, 0]], 1))
    assert np.abs(R[:3 * N] - expect.ravel()).max() <= 1e-14
    assert np.abs(R[3 * N:]).max() <= 1e-15  # div v = 0


def test_mass_term_closed_form():
    c = _box_case(3, vdot=lambda X: np.stack([X[:, 0] + 2 * X[:, 1], -X[:, 2], 3.0 + 0 * X[:, 0]], 1))
    ph = dz.Physics(1.06, 0.0, 1e-3, 0.5)
    R = _res(c, ph)
    expect = 1.06 * _mass_apply(c, c.vdot)
    assert np.abs(R[:3 * c.n_nodes] - expect.ravel()).max() <= 1e-14


def test_viscous_term_rigid_rotation_and_shear():
    """2 mu eps(w):eps(v) vanishes element by element for a rigid rotation;
    a plain grad(w):grad(v) form would not."""
    om = np.array([0.3, -1.1, 0.7])
    c = _box_case(3, v=lambda X: np.cross(om, X))
    ph = dz.Physics(1e-30, 0.5, 1e-3, 0.5)
    R = _res(c, ph)
    assert np.abs(R).max() <= 1e-14
    # shear v = (y, 0, 0): per element mu V sum_l dN_a/dx_l (d_l v_i + d_i v_l)
    c2 = _box_case(2, v=lambda X: np.stack([X[:, 1], 0 * X[:, 0], 0 * X[:, 0]], 1))
    R2 = _res(c2, ph)
    expect = np.zeros((c2.n_nodes, 3))
    gv = np.zeros((3, 3))
    gv[0, 1] = 1.0  # d v_x / d y
    for t in c2.tets:
        g, V = _grads(c2.xyz[t])
        for a in range(4):
            expect[t[a]] += ph.mu * V * ((gv + gv.T) @ g[a])
    assert np.abs(R2[:3 * c2.n_nodes] - expect.ravel()).max() <= 1e-14


def test_pressure_and_reynolds_stress_terms():
    """v = 0, p linear, tau on: v' = -tau_M grad p, so per element
    R_m[a,i] = -V p(centroid) dN_a/dx_i - rho V tau_M^2 d_i p (grad p . grad N_a),
    R_p[a]   = V tau_M grad N_a . grad p,
    with tau_M = rho^-1 (C_T/dt^2 + C_I (mu/rho)^2 G:G)^(-1/2)."""
    gp = np.array([0.4, -1.2, 2.0])
    c = _box_case(2, p=lambda X: 1.5 + X @ gp)
    ph = dz.Physics(1.06, 0.04, 1e-3, 0.5)
    R = _res(c, ph, tau_off=False)
    N = c.n_nodes
    Rm = np.zeros((N, 3))
    Rp = np.zeros(N)
    Mq = (2 ** (1 / 3) / 2) * np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]])
    for t in c.tets:
        X = c.xyz[t]
        g, V = _grads(X)
        Jinv = np.linalg.inv(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1))
        G = Jinv.T @ Mq @ Jinv
        tM = (1 / ph.rho) / np.sqrt(4.0 / ph.dt ** 2 + 36.0 * (ph.mu / ph.rho) ** 2 * np.sum(G * G))
        pc = c.p[t].mean()
        for a in range(4):
            Rm[t[a]] += -V * pc * g[a] - ph.rho * V * tM ** 2 * gp * (gp @ g[a])
            Rp[t[a]] += V * tM * (g[a] @ gp)
    assert np.abs(R[:3 * N] - Rm.ravel()).max() <= 1e-13 * np.abs(Rm).max()
    assert np.abs(R[3 * N:] - Rp).max() <= 1e-13 * np.abs(Rp).max()


def _tau_M_closed(X, ph, U=np.zeros(3)):
    """tau_M of one element for a velocity U that is uniform over it (Sec. 2.3):
    rho^-1 (C_T/dt^2 + U.G.U + C_I (mu/rho)^2 G:G)^(-1/2), G from the simplex matrix."""
    Mq = (2 ** (1 / 3) / 2) * np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]])
    Jinv = np.linalg.inv(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1))
    G = Jinv.T @ Mq @ Jinv
    return (1 / ph.rho) / np.sqrt(4.0 / ph.dt ** 2 + U @ G @ U + 36.0 * (ph.mu / ph.rho) ** 2 * np.sum(G * G))


def test_supg_term_uniform_velocity():
    """SUPG term of B_m^vol: v = U uniform, p linear, vdot = 0, tau on.  Then
    grad v = 0, r_M = grad p and v' = -tau_M grad p (tau_M constant per element,
    with the U.G.U term), so per element
      R_m[a,i] = -V p(centroid) dN_a/dx_i + rho V tau_M d_i p (U . grad N_a)
                 - rho V tau_M^2 d_i p (grad p . grad N_a),
      R_p[a]   = V tau_M grad N_a . grad p.
    The second term is -rho v'_i (v.grad N_a); its sign, and the v.grad N_a
    contraction, are what this pins (the cross-stress term is zero here)."""
    U = np.array([0.8, -0.5, 1.3])
    gp = np.array([0.4, -1.2, 2.0])
    c = _box_case(2, v=lambda X: np.broadcast_to(U, X.shape).copy(), p=lambda X: 0.2 + X @ gp)
    ph = dz.Physics(1.06, 0.004, 0.5, 0.5)  # a long step: tau_M ~ h / |U|, so the SUPG term is O(1)
    R = _res(c, ph, tau_off=False)
    N = c.n_nodes
    Rm = np.zeros((N, 3))
    Rp = np.zeros(N)
    supg = np.zeros((N, 3))
    for t in c.tets:
        X = c.xyz[t]
        g, V = _grads(X)
        tM = _tau_M_closed(X, ph, U)
        pc = c.p[t].mean()
        for a in range(4):
            s = ph.rho * V * tM * gp * (U @ g[a])
            supg[t[a]] += s
            Rm[t[a]] += -V * pc * g[a] + s - ph.rho * V * tM ** 2 * gp * (gp @ g[a])
            Rp[t[a]] += V * tM * (g[a] @ gp)
    # the SUPG contribution is a sizeable part of the row, so a flipped or dropped term shows
    assert np.abs(supg).max() > 0.05 * np.abs(Rm).max()
    assert np.abs(R[:3 * N] - Rm.ravel()).max() <= 1e-13 * np.abs(Rm).max()
    assert np.abs(R[3 * N:] - Rp).max() <= 1e-13 * np.abs(Rp).max()


def test_cross_stress_term_shear_flow():
    """Cross-stress term of B_m^vol: the shear v = (y, 0, 0), p linear, vdot = 0,
    with tau_M = t and tau_C held fixed (the frozen-tau residual).  Then
    (v.grad)v = 0, div v = 0, r_M = grad p, v' = -t grad p, and
    (v'.grad)v_i = v'_y delta_ix, so with the exact integrals int N_a = V/4 and
    int y = V y_c (centroid) per element
      R_m[a,i] = -V p_c d_iN_a + mu V (d_yN_a delta_ix + d_xN_a delta_iy)
                 + rho t V y_c d_i p d_xN_a          (SUPG,  -rho v'_i (v.grad N_a))
                 - rho t (V/4) d_y p delta_ix        (cross, +rho N_a (v'.grad) v_i)
                 - rho t^2 V d_i p (grad p . grad N_a)  (Reynolds stress),
      R_p[a]   = V t grad N_a . grad p.
    A transposed cross term (v'_l d_i v_l) would put -rho t (V/4) d_x p in the
    y rows instead."""
    gp = np.array([0.7, -1.1, 0.5])
    c = _box_case(2, v=lambda X: np.stack([X[:, 1], 0 * X[:, 0], 0 * X[:, 0]], 1), p=lambda X: -0.3 + X @ gp)
    ph = dz.Physics(1.3, 0.02, 1e-3, 0.5)
    E, N = c.n_elems, c.n_nodes
    t = 0.37
    R = dz.residual_only(c, c.v, c.p, c.vdot, np.zeros(0), ph, tau_fixed=(np.full((E, 4), t), np.full((E, 4), 2.9)))
    Rm = np.zeros((N, 3))
    Rp = np.zeros(N)
    cross = np.zeros((N, 3))
    ex, ey = np.eye(3)[0], np.eye(3)[1]
    for tt in c.tets:
        X = c.xyz[tt]
        g, V = _grads(X)
        pc = c.p[tt].mean()
        yc = X[:, 1].mean()
        for a in range(4):
            cr = -ph.rho * t * (V / 4) * gp[1] * ex
            cross[tt[a]] += cr
            Rm[tt[a]] += (-V * pc * g[a] + ph.mu * V * (g[a][1] * ex + g[a][0] * ey)
                          + ph.rho * t * V * yc * gp * g[a][0] + cr - ph.rho * t ** 2 * V * gp * (gp @ g[a]))
            Rp[tt[a]] += V * t * (g[a] @ gp)
    assert np.abs(cross).max() > 0.05 * np.abs(Rm).max()
    assert np.abs(R[:3 * N] - Rm.ravel()).max() <= 1e-13 * np.abs(Rm).max()
    assert np.abs(R[3 * N:] - Rp).max() <= 1e-13 * np.abs(Rp).max()


def test_grad_div_term_tau_C():
    """rho -> 0, mu > 0, v = (x, 0, 0): v' -> 0 and p' = -tau_C div v with
    tau_C = 1/(tau_M tr G), tau_M -> 1/(mu sqrt(C_I G:G))."""
    c = _box_case(2, v=lambda X: np.stack([X[:, 0], 0 * X[:, 0], 0 * X[:, 0]], 1))
    ph = dz.Physics(1e-30, 0.3, 1e-3, 0.5)
    R = _res(c, ph, tau_off=False)
    N = c.n_nodes
    Rm = np.zeros((N, 3))
    Mq = (2 ** (1 / 3) / 2) * np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]])
    gv = np.zeros((3, 3))
    gv[0, 0] = 1.0
    for t in c.tets:
        X = c.xyz[t]
        g, V = _grads(X)
        Jinv = np.linalg.inv(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1))
        G = Jinv.T @ Mq @ Jinv
        tC = ph.mu * np.sqrt(36.0 * np.sum(G * G)) / np.trace(G)
        for a in range(4):
            Rm[t[a]] += V * (tC * 1.0 * g[a] + ph.mu * (g[a] @ (gv + gv.T).T))
    assert np.abs(R[:3 * N] - Rm.ravel()).max() <= 1e-10 * np.abs(Rm).max()


def test_couette_full_vms_residual_vanishes():
    """v = (U z, 0, 0), p = const, a = 0 solves the steady NS equations with
    r_M = 0, so v' = p' = 0 and the full VMS residual is zero at interior rows."""
    c = _box_case(4, v=lambda X: np.stack([2.5 * X[:, 2], 0 * X[:, 0], 0 * X[:, 0]], 1), p=lambda X: 3.0 + 0 * X[:, 0])
    ph = dz.Physics(1.0, 0.04, 1e-3, 0.5)
    R = _res(c, ph, tau_off=False)
    N = c.n_nodes
    it = _interior(c.xyz)
    Rm = R[:3 * N].reshape(N, 3)
    assert np.abs(Rm[it]).max() <= 1e-15
    assert np.abs(R[3 * N:]).max() <= 1e-15
    # a non-solution (U z^2 profile) leaves a visible residual
    c.v[:, 0] = 2.5 * c.xyz[:, 2] ** 2
    assert np.abs(_res(c, ph, tau_off=False)[:3 * N].reshape(N, 3)[it]).max() > 1e-4


def test_plane_poiseuille_galerkin_residual_vanishes():
    """tau off: v = (4U z(1-z), 0, 0), p = -8 mu U x on the Kuhn lattice."""
    U, mu = 1.3, 0.04
    c = _box_case(4, v=lambda X: np.stack([4 * U * X[:, 2] * (1 - X[:, 2]), 0 * X[:, 0], 0 * X[:, 0]], 1),
                  p=lambda X: -8 * mu * U * X[:, 0] + 0.7)
    ph = dz.Physics(1.0, mu, 1e-3, 0.5)
    R = _res(c, ph, tau_off=True)
    N = c.n_nodes
    it = _interior(c.xyz)
    assert np.abs(R[:3 * N].reshape(N, 3)[it]).max() <= 1e-15
    # a wrong pressure gradient (sign flipped) does not
    c.p[:] = 8 * mu * U * c.xyz[:, 0]
    assert np.abs(_res(c, ph)[:3 * N].reshape(N, 3)[it]).max() > 1e-3


def test_backflow_term_closed_form():
    """One outlet triangle with uniform inflow v = -s n: (v.n)_- = -s, so the
    face rows are rho beta s^2 (|f|/3) (-n) per node; outflow gives zero."""
    xyz = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0], [0.0, 0, -1]])
    tets = np.array([[0, 1, 2, 3]], np.int32)
    tets = meshes._orient(xyz, tets)
    faces = np.array([[0, 1, 2]], np.int32)  # normal +z: outward (tet lies below)
    for s, expect_zero in [(2.0, False), (-2.0, True)]:
        v = np.zeros((4, 3))
        v[:3] = -s * np.array([0, 0, 1.0])
        c = Case("f", xyz, tets, np.zeros((4, 4), np.uint8), np.array([0, 1], np.int32), faces, v, np.zeros(4),
                 np.zeros((4, 3)), 1.0, 0.0, 1e-3, 0.5, np.zeros(1), {})
        ph = dz.Physics(1.0, 0.0, 1e-3, 0.5)
        tau = (np.zeros((1, 4)), np.zeros((1, 4)))
        Rf = dz.residual_only(c, c.v, c.p, c.vdot, np.zeros(1), ph, tau_fixed=tau)
        Rv = dz.residual_only(c, c.v, c.p, c.vdot, np.zeros(1), ph, tau_fixed=tau) * 0
        c0 = Case("f", xyz, tets, c.mask, np.array([0], np.int32), np.zeros((0, 3), np.int32), v, np.zeros(4),
                  np.zeros((4, 3)), 1.0, 0.0, 1e-3, 0.5, np.zeros(0), {})
        Rv = dz.residual_only(c0, c0.v, c0.p, c0.vdot, np.zeros(0), ph, tau_fixed=tau)
        face = (Rf - Rv)[:9].reshape(3, 3)
        if expect_zero:
            assert np.abs(face).max() == 0.0
        else:
            exp = 1.0 * 0.2 * s * s * (0.5 / 3) * np.array([0, 0, -1.0])
            assert np.abs(face - exp).max() <= 1e-15


def test_outlet_vectors_closed_form():
    c = get_case("pipe_tiny")
    a, w, area = dz.outlet_vectors(c)
    f = c.faces
    poly = 0.5 * np.abs(np.cross(c.xyz[f[:, 1]] - c.xyz[f[:, 0]], c.xyz[f[:, 2]] - c.xyz[f[:, 0]])[:, 2]).sum()
    assert area[0] == pytest.approx(poly, rel=1e-14)
    # planar outlet: sum_A a_A = |Gamma| n, n = +z
    assert a[0].sum(axis=0) == pytest.approx([0.0, 0.0, area[0]], abs=1e-14)
    assert w[0].sum() == pytest.approx(area[0], rel=1e-14)
    # flow rate of a linear axial profile v_z = 1 + x is exact: |Gamma| + int x
    X = c.xyz
    cx = sum((X[f[:, 0], 0] + X[f[:, 1], 0] + X[f[:, 2], 0]) / 3
             * 0.5 * np.abs(np.cross(X[f[:, 1]] - X[f[:, 0]], X[f[:, 2]] - X[f[:, 0]])[:, 2]))
    v = np.zeros_like(X)
    v[:, 2] = 1 + X[:, 0]
    assert np.sum(a[0] * v) == pytest.approx(area[0] + cx, rel=1e-13)


# --------------------------------------------------------------------------- tangent


@pytest.mark.parametrize("name", ["cube", "channel2", "unstr_channel"])
def test_tangent_matches_central_differences(name):
    c = get_case(name)
    S = get_assembled(name)
    ph = dz.physics_of(c)
    am, af, g = ph.alphas
    cf = af * g * ph.dt
    tau = dz.frozen_tau(c, c.v)
    N = c.n_nodes
    d = np.random.default_rng(0).standard_normal(4 * N)
    dm = np.concatenate([c.mask[:, :3].ravel(), c.mask[:, 3]]).astype(bool)
    d[dm] = 0
    P = c.R * S.Q

    def R(s):
        dv = (s * d[:3 * N]).reshape(N, 3)
        return dz.residual_only(c, c.v + cf * dv, c.p + cf * s * d[3 * N:], c.vdot + am * dv, P, tau_fixed=tau)

    h = 0.1
    fd = (R(h) - R(-h)) / (2 * h)
    # tangent without the rank-one term (the outlet pressure is held fixed here)
    Jd = np.concatenate([S.A_F @ d[:3 * N] + S.B @ d[3 * N:], S.C @ d[:3 * N] + S.D @ d[3 * N:]])
    fd[dm] = 0
    Jd[dm] = 0
    assert np.linalg.norm(fd - Jd) <= 1e-10 * np.linalg.norm(Jd)


def test_tangent_invariants():
    S = get_assembled("cube")
    assert abs(S.D - S.D.T).max() <= 1e-15 * abs(S.D).max()
    # Stokes limit (v = a = p = 0): A symmetric, C + B^T = c_m rho int tau_M N_b d_j N_a
    c = get_case("cube")
    c0 = Case(c.name, c.xyz, c.tets, np.zeros_like(c.mask), c.outlet_ptr, c.faces, np.zeros_like(c.v),
              np.zeros_like(c.p), np.zeros_like(c.v), c.rho, c.mu, c.dt, c.rho_inf, c.R, {})
    S0 = dz.assemble(c0)
    assert abs(S0.A_F - S0.A_F.T).max() <= 1e-14 * abs(S0.A_F).max()
    ph = dz.physics_of(c0)
    N = c0.n_nodes
    CB = (S0.C + S0.B.T).toarray()
    expect = np.zeros((N, 3 * N))
    vol, gN, G = dz.tet_geometry(c0.xyz, c0.tets)
    tM = (1 / ph.rho) / np.sqrt(4.0 / ph.dt ** 2 + 36 * (ph.mu / ph.rho) ** 2 * np.einsum("eij,eij->e", G, G))
    for e, t in enumerate(c0.tets):
        # int N_b = V/4 for each b
        for a in range(4):
            for b in range(4):
                expect[t[a], 3 * t[b]:3 * t[b] + 3] += ph.c_m * ph.rho * tM[e] * vol[e] / 4 * gN[e, a]
    assert np.abs(CB - expect).max() <= 1e-13 * np.abs(expect).max()


def test_rank_one_term():
    S = get_assembled("channel2")
    c = get_case("channel2")
    ph = dz.physics_of(c)
    K = sum(ck * np.outer(ak, ak) for ak, ck in zip(S.a, S.c))
    assert np.linalg.matrix_rank(K) == c.n_outlets
    assert np.allclose(K, K.T, rtol=0, atol=0)
    assert S.c == pytest.approx(ph.alphas[1] * ph.alphas[2] * ph.dt * c.R, rel=1e-15)


def test_dirichlet_elimination():
    S = get_assembled("cube")
    c = get_case("cube")
    dm = np.concatenate([c.mask[:, :3].ravel(), c.mask[:, 3]]).astype(bool)
    Ad = S.dense()
    assert np.all(Ad[dm][:, dm] == np.eye(int(dm.sum())))
    assert np.all(Ad[dm][:, ~dm] == 0) and np.all(Ad[~dm][:, dm] == 0)
    assert np.all(S.rhs[dm] == 0)


# --------------------------------------------------------------------------- preconditioner pieces


def test_schur_sparse_approximation_brute_force():
    S = get_assembled("channel2")
    ns = kr.NestedSolver(S, amg.node_adjacency(get_case("channel2").n_nodes, get_case("channel2").tets),
                         kr.SolveOpts())
    Bd, Cd, Dd = S.B.toarray(), S.C.toarray(), S.D.toarray()
    dA = np.diag(S.dense()[:3 * S.n_nodes, :3 * S.n_nodes])
    N = S.n_nodes
    Sh = np.zeros((N, N))
    for i in range(N):
        for j in range(N):
            acc = Dd[i, j]
            for k in range(3 * N):
                if Cd[i, k] != 0.0 and Bd[k, j] != 0.0:
                    acc -= Cd[i, k] * Bd[k, j] / dA[k]
            Sh[i, j] = acc
    assert np.abs(ns.Shat.toarray() - Sh).max() <= 1e-14 * np.abs(Sh).max()


def test_matrix_free_schur_matches_dense_schur():
    S = get_assembled("channel2")
    c = get_case("channel2")
    o = kr.SolveOpts(rtol_I=1e-14)
    ns = kr.NestedSolver(S, amg.node_adjacency(c.n_nodes, c.tets), o)
    n3 = 3 * S.n_nodes
    Ad = S.dense()
    A, B, C, D = Ad[:n3, :n3], Ad[:n3, n3:], Ad[n3:, :n3], Ad[n3:, n3:]
    Sd = D - C @ np.linalg.solve(A, B)
    x = np.random.default_rng(5).standard_normal(S.n_nodes)
    y = ns.schur_apply(x, kr.Schedule())
    assert np.linalg.norm(y - Sd @ x) <= 1e-10 * np.linalg.norm(Sd @ x)


@pytest.mark.parametrize("name", ["cube", "channel2", "unstr_channel"])
def test_exact_subsolves_make_scr_exact(name):
    """With delta_A = delta_S = delta_I -> 0 the SCR preconditioner is the block
    LDU factorisation of the tangent, so FGMRES needs one iteration."""
    S = get_assembled(name)
    c = get_case(name)
    o = kr.SolveOpts(rtol=1e-10, rtol_A=1e-14, rtol_S=1e-14, rtol_I=1e-14)
    ns = kr.NestedSolver(S, amg.node_adjacency(c.n_nodes, c.tets), o)
    x, info = ns.solve(S.rhs)
    assert info["outer"] == 1
    xs = np.linalg.solve(S.dense(), S.rhs)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)


@pytest.mark.parametrize("name", ["cube", "channel2", "unstr_channel"])
def test_nested_solve_matches_dense_lu(name):
    S = get_assembled(name)
    c = get_case(name)
    ns = kr.NestedSolver(S, amg.node_adjacency(c.n_nodes, c.tets), kr.SolveOpts(rtol=1e-8))
    x, info = ns.solve(S.rhs)
    Ad = S.dense()
    assert np.linalg.norm(S.rhs - Ad @ x) <= 1e-8 * np.linalg.norm(S.rhs)
    assert info["converged"] and info["true_rel_res"] <= 1e-8
    xs = np.linalg.solve(Ad, S.rhs)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(x - xs) <= kappa * 1e-8 * np.linalg.norm(xs)
    # replaying the logged iteration counts reproduces the same iterate
    x2, info2 = ns.solve(S.rhs, replay=info["schedule"])
    assert np.array_equal(x, x2) and info2["schedule"] == info["schedule"]


@pytest.mark.parametrize("name,transposed", [("cube", False), ("channel2", False), ("channel2", True)])
def test_exact_subsolves_make_simple_the_factored_product(name, transposed):
    """With exact A- and S_hat-solves the SIMPLE preconditioner is the product of
    its three factors, [A  A diag(A)^{-1} B; C  D] (Sec. 3.2): applying the
    oracle's P_SIMPLE^{-1} and then that dense matrix returns the input."""
    S = get_assembled(name)
    if transposed:
        S = S.transposed()
    c = get_case(name)
    o = kr.SolveOpts(pc="simple", rtol_A=1e-14, rtol_S=1e-14)
    ns = kr.NestedSolver(S, amg.node_adjacency(c.n_nodes, c.tets), o)
    n3 = 3 * S.n_nodes
    Ad = S.dense()
    A, B, C, D = Ad[:n3, :n3], Ad[:n3, n3:], Ad[n3:, :n3], Ad[n3:, n3:]
    dA = np.diag(A)
    P = np.block([[A, A @ (B / dA[:, None])], [C, D]])
    s = np.random.default_rng(11).standard_normal(4 * S.n_nodes)
    y = ns.simple_apply(s, kr.Schedule())
    assert np.linalg.norm(P @ y - s) <= 1e-10 * np.linalg.norm(s)
    # and it is not the tangent's inverse (the (1,2) block differs)
    assert np.linalg.norm(Ad @ y - s) > 1e-6 * np.linalg.norm(s)


@pytest.mark.parametrize("name", ["cube", "channel2"])
def test_simple_outer_solve_matches_dense_lu(name):
    S = get_assembled(name)
    c = get_case(name)
    ns = kr.NestedSolver(S, amg.node_adjacency(c.n_nodes, c.tets), kr.SolveOpts(rtol=1e-8, pc="simple"))
    x, info = ns.solve(S.rhs)
    Ad = S.dense()
    assert info["converged"] and np.linalg.norm(S.rhs - Ad @ x) <= 1e-8 * np.linalg.norm(S.rhs)
    xs = np.linalg.solve(Ad, S.rhs)
    assert np.linalg.norm(x - xs) <= np.linalg.cond(Ad) * 1e-8 * np.linalg.norm(xs)
    # two Krylov calls per preconditioner application (A, then S_hat), replayable
    assert len(info["schedule"]) == 1 + 2 * info["outer"]
    x2, info2 = ns.solve(S.rhs, replay=info["schedule"])
    assert np.array_equal(x, x2)


def test_jacobi_variant_converges():
    S = get_assembled("channel2")
    c = get_case("channel2")
    ns = kr.NestedSolver(S, amg.node_adjacency(c.n_nodes, c.tets), kr.SolveOpts(pc_A="jacobi"))
    x, info = ns.solve(S.rhs)
    assert info["converged"]


def test_gmres_on_spd_system_matches_solution():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    M = Q @ np.diag(np.linspace(1, 10, 30)) @ Q.T
    b = rng.standard_normal(30)
    x, its = kr.gmres_left(lambda v: M @ v, lambda v: v, b, 1e-12, 40, 40, kr.Schedule())
    assert np.linalg.norm(M @ x - b) <= 1e-11 * np.linalg.norm(b)
    assert its <= 30
    # restarted GMRES(5) still converges
    x5, its5 = kr.gmres_left(lambda v: M @ v, lambda v: v, b, 1e-10, 5, 400, kr.Schedule())
    assert np.linalg.norm(M @ x5 - b) <= 1e-9 * np.linalg.norm(b) and its5 > 5


def test_greedy_matching_hand_example():
    # path 0-1-2-3-4: first pass pairs (0,1), (2,3), single 4
    path = [np.array([1]), np.array([0, 2]), np.array([1, 3]), np.array([2, 4]), np.array([3])]
    agg, nc = amg.greedy_matching(path)
    assert list(agg) == [0, 0, 1, 1, 2] and nc == 3
    q = amg.quotient(path, agg, nc)
    assert [list(x) for x in q] == [[1], [0, 2], [1]]
    aggs = amg.build_aggregates(path, coarse_nodes=1)
    assert list(aggs[0]) == [0, 0, 0, 0, 1]


def test_power_start_vector_values():
    x = amg.power_start(3)
    assert x[0] == 0.5
    assert x[1] == 0.5 + 2654435761 / 2 ** 32
    assert x[2] == 0.5 + ((2 * 2654435761) % 2 ** 32) / 2 ** 32


def test_gershgorin_bound_brute_force():
    """Row sums of |D^{-1} M| by explicit loops over a small dense matrix."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((7, 7)) + 6 * np.eye(7)
    A[A < -1.0] = 0.0
    d = 1.0 / np.diag(A)
    want = max(sum(abs(d[i] * A[i, j]) for j in range(7)) for i in range(7))
    assert amg.gershgorin_bound(sp.csr_matrix(A), d) == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("name", ["cube", "channel2", "pipe_tiny", "unstr_channel"])
def test_smoother_bound_covers_spectrum(name):
    """The smoother interval's upper end bounds the spectral radius of
    D^{-1} M on every smoothed level (dense eigenvalues), for both
    hierarchies; a smaller value would make the damped Jacobi step amplify the
    top modes."""
    c = get_case(name)
    S = get_assembled(name)
    ns = kr.NestedSolver(S, amg.node_adjacency(c.n_nodes, c.tets), kr.SolveOpts(coarse_nodes=16))
    for h in (ns.amgA, ns.amgS):
        assert h.n_levels >= 2
        for Ml, di, lm in zip(h.M[:-1], h.dinv, h.lmax):
            rho = np.abs(np.linalg.eigvals(np.diag(di) @ Ml.toarray())).max()
            assert rho <= lm <= amg.gershgorin_bound(Ml, di) * (1 + 1e-15)


def test_chebyshev_matches_scalar_polynomial():
    """For M = diag(lam), D = M... use D = I via a unit diagonal: x = (1 - p(lam)) b / lam
    with p(t) = T_k((theta - t)/delta) / T_k(theta/delta)."""
    lam = np.linspace(0.2, 3.0, 9)
    M = sp.diags(lam).tocsr()
    b = np.arange(1.0, 10.0)
    lmin, lmax = 0.1, 3.3
    th, de = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    for k in [1, 2, 3]:
        x = amg.chebyshev(M, np.ones(9), b, None, k, lmin, lmax)
        Tk = lambda s: np.cos(k * np.arccos(s)) if abs(s) <= 1 else np.cosh(k * np.arccosh(abs(s))) * np.sign(s) ** k
        p = np.array([Tk((th - t) / de) for t in lam]) / Tk(th / de)
        assert x == pytest.approx((1 - p) * b / lam, rel=1e-12)


def test_amg_two_level_galerkin_and_exact_coarse():
    S = get_assembled("channel2")
    c = get_case("channel2")
    adj = amg.node_adjacency(c.n_nodes, c.tets)
    aggs = amg.build_aggregates(adj, coarse_nodes=10 ** 9)
    assert aggs == []
    h = amg.AMG(S.A_F, 3, aggs)
    b = np.random.default_rng(2).standard_normal(3 * S.n_nodes)
    assert h.vcycle(b) == pytest.approx(np.linalg.solve(S.A_F.toarray(), b), rel=1e-10)
    aggs = amg.build_aggregates(adj, coarse_nodes=60)
    h = amg.AMG(S.A_F, 3, aggs)
    Pn = np.zeros((c.n_nodes, int(aggs[0].max()) + 1))
    Pn[np.arange(c.n_nodes), aggs[0]] = 1
    P = np.kron(Pn, np.eye(3))
    assert np.abs(h.M[1].toarray() - P.T @ S.A_F.toarray() @ P).max() <= 1e-15 * abs(S.A_F).max()
    # every aggregate has at most 4 nodes and is connected by construction
    assert np.bincount(aggs[0]).max() <= 4


@pytest.mark.parametrize("cc", [1.0, 1.7])
def test_amg_two_level_cycle_dense_formula(cc):
    """Two levels, degree-1 smoothing (x += D^-1 r / theta), exact coarse
    solve and the coarse-grid correction scaled by cc: the cycle is the dense
    matrix B = X + T (I - M X) with X = T + cc P (P^T M P)^-1 P^T (I - M T),
    T = D^-1 / theta, theta the centre of [lambda/10, lambda]."""
    S = get_assembled("channel2")
    c = get_case("channel2")
    adj = amg.node_adjacency(c.n_nodes, c.tets)
    aggs = amg.build_aggregates(adj, coarse_nodes=60)[:1]
    h = amg.AMG(S.A_F, 3, aggs, cheb_degree=1, cc_scale=cc)
    M = S.A_F.toarray()
    n = M.shape[0]
    Pn = np.zeros((c.n_nodes, int(aggs[0].max()) + 1))
    Pn[np.arange(c.n_nodes), aggs[0]] = 1
    P = np.kron(Pn, np.eye(3))
    lam = h.lmax[0]
    T = np.diag(1.0 / np.diag(M)) / (0.5 * (lam + lam / 10.0))
    I = np.eye(n)
    Cc = cc * P @ np.linalg.solve(P.T @ M @ P, P.T)
    pre = T                                   # x1 = T b
    mid = pre + Cc @ (I - M @ pre)            # x2 = x1 + cc P Mc^-1 P^T (b - M x1)
    B = mid + T @ (I - M @ mid)               # x3 = x2 + T (b - M x2)
    b = np.random.default_rng(4).standard_normal(n)
    assert np.abs(h.vcycle(b) - B @ b).max() <= 1e-10 * np.abs(B @ b).max()


@pytest.mark.parametrize("gamma", [1, 2, 3])
def test_amg_three_level_cycle_index_dense_formula(gamma):
    """Three levels, degree-1 smoothing (T_l = D_l^-1 / theta_l), exact coarsest
    solve: the finest level takes one coarse-grid correction, level 1 takes
    gamma (each followed by its post-smoothing), written as dense matrices:
    B_1 = X with X <- T_1, then gamma times X <- X + P_1 M_2^-1 P_1^T (I - M_1 X),
    X <- X + T_1 (I - M_1 X); B_0 likewise with B_1 in place of M_2^-1, once."""
    S = get_assembled("channel2")
    c = get_case("channel2")
    adj = amg.node_adjacency(c.n_nodes, c.tets)
    aggs = amg.build_aggregates(adj, coarse_nodes=8)[:2]
    assert len(aggs) == 2
    h = amg.AMG(S.A_F, 3, aggs, cheb_degree=1, cycle_index=gamma)
    Ms = [m.toarray() for m in h.M]
    Ps = [p.toarray() for p in h.P]
    Ts = [np.diag(1.0 / np.diag(Ms[l])) / (0.5 * (h.lmax[l] + h.lmax[l] / 10.0)) for l in range(2)]

    def level(l, Bc, reps):
        n = Ms[l].shape[0]
        X = Ts[l].copy()
        for _ in range(reps):
            X = X + Ps[l] @ Bc @ Ps[l].T @ (np.eye(n) - Ms[l] @ X)
            X = X + Ts[l] @ (np.eye(n) - Ms[l] @ X)
        return X

    B1 = level(1, np.linalg.inv(Ms[2]), gamma)
    B0 = level(0, B1, 1)
    b = np.random.default_rng(6).standard_normal(Ms[0].shape[0])
    assert np.abs(h.vcycle(b) - B0 @ b).max() <= 1e-9 * np.abs(B0 @ b).max()


# --------------------------------------------------------------------------- adjoint


def test_transpose_identity_and_adjoint_gradient():
    c = get_case("channel2")
    S = get_assembled("channel2")
    Ad = S.dense()
    rng = np.random.default_rng(9)
    lam, x = rng.standard_normal(4 * c.n_nodes), rng.standard_normal(4 * c.n_nodes)
    St = S.transposed()
    assert abs(St.apply(lam) @ x - lam @ S.apply(x)) <= 1e-14 * np.linalg.norm(Ad) * np.linalg.norm(x) * np.linalg.norm(lam)
    ph = dz.physics_of(c)
    am, af, g = ph.alphas
    cf = af * g * ph.dt
    adj = amg.node_adjacency(c.n_nodes, c.tets)
    o = kr.SolveOpts(rtol=1e-12)
    x, _ = kr.NestedSolver(S, adj, o).solve(S.rhs)
    gJ = adj_mod.mean_outlet_pressure_weights(S, 0, g * ph.dt) + 0.5 * adj_mod.mean_outlet_pressure_weights(S, 1, g * ph.dt)
    lam, info = adj_mod.adjoint_solve(S, adj, gJ, o)
    lam_d = np.linalg.solve(Ad.T, gJ)
    assert np.linalg.norm(lam - lam_d) <= 1e-9 * np.linalg.norm(lam_d)
    gr = adj_mod.grad_R(S, x, lam, af, cf)
    Pn = c.R * S.Q

    def L(R):
        S2 = dz.assemble(c, P_af=(1 - af) * Pn + af * R * S.Q, R=R)
        return gJ @ np.linalg.solve(S2.dense(), S2.rhs)

    for k in range(2):
        h = 1e-6 * c.R[k]
        Rp, Rm = c.R.copy(), c.R.copy()
        Rp[k] += h
        Rm[k] -= h
        fd = (L(Rp) - L(Rm)) / (2 * h)
        assert gr[k] == pytest.approx(fd, rel=1e-7)


# --------------------------------------------------------------------------- time step (predictor multi-corrector)

from oracle import newton as nt  # noqa: E402


def test_windkessel_rk4_matches_closed_form():
    """dPi/dt = -Pi/(Rd C) + Q(t)/C with Q linear over the step has the closed
    form Pi(T) = Pi_0 e^{-T/tau} + (1/C) int_0^T e^{-(T-s)/tau} (a + b s) ds."""
    Rp, C, Rd, Pd = 120.0, 1.5e-3, 900.0, 7.0
    Pi0, Qa, Qb, T = 40.0, 2.0, 3.5, 0.01
    tau = Rd * C
    e = np.exp(-T / tau)
    a, b = Qa, (Qb - Qa) / T
    integral = a * tau * (1 - e) + b * (tau * T - tau ** 2 * (1 - e))
    Pi_exact = Pi0 * e + integral / C
    P, Pi = nt.windkessel(Rp, C, Rd, Pd, Pi0, Qa, Qb, 100, T)
    assert Pi == pytest.approx(Pi_exact, rel=1e-12)
    assert P == pytest.approx(Rp * Qb + Pi_exact + Pd, rel=1e-12)
    # fourth order: over a step of ~1 time constant the error falls ~16x
    # when the sub-step is halved
    T = 1.0
    e = np.exp(-T / tau)
    b = (Qb - Qa) / T
    Pi_exact = Pi0 * e + (a * tau * (1 - e) + b * (tau * T - tau ** 2 * (1 - e))) / C
    e1 = abs(nt.windkessel(Rp, C, Rd, Pd, Pi0, Qa, Qb, 5, T)[1] - Pi_exact)
    e2 = abs(nt.windkessel(Rp, C, Rd, Pd, Pi0, Qa, Qb, 10, T)[1] - Pi_exact)
    assert 13.0 < e1 / e2 < 19.0


def test_windkessel_limits():
    """Constant flow for many time constants: P -> (Rp + Rd) Q + Pd, the
    resistance model; zero compliance is that model at once."""
    Rp, C, Rd, Pd, Q = 100.0, 1e-3, 1000.0, 5.0, 2.0
    Pi = 0.0
    for _ in range(1000):  # 50 time constants R_d C
        P, Pi = nt.windkessel(Rp, C, Rd, Pd, Pi, Q, Q, 20, 0.05)
    assert P == pytest.approx((Rp + Rd) * Q + Pd, rel=1e-12)
    assert nt.windkessel(Rp, 0.0, Rd, Pd, 123.0, 9.0, Q, 20, 0.05) == ((Rp + Rd) * Q + Pd, 0.0)


def _step_inputs(name, seed=3):
    c = get_case(name)
    N = c.n_nodes
    y_n = np.concatenate([c.v.ravel(), c.p])
    rng = np.random.default_rng(seed)
    ydot_n = rng.standard_normal(4 * N) * 0.5
    dm = np.concatenate([c.mask[:, :3].ravel(), c.mask[:, 3]]).astype(bool)
    ydot_n[dm] = 0.0
    a_raw, _, _ = dz.outlet_vectors(c)
    Q_n = np.array([np.sum(a_raw[k] * c.v) for k in range(c.n_outlets)])
    model = nt.OutletModel(Rp=c.R.copy(), C=np.zeros(c.n_outlets), Rd=np.zeros(c.n_outlets),
                           Pd=np.zeros(c.n_outlets), Pi=np.zeros(c.n_outlets), P=c.R * Q_n, Q=Q_n)
    return c, y_n, ydot_n, model


def test_time_step_update_and_converged_residual():
    """The predictor and every update keep y = y_n + dt ydot_n + gamma dt
    (ydot - ydot_n); the accepted state's residual, evaluated at the
    generalized-alpha intermediate states built here from their definitions,
    meets the tolerance; a resistance outlet ends with P = R Q."""
    c, y_n, ydot_n, model = _step_inputs("channel2")
    ph = dz.physics_of(c)
    am, af, gam = ph.alphas
    y, ydot, info, out = nt.time_step(c, y_n, ydot_n, model, nt.NewtonOpts(tol_R=1e-9, tol_A=1e-14),
                                      kr.SolveOpts(rtol=1e-12, rtol_A=1e-10, rtol_S=1e-10, rtol_I=1e-10))
    assert info["converged"] and info["iterations"] >= 2
    assert np.allclose(y, y_n + ph.dt * ydot_n + gam * ph.dt * (ydot - ydot_n), rtol=0, atol=1e-13 * np.abs(y).max())
    N = c.n_nodes
    yaf = y_n + af * (y - y_n)
    ydam = ydot_n + am * (ydot - ydot_n)
    a_raw, _, _ = dz.outlet_vectors(c)
    Q = np.array([np.sum(a_raw[k] * y[:3 * N].reshape(N, 3)) for k in range(c.n_outlets)])
    Paf = (1 - af) * model.P + af * c.R * Q
    S = dz.assemble(c, P_af=Paf, R=c.R, v=yaf[:3 * N].reshape(N, 3), p=yaf[3 * N:], vdot=ydam[:3 * N].reshape(N, 3))
    assert np.linalg.norm(S.rhs) <= 1e-9 * info["res0"]
    assert np.allclose(out.Q, Q, rtol=1e-14) and np.allclose(out.P, c.R * Q, rtol=1e-14)
    # the residual history decreases at every corrector
    h = info["res_hist"]
    assert all(b < a for a, b in zip(h, h[1:]))


def test_time_step_nested_matches_dense_newton():
    """The same corrector loop with every linear system solved densely gives
    the same iterates as with the nested solver at tight tolerances."""
    c, y_n, ydot_n, model = _step_inputs("channel2")
    tight = kr.SolveOpts(rtol=1e-13, rtol_A=1e-11, rtol_S=1e-11, rtol_I=1e-11)
    nopt = nt.NewtonOpts(tol_R=1e-10, tol_A=1e-15, l_max=6)
    y1, yd1, i1, _ = nt.time_step(c, y_n, ydot_n, model, nopt, tight)
    y2, yd2, i2, _ = nt.time_step(c, y_n, ydot_n, model, nopt, tight,
                                  linear_solve=lambda S: np.linalg.solve(S.dense(), S.rhs))
    assert i1["iterations"] == i2["iterations"]
    assert np.allclose(i1["res_hist"], i2["res_hist"], rtol=1e-6, atol=1e-12 * i1["res0"])
    assert np.linalg.norm(y1 - y2) <= 1e-10 * np.linalg.norm(y2)
    assert np.linalg.norm(yd1 - yd2) <= 1e-8 * np.linalg.norm(yd2)


def test_time_step_windkessel_derivative_gives_newton_convergence():
    """With three-element Windkessel outlets and dense linear solves the
    corrector is Newton's method on the coupled problem only if m^k is the
    derivative of the reduced model's outlet pressure: the residual then
    falls from 1e3 to 1e-10 relative in three corrections (each factor at
    most 1e-4 after the first), where an m^k off by 10 % (or m^k = R_p alone)
    only contracts linearly, by 1e-2 per correction."""
    c, y_n, ydot_n, _ = _step_inputs("channel2")
    a_raw, _, _ = dz.outlet_vectors(c)
    no = c.n_outlets
    Q_n = np.array([np.sum(a_raw[k] * c.v) for k in range(no)])
    Rp, Rd = 0.1 * c.R, 0.9 * c.R
    C = 10 * c.dt / Rd
    Pi = Rd * Q_n
    model = nt.OutletModel(Rp=Rp, C=C, Rd=Rd, Pd=np.full(no, 2.0), Pi=Pi, P=Rp * Q_n + Pi + 2.0, Q=Q_n, n_ts=50)
    nopt = nt.NewtonOpts(tol_R=1e-12, tol_A=1e-15, l_max=6)
    _, _, info, _ = nt.time_step(c, y_n, ydot_n, model, nopt, kr.SolveOpts(),
                                 linear_solve=lambda S: np.linalg.solve(S.dense(), S.rhs))
    h = np.array(info["res_hist"])
    assert info["converged"] and info["iterations"] <= 3
    assert h[-1] <= 1e-12 * h[0]
    assert np.all(h[2:] / h[1:-1] <= 1e-4)


def test_time_step_exhausted_correctors_report_the_returned_state():
    """With l_max solves used up, the last history entry is the residual of the
    returned state (assembled here from its definition) and the step is not
    converged."""
    c, y_n, ydot_n, model = _step_inputs("channel2")
    ph = dz.physics_of(c)
    am, af, gam = ph.alphas
    y, ydot, info, _ = nt.time_step(c, y_n, ydot_n, model, nt.NewtonOpts(tol_R=1e-30, tol_A=1e-300, l_max=1),
                                    kr.SolveOpts())
    assert not info["converged"] and info["iterations"] == 1 and len(info["res_hist"]) == 2
    N = c.n_nodes
    yaf = y_n + af * (y - y_n)
    ydam = ydot_n + am * (ydot - ydot_n)
    a_raw, _, _ = dz.outlet_vectors(c)
    Q = np.array([np.sum(a_raw[k] * y[:3 * N].reshape(N, 3)) for k in range(c.n_outlets)])
    S = dz.assemble(c, P_af=(1 - af) * model.P + af * c.R * Q, R=c.R, v=yaf[:3 * N].reshape(N, 3), p=yaf[3 * N:],
                    vdot=ydam[:3 * N].reshape(N, 3))
    assert np.isclose(info["res_hist"][-1], np.linalg.norm(S.rhs), rtol=1e-12)
    assert info["res_hist"][-1] < info["res_hist"][0]
