"""Seeded synthetic workloads: mesh + boundary data + flow state + physics.

Each builder returns a :class:`Case`.  Nothing here evaluates the VMS
discretisation or the solver; a case is only the data one Newton step starts
from (the state the step linearises about, with y_{n+af} = y and the
acceleration at n+am equal to zero, as the predictor gives for a state at rest
in time).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import meshes


@dataclasses.dataclass
class Case:
    name: str
    xyz: np.ndarray          # f64 [N, 3]
    tets: np.ndarray         # i32 [E, 4]
    mask: np.ndarray         # u8  [N, 4]  Dirichlet flags (u, v, w, p)
    outlet_ptr: np.ndarray   # i32 [n_out + 1]
    faces: np.ndarray        # i32 [F, 3] outward oriented outlet triangles
    v: np.ndarray            # f64 [N, 3] velocity at n+af (Dirichlet values imposed)
    p: np.ndarray            # f64 [N]    pressure at n+af
    vdot: np.ndarray         # f64 [N, 3] acceleration at n+am
    rho: float
    mu: float
    dt: float
    rho_inf: float
    R: np.ndarray            # f64 [n_out] outlet resistances
    meta: dict

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_outlets(self) -> int:
        return int(self.outlet_ptr.shape[0] - 1)

    @property
    def n_dof(self) -> int:
        return 4 * self.n_nodes


def _finish(name, xyz, tets, mask, outlet_faces, v, p, rho, mu, dt, rho_inf, R, meta):
    ptr = [0]
    for f in outlet_faces:
        ptr.append(ptr[-1] + len(f))
    faces = (np.concatenate(outlet_faces, axis=0) if outlet_faces else np.zeros((0, 3))).astype(np.int32)
    v = v.copy()
    return Case(name=name, xyz=np.ascontiguousarray(xyz, dtype=np.float64),
                tets=np.ascontiguousarray(tets, dtype=np.int32),
                mask=np.ascontiguousarray(mask, dtype=np.uint8),
                outlet_ptr=np.asarray(ptr, dtype=np.int32), faces=np.ascontiguousarray(faces),
                v=np.ascontiguousarray(v, dtype=np.float64), p=np.ascontiguousarray(p, dtype=np.float64),
                vdot=np.zeros_like(v, dtype=np.float64), rho=float(rho), mu=float(mu), dt=float(dt),
                rho_inf=float(rho_inf), R=np.asarray(R, dtype=np.float64), meta=meta)


# ----------------------------------------------------------------------------
# Lid-driven unit cube (Kuhn lattice)
# ----------------------------------------------------------------------------


def cube_lid(n: int = 8, seed: int = 1, amp: float = 0.1) -> Case:
    """[0,1]^3, n^3 hexes x 6 tets; lid u=(1,0,0) on z=1 (edges and corners
    included), no-slip elsewhere, pressure pinned at node 0; interior velocity
    components ~ U(-amp, amp); p = 0."""
    xyz, tets = meshes.kuhn_box(n, n, n)
    N = len(xyz)
    tol = 1e-12
    on_bnd = np.any((xyz < tol) | (xyz > 1 - tol), axis=1)
    lid = xyz[:, 2] > 1 - tol
    mask = np.zeros((N, 4), np.uint8)
    mask[on_bnd, :3] = 1
    mask[0, 3] = 1
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.uniform(-amp, amp, size=(N, 3))
    v[on_bnd] = 0.0
    v[lid] = (1.0, 0.0, 0.0)
    return _finish(f"cube{n}", xyz, tets, mask, [], v, np.zeros(N), 1.0, 0.04, 1e-3, 0.5,
                   np.zeros(0), {"seed": seed, "pressure": "p = 0 everywhere"})


# ----------------------------------------------------------------------------
# Tiny two-outlet box channel (dense-checkable)
# ----------------------------------------------------------------------------


def channel2(nx: int = 8, ny: int = 4, nz: int = 4, seed: int = 2, R=(1.5e3, 3.0e3),
             umax: float = 10.0, noise: float = 0.01) -> Case:
    """Box [0,2]x[0,1]x[0,1]; inlet x=0 with u = umax*16 y(1-y) z(1-z);
    outlet 1 is the face x=2, outlet 2 the patch x in [0.75, 1.25] of the
    face y=1; every other boundary point (and every outlet rim) is no-slip.
    State: the inlet profile continued along x, scaled near the side outlet,
    plus seeded Gaussian noise (``noise`` * umax) on free components."""
    lx, ly, lz = 2.0, 1.0, 1.0
    xyz, tets = meshes.kuhn_box(nx, ny, nz, lx, ly, lz)
    N = len(xyz)
    tol = 1e-12
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    bfaces = meshes.boundary_faces(xyz, tets)
    fx = xyz[bfaces]
    out1 = np.all(np.abs(fx[:, :, 0] - lx) < tol, axis=1)
    out2 = (np.all(np.abs(fx[:, :, 1] - ly) < tol, axis=1)
            & np.all(fx[:, :, 0] > 0.75 - tol, axis=1) & np.all(fx[:, :, 0] < 1.25 + tol, axis=1))
    # free boundary nodes: interior points of the outlet patches
    free1 = (np.abs(x - lx) < tol) & (y > tol) & (y < ly - tol) & (z > tol) & (z < lz - tol)
    free2 = (np.abs(y - ly) < tol) & (x > 0.75 + tol) & (x < 1.25 - tol) & (z > tol) & (z < lz - tol)
    on_bnd = np.any((xyz < tol) | (xyz > np.array([lx, ly, lz]) - tol), axis=1)
    dir_nodes = on_bnd & ~free1 & ~free2
    mask = np.zeros((N, 4), np.uint8)
    mask[dir_nodes, :3] = 1
    prof = umax * 16.0 * y * (1 - y) * z * (1 - z)
    v = np.zeros((N, 3))
    v[:, 0] = prof
    rng = np.random.Generator(np.random.PCG64(seed))
    v[~dir_nodes] += rng.normal(0.0, noise * umax, size=(int((~dir_nodes).sum()), 3))
    inlet = np.abs(x) < tol
    v[dir_nodes] = 0.0
    v[inlet, 0] = prof[inlet]
    return _finish("channel2", xyz, tets, mask, [bfaces[out1], bfaces[out2]], v, np.zeros(N),
                   1.06, 0.04, 1e-3, 0.5, np.asarray(R, float),
                   {"seed": seed, "pressure": "p = 0 everywhere"})


UNSTR_SIZES = {
    "unstr_channel": (16, 8, 8),    # 1 377 nodes (parity tests)
    "unstr_200k": (96, 48, 48),     # 232 897 nodes, 1.48M tets (the Delaunay step takes ~1 min)
}


def unstructured_channel(size: str = "unstr_channel", seed: int = 7, R: float = 2.0e3,
                         umax: float = 10.0, noise: float = 0.01, jitter: float = 0.3) -> Case:
    """Box [0,2]x[0,1]x[0,1] meshed by ``meshes.delaunay_box`` (unstructured:
    irregular node degrees and row lengths); inlet x=0 with u = umax*16
    y(1-y) z(1-z); outlet the face x=2; every other boundary point (and the
    outlet rim) is no-slip.  State: the inlet profile continued along x plus
    seeded Gaussian noise (``noise`` * umax) on free components; p = 0."""
    nx, ny, nz = UNSTR_SIZES[size]
    lx, ly, lz = 2.0, 1.0, 1.0
    xyz, tets = meshes.delaunay_box(nx, ny, nz, lx, ly, lz, jitter=jitter, seed=seed)
    N = len(xyz)
    tol = 1e-12
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    bfaces = meshes.boundary_faces(xyz, tets)
    out = np.all(np.abs(xyz[bfaces][:, :, 0] - lx) < tol, axis=1)
    free = (np.abs(x - lx) < tol) & (y > tol) & (y < ly - tol) & (z > tol) & (z < lz - tol)
    on_bnd = np.any((xyz < tol) | (xyz > np.array([lx, ly, lz]) - tol), axis=1)
    dir_nodes = on_bnd & ~free
    mask = np.zeros((N, 4), np.uint8)
    mask[dir_nodes, :3] = 1
    prof = umax * 16.0 * y * (1 - y) * z * (1 - z)
    v = np.zeros((N, 3))
    v[:, 0] = prof
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    v[~dir_nodes] += rng.normal(0.0, noise * umax, size=(int((~dir_nodes).sum()), 3))
    inlet = np.abs(x) < tol
    v[dir_nodes] = 0.0
    v[inlet, 0] = prof[inlet]
    return _finish(size, xyz, tets, mask, [bfaces[out]], v, np.zeros(N), 1.06, 0.04, 1e-3, 0.5,
                   np.asarray([R], float), {"seed": seed, "jitter": jitter, "pressure": "p = 0 everywhere"})


# ----------------------------------------------------------------------------
# Straight circular pipe (swept O-grid)
# ----------------------------------------------------------------------------

PIPE_SIZES = {
    # name: (m, nr, layers) -> nodes = ((m+1)^2 + 4 m nr) * (layers + 1)
    "pipe_tiny": (4, 2, 12),
    "pipe_small": (8, 4, 40),
    "pipe_20k": (10, 5, 60),
    "pipe_40k": (12, 6, 96),
    "pipe_200k": (20, 10, 160),
    "pipe_2m": (44, 22, 340),
}


def pipe(size: str = "pipe_200k", seed: int = 2, R: float = 1e3, radius: float = 0.3,
         length: float = 3.0, umax: float = 30.0, noise: float = 0.01,
         rho: float = 1.06, mu: float = 0.04, dt: float = 1e-3) -> Case:
    """Pipe along z: parabolic inflow v_z = umax (1 - r^2/radius^2) at z=0,
    no-slip wall, resistance outlet at z=length.  State: Poiseuille profile
    plus N(0, (noise*umax)^2) on every free velocity component; p = 0."""
    m, nr, layers = PIPE_SIZES[size]
    zn = np.linspace(0.0, length, layers + 1)
    xyz, tets, rim, layer_of, _, out_faces = meshes.swept_tube(lambda z: radius, zn, m, nr)
    N = len(xyz)
    inlet = layer_of == 0
    mask = np.zeros((N, 4), np.uint8)
    mask[rim | inlet, :3] = 1
    r2 = (xyz[:, 0] ** 2 + xyz[:, 1] ** 2) / radius ** 2
    v = np.zeros((N, 3))
    v[:, 2] = umax * np.clip(1.0 - r2, 0.0, None)
    v[rim] = 0.0
    free = mask[:, 0] == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    v[free] += rng.normal(0.0, noise * umax, size=(int(free.sum()), 3))
    return _finish(size, xyz, tets, mask, [out_faces], v, np.zeros(N), rho, mu, dt, 0.5,
                   np.asarray([R], float),
                   {"seed": seed, "m": m, "nr": nr, "layers": layers, "pressure": "p = 0 everywhere"})


# ----------------------------------------------------------------------------
# Y-bifurcation (carved Kuhn lattice)
# ----------------------------------------------------------------------------

YBIF_SIZES = {
    # name: lattice spacing -> about 7e3 / 1e6 nodes
    "ybif_small": 0.1,
    "ybif_1m": 0.0176,
}


def ybif(size: str = "ybif_1m", seed: int = 4, R=(1.5e3, 3.0e3), umax: float = 30.0, noise: float = 0.01,
         rho: float = 1.06, mu: float = 0.04, dt: float = 1e-3) -> Case:
    """Parent tube r = 0.5 along z over [0, 4]; two daughters r = 0.35 from
    (0, 0, 4) at +-30 degrees from z in the x-z plane, cut by the plane
    z = 4 + 3 cos 30 deg (planar, disjoint outlet caps: outlet 1 at x < 0,
    outlet 2 at x > 0).  Mesh: the Kuhn tetrahedra of the lattice cells whose
    centre is inside (staircase wall).  Inflow: parabolic v_z with peak umax
    over the parent radius; no-slip on the rest of the boundary (outlet rims
    included).  State: per-branch axial Poiseuille (each daughter carries half
    the parent flow) plus N(0, (noise*umax)^2) on free components; p = 0."""
    h = YBIF_SIZES[size]
    rp, rd, lp, ld = 0.5, 0.35, 4.0, 3.0
    th = np.radians(30.0)
    ztop = lp + ld * np.cos(th)
    P0 = np.array([0.0, 0.0, lp])
    dirs = [np.array([-np.sin(th), 0.0, np.cos(th)]), np.array([np.sin(th), 0.0, np.cos(th)])]

    def axial(p):
        """branch (0 parent, 1/2 daughters), radial distance, unit axis"""
        q = p - P0
        br = np.zeros(len(p), np.int64)
        rad = np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2)
        for b, d in enumerate(dirs, start=1):
            a = q @ d
            rr = np.linalg.norm(q - a[:, None] * d, axis=1)
            sel = (p[:, 2] > lp) & ((p[:, 0] < 0) if b == 1 else (p[:, 0] >= 0))
            br[sel] = b
            rad[sel] = rr[sel]
        return br, rad

    def inside(c):
        inp = (c[:, 0] ** 2 + c[:, 1] ** 2 <= rp ** 2) & (c[:, 2] <= lp)
        q = c - P0
        for d in dirs:
            a = q @ d
            rr = np.linalg.norm(q - a[:, None] * d, axis=1)
            inp |= (a >= 0.0) & (rr <= rd)
        return inp & (c[:, 2] >= 0.0) & (c[:, 2] <= ztop)

    xmax = ld * np.sin(th) + rd / np.cos(th) + h
    lo, hi = (-xmax, -rp, 0.0), (xmax, rp, ztop)
    shape = (int(round(2 * xmax / h)), int(round(2 * rp / h)), int(round(ztop / h)))
    xyz, tets = meshes.carved_kuhn(inside, lo, hi, shape)
    N = len(xyz)
    tol = 1e-9
    bf = meshes.boundary_faces(xyz, tets)
    fz = xyz[bf][:, :, 2]
    inl = np.all(np.abs(fz) < tol, axis=1)
    outl = np.all(np.abs(fz - ztop) < tol, axis=1)
    fx = xyz[bf][:, :, 0].mean(axis=1)
    wall = np.zeros(N, bool)
    wall[bf[~inl & ~outl].ravel()] = True
    inlet = np.zeros(N, bool)
    inlet[bf[inl].ravel()] = True
    dirn = wall | inlet
    mask = np.zeros((N, 4), np.uint8)
    mask[dirn, :3] = 1
    br, rad = axial(xyz)
    qp = np.pi * rp ** 2 * umax / 2.0          # parent flow (Poiseuille mean = peak/2)
    ud = 2.0 * (qp / 2.0) / (np.pi * rd ** 2)  # daughter peak carrying half of it
    v = np.zeros((N, 3))
    par = br == 0
    v[par, 2] = umax * np.clip(1.0 - rad[par] ** 2 / rp ** 2, 0.0, None)
    for b, d in enumerate(dirs, start=1):
        s = br == b
        v[s] = (ud * np.clip(1.0 - rad[s] ** 2 / rd ** 2, 0.0, None))[:, None] * d[None, :]
    v[wall] = 0.0
    free = ~dirn
    rng = np.random.Generator(np.random.PCG64(seed))
    v[free] += rng.normal(0.0, noise * umax, size=(int(free.sum()), 3))
    outs = [bf[outl & (fx < 0)], bf[outl & (fx >= 0)]]
    return _finish(size, xyz, tets, mask, outs, v, np.zeros(N), rho, mu, dt, 0.5, np.asarray(R, float),
                   {"seed": seed, "h": h, "lattice": shape, "pressure": "p = 0 everywhere",
                    "wall": "staircase (cells with centre inside)"})


# ----------------------------------------------------------------------------
# Contraction-expansion tube (swept O-grid with a sudden expansion)
# ----------------------------------------------------------------------------

CONEXP_SIZES = {
    # name: (m, nr, annulus rings, cone layers, throat layers, expansion layers)
    "conexp_small": (6, 3, 4, 6, 10, 16),
    "conexp_60k": (8, 4, 6, 20, 40, 120),     # a CPU-sized sample of the same recipe (61 061 nodes)
    "conexp_150k": (10, 5, 8, 30, 60, 180),   # the size of the paper's nozzle mesh (~1.4e5 vertices)
    "conexp_4m": (24, 10, 20, 100, 200, 1000),
}


def conexp(size: str = "conexp_4m", seed: int = 5, R: float = 1e5, re_t: float = 3500.0,
           rho: float = 1.0, mu: float = 0.0035, dt: float = 5e-4, n_modes: int = 16,
           rms: float = 0.05) -> Case:
    """Inlet r = 0.6, cone of 20 deg included angle to a throat r = 0.2 of
    length 4, sudden expansion to r = 0.6 for length 12.  Throat Reynolds
    number re_t fixes the throat mean velocity u_t = re_t mu / (rho 2 r_t);
    the inflow is parabolic with the same flow rate.  Axial layers: uniform in
    the cone and throat, geometrically graded after the step (finest at the
    step plane).  State: the local-radius Poiseuille profile carrying that
    flow, plus ``n_modes`` divergence-free Fourier modes (wavelengths
    U[2 r_t, 8 r_t], random directions and phases) scaled to an RMS of
    rms * u_t over the free components; zero at Dirichlet DOFs; p = 0."""
    m, nr, nrings, kc, kt, kw = CONEXP_SIZES[size]
    ri, rt, rw, lt, lw = 0.6, 0.2, 0.6, 4.0, 12.0
    lc = (ri - rt) / np.tan(np.radians(10.0))
    zs = lc + lt

    def r_of(z):
        return ri + (rt - ri) * min(max(z / lc, 0.0), 1.0) if z < lc else rt

    z_narrow = np.concatenate([np.linspace(0.0, lc, kc + 1)[:-1], np.linspace(lc, zs, kt + 1)])
    beta = 2.5
    t = np.linspace(0.0, 1.0, kw + 1)
    z_wide = zs + lw * (np.expm1(beta * t) / np.expm1(beta))
    xyz, tets, wall, inl_faces, out_faces, layer_of = meshes.swept_step_tube(
        r_of, z_narrow, z_wide, rt, rw, m, nr, nrings)
    N = len(xyz)
    inlet = layer_of == 0
    mask = np.zeros((N, 4), np.uint8)
    dirn = wall | inlet
    mask[dirn, :3] = 1
    u_t = re_t * mu / (rho * 2.0 * rt)
    q = np.pi * rt ** 2 * u_t
    z = xyz[:, 2]
    rloc = np.where(z < lc, ri + (rt - ri) * np.clip(z / lc, 0.0, 1.0), rt)
    rloc = np.where(z < zs - 1e-12, rloc, rw)
    rad2 = (xyz[:, 0] ** 2 + xyz[:, 1] ** 2) / rloc ** 2
    v = np.zeros((N, 3))
    v[:, 2] = 2.0 * q / (np.pi * rloc ** 2) * np.clip(1.0 - rad2, 0.0, None)
    rng = np.random.Generator(np.random.PCG64(seed))
    pert = np.zeros((N, 3))
    for _ in range(n_modes):
        lam = rng.uniform(2 * rt, 8 * rt)
        kdir = rng.normal(size=3)
        kdir /= np.linalg.norm(kdir)
        e = np.cross(kdir, rng.normal(size=3))
        e /= np.linalg.norm(e)
        phase = rng.uniform(0.0, 2 * np.pi)
        pert += np.cos((2 * np.pi / lam) * (xyz @ kdir) + phase)[:, None] * e[None, :]
    free = ~dirn
    scale = rms * u_t / np.sqrt(np.mean(pert[free] ** 2))
    v[free] += scale * pert[free]
    v[wall] = 0.0
    return _finish(size, xyz, tets, mask, [out_faces], v, np.zeros(N), rho, mu, dt, 0.5, np.asarray([R], float),
                   {"seed": seed, "m": m, "nr": nr, "rings": nrings, "layers": (kc, kt, kw), "u_t": u_t,
                    "pressure": "p = 0 everywhere"})


# ----------------------------------------------------------------------------
# Box with a perforated top: many resistance / Windkessel outlets
# ----------------------------------------------------------------------------

PLATE_SIZES = {
    # name: (patches per side, quads per patch side, layers) -> patches^2 outlets
    "plate_small": (4, 3, 4),
    "plate_784": (28, 3, 10),    # as many outlets as the paper's pulmonary model (772)
}


def plate(size: str = "plate_784", seed: int = 6, umax: float = 10.0, noise: float = 0.01, height: float = 0.5,
          R_range=(1e4, 1e5), tau_range=(0.05, 0.5), rho: float = 1.06, mu: float = 0.04, dt: float = 1e-3) -> Case:
    """Box [0,1]^2 x [0,height] (Kuhn lattice); inflow v_z = umax 16 x(1-x)
    y(1-y) at z = 0; no-slip side walls.  The top z = height carries
    patches^2 square outlet patches of q x q quads on a grid of cells of
    (q+1) x (q+1) quads: one quad row of no-slip wall separates neighbouring
    patches (and the patches from the side walls), so the outlets share no
    node and every patch rim is wall.  Outlet parameters (seeded,
    log-uniform): R_k in R_range; for the three-element Windkessel
    Rp = R/10, Rd = 9R/10 and C = tau/Rd with tau in tau_range (meta['rcr']).
    State: the inflow profile continued along z plus N(0, (noise umax)^2) on
    free components; p = 0."""
    npch, q, nz = PLATE_SIZES[size]
    c = q + 1
    n = npch * c + 1
    xyz, tets = meshes.kuhn_box(n, n, nz, 1.0, 1.0, height)
    N = len(xyz)
    tol = 1e-12
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    ix = np.rint(x * n).astype(int)
    iy = np.rint(y * n).astype(int)
    top = np.abs(z - height) < tol

    def inner(i):  # node index strictly inside a patch along one axis
        t = (i - 1) % c
        return (i >= 1) & (i <= n - 1) & (t >= 1) & (t <= q - 1)

    free_top = top & inner(ix) & inner(iy)
    side = (x < tol) | (x > 1 - tol) | (y < tol) | (y > 1 - tol)
    bottom = z < tol
    dir_nodes = side | bottom | (top & ~free_top)
    mask = np.zeros((N, 4), np.uint8)
    mask[dir_nodes, :3] = 1
    bf = meshes.boundary_faces(xyz, tets)
    on_top = np.all(np.abs(xyz[bf][:, :, 2] - height) < tol, axis=1)
    tf = bf[on_top]
    u = xyz[tf].mean(axis=1)[:, :2] * n - 1.0    # face centroid in quad units from the first gap
    cell = np.floor(u / c).astype(int)
    inpatch = np.all((u - cell * c) < q, axis=1) & np.all(u > 0, axis=1)
    pid = cell[:, 0] * npch + cell[:, 1]
    outlets = [tf[inpatch & (pid == k)] for k in range(npch * npch)]
    prof = umax * 16.0 * x * (1 - x) * y * (1 - y)
    v = np.zeros((N, 3))
    v[:, 2] = prof
    rng = np.random.Generator(np.random.PCG64(seed))
    free = ~dir_nodes
    v[free] += rng.normal(0.0, noise * umax, size=(int(free.sum()), 3))
    v[dir_nodes] = 0.0
    v[bottom & ~side, 2] = prof[bottom & ~side]
    n_out = npch * npch
    R = np.exp(rng.uniform(np.log(R_range[0]), np.log(R_range[1]), size=n_out))
    tau = np.exp(rng.uniform(np.log(tau_range[0]), np.log(tau_range[1]), size=n_out))
    Rd = 0.9 * R
    rcr = {"Rp": 0.1 * R, "Rd": Rd, "C": tau / Rd}
    return _finish(size, xyz, tets, mask, outlets, v, np.zeros(N), rho, mu, dt, 0.5, R,
                   {"seed": seed, "patches": npch, "q": q, "layers": nz, "rcr": rcr,
                    "pressure": "p = 0 everywhere"})


def build(name: str, **kw) -> Case:
    if name.startswith("cube"):
        return cube_lid(**kw)
    if name == "channel2":
        return channel2(**kw)
    if name in UNSTR_SIZES:
        return unstructured_channel(name, **kw)
    if name in PIPE_SIZES:
        return pipe(name, **kw)
    if name in YBIF_SIZES:
        return ybif(name, **kw)
    if name in CONEXP_SIZES:
        return conexp(name, **kw)
    if name in PLATE_SIZES:
        return plate(name, **kw)
    raise KeyError(name)
