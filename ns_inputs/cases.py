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


# ----------------------------------------------------------------------------
# Straight circular pipe (swept O-grid)
# ----------------------------------------------------------------------------

PIPE_SIZES = {
    # name: (m, nr, layers) -> nodes = ((m+1)^2 + 4 m nr) * (layers + 1)
    "pipe_tiny": (4, 2, 12),
    "pipe_small": (8, 4, 40),
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


def build(name: str, **kw) -> Case:
    if name.startswith("cube"):
        return cube_lid(**kw)
    if name == "channel2":
        return channel2(**kw)
    if name in PIPE_SIZES:
        return pipe(name, **kw)
    raise KeyError(name)
