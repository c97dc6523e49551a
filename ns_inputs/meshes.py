"""Seeded synthetic P1 tetrahedral meshes and their boundary descriptions.

This module only builds geometry, connectivity, boundary masks and states.  It
holds none of the discretisation or solver arithmetic, so both the CPU oracle
and the GPU path can take their inputs from it without sharing method code.

Conventions
-----------
* ``xyz``   float64 [N, 3] node coordinates.
* ``tets``  int32   [E, 4] vertex indices, positively oriented (det > 0).
* ``faces`` int32   [F, 3] outlet triangles, ordered so that the right-hand
  normal points out of the domain; ``outlet_ptr`` (int32 [n_out + 1]) is the
  CSR offset of each outlet's triangles into ``faces``.
* ``mask``  uint8   [N, 4] Dirichlet flags for (u, v, w, p).
"""
from __future__ import annotations

import itertools

import numpy as np

# ----------------------------------------------------------------------------
# Structured Kuhn lattice (each hexahedron cut into 6 tetrahedra that share the
# cell diagonal from its lowest to its highest corner).
# ----------------------------------------------------------------------------


def _orient(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap two vertices of every negatively oriented tetrahedron."""
    p = xyz[tets]
    det = np.einsum("ei,ei->e", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    if np.any(det == 0.0):
        raise ValueError("degenerate tetrahedron")
    tets = tets.copy()
    neg = det < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets.astype(np.int32)


def kuhn_box(nx: int, ny: int, nz: int, lx: float = 1.0, ly: float = 1.0, lz: float = 1.0):
    """Kuhn subdivision of an nx*ny*nz grid of boxes of size lx*ly*lz.

    Node (i, j, k) has index i + (nx+1)*(j + (ny+1)*k) (x fastest).
    """
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    order = np.lexsort((ii, jj, kk))  # cells in k-major, then j, then i
    ii, jj, kk = ii[order], jj[order], kk[order]
    tets = []
    for perm in itertools.permutations(range(3)):
        c = [np.zeros_like(ii), np.zeros_like(ii), np.zeros_like(ii)]
        verts = [nid(ii, jj, kk)]
        for axis in perm:
            c[axis] = c[axis] + 1
            verts.append(nid(ii + c[0], jj + c[1], kk + c[2]))
        tets.append(np.stack(verts, axis=1))
    tets = np.stack(tets, axis=1).reshape(-1, 4)
    return xyz, _orient(xyz, tets)


def delaunay_box(nx: int, ny: int, nz: int, lx: float = 1.0, ly: float = 1.0, lz: float = 1.0,
                 jitter: float = 0.3, seed: int = 0):
    """Unstructured mesh of a box: the Delaunay tetrahedralisation of an
    (nx+1)(ny+1)(nz+1) lattice whose points move by up to ``jitter`` lattice
    spacings (boundary points only within their faces, so the boundary stays
    the box surface).  Node degrees spread well beyond the Kuhn lattice's
    (up to ~30 neighbours).  Flat tetrahedra that the triangulation leaves on
    the planar faces are dropped; every lattice point stays a vertex."""
    from scipy.spatial import Delaunay
    L = np.array([lx, ly, lz])
    h = L / np.array([nx, ny, nz])
    xs = [np.linspace(0.0, L[a], n + 1) for a, n in enumerate((nx, ny, nz))]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.uniform(-jitter, jitter, size=xyz.shape) * h
    tol = 1e-12
    on_face = (xyz < tol) | (xyz > L - tol)
    d[on_face] = 0.0
    xyz = xyz + d
    tets = Delaunay(xyz).simplices.astype(np.int64)
    p = xyz[tets]
    vol = np.einsum("ei,ei->e", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6.0
    tets = tets[np.abs(vol) > 1e-9 * float(np.prod(h))]
    if np.unique(tets).size != len(xyz):
        raise ValueError("a lattice point is not a vertex of the triangulation")
    return xyz, _orient(xyz, tets)


# ----------------------------------------------------------------------------
# Boundary faces
# ----------------------------------------------------------------------------


def boundary_faces(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """All boundary triangles, oriented with the outward right-hand normal."""
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    tri = tets[:, loc].reshape(-1, 3)
    opp = tets.reshape(-1)  # vertex opposite to each local face
    key = np.sort(tri, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    bmask = cnt[inv] == 1
    tri = tri[bmask]
    opp = opp[bmask]
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    inward = np.einsum("fi,fi->f", nrm, xyz[opp] - p0) > 0
    tri = tri.copy()
    tri[inward, 1], tri[inward, 2] = tri[inward, 2].copy(), tri[inward, 1].copy()
    return tri.astype(np.int32)


def face_normals(xyz: np.ndarray, faces: np.ndarray) -> np.ndarray:
    p0, p1, p2 = xyz[faces[:, 0]], xyz[faces[:, 1]], xyz[faces[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


# ----------------------------------------------------------------------------
# Swept circular cross-sections (O-grid disk, prisms cut into 3 tetrahedra)
# ----------------------------------------------------------------------------


def ogrid_disk(m: int, nr: int, core_frac: float = 0.5):
    """Unit-radius O-grid disk: an m*m core square plus 4 ring sectors.

    Returns (pts [n, 2], tris [t, 3], rim_mask [n]).  The core square has
    half-side ``core_frac / sqrt(2)``; ring layers blend linearly from the core
    boundary to the unit circle.
    """
    s = core_frac / np.sqrt(2.0)
    idx = {}
    pts = []

    def add(key, p):
        if key not in idx:
            idx[key] = len(pts)
            pts.append(p)
        return idx[key]

    g = np.linspace(-s, s, m + 1)
    for j in range(m + 1):
        for i in range(m + 1):
            add(("c", i, j), (g[i], g[j]))
    # boundary walk of the core square, counter-clockwise, 4*m points
    walk = []
    for i in range(m):
        walk.append(("c", i, 0))
    for j in range(m):
        walk.append(("c", m, j))
    for i in range(m, 0, -1):
        walk.append(("c", i, m))
    for j in range(m, 0, -1):
        walk.append(("c", 0, j))
    nb = len(walk)
    for t in range(nb):
        sq = np.array(pts[idx[walk[t]]])
        ang = np.arctan2(sq[1], sq[0])
        circ = np.array([np.cos(ang), np.sin(ang)])
        for r in range(1, nr + 1):
            f = r / nr
            add(("r", t, r), tuple((1 - f) * sq + f * circ))
    tris = []

    def ring(t, r):
        return idx[walk[t % nb]] if r == 0 else idx[("r", t % nb, r)]

    for j in range(m):
        for i in range(m):
            a, b = idx[("c", i, j)], idx[("c", i + 1, j)]
            c, d = idx[("c", i + 1, j + 1)], idx[("c", i, j + 1)]
            tris += [(a, b, c), (a, c, d)]
    for t in range(nb):
        for r in range(nr):
            a, b = ring(t, r), ring(t + 1, r)
            c, d = ring(t + 1, r + 1), ring(t, r + 1)
            tris += [(a, b, c), (a, c, d)]
    pts = np.array(pts, dtype=np.float64)
    tris = np.array(tris, dtype=np.int64)
    # counter-clockwise orientation
    e1 = pts[tris[:, 1]] - pts[tris[:, 0]]
    e2 = pts[tris[:, 2]] - pts[tris[:, 0]]
    cw = (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]) < 0
    tris[cw, 1], tris[cw, 2] = tris[cw, 2].copy(), tris[cw, 1].copy()
    rim = np.zeros(len(pts), dtype=bool)
    for t in range(nb):
        rim[ring(t, nr)] = True
    return pts, tris.astype(np.int32), rim


def sweep_prisms(n_disk: int, tris: np.ndarray, layers: int) -> np.ndarray:
    """Cut the prisms of a swept triangle mesh into 3 tetrahedra each.

    Node (layer l, disk node a) has index l*n_disk + a.  With the disk
    vertices of a triangle sorted a < b < c, the prism is cut into
    (a0 b0 c0 c1), (a0 b0 b1 c1), (a0 a1 b1 c1); every quad side face is then
    split along the diagonal from its lower-indexed bottom vertex to the other
    top vertex, so neighbouring prisms always agree (conforming mesh).
    """
    st = np.sort(tris.astype(np.int64), axis=1)
    a, b, c = st[:, 0], st[:, 1], st[:, 2]
    base = np.stack([np.stack([a, b, c, c + n_disk], 1),
                     np.stack([a, b, b + n_disk, c + n_disk], 1),
                     np.stack([a, a + n_disk, b + n_disk, c + n_disk], 1)], axis=1)  # [T, 3, 4]
    off = (np.arange(layers, dtype=np.int64) * n_disk)[:, None, None, None]
    return (base[None] + off).reshape(-1, 4)  # layer-major element order


def swept_tube(radius_of_z, z_nodes: np.ndarray, m: int, nr: int):
    """Tube along z whose radius is ``radius_of_z(z)``.

    Returns xyz, tets, disk-rim mask [N], layer index per node [N].
    """
    pts, tris, rim = ogrid_disk(m, nr)
    nd = len(pts)
    layers = len(z_nodes) - 1
    xyz = np.empty(((layers + 1) * nd, 3))
    for lay, z in enumerate(z_nodes):
        r = radius_of_z(z)
        xyz[lay * nd:(lay + 1) * nd, 0] = r * pts[:, 0]
        xyz[lay * nd:(lay + 1) * nd, 1] = r * pts[:, 1]
        xyz[lay * nd:(lay + 1) * nd, 2] = z
    tets = sweep_prisms(nd, tris, layers)
    tets = _orient(xyz, tets)
    rim_all = np.tile(rim, layers + 1)
    layer_of = np.repeat(np.arange(layers + 1), nd)
    # end caps: disk triangles are counter-clockwise seen from +z
    inlet_faces = tris[:, [0, 2, 1]].astype(np.int32)
    outlet_faces = (tris + layers * nd).astype(np.int32)
    return xyz, tets, rim_all, layer_of, inlet_faces, outlet_faces


# ----------------------------------------------------------------------------
# Carved Kuhn lattice (cells whose centre lies inside a region)
# ----------------------------------------------------------------------------


def carved_kuhn(inside, lo, hi, shape):
    """Kuhn tetrahedra of the lattice cells of the box [lo, hi] (``shape`` =
    cells per axis) whose centre satisfies ``inside(centres [n, 3]) -> bool``.

    Unused lattice nodes are dropped; node order follows the lattice index
    (x fastest, then y, then z).  Returns xyz, tets (positively oriented).
    """
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    nx, ny, nz = (int(s) for s in shape)
    h = (hi - lo) / np.array([nx, ny, nz], float)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    cen = lo + (np.stack([ii, jj, kk], 1) + 0.5) * h
    keep = inside(cen)
    ii, jj, kk = ii[keep], jj[keep], kk[keep]

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k.astype(np.int64))

    tets = []
    for perm in itertools.permutations(range(3)):
        c = [np.zeros_like(ii), np.zeros_like(ii), np.zeros_like(ii)]
        verts = [nid(ii, jj, kk)]
        for axis in perm:
            c[axis] = c[axis] + 1
            verts.append(nid(ii + c[0], jj + c[1], kk + c[2]))
        tets.append(np.stack(verts, axis=1))
    tets = np.stack(tets, axis=1).reshape(-1, 4)
    used, tets = np.unique(tets, return_inverse=True)
    tets = tets.reshape(-1, 4)
    i = used % (nx + 1)
    j = (used // (nx + 1)) % (ny + 1)
    k = used // ((nx + 1) * (ny + 1))
    xyz = lo + np.stack([i, j, k], 1).astype(np.float64) * h
    return xyz, _orient(xyz, tets)


# ----------------------------------------------------------------------------
# Swept tube with a sudden expansion: an O-grid core disk swept through a
# variable-radius section, then the core plus annulus rings (so the step
# plane conforms) swept through the wide section.
# ----------------------------------------------------------------------------


def annulus_rings(pts, rim_walk, n_rings: int, r_out: float):
    """Rings outside the unit disk: points at radii 1 + (r_out - 1) k / n_rings
    (k = 1..n_rings) along the angles of the rim walk, and the triangles
    between consecutive rings.  Returns (new points [n, 2], triangles [t, 3]
    indexed into the concatenation [pts; new points], outer-rim mask of the
    concatenation)."""
    nb = len(rim_walk)
    base = len(pts)
    ang = np.arctan2(pts[rim_walk, 1], pts[rim_walk, 0])
    new = []
    for k in range(1, n_rings + 1):
        r = 1.0 + (r_out - 1.0) * k / n_rings
        new.append(np.stack([r * np.cos(ang), r * np.sin(ang)], 1))
    new = np.concatenate(new, 0)

    def idx(t, k):
        t = t % nb
        return rim_walk[t] if k == 0 else base + (k - 1) * nb + t

    tris = []
    for k in range(n_rings):
        for t in range(nb):
            a, b, c, d = idx(t, k), idx(t + 1, k), idx(t + 1, k + 1), idx(t, k + 1)
            tris += [(a, b, c), (a, c, d)]
    tris = np.array(tris, dtype=np.int64)
    allp = np.concatenate([pts, new], 0)
    e1 = allp[tris[:, 1]] - allp[tris[:, 0]]
    e2 = allp[tris[:, 2]] - allp[tris[:, 0]]
    cw = (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]) < 0
    tris[cw, 1], tris[cw, 2] = tris[cw, 2].copy(), tris[cw, 1].copy()
    outer = np.zeros(len(allp), dtype=bool)
    outer[base + (n_rings - 1) * nb:] = True
    return new, tris.astype(np.int32), outer


def _prisms(tris, gid_lo, gid_hi):
    """Three tetrahedra per prism (as sweep_prisms, cut by the 2-D vertex
    order so neighbouring prisms agree), with per-layer index maps."""
    st = np.sort(tris.astype(np.int64), axis=1)
    a, b, c = st[:, 0], st[:, 1], st[:, 2]
    L, H = gid_lo, gid_hi
    return np.concatenate([np.stack([L[a], L[b], L[c], H[c]], 1),
                           np.stack([L[a], L[b], H[b], H[c]], 1),
                           np.stack([L[a], H[a], H[b], H[c]], 1)], 0)


def swept_step_tube(radius_of_z, z_narrow: np.ndarray, z_wide: np.ndarray, r_step: float, r_wide: float,
                    m: int, nr: int, n_rings: int):
    """Tube along z: the core disk scaled to ``radius_of_z`` at the layers
    ``z_narrow`` (ending at the step plane z_narrow[-1] == z_wide[0] where the
    radius is r_step), then core + annulus (out to r_wide) at the layers
    ``z_wide``.  Returns xyz, tets, wall-node mask, inlet faces, outlet faces,
    layer index per node (narrow layers first)."""
    pts, tris, rim = ogrid_disk(m, nr)
    nd = len(pts)
    # rim walk in angular order (the rim points of the O-grid, counter-clockwise)
    rim_idx = np.nonzero(rim)[0]
    ang = np.arctan2(pts[rim_idx, 1], pts[rim_idx, 0])
    walk = rim_idx[np.argsort(ang)]
    new, atris, outer = annulus_rings(pts, walk, n_rings, r_wide / r_step)
    nfull = nd + len(new)
    full_pts = np.concatenate([pts, new], 0)
    all_tris = np.concatenate([tris, atris], 0)
    K1 = len(z_narrow) - 1          # narrow layers below the step plane
    K2 = len(z_wide) - 1
    # node ids: narrow layers 0..K1-1 hold nd nodes; wide layers 0..K2 hold nfull
    n_narrow = K1 * nd
    N = n_narrow + (K2 + 1) * nfull
    xyz = np.empty((N, 3))
    layer_of = np.empty(N, np.int64)
    for lay in range(K1):
        z = z_narrow[lay]
        r = radius_of_z(z)
        s = slice(lay * nd, (lay + 1) * nd)
        xyz[s, 0], xyz[s, 1], xyz[s, 2] = r * pts[:, 0], r * pts[:, 1], z
        layer_of[s] = lay
    for lay in range(K2 + 1):
        z = z_wide[lay]
        s = slice(n_narrow + lay * nfull, n_narrow + (lay + 1) * nfull)
        xyz[s, 0], xyz[s, 1], xyz[s, 2] = r_step * full_pts[:, 0], r_step * full_pts[:, 1], z
        layer_of[s] = K1 + lay

    def gid_narrow(lay):  # disk nodes of narrow layer lay (lay == K1: the step layer)
        if lay < K1:
            return np.arange(lay * nd, (lay + 1) * nd)
        return n_narrow + np.arange(nd)

    def gid_wide(lay):
        return n_narrow + lay * nfull + np.arange(nfull)

    tets = [_prisms(tris, gid_narrow(l), gid_narrow(l + 1)) for l in range(K1)]
    tets += [_prisms(all_tris, gid_wide(l), gid_wide(l + 1)) for l in range(K2)]
    tets = _orient(xyz, np.concatenate(tets, 0))
    wall = np.zeros(N, dtype=bool)
    for lay in range(K1):
        wall[lay * nd + np.nonzero(rim)[0]] = True
    for lay in range(K2 + 1):
        wall[n_narrow + lay * nfull + np.nonzero(outer)[0]] = True
    # the step plane: the core rim (the corner of the step) and the annulus
    # nodes of the first wide layer (r_step <= r <= r_wide) are wall
    wall[n_narrow + np.nonzero(rim)[0]] = True
    wall[n_narrow + nd + np.arange(len(new))] = True
    inlet_faces = tris[:, [0, 2, 1]].astype(np.int32)
    outlet_faces = (all_tris + n_narrow + K2 * nfull).astype(np.int32)
    return xyz, tets, wall, inlet_faces, outlet_faces, layer_of
