"""Validity of the seeded synthetic workloads (CPU): conforming positively
oriented tetrahedra, outlet caps that are planar, outward oriented and
disjoint, and Dirichlet sets that cover the wall.  The large workloads share
their generators with the small ones checked here."""
import numpy as np
import pytest

from ns_inputs import build, meshes

SMALL = ["cube", "channel2", "pipe_tiny", "ybif_small", "conexp_small", "plate_small", "unstr_channel"]


def _faces(tets):
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    return np.sort(tets[:, loc].reshape(-1, 3), axis=1)


@pytest.mark.parametrize("name", SMALL)
def test_mesh_conforming_and_oriented(name):
    c = build(name)
    p = c.xyz[c.tets]
    det = np.einsum("ei,ei->e", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    assert (det > 0).all()
    _, cnt = np.unique(_faces(c.tets), axis=0, return_counts=True)
    assert cnt.max() <= 2
    # every node belongs to an element
    assert len(np.unique(c.tets)) == c.n_nodes


@pytest.mark.parametrize("name", ["channel2", "pipe_tiny", "ybif_small", "conexp_small", "plate_small",
                                  "unstr_channel"])
def test_outlets_planar_outward_disjoint(name):
    c = build(name)
    bf = {tuple(f) for f in np.sort(meshes.boundary_faces(c.xyz, c.tets), axis=1)}
    seen = set()
    for k in range(c.n_outlets):
        f = c.faces[c.outlet_ptr[k]:c.outlet_ptr[k + 1]]
        assert len(f) > 0
        assert all(tuple(t) in bf for t in np.sort(f, axis=1))   # on the boundary
        nodes = set(np.unique(f).tolist())
        assert not (nodes & seen)                                 # disjoint caps
        seen |= nodes
        n = meshes.face_normals(c.xyz, f)
        assert np.allclose(n, n[0], atol=1e-12)                   # planar
        cen = c.xyz[f].mean(axis=1)
        # outward: the normal points away from the mesh centroid side
        inner = c.xyz[np.unique(c.tets)].mean(axis=0)
        assert np.all(np.einsum("fi,i->f", cen - inner, n[0]) > 0)


@pytest.mark.parametrize("name", ["pipe_tiny", "ybif_small", "conexp_small", "plate_small"])
def test_wall_is_dirichlet_and_outlet_interior_is_free(name):
    c = build(name)
    bf = meshes.boundary_faces(c.xyz, c.tets)
    key = {tuple(t) for t in np.sort(c.faces, axis=1)}
    zmin = c.xyz[:, 2].min()
    inlet = np.all(np.abs(c.xyz[bf][:, :, 2] - zmin) < 1e-9, axis=1)
    out = np.array([tuple(t) in key for t in np.sort(bf, axis=1)])
    wall_nodes = np.unique(bf[~inlet & ~out])
    assert c.mask[wall_nodes, :3].all()
    assert c.mask[np.unique(bf[inlet]), :3].all()
    assert (c.v[wall_nodes] == 0).all()
    free_out = np.setdiff1d(np.unique(c.faces), wall_nodes)
    assert len(free_out) > 0 and not c.mask[free_out, :3].any()
    assert not c.mask[:, 3].any()                                 # outlets fix the pressure level


def test_ybif_branch_flow_split():
    c = build("ybif_small")
    # the imposed inflow, integrated over the inlet cap, is shared equally by
    # the daughters in the state (before noise): check the outlet-normal flux
    # of the state over each cap agrees within the noise and staircase error
    flux = []
    for k in range(2):
        f = c.faces[c.outlet_ptr[k]:c.outlet_ptr[k + 1]]
        n = np.cross(c.xyz[f[:, 1]] - c.xyz[f[:, 0]], c.xyz[f[:, 2]] - c.xyz[f[:, 0]]) / 2.0
        flux.append(np.sum(np.einsum("fi,fi->f", c.v[f].mean(axis=1), n)))
    assert flux[0] > 0 and flux[1] > 0
    assert abs(flux[0] - flux[1]) <= 0.1 * max(flux)


def test_conexp_throat_reynolds_number():
    c = build("conexp_small")
    u_t = c.meta["u_t"]
    assert np.isclose(u_t * 2 * 0.2 * c.rho / c.mu, 3500.0)
    zmin = c.xyz[:, 2].min()
    inlet = np.abs(c.xyz[:, 2] - zmin) < 1e-12
    r = np.hypot(c.xyz[inlet, 0], c.xyz[inlet, 1])
    # parabolic inflow with the throat's flow rate: peak 2 u_t (r_t / r_i)^2
    assert np.isclose(c.v[inlet, 2].max(), 2 * u_t * (0.2 / 0.6) ** 2, rtol=1e-12)
    assert np.all(c.v[inlet][r > 0.6 - 1e-9] == 0)


def test_plate_outlet_patches():
    c = build("plate_small")
    npch, q = c.meta["patches"], c.meta["q"]
    assert c.n_outlets == npch * npch
    rcr = c.meta["rcr"]
    assert np.allclose(rcr["Rp"] + rcr["Rd"], c.R) and (rcr["C"] > 0).all()
    for k in range(c.n_outlets):
        f = c.faces[c.outlet_ptr[k]:c.outlet_ptr[k + 1]]
        assert len(f) == 2 * q * q                                # q x q quads, two triangles each
        nodes = np.unique(f)
        assert (c.mask[nodes, 0] == 0).sum() == (q - 1) ** 2      # interior nodes are free, the rim is wall
        area = 0.5 * np.linalg.norm(np.cross(c.xyz[f[:, 1]] - c.xyz[f[:, 0]], c.xyz[f[:, 2]] - c.xyz[f[:, 0]]),
                                    axis=1).sum()
        n_quads = npch * (q + 1) + 1
        assert np.isclose(area, (q / n_quads) ** 2)


def test_unstructured_channel_is_irregular_and_fills_the_box():
    """The Delaunay channel fills [0,2]x[0,1]x[0,1] exactly, its boundary is
    the box surface, and its node degrees exceed the Kuhn lattice's (so rows
    longer than 16 blocks and S_hat rows of irregular length occur)."""
    c = build("unstr_channel")
    p = c.xyz[c.tets]
    vol = np.einsum("ei,ei->e", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6.0
    assert abs(vol.sum() - 2.0) < 1e-12
    fx = c.xyz[meshes.boundary_faces(c.xyz, c.tets)]
    on = np.zeros(len(fx), bool)
    for a, L in enumerate((2.0, 1.0, 1.0)):
        on |= np.all(np.abs(fx[:, :, a]) < 1e-12, axis=1) | np.all(np.abs(fx[:, :, a] - L) < 1e-12, axis=1)
    assert on.all()
    nbr = [set() for _ in range(c.n_nodes)]
    for t in c.tets:
        for a in t:
            nbr[a].update(t.tolist())
    deg = np.array([len(s) for s in nbr])
    assert deg.max() > 16 and deg.min() < 10
    # the wall (every boundary node off the outlet interior) is no-slip
    x, y, z = c.xyz.T
    outlet_interior = (np.abs(x - 2.0) < 1e-12) & (y > 1e-12) & (y < 1 - 1e-12) & (z > 1e-12) & (z < 1 - 1e-12)
    bnd = np.unique(meshes.boundary_faces(c.xyz, c.tets))
    wall = np.setdiff1d(bnd, np.nonzero(outlet_interior)[0])
    assert c.mask[wall, :3].all() and not c.mask[outlet_interior, :3].any()
