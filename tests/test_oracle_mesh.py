"""Pins of the oracle's mesh-given 3D surfaces (closed triangle meshes with local quadratic
coordinate systems).

Checked against what geometry fixes: an icosphere on a sphere (exact normals R^-1 x and
shape operator P_n / R), grid-node sides against the exact ball, crossings on the sphere,
the direction of the triangles and the tissue side, mesh validity checks, and the
manufactured solution on a mesh ellipsoid (second order, no worse than the analytic
ellipsoid with as many nodes)."""
import numpy as np
import pytest

from oracle import geometry as og
from oracle import kfbi as ok
from oracle.mesh import MeshError, TriMesh
from paper_2104_05024_amd import workloads as W


def test_vertex_normals_and_curvature_on_a_sphere_converge():
    en, eW = [], []
    for L in (3, 4):
        tm = TriMesh(W.mesh_sphere(0.5, L).surfaces[0])
        X, n, Wm = tm.vertex_geometry()
        u = X / np.linalg.norm(X, axis=1)[:, None]
        en.append(np.max(np.linalg.norm(n - u, axis=1)))
        P = np.eye(3)[None] - n[:, :, None] * n[:, None, :]
        eW.append(np.max(np.abs(Wm - P / 0.5)))
        assert np.max(np.abs(np.einsum("nij,nj->ni", Wm, n))) < 1e-12      # W annihilates n
        assert np.max(np.abs(Wm - np.transpose(Wm, (0, 2, 1)))) < 1e-12     # and is symmetric
    assert en[-1] < 2e-5 and en[0] / en[1] > 6          # normals O(h^3) on the symmetric mesh
    assert eW[-1] < 5e-3 and eW[0] / eW[1] > 3          # curvature O(h^2)


def test_sides_and_crossings_on_a_sphere():
    errs = []
    for L, cells in ((3, 32), (4, 64)):
        iface, grid = W.mesh_sphere(0.5, L), W.box(3, cells)
        side = og.classify(iface, grid)
        pts = og.grid_points(grid)
        r = np.linalg.norm(pts, axis=1)
        differ = side[0] != (r <= 0.5)
        # the flat mesh lies within (edge length)^2 / (8 R) of the sphere: only nodes that close
        assert np.all(np.abs(r[differ] - 0.5) < 2e-3)
        cr = og.Crossings(iface, grid, side)
        N = grid.n
        ins = cr.inside.reshape(N, N, N)
        flips = sum(np.count_nonzero(np.diff(ins, axis=ax)) for ax in range(3))
        assert flips == cr.count
        dist = np.abs(np.linalg.norm(cr.z, axis=1) - 0.5)
        errs.append(np.max(dist))
        u = cr.z / np.linalg.norm(cr.z, axis=1)[:, None]
        assert np.max(np.linalg.norm(cr.n - u, axis=1)) < 2e-3
        # every crossing lies on its arm
        for c in range(0, cr.count, 7):
            a = cr.axis[c]
            za = sorted(grid.lo + ((p // N ** a) % N + 1) * grid.h for p in (cr.p_in[c], cr.p_out[c]))
            assert za[0] - 1e-12 <= cr.z[c, a] <= za[1] + 1e-12
    assert errs[1] < 3e-6 and errs[0] / errs[1] > 8        # the six-point patches: O(h^3) or better


def test_triangle_direction_and_tissue_side():
    grid = W.box(3, 32)
    a = W.mesh_ellipsoid(level=3)
    b = W.mesh_ellipsoid(level=3, flip=True)
    oa, ob = ok.Problem(a, grid, W.scalar_coeffs(3)), ok.Problem(b, grid, W.scalar_coeffs(3))
    assert np.allclose(oa.nodes.n, ob.nodes.n, atol=1e-13) and np.allclose(oa.nodes.W, ob.nodes.W, atol=1e-12)
    assert np.array_equal(oa.inside, ob.inside) and np.allclose(oa.cross.z, ob.cross.z, atol=1e-14)
    s = a.surfaces[0]
    out = W.mesh_surface(s.points, s.tris, orient=-1)
    tm_in, tm_out = TriMesh(s), TriMesh(out)
    _, n1, W1 = tm_in.vertex_geometry()
    _, n2, W2 = tm_out.vertex_geometry()
    assert np.allclose(n2, -n1, atol=1e-15) and np.allclose(W2, -W1, atol=1e-15)
    side_in = og.classify(W.Interface(3, [s]), grid)[0]
    side_out = og.classify(W.Interface(3, [out]), grid)[0]
    assert np.array_equal(side_out, ~side_in)              # no grid node lies on this mesh


def test_invalid_meshes_are_rejected():
    V, F = W.icosphere(1)
    with pytest.raises(MeshError):
        TriMesh(W.mesh_surface(V, F[:-1]))                  # a hole
    G = F.copy()
    G[0] = G[0, ::-1]
    with pytest.raises(MeshError):
        TriMesh(W.mesh_surface(V, G))                       # one triangle turned over
    with pytest.raises(MeshError):
        TriMesh(W.mesh_surface(V, np.where(F == 3, 99, F)))  # index out of range


def _mms3(o, grid, kappa):
    pts = og.grid_points(grid)
    ue = np.exp(pts[:, 0]) * np.sin(np.pi * pts[:, 1]) * np.cos(pts[:, 2])
    X, n = o.nodes.X, o.nodes.n
    g = np.stack([np.exp(X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.cos(X[:, 2]),
                  np.pi * np.exp(X[:, 0]) * np.cos(np.pi * X[:, 1]) * np.cos(X[:, 2]),
                  -np.exp(X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(X[:, 2])], 1)
    return (np.pi ** 2 + kappa) * ue, np.sum(n * g, 1), ue


def test_manufactured_solution_on_a_mesh_ellipsoid():
    """u = e^x sin(pi y) cos z, kappa = 400: the error on the mesh ellipsoid falls at about second
    order and stays within 10% of the analytic ellipsoid's with as many nodes."""
    errs = []
    for L, cells in ((3, 32), (4, 64)):
        grid = W.box(3, cells)
        co = W.scalar_coeffs(3, 1.0, 400.0)
        res = []
        for iface in (W.mesh_ellipsoid(level=L), W.ellipsoid(n_nodes=10 * 4 ** L + 2)):
            o = ok.Problem(iface, grid, co)
            f, g, ue = _mms3(o, grid, co.kappa)
            u, _, info = o.solve_neumann(g[None], f[None], tol=1e-12)
            res.append(np.max(np.abs(u[0] - ue)[o.inside]))
        errs.append(res[0])
        assert res[0] < 1.1 * res[1]
        assert res[0] < 0.3 * grid.h ** 2
    assert np.log2(errs[0] / errs[1]) > 1.5


def test_six_point_transfer_of_a_linear_function():
    """psi = x on a sphere mesh: on the six-point patches x is itself the quadratic interpolant,
    so psi at the crossings is exact; the surface gradient P_n e_x converges at about third
    order at crossings and vertices; unused slots carry no weight."""
    errs_c, errs_q = [], []
    for L, cells in ((3, 32), (4, 64)):
        o = ok.Problem(W.mesh_sphere(0.5, L), W.box(3, cells), W.scalar_coeffs(3))
        psi = o.nodes.X[:, 0]
        p0 = np.sum(o.z_w0 * psi[o.z_idx], axis=1)
        assert np.max(np.abs(p0 - o.cross.z[:, 0])) < 1e-13
        assert np.all(o.z_w0[:, 6:] == 0) and np.all(o.z_wg[:, 6:] == 0)
        u = o.cross.z / np.linalg.norm(o.cross.z, axis=1)[:, None]
        g = np.einsum("nk,nkd->nd", psi[o.z_idx], o.z_wg)
        errs_c.append(np.max(np.abs(g - (np.array([1.0, 0, 0])[None] - u * u[:, :1]))))
        un = o.nodes.X / np.linalg.norm(o.nodes.X, axis=1)[:, None]
        gq = np.einsum("nk,nkd->nd", psi[o.q_idx], o.q_wg)
        errs_q.append(np.max(np.abs(gq - (np.array([1.0, 0, 0])[None] - un * un[:, :1]))))
        # the gradient is tangent to the patch: orthogonal to the patch normal at the crossing
        assert np.max(np.abs(np.sum(g * o.cross.n, axis=1))) < 1e-12
    assert errs_c[1] < 1e-4 and errs_c[0] / errs_c[1] > 5
    assert errs_q[1] < 1.5e-5 and errs_q[0] / errs_q[1] > 5
