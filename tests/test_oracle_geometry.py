"""Pins for oracle.geometry against closed forms and finite differences (CPU only)."""
import math

import numpy as np
import pytest

from oracle import geometry
from paper_2104_05024_amd import workloads as W


def _surfaces():
    return [W.star2d().surfaces[0], W.ellipsoid().surfaces[0],
            W.perturbed_sphere().surfaces[0]] + W.thick_shell().surfaces


@pytest.mark.parametrize("k", range(5))
def test_radial_derivatives_match_finite_differences(k):
    surf = _surfaces()[k]
    d = len(surf.axes)
    rng = np.random.default_rng(k)
    u = rng.normal(size=(7, d))
    u /= np.linalg.norm(u, axis=1)[:, None]
    G, g, H = geometry.radial(surf, u)
    eps = 1e-5
    for a in range(d):
        e = np.zeros(d)
        e[a] = eps
        Gp, gp, _ = geometry.radial(surf, u + e)
        Gm, gm, _ = geometry.radial(surf, u - e)
        np.testing.assert_allclose((Gp - Gm) / (2 * eps), g[:, a], rtol=1e-7, atol=1e-8)
        np.testing.assert_allclose((gp - gm) / (2 * eps), H[:, :, a], rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("k", range(5))
def test_levelset_gradient_and_hessian_match_finite_differences(k):
    surf = _surfaces()[k]
    d = len(surf.axes)
    rng = np.random.default_rng(10 + k)
    x = rng.uniform(-0.9, 0.9, size=(6, d))
    _, grad, hess = geometry.levelset(surf, x, order=2)
    eps = 1e-5
    for a in range(d):
        e = np.zeros(d)
        e[a] = eps
        fp, gp = geometry.levelset(surf, x + e, order=1)
        fm, gm = geometry.levelset(surf, x - e, order=1)
        np.testing.assert_allclose((fp - fm) / (2 * eps), grad[:, a], rtol=1e-7, atol=1e-8)
        np.testing.assert_allclose((gp - gm) / (2 * eps), hess[:, :, a], rtol=1e-6, atol=1e-6)


def test_star_curvature_matches_polar_formula():
    """Curvature of r(t) = 0.7 + 0.15 cos 5t: (r^2 + 2r'^2 - r r'') / (r^2 + r'^2)^{3/2}."""
    surf = W.star2d().surfaces[0]
    t = np.linspace(0, 2 * np.pi, 101)
    u = np.stack([np.cos(t), np.sin(t)], 1)
    G, _, _ = geometry.radial(surf, u)
    r, rp, rpp = 0.7 + 0.15 * np.cos(5 * t), -0.75 * np.sin(5 * t), -3.75 * np.cos(5 * t)
    np.testing.assert_allclose(G, r, atol=1e-15)
    n, Wm = geometry.normal_and_shape(surf, G[:, None] * u)
    c = (r * r + 2 * rp * rp - r * rpp) / (r * r + rp * rp) ** 1.5
    np.testing.assert_allclose(np.trace(Wm, axis1=1, axis2=2), c, rtol=1e-12, atol=1e-12)
    # outward normal: n . x > 0 for a star-shaped curve
    assert np.all(np.sum(n * u, axis=1) > 0)


def test_ellipsoid_gauss_and_mean_curvature():
    """Gaussian curvature 1/(a^2 b^2 c^2 (x^2/a^4 + y^2/b^4 + z^2/c^4)^2) and mean curvature."""
    a, b, c = 0.9, 0.7, 0.5
    surf = W.ellipsoid(a, b, c).surfaces[0]
    u = geometry.node_directions(3, 200)
    G, _, _ = geometry.radial(surf, u)
    x = G[:, None] * u
    np.testing.assert_allclose(np.sum(x * x / np.array([a, b, c]) ** 2, axis=1), 1.0, atol=1e-14)
    n, Wm = geometry.normal_and_shape(surf, x)
    q = x[:, 0] ** 2 / a ** 4 + x[:, 1] ** 2 / b ** 4 + x[:, 2] ** 2 / c ** 4
    K = 1.0 / (a * a * b * b * c * c * q * q)
    ev = np.linalg.eigvalsh(Wm)                  # one eigenvalue is 0 (normal direction)
    ev = np.sort(ev, axis=1)
    kprod = np.where(np.abs(ev[:, 0]) < 1e-12, ev[:, 1] * ev[:, 2], ev[:, 0] * ev[:, 1])
    np.testing.assert_allclose(kprod, K, rtol=1e-10)
    # mean curvature: |x|^2 - a^2 - b^2 - c^2 form (e.g. standard closed form)
    Hm = (np.sum(x * x, axis=1) - a * a - b * b - c * c) / (2 * (a * b * c) ** 2 * q ** 1.5)
    np.testing.assert_allclose(np.trace(Wm, axis1=1, axis2=2) / 2, -Hm, rtol=1e-10)
    np.testing.assert_allclose(np.einsum("nij,nj->ni", Wm, n), 0.0, atol=1e-12)


def test_sphere_shape_operator_and_inner_orientation():
    R = 0.6
    outer = W.sphere(R).surfaces[0]
    inner = W.Surface((R, R, R), -1, 10, [])
    u = geometry.node_directions(3, 50)
    x = R * u
    n, Wm = geometry.normal_and_shape(outer, x)
    P = np.eye(3)[None] - u[:, :, None] * u[:, None, :]
    np.testing.assert_allclose(n, u, atol=1e-14)
    np.testing.assert_allclose(Wm, P / R, atol=1e-13)
    n2, W2 = geometry.normal_and_shape(inner, x)
    np.testing.assert_allclose(n2, -u, atol=1e-14)
    np.testing.assert_allclose(W2, -P / R, atol=1e-13)


def test_nodes_lie_on_surfaces():
    iface = W.thick_shell(n_nodes=4000)
    nd = geometry.Nodes(iface)
    assert nd.M == 4000
    for s, surf in enumerate(iface.surfaces):
        m = nd.surf == s
        np.testing.assert_allclose(geometry.levelset(surf, nd.X[m]), 0.0, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(nd.n, axis=1), 1.0, atol=1e-14)


def test_fibonacci_directions_are_unit_and_balanced():
    u = geometry.node_directions(3, 1000)
    np.testing.assert_allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-14)
    assert abs(np.mean(u[:, 2])) < 1e-12
    assert np.all(np.abs(np.mean(u, axis=0)) < 5e-3)


@pytest.mark.parametrize("name,cells", [("star", 64), ("ellipsoid", 32), ("shell", 32)])
def test_crossings_are_on_the_surface_and_between_sides(name, cells):
    if name == "star":
        iface, grid = W.star2d(n_nodes=128), W.box(2, cells)
    elif name == "ellipsoid":
        iface, grid = W.ellipsoid(n_nodes=512), W.box(3, cells)
    else:
        iface, grid = W.thick_shell(n_nodes=1000), W.box(3, cells)
    side = geometry.classify(iface, grid)
    cr = geometry.Crossings(iface, grid, side)
    inside = np.all(side, axis=0)
    assert cr.count > 0
    assert np.all(inside[cr.p_in]) and not np.any(inside[cr.p_out])
    for s, surf in enumerate(iface.surfaces):
        m = cr.surf == s
        np.testing.assert_allclose(geometry.levelset(surf, cr.z[m]), 0.0, atol=1e-13)
    # the number of crossings equals the number of side changes along grid lines
    N, d = grid.n, grid.dim
    ins = inside.reshape((N,) * d)
    changes = sum(int(np.sum(np.diff(ins.astype(np.int8), axis=ax) != 0)) for ax in range(d))
    assert changes == cr.count
    # z lies on the arm between the two nodes
    pts = geometry.grid_points(grid)
    lo = np.minimum(pts[cr.p_in], pts[cr.p_out]) - 1e-15
    hi = np.maximum(pts[cr.p_in], pts[cr.p_out]) + 1e-15
    assert np.all((cr.z >= lo) & (cr.z <= hi))


def test_batch_2d_draws_are_seeded_and_resolved():
    """The batch generator is deterministic, covers the sizes, and every drawn star keeps its
    smallest radius of curvature above 2h, checked with the oracle's shape operator (in 2D
    tr W is the curvature) on points of the curve, independently of the generator's formula."""
    a, b = W.batch_2d(), W.batch_2d()
    assert len(a) == 64
    assert [(g.cells, c.kappa) for _, g, c in a] == [(g.cells, c.kappa) for _, g, c in b]
    assert {g.cells for _, g, _ in a} == {64, 128, 256, 512, 1024}
    t = np.linspace(0, 2 * np.pi, 4096, endpoint=False)
    u = np.stack([np.cos(t), np.sin(t)], axis=1)
    for iface, grid, co in a:
        assert 50.0 <= co.kappa <= 2000.0
        assert iface.n_nodes == 2 * grid.cells
        surf = iface.surfaces[0]
        G, _, _ = geometry.radial(surf, u)
        _, Wm = geometry.normal_and_shape(surf, G[:, None] * u)
        curv = np.abs(np.trace(Wm, axis1=1, axis2=2))
        assert 1.0 / np.max(curv) >= 2.0 * grid.h * (1 - 1e-3)
