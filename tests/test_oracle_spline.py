"""Pins of the oracle's node-given 2D curves (periodic cubic splines through the nodes).

Checked against what geometry fixes: a circle's normals and curvature, the direction of
travel and the tissue side, grid-node sides against a brute-force point-in-polygon test of a
dense polyline, crossings that lie on the curve inside their arm, the analytic star that the
spline interpolates, and second-order convergence of a manufactured solution on spline
domains (the method's order, Sec. 7)."""
import numpy as np
import pytest

from oracle import geometry as og
from oracle import kfbi as ok
from oracle.spline import SplineCurve
from paper_2104_05024_amd import workloads as W


def test_circle_normals_and_curvature_converge():
    errs_n, errs_k = [], []
    for m in (64, 128, 256):
        cv = SplineCurve(W.spline_circle(0.5, m).surfaces[0])
        t = np.arange(m, dtype=np.float64)
        X = cv.X(t)
        n, Wm = cv.normal_and_shape(t)
        errs_n.append(np.max(np.abs(n - X / 0.5)))
        errs_k.append(np.max(np.abs(np.einsum("nii->n", Wm) - 2.0)))
        # W = k tau tau^T annihilates n
        assert np.max(np.abs(np.einsum("nij,nj->ni", Wm, n))) < 1e-12
    assert max(errs_n) < 1e-12                 # nodes on the circle: the normal is exact by symmetry
    rate = np.log2(errs_k[0] / errs_k[-1]) / 2
    assert errs_k[-1] < 2e-4 and rate > 1.8    # curvature error O(dt^2)


def test_direction_of_travel_and_tissue_side():
    t = np.arange(128, dtype=np.float64)
    ccw = SplineCurve(W.spline_circle(0.5, 128).surfaces[0])
    cw = SplineCurve(W.spline_circle(0.5, 128, clockwise=True).surfaces[0])
    out = SplineCurve(W.spline_circle(0.5, 128, orient=-1).surfaces[0])
    n1, W1 = ccw.normal_and_shape(t)
    n2, W2 = cw.normal_and_shape(t)
    n3, W3 = out.normal_and_shape(t)
    X1, X2 = ccw.X(t), cw.X(t)
    assert np.allclose(n1, X1 / 0.5, atol=1e-12) and np.allclose(n2, X2 / 0.5, atol=1e-12)
    assert np.allclose(np.einsum("nii->n", W1), np.einsum("nii->n", W2), atol=1e-12)
    assert np.allclose(n3, -n1, atol=1e-15) and np.allclose(W3, -W1, atol=1e-15)
    pts = np.array([[0.0, 0.1], [0.45, 0.0], [0.7, 0.2], [0.0, -0.55]])
    assert list(ccw.tissue(pts)) == [True, True, False, False]
    assert list(cw.tissue(pts)) == [True, True, False, False]
    assert list(out.tissue(pts)) == [False, False, True, True]


def _polygon_inside(poly, pts):
    """Even-odd ray casting against a closed polyline (brute force)."""
    x0, y0 = poly[:, 0], poly[:, 1]
    x1, y1 = np.roll(x0, -1), np.roll(y0, -1)
    inside = np.zeros(pts.shape[0], dtype=bool)
    for i in range(pts.shape[0]):
        px, py = pts[i]
        c = (y0 > py) != (y1 > py)
        xs = x0[c] + (py - y0[c]) * (x1[c] - x0[c]) / (y1[c] - y0[c])
        inside[i] = np.count_nonzero(xs > px) % 2 == 1
    return inside


def test_sides_match_a_dense_polygon():
    iface, grid = W.heart2d(256), W.box(2, 64)
    cv = og.curve_of(iface.surfaces[0])
    side = og.classify(iface, grid)[0]
    tt, dense = cv.samples(256)
    pts = og.grid_points(grid)
    ref = _polygon_inside(dense, pts)
    sd = cv.signed_distance(pts)
    # the polyline is within ~1e-9 of the spline: only nodes that close could differ
    differ = side != ref
    assert np.all(np.abs(sd[differ]) < 1e-8)
    assert np.count_nonzero(differ) == 0
    assert 0.25 < side.mean() < 0.35           # heart area about 1.7 in the 2.4^2 box


def test_crossings_lie_on_the_curve_inside_their_arm():
    iface, grid = W.heart2d(256), W.box(2, 128)
    o = ok.Problem(iface, grid, W.scalar_coeffs(2))
    cr = o.cross
    cv = og.curve_of(iface.surfaces[0])
    assert np.max(np.abs(cv.X(cr.tparam) - cr.z)) < 1e-12
    for c in range(cr.count):
        a = cr.axis[c]
        za = o.node_coord(cr.p_in[c], a), o.node_coord(cr.p_out[c], a)
        assert min(za) - 1e-12 <= cr.z[c, a] <= max(za) + 1e-12
    # every arm with ends on different sides has exactly one crossing, and no other arm has one
    N = grid.n
    ins = o.inside.reshape(N, N)
    flips = np.count_nonzero(ins[:, 1:] != ins[:, :-1]) + np.count_nonzero(ins[1:, :] != ins[:-1, :])
    assert flips == cr.count
    # normals point out of the tissue: stepping along n leaves it
    step = cr.z + 1e-4 * cr.n
    assert not np.any(cv.tissue(step))


def test_spline_through_star_nodes_approaches_the_analytic_star():
    """The spline through the analytic star's own nodes converges to it: normals, shape operators
    and the operator A psi on the same density."""
    grid = W.box(2, 128)
    co = W.scalar_coeffs(2, 1.0, 400.0)
    errs = []
    for m in (256, 512):
        a = ok.Problem(W.star2d(n_nodes=m), grid, co)
        s = ok.Problem(W.spline_star(n_nodes=m), grid, co)
        assert np.allclose(a.nodes.X, s.nodes.X, atol=1e-15)
        assert np.max(np.abs(a.nodes.n - s.nodes.n)) < 5e-4 * (256 / m) ** 2
        assert np.array_equal(a.inside, s.inside)
        assert a.cross.count == s.cross.count
        assert np.max(np.abs(a.cross.z - s.cross.z)) < 1e-6
        t = 2 * np.pi * np.arange(m) / m
        psi = np.cos(3 * t) + 0.5 * np.sin(t)
        ra, rs = a.apply(psi[None])[0], s.apply(psi[None])[0]
        errs.append(np.linalg.norm(ra - rs) / np.linalg.norm(ra))
    assert errs[1] < errs[0] / 3 and errs[1] < 1e-3


@pytest.mark.parametrize("shape", ["heart", "circle"])
def test_manufactured_solution_second_order_on_spline_domains(shape):
    """u = e^x sin(pi y), kappa = 400, Neumann data from the exact gradient at the nodes:
    max-norm error in the tissue falls like h^2."""
    errs = []
    for cells in (64, 128):
        iface = W.heart2d(2 * cells) if shape == "heart" else W.spline_circle(0.6, 2 * cells)
        grid = W.box(2, cells)
        co = W.scalar_coeffs(2, 1.0, 400.0)
        o = ok.Problem(iface, grid, co)
        pts = og.grid_points(grid)
        ue = np.exp(pts[:, 0]) * np.sin(np.pi * pts[:, 1])
        X, n = o.nodes.X, o.nodes.n
        grad = np.stack([np.exp(X[:, 0]) * np.sin(np.pi * X[:, 1]),
                         np.pi * np.exp(X[:, 0]) * np.cos(np.pi * X[:, 1])], 1)
        f = (np.pi ** 2 - 1 + co.kappa) * ue
        u, _, info = o.solve_neumann(np.sum(n * grad, 1)[None], f[None], tol=1e-12)
        errs.append(np.max(np.abs(u[0] - ue)[o.inside]))
        assert errs[-1] < 0.4 * grid.h ** 2
    assert np.log2(errs[0] / errs[1]) > 1.7
