"""Interface geometry for the oracle (FP64, NumPy).  Test infrastructure only.

Follows the implementation paragraph after Algorithm 1 (Sec. 6): place
quasi-uniform nodes on the boundary, compute normals / tangents / curvatures
there, classify grid nodes as lying in the tissue Omega ("+") or in its
complement ("-"), and locate every intersection of the boundary with the grid
lines (Sec. 5.3 assumes one crossing per stencil arm, at a point z with
x_k <= z < x_{k+1}).

Analytic shapes are star-shaped surfaces r = G(u), u = x/|x| (see the
workloads module); the level set of one surface is  phi = orient * (|x| - G(x/|x|)),
negative (or within 1e-12) in the tissue.  2D curves given by their nodes go
through the periodic cubic spline of the ``spline`` module instead.
"""
from __future__ import annotations

import math

import numpy as np

from .mesh import MeshError, TriMesh
from .spline import SplineCurve

SIDE_TOL = 1e-12          # nodes with phi <= SIDE_TOL count as tissue ("+")


class GeometryError(ValueError):
    pass


_CURVES = {}


def curve_of(surf):
    """The spline of a node-given 2D curve (built once per surface object)."""
    key = id(surf)
    hit = _CURVES.get(key)
    if hit is None or hit[0] is not surf:
        hit = (surf, SplineCurve(surf))
        _CURVES[key] = hit
    return hit[1]


def is_spline(surf):
    return getattr(surf, "kind", "analytic") == "spline"


def is_mesh(surf):
    return getattr(surf, "kind", "analytic") == "mesh"


_MESHES = {}


def trimesh_of(surf):
    """The triangle mesh of a mesh-given 3D surface (built once per surface object)."""
    key = id(surf)
    hit = _MESHES.get(key)
    if hit is None or hit[0] is not surf:
        try:
            hit = (surf, TriMesh(surf))
        except MeshError as e:
            raise GeometryError(str(e))
        _MESHES[key] = hit
    return hit[1]


def mesh_lines(tm, grid):
    """Crossings of the mesh with every grid line, per axis (cached per grid on the mesh)."""
    key = (grid.lo, grid.cells)
    cache = getattr(tm, "_lines", None)
    if cache is None or cache[0] != key:
        c = grid_coords(grid)
        tm._lines = (key, [tm.line_hits(a, c, c) for a in range(3)])
    return tm._lines[1]


def mesh_sides(tm, grid):
    """Tissue flags of the grid nodes for one mesh: parity of the crossings beyond the node on
    its x line; a node within 1e-12 of a crossing on any of its three lines is on the surface."""
    N = grid.n
    c = grid_coords(grid)
    lines = mesh_lines(tm, grid)
    interior = np.zeros((N, N, N), dtype=bool)           # [z][y][x]
    on = np.zeros((N, N, N), dtype=bool)
    for (iy, iz), hits in lines[0].items():
        xs = np.array([x for x, _ in hits])
        beyond = len(xs) - np.searchsorted(xs, c, side="right")
        interior[iz, iy, :] = beyond % 2 == 1
    for a in range(3):
        for (ib, ic), hits in lines[a].items():
            for x, _ in hits:
                k = int(round((x - grid.lo) / grid.h)) - 1
                if 0 <= k < N and abs(x - c[k]) <= SIDE_TOL:
                    idx = [0, 0, 0]
                    others = [b for b in range(3) if b != a]
                    idx[a], idx[others[0]], idx[others[1]] = k, ib, ic
                    on[idx[2], idx[1], idx[0]] = True
    return on, interior


# ----------------------------------------------------------------------------- radial function

def _pow(u, k):
    return u ** k if k >= 0 else np.zeros_like(u)


def radial(surf, u):
    """G(u) = E(u) (1 + P(u)) with its ambient gradient and Hessian at points u (n, d)."""
    u = np.asarray(u, dtype=np.float64)
    n, d = u.shape
    a2 = np.asarray(surf.axes, dtype=np.float64) ** 2
    q = np.sum(u * u / a2, axis=1)
    E = q ** -0.5
    c = u / a2
    gE = -(E ** 3)[:, None] * c
    HE = 3.0 * (E ** 5)[:, None, None] * c[:, :, None] * c[:, None, :] \
        - (E ** 3)[:, None, None] * np.diag(1.0 / a2)[None, :, :]
    P = np.zeros(n)
    gP = np.zeros((n, d))
    HP = np.zeros((n, d, d))
    for coef, e in surf.terms:
        e = list(e)
        P += coef * np.prod([_pow(u[:, i], e[i]) for i in range(d)], axis=0)
        for j in range(d):
            if e[j] == 0:
                continue
            ej = list(e)
            ej[j] -= 1
            gP[:, j] += coef * e[j] * np.prod([_pow(u[:, i], ej[i]) for i in range(d)], axis=0)
            for k in range(d):
                if ej[k] == 0:
                    continue
                ejk = list(ej)
                ejk[k] -= 1
                HP[:, j, k] += coef * e[j] * ej[k] * np.prod([_pow(u[:, i], ejk[i]) for i in range(d)], axis=0)
    G = E * (1.0 + P)
    g = (1.0 + P)[:, None] * gE + E[:, None] * gP
    H = (1.0 + P)[:, None, None] * HE + gE[:, :, None] * gP[:, None, :] \
        + gP[:, :, None] * gE[:, None, :] + E[:, None, None] * HP
    return G, g, H


def levelset(surf, x, order=0):
    """phi = orient (r - G(x/r)) and, for order >= 1/2, its gradient and Hessian.

    With rho(x) = G(x/r):  grad rho = P_u g / r  and
    Hess rho = (P_u H P_u - s P_u - u g_t^T - g_t u^T) / r^2,  s = u.g, g_t = P_u g.
    """
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(np.sum(x * x, axis=1))
    zero = r == 0.0
    u = x / np.where(zero, 1.0, r)[:, None]
    u[zero, 0] = 1.0                      # any direction at the origin (phi only)
    G, g, H = radial(surf, u)
    o = float(surf.orient)
    phi = o * (r - G)
    if order == 0:
        return phi
    d = x.shape[1]
    I = np.eye(d)[None]
    Pu = I - u[:, :, None] * u[:, None, :]
    gt = np.einsum("nij,nj->ni", Pu, g)
    grad = o * (u - gt / r[:, None])
    if order == 1:
        return phi, grad
    s = np.sum(u * g, axis=1)
    PHP = np.einsum("nij,njk,nkl->nil", Pu, H, Pu)
    hess_rho = (PHP - s[:, None, None] * Pu - u[:, :, None] * gt[:, None, :]
                - gt[:, :, None] * u[:, None, :]) / (r ** 2)[:, None, None]
    hess = o * (Pu / r[:, None, None] - hess_rho)
    return phi, grad, hess


def normal_and_shape(surf, x):
    """Unit normal n (out of the tissue) and shape operator W = P_n Hess(phi) P_n / |grad phi|.

    W is symmetric, annihilates n, and equals (1/R) on the tangent plane of a
    sphere of radius R that bounds the tissue from outside.
    """
    _, grad, hess = levelset(surf, x, order=2)
    gn = np.sqrt(np.sum(grad * grad, axis=1))
    n = grad / gn[:, None]
    d = x.shape[1]
    Pn = np.eye(d)[None] - n[:, :, None] * n[:, None, :]
    W = np.einsum("nij,njk,nkl->nil", Pn, hess, Pn) / gn[:, None, None]
    return n, W


# ----------------------------------------------------------------------------- interface nodes

def node_directions(dim, m):
    """Unit directions of the M nodes of one surface.

    2D: equally spaced angles t_j = 2 pi j / M.  3D: spherical Fibonacci
    lattice z_j = 1 - (2j+1)/M, azimuth j * pi (3 - sqrt 5).
    """
    j = np.arange(m, dtype=np.float64)
    if dim == 2:
        t = 2.0 * math.pi * j / m
        return np.stack([np.cos(t), np.sin(t)], axis=1)
    z = 1.0 - (2.0 * j + 1.0) / m
    az = j * (math.pi * (3.0 - math.sqrt(5.0)))
    rho = np.sqrt(1.0 - z * z)
    return np.stack([rho * np.cos(az), rho * np.sin(az), z], axis=1)


class Nodes:
    """All interface nodes, surfaces concatenated in descriptor order."""

    def __init__(self, iface):
        self.dim = iface.dim
        X, N, W, sid, par = [], [], [], [], []
        self.offsets = [0]
        for s, surf in enumerate(iface.surfaces):
            if is_spline(surf):
                cv = curve_of(surf)
                t = np.arange(cv.m, dtype=np.float64)
                x = cv.X(t)
                n, w = cv.normal_and_shape(t)
            elif is_mesh(surf):
                x, n, w = trimesh_of(surf).vertex_geometry()
            else:
                u = node_directions(iface.dim, surf.n_nodes)
                G, _, _ = radial(surf, u)
                x = G[:, None] * u
                n, w = normal_and_shape(surf, x)
            X.append(x), N.append(n), W.append(w)
            sid.append(np.full(surf.n_nodes, s))
            self.offsets.append(self.offsets[-1] + surf.n_nodes)
        self.X = np.concatenate(X)
        self.n = np.concatenate(N)
        self.W = np.concatenate(W)
        self.surf = np.concatenate(sid)
        self.M = self.X.shape[0]


def curve_tangent(surf, t):
    """2D: unit tangent (direction of increasing t) and speed |X'(t)| of X(t) = G(u(t)) u(t)."""
    t = np.asarray(t, dtype=np.float64)
    u = np.stack([np.cos(t), np.sin(t)], axis=1)
    up = np.stack([-np.sin(t), np.cos(t)], axis=1)
    G, g, _ = radial(surf, u)
    Xp = np.sum(g * up, axis=1)[:, None] * u + G[:, None] * up
    speed = np.sqrt(np.sum(Xp * Xp, axis=1))
    return Xp / speed[:, None], speed


# ----------------------------------------------------------------------------- grid

def grid_coords(grid):
    """Coordinates of the interior nodes along one axis: x_k = lo + k h, k = 1..I-1."""
    return grid.lo + grid.h * np.arange(1, grid.cells, dtype=np.float64)


def grid_points(grid):
    """(N^d, d) coordinates of all interior nodes in [z][y][x] order (x fastest)."""
    c = grid_coords(grid)
    if grid.dim == 2:
        yy, xx = np.meshgrid(c, c, indexing="ij")
        return np.stack([xx.ravel(), yy.ravel()], axis=1)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def linear_index(grid, idx):
    """Linear index of interior node with 0-based per-axis indices idx[..., a] (a=0 is x)."""
    N = grid.n
    lin = np.zeros(idx.shape[:-1], dtype=np.int64)
    for a in reversed(range(grid.dim)):
        lin = lin * N + idx[..., a]
    return lin


def classify(iface, grid):
    """Per-surface side flags (True = tissue side) at every interior node, shape (S, N^d)."""
    pts = grid_points(grid)
    out = np.zeros((len(iface.surfaces), pts.shape[0]), dtype=bool)
    chunk = 1 << 20
    for s, surf in enumerate(iface.surfaces):
        for i in range(0, pts.shape[0], chunk):
            if is_mesh(surf):
                on, interior = mesh_sides(trimesh_of(surf), grid)
                tissue = on | (interior if surf.orient == 1 else ~interior)
                out[s] = tissue.ravel()
                break
            if is_spline(surf):
                out[s, i:i + chunk] = curve_of(surf).tissue(pts[i:i + chunk])
            else:
                out[s, i:i + chunk] = levelset(surf, pts[i:i + chunk]) <= SIDE_TOL
    return out


def check_box_clearance(iface, grid, margin_cells=3):
    """The boundary must stay at least 3h inside the box (the stencils never reach it)."""
    lim = grid.hi - margin_cells * grid.h
    lim_lo = grid.lo + margin_cells * grid.h
    for surf in iface.surfaces:
        if is_spline(surf):
            _, x = curve_of(surf).samples(16)
        elif is_mesh(surf):
            x = trimesh_of(surf).V
        else:
            u = node_directions(iface.dim, max(surf.n_nodes, 4096 if iface.dim == 3 else 1024))
            G, _, _ = radial(surf, u)
            x = G[:, None] * u
        if np.any(x > lim) or np.any(x < lim_lo):
            raise GeometryError("interface closer than 3h to the box boundary")


def _root_on_arm(surf, p, axis, h, iters=80):
    """Safeguarded Newton for phi(p + t h e_axis) = 0, t in [0, 1], vectorised over arms.

    An end point with |phi| <= SIDE_TOL is taken as the crossing itself."""
    n = p.shape[0]

    def f(t):
        x = p.copy()
        x[:, axis] += t * h
        ph, gr = levelset(surf, x, order=1)
        return ph, gr[:, axis] * h

    f0, _ = f(np.zeros(n))
    f1, _ = f(np.ones(n))
    t = np.where(np.abs(f0) <= np.abs(f1), 0.0, 1.0)
    # an end point on the boundary (|phi| <= SIDE_TOL) is the crossing itself: near such a
    # node phi grows like t^2 along a tangent arm and the root is ill-conditioned
    on0, on1 = np.abs(f0) <= SIDE_TOL, np.abs(f1) <= SIDE_TOL
    t = np.where(on0, 0.0, np.where(on1, 1.0, t))
    bracket = (f0 * f1 <= 0.0) & ~on0 & ~on1
    # orient so that f(lo) <= 0 <= f(hi)
    lo = np.where(f0 <= 0.0, 0.0, 1.0)
    hi = 1.0 - lo
    denom = f1 - f0
    safe = np.where(denom != 0.0, denom, 1.0)
    t = np.where(bracket & (denom != 0.0), np.clip(-f0 / safe, 0.0, 1.0), t)
    active = bracket.copy()
    for _ in range(iters):
        if not np.any(active):
            break
        ft, dft = f(t)
        zero = ft == 0.0
        neg = ft < 0.0
        lo = np.where(active & neg, t, lo)
        hi = np.where(active & ~neg & ~zero, t, hi)
        dsafe = np.where(dft != 0.0, dft, 1.0)
        tn = t - ft / dsafe
        a, b = np.minimum(lo, hi), np.maximum(lo, hi)
        bad = (dft == 0.0) | ~((tn > a) & (tn < b))
        tn = np.where(bad, 0.5 * (lo + hi), tn)
        done = zero | (np.abs(tn - t) <= 1e-15)
        t = np.where(active & ~zero, tn, t)
        active = active & ~done
    return t


def _spline_roots_on_arms(cv, p0, axis, h, tol=1e-12):
    """Crossing of a spline curve with each arm from p0 to p0 + h e_axis: the arm fraction
    and the curve parameter.  An end point on the curve (|signed distance| <= 1e-12) is the
    crossing itself; otherwise exactly one root of the curve may lie on the arm."""
    other = 1 - axis
    frac = np.zeros(p0.shape[0])
    tpar = np.zeros(p0.shape[0])
    p1 = p0.copy()
    p1[:, axis] += h
    sd0, t0 = cv.closest(p0)
    sd1, t1 = cv.closest(p1)
    cache = {}
    for i in range(p0.shape[0]):
        if abs(sd0[i]) <= SIDE_TOL or abs(sd1[i]) <= SIDE_TOL:
            end0 = abs(sd0[i]) <= SIDE_TOL
            frac[i] = 0.0 if end0 else 1.0
            tpar[i] = t0[i] if end0 else t1[i]
            continue
        c = p0[i, other]
        if c not in cache:
            r = cv.line_roots(other, c)
            cache[c] = (r, cv.X(r)[:, axis] if r.size else np.zeros(0))
        r, xa = cache[c]
        on = (xa >= p0[i, axis] - tol) & (xa <= p0[i, axis] + h + tol)
        if np.count_nonzero(on) != 1:
            raise GeometryError("grid arm crossed more than once")
        k = int(np.flatnonzero(on)[0])
        frac[i] = min(1.0, max(0.0, (xa[k] - p0[i, axis]) / h))
        tpar[i] = r[k]
    return frac, tpar


def _mesh_roots_on_arms(tm, grid, idx0, p0, axis, h):
    """Crossing of a triangle mesh with each arm from p0 to p0 + h e_axis, moved onto the local
    quadratic patch of the triangle it passes through: arm fraction, n and W.  An end point on
    the surface is the crossing itself; otherwise exactly one crossing may lie on the arm."""
    lines = mesh_lines(tm, grid)[axis]
    others = [b for b in range(3) if b != axis]
    c = grid_coords(grid)
    n_arm = p0.shape[0]
    frac = np.zeros(n_arm)
    tri = np.zeros(n_arm, dtype=np.int64)
    nn = np.zeros((n_arm, 3))
    WW = np.zeros((n_arm, 3, 3))
    for i in range(n_arm):
        hits = lines.get((int(idx0[i, others[0]]), int(idx0[i, others[1]])), [])
        k0 = int(idx0[i, axis])
        x0, x1 = c[k0], c[k0 + 1]
        end = [(x, t) for x, t in hits if abs(x - x0) <= SIDE_TOL or abs(x - x1) <= SIDE_TOL]
        if end:
            x, t = min(end, key=lambda e: min(abs(e[0] - x0), abs(e[0] - x1)))
            at0 = abs(x - x0) <= SIDE_TOL
            z = p0[i].copy()
            if not at0:
                z[axis] = x1
            frac[i] = 0.0 if at0 else 1.0
            tri[i] = t
            nn[i], WW[i] = tm.patch_geometry(t, z)
            continue
        inarm = [(x, t) for x, t in hits if x0 - SIDE_TOL <= x <= x1 + SIDE_TOL]
        if len(inarm) != 1:
            raise GeometryError("grid arm crossed more than once")
        x, t = inarm[0]
        z, s, nn[i], WW[i] = tm.onto_patch(t, p0[i], axis, x - x0, h)
        frac[i] = s / h
        tri[i] = t
    return frac, nn, WW, tri


class Crossings:
    """All grid-arm / boundary intersections.

    For every arm between interior nodes p and p + e_axis whose end points lie
    on different sides of one surface: the surface id, the axis, the
    intersection z, the linear indices of its tissue-side ("plus") and
    complement-side ("minus") end points, and n, W at z.  ``tparam`` holds the spline
    parameter of the crossing on a spline curve, the index of the triangle it lies in on a
    mesh, NaN on an analytic surface.
    """

    def __init__(self, iface, grid, side):
        d, N, h = grid.dim, grid.n, grid.h
        shape = (N,) * d
        inside_all = np.all(side, axis=0)
        surf_l, axis_l, z_l, pin_l, pout_l, tparam_l = [], [], [], [], [], []
        mesh_nw = {}
        for s, surf in enumerate(iface.surfaces):
            sd = side[s].reshape(shape)
            others = np.all(np.delete(side, s, axis=0), axis=0).reshape(shape) \
                if side.shape[0] > 1 else np.ones(shape, dtype=bool)
            for a in range(d):
                ax = d - 1 - a                       # numpy axis of spatial axis a
                sl0 = [slice(None)] * d
                sl1 = [slice(None)] * d
                sl0[ax] = slice(0, N - 1)
                sl1[ax] = slice(1, N)
                diff = sd[tuple(sl0)] != sd[tuple(sl1)]
                if not np.any(diff):
                    continue
                if not np.all(others[tuple(sl0)][diff] & others[tuple(sl1)][diff]):
                    raise GeometryError("grid arm crosses two surfaces")
                base = np.argwhere(diff)             # numpy-order indices of the lower node
                idx0 = base[:, ::-1].copy()          # per spatial axis (x first)
                idx1 = idx0.copy()
                idx1[:, a] += 1
                p0 = grid.lo + (idx0 + 1) * h
                if is_spline(surf):
                    t, tp = _spline_roots_on_arms(curve_of(surf), p0, a, h)
                    tparam_l.append(tp)
                elif is_mesh(surf):
                    t, mn, mW, mt = _mesh_roots_on_arms(trimesh_of(surf), grid, idx0, p0, a, h)
                    tparam_l.append(mt.astype(np.float64))
                    mesh_nw[(s, a)] = (mn, mW)
                else:
                    t = _root_on_arm(surf, p0, a, h)
                    tparam_l.append(np.full(len(t), np.nan))
                # reject arms that the surface crosses more than once
                if not is_spline(surf) and not is_mesh(surf):
                    ts = np.linspace(0.0, 1.0, 9)
                    sides = []
                    for tt in ts:
                        x = p0.copy()
                        x[:, a] += tt * h
                        sides.append(levelset(surf, x) <= SIDE_TOL)
                    sides = np.stack(sides, axis=1)
                    if np.any(np.sum(sides[:, 1:] != sides[:, :-1], axis=1) != 1):
                        raise GeometryError("grid arm crossed more than once")
                z = p0.copy()
                z[:, a] += t * h
                lin0 = linear_index(grid, idx0)
                lin1 = linear_index(grid, idx1)
                in0 = sd[tuple(base.T)]
                surf_l.append(np.full(len(t), s))
                axis_l.append(np.full(len(t), a))
                z_l.append(z)
                pin_l.append(np.where(in0, lin0, lin1))
                pout_l.append(np.where(in0, lin1, lin0))
        if surf_l:
            self.surf = np.concatenate(surf_l)
            self.axis = np.concatenate(axis_l)
            self.z = np.concatenate(z_l)
            self.p_in = np.concatenate(pin_l)
            self.p_out = np.concatenate(pout_l)
            self.tparam = np.concatenate(tparam_l)
        else:
            self.surf = np.zeros(0, dtype=np.int64)
            self.axis = np.zeros(0, dtype=np.int64)
            self.z = np.zeros((0, d))
            self.p_in = np.zeros(0, dtype=np.int64)
            self.p_out = np.zeros(0, dtype=np.int64)
            self.tparam = np.zeros(0)
        self.count = len(self.surf)
        self.n = np.zeros((self.count, d))
        self.W = np.zeros((self.count, d, d))
        for s, surf in enumerate(iface.surfaces):
            m = self.surf == s
            if np.any(m) and is_mesh(surf):
                for a in range(d):
                    ma = m & (self.axis == a)
                    if np.any(ma):
                        self.n[ma], self.W[ma] = mesh_nw[(s, a)]
            elif np.any(m):
                if is_spline(surf):
                    self.n[m], self.W[m] = curve_of(surf).normal_and_shape(self.tparam[m])
                else:
                    self.n[m], self.W[m] = normal_and_shape(surf, self.z[m])
        self.inside = inside_all


def irregular_nodes(grid, crossings):
    """Sorted linear indices of the grid nodes whose stencil meets the boundary (Sec. 5.3)."""
    return np.unique(np.concatenate([crossings.p_in, crossings.p_out]))
