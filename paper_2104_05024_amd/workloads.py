"""Seeded synthetic workloads: interface, grid and coefficient descriptors.

This module only *describes* problems (shapes as coefficient lists, grid sizes,
physical constants, seeded random numbers).  It holds none of the method's
arithmetic, so both the HIP path and the FP64 CPU checker take their inputs
from here without sharing any computation.

Every interface is a union of closed surfaces (curves in 2D).  A surface is
either analytic, star-shaped in polar form  r = R(u),  u = x/|x|,

    R(u) = E(u) * (1 + sum_t c_t * prod_i u_i**e_ti),
    E(u) = (sum_i u_i**2 / a_i**2) ** (-1/2)          (ellipse / ellipsoid)

or given only by its nodes: a closed 2D curve through ordered points (the method
interpolates them with a periodic cubic spline), or a closed 3D triangle mesh
(vertices and triangles).  ``orient = +1`` puts the tissue (the "+" side) inside
the surface, ``-1`` outside it (the inner wall of a shell).  The tissue region
is the intersection of the per-surface regions.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Surface:
    axes: Tuple[float, ...]
    orient: int
    n_nodes: int
    terms: List[Tuple[float, Tuple[int, ...]]] = field(default_factory=list)
    kind: str = "analytic"              # "analytic", "spline" (2D points) or "mesh" (3D triangles)
    points: Optional[np.ndarray] = None  # (n_nodes, dim) node coordinates of a spline / mesh
    tris: Optional[np.ndarray] = None    # (n_tris, 3) vertex indices of a mesh


@dataclass
class Interface:
    dim: int
    surfaces: List[Surface]

    @property
    def n_nodes(self) -> int:
        return sum(s.n_nodes for s in self.surfaces)


@dataclass
class Grid:
    dim: int
    lo: float
    hi: float
    cells: int          # I intervals per axis; unknowns are the (I-1)^dim interior nodes

    @property
    def n(self) -> int:
        return self.cells - 1

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.cells


@dataclass
class Coeffs:
    ncomp: int
    D: List[List[float]]      # D[c][axis]
    kappa: float


@dataclass
class BidomainParams:
    Cm: float = 1.0
    beta: float = 1.0
    H: float = 100.0          # FitzHugh-Nagumo: I_ion = H (q - V (V - theta)(1 - V))
    theta: float = 0.13
    alpha: float = 0.25       # M(V, q) = alpha V - zeta q
    zeta: float = 1.0
    sigma_i: float = 1.0
    sigma_e: float = 2.0
    newton_tol: float = 1e-10
    newton_maxit: int = 50


# ----------------------------------------------------------------------------- shapes

def _star_terms(R0: float, A: float, L: int):
    """Terms of (A/R0) * Re((u_x + i u_y)^L): the polar curve R0 + A cos(L t)."""
    terms = []
    for k in range(0, L + 1, 2):
        c = math.comb(L, k) * (-1) ** (k // 2) * A / R0
        terms.append((float(c), (L - k, k)))
    return terms


def star2d(R0=0.7, A=0.15, L=5, n_nodes=256) -> Interface:
    return Interface(2, [Surface((R0, R0), +1, n_nodes, _star_terms(R0, A, L))])


def circle2d(R=0.5, n_nodes=256) -> Interface:
    return Interface(2, [Surface((R, R), +1, n_nodes, [])])


def spline_curve(points, orient=+1) -> Surface:
    """A closed curve through the ordered points (n, 2), either direction of travel."""
    P = np.ascontiguousarray(points, dtype=np.float64)
    return Surface((1.0, 1.0), orient, P.shape[0], [], kind="spline", points=P)


def _resample_closed(x, y, n, jitter, seed):
    """n quasi-uniform points on a densely sampled closed curve: equal arc-length steps, each
    moved by a seeded fraction (|.| <= jitter) of the step along the curve."""
    xc, yc = np.append(x, x[0]), np.append(y, y[0])
    s = np.concatenate([[0.0], np.cumsum(np.hypot(np.diff(xc), np.diff(yc)))])
    u = (np.arange(n) + np.random.default_rng(seed).uniform(-jitter, jitter, size=n)) * (s[-1] / n)
    return np.stack([np.interp(u, s, xc), np.interp(u, s, yc)], axis=1)


def heart_points(n_nodes=256, scale=0.72, jitter=0.1, seed=3, samples=1 << 16):
    """Quasi-uniform nodes on a smooth heart-shaped curve (counter-clockwise): the polar curve
    r(t) = scale (1 - 0.28 g(t - pi/2, 0.45) + 0.22 g(t - 3 pi/2, 0.5)), g(s, w) = exp(-(s/w)^2)
    (s wrapped to [-pi, pi)), a dimple at the top and a rounded tip at the bottom, shifted up
    by 0.15.  Smallest radius of curvature 0.18."""
    t = np.linspace(0.0, 2.0 * np.pi, samples, endpoint=False)

    def g(c, w):
        return np.exp(-((np.mod(t - c + np.pi, 2.0 * np.pi) - np.pi) / w) ** 2)

    r = scale * (1.0 - 0.28 * g(0.5 * np.pi, 0.45) + 0.22 * g(1.5 * np.pi, 0.5))
    return _resample_closed(r * np.cos(t), r * np.sin(t) + 0.15, n_nodes, jitter, seed)


def heart2d(n_nodes=256, jitter=0.1, seed=3) -> Interface:
    return Interface(2, [spline_curve(heart_points(n_nodes, jitter=jitter, seed=seed))])


def spline_circle(R=0.5, n_nodes=256, clockwise=False, orient=+1) -> Interface:
    """Circle of radius R through n equally spaced points (angle offset half a step)."""
    t = 2.0 * np.pi * (np.arange(n_nodes) + 0.5) / n_nodes
    if clockwise:
        t = -t
    return Interface(2, [spline_curve(np.stack([R * np.cos(t), R * np.sin(t)], axis=1), orient)])


def spline_star(R0=0.7, A=0.15, L=5, n_nodes=256) -> Interface:
    """The star r = R0 + A cos(L t) through its points at t_j = 2 pi j / n (the analytic
    surface's own nodes), as a spline curve."""
    t = 2.0 * np.pi * np.arange(n_nodes) / n_nodes
    r = R0 + A * np.cos(L * t)
    return Interface(2, [spline_curve(np.stack([r * np.cos(t), r * np.sin(t)], axis=1))])


def ellipsoid(a=0.9, b=0.7, c=0.5, n_nodes=8192) -> Interface:
    return Interface(3, [Surface((a, b, c), +1, n_nodes, [])])


def sphere(R=0.5, n_nodes=2048) -> Interface:
    return Interface(3, [Surface((R, R, R), +1, n_nodes, [])])


def perturbed_sphere(R=0.8, eps=0.1, n_nodes=32768) -> Interface:
    """r = R (1 + eps cos(3 theta) sin(2 phi) sin^2(phi))  (theta azimuth, phi polar).

    cos(3 theta) sin^3(phi) = x^3 - 3 x y^2 and sin(2 phi) = 2 sin(phi) z on the
    unit sphere, so the perturbation is the polynomial 2 eps z (x^3 - 3 x y^2).
    """
    terms = [(2 * eps, (3, 0, 1)), (-6 * eps, (1, 2, 1))]
    return Interface(3, [Surface((R, R, R), +1, n_nodes, terms)])


def shell_noise_terms(seed=1, n_terms=8, max_degree=4, amplitude=0.08):
    """Seeded smooth radial noise: a random polynomial in the unit vector.

    ``n_terms`` monomials of total degree 1..max_degree with random signs and
    weights, scaled so that sum |c| = amplitude (hence |noise| <= amplitude).
    """
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(n_terms):
        deg = int(rng.integers(1, max_degree + 1))
        cut = np.sort(rng.integers(0, deg + 1, size=2))
        e = (int(cut[0]), int(cut[1] - cut[0]), int(deg - cut[1]))
        terms.append([float(rng.uniform(0.3, 1.0) * rng.choice([-1.0, 1.0])), e])
    s = sum(abs(t[0]) for t in terms)
    return [(t[0] * amplitude / s, tuple(t[1])) for t in terms]


def thick_shell(outer=(0.9, 0.7, 0.6), inner_scale=0.6, n_nodes=40960, seed=1) -> Interface:
    """Closed thick shell: tissue between an outer ellipsoid and a noisy inner wall.

    Nodes are split in proportion to the (noise-free) areas, i.e. 1 : inner_scale^2.
    """
    frac = inner_scale ** 2 / (1.0 + inner_scale ** 2)
    n_in = int(round(n_nodes * frac))
    n_out = n_nodes - n_in
    inner_axes = tuple(inner_scale * a for a in outer)
    return Interface(3, [Surface(tuple(outer), +1, n_out, []),
                         Surface(inner_axes, -1, n_in, shell_noise_terms(seed))])


def _radius(surface: Surface, u):
    """Plain polar radius of a surface in direction u (workload placement only)."""
    u = np.asarray(u, dtype=np.float64)
    E = 1.0 / math.sqrt(sum(u[i] ** 2 / surface.axes[i] ** 2 for i in range(len(u))))
    P = sum(c * np.prod([u[i] ** e[i] for i in range(len(u))]) for c, e in surface.terms)
    return E * (1.0 + P)


def icosphere(level: int):
    """Unit-sphere triangulation: the icosahedron with each triangle split into 4 per level
    (10 4^level + 2 vertices), triangles oriented with outward (counter-clockwise) normals."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                mid[key] = len(V) - 1
            return mid[key]

        G = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            G += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = G
    return np.array(V), np.array(F, dtype=np.int32)


def _rotation(seed):
    """Seeded rotation matrix (QR of a Gaussian matrix, determinant +1)."""
    Q, R = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def mesh_surface(points, tris, orient=+1) -> Surface:
    """A closed, consistently oriented triangle mesh (either orientation)."""
    P = np.ascontiguousarray(points, dtype=np.float64)
    Tr = np.ascontiguousarray(tris, dtype=np.int32)
    return Surface((1.0, 1.0, 1.0), orient, P.shape[0], [], kind="mesh", points=P, tris=Tr)


def mesh_of(surface: Surface, level: int, seed=5, flip=False) -> Surface:
    """Triangle mesh of an analytic star-shaped surface: the icosphere's vertex directions,
    rotated by a seeded rotation, placed at the surface's radius (triangles reversed if flip)."""
    U, F = icosphere(level)
    U = U @ _rotation(seed).T
    X = np.stack([_radius(surface, u) * u for u in U])
    if flip:
        F = F[:, ::-1]
    return mesh_surface(X, F, surface.orient)


def mesh_sphere(R=0.5, level=4, seed=5) -> Interface:
    return Interface(3, [mesh_of(Surface((R, R, R), +1, 0, []), level, seed)])


def mesh_ellipsoid(a=0.9, b=0.7, c=0.5, level=5, seed=5, flip=False) -> Interface:
    return Interface(3, [mesh_of(Surface((a, b, c), +1, 0, []), level, seed, flip)])


def mesh_perturbed_sphere(R=0.8, eps=0.1, level=5, seed=5) -> Interface:
    return Interface(3, [mesh_of(perturbed_sphere(R, eps, 1).surfaces[0], level, seed)])


def mesh_shell(outer=(0.9, 0.7, 0.6), inner_scale=0.6, level_out=5, level_in=4, seed=1) -> Interface:
    """The thick shell with both walls given as triangle meshes."""
    sh = thick_shell(outer, inner_scale, 1000, seed)
    return Interface(3, [mesh_of(sh.surfaces[0], level_out, seed + 4), mesh_of(sh.surfaces[1], level_in, seed + 5)])


def stimulus_center(iface: Interface, seed=0):
    """Seeded centre of the initial V=1 ball: inside the tissue, mid-wall for a shell."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=iface.dim)
    u = v / np.linalg.norm(v)
    if len(iface.surfaces) == 1:
        r = 0.5 * _radius(iface.surfaces[0], u)
    else:
        r = 0.5 * (_radius(iface.surfaces[0], u) + _radius(iface.surfaces[1], u))
    return tuple(float(x) for x in r * u)


def box(dim, cells, lo=-1.2, hi=1.2) -> Grid:
    return Grid(dim, lo, hi, cells)


def scalar_coeffs(dim, sigma=1.0, kappa=400.0) -> Coeffs:
    return Coeffs(1, [[sigma] * dim], kappa)


def bidomain_coeffs(dim, params: BidomainParams, dt: float) -> Coeffs:
    kappa = 2.0 * params.Cm * params.beta / dt
    return Coeffs(2, [[params.sigma_i] * dim, [params.sigma_e] * dim], kappa)


# ----------------------------------------------------------------------------- the paper's examples

def paper_params() -> BidomainParams:
    """The parameters of the paper's numerical section: C_m = 1, beta = 1000, FitzHugh-Nagumo with
    H = 100, theta = 0.25, alpha = 5/20, zeta = 1, Newton tolerance 1e-10."""
    return BidomainParams(Cm=1.0, beta=1000.0, H=100.0, theta=0.25, alpha=0.25, zeta=1.0)


def paper_circle_example(cells, R=0.8):
    """Example 1 (2D circle) with dt = h.  Box [-1, 1]^2 (the paper's trajectory points
    (0.5625..0.71875, 0) are grid nodes of that box) and a circle of radius R = 0.8 (not stated; it
    must hold those points), given by `cells` quasi-uniform nodes through a periodic cubic spline;
    D_i = diag(30, 5), D_e = diag(20, 10) (fibers along x); kappa = 2 C_m beta / dt; the virtual
    electrode: anode (-0.3, 0), cathode (0.3, 0), radius 0.25, V_stim = 10.
    Returns (interface, grid, coeffs, params, dt, I_stim on the box nodes)."""
    grid = box(2, cells, -1.0, 1.0)
    p = paper_params()
    dt = grid.h
    co = Coeffs(2, [[30.0, 5.0], [20.0, 10.0]], 2.0 * p.Cm * p.beta / dt)
    stim = virtual_electrode(grid, (-0.3, 0.0), (0.3, 0.0), radius=0.25, amplitude=10.0)
    return spline_circle(R, n_nodes=cells), grid, co, p, dt, stim


def paper_sphere_example(cells, R=0.9, n_nodes=None):
    """Example 3 (3D sphere) with dt = h.  Box [-1, 1]^3 (the trajectory points (0.5625..0.875, 0, 0)
    are grid nodes of that box), a sphere of radius R = 0.9 (not stated; it must hold them) with
    (cells/8)^2 + 2 nodes (the paper's 66 at 64^3, 258 at 128^3) unless n_nodes is given; D_i = diag(30, 5, 5),
    D_e = diag(20, 10, 10); kappa = 2 C_m beta / dt; virtual electrode at (-0.3, 0, 0) / (0.3, 0, 0),
    radius 0.25, V_stim = 10.  Returns (interface, grid, coeffs, params, dt, I_stim)."""
    grid = box(3, cells, -1.0, 1.0)
    p = paper_params()
    dt = grid.h
    co = Coeffs(2, [[30.0, 5.0, 5.0], [20.0, 10.0, 10.0]], 2.0 * p.Cm * p.beta / dt)
    stim = virtual_electrode(grid, (-0.3, 0.0, 0.0), (0.3, 0.0, 0.0), radius=0.25, amplitude=10.0)
    m = n_nodes if n_nodes is not None else (cells // 8) ** 2 + 2
    return sphere(R, n_nodes=m), grid, co, p, dt, stim


# ----------------------------------------------------------------------------- named configs

def config(name: str):
    """Named workloads (interface, grid, coeffs-or-params) used by tests and the bench."""
    if name == "star2d_128":
        return star2d(n_nodes=256), box(2, 128), scalar_coeffs(2, 1.0, 400.0)
    if name == "ellipsoid_128":
        return ellipsoid(n_nodes=8192), box(3, 128), scalar_coeffs(3, 1.0, 400.0)
    if name == "psphere_256":
        return perturbed_sphere(n_nodes=32768), box(3, 256), scalar_coeffs(3, 1.0, 400.0)
    if name == "shell_256":
        return thick_shell(n_nodes=40960), box(3, 256), BidomainParams()
    if name == "heart2d_128":
        return heart2d(n_nodes=256), box(2, 128), scalar_coeffs(2, 1.0, 400.0)
    if name == "ellipsoid_bidomain_128":
        return ellipsoid(n_nodes=8192), box(3, 128), BidomainParams()
    raise KeyError(name)


def _min_curvature_radius(R0, A, L, samples=4096):
    """Smallest radius of curvature of the polar curve r = R0 + A cos(L t) (draw check only)."""
    t = np.linspace(0.0, 2.0 * np.pi, samples, endpoint=False)
    r = R0 + A * np.cos(L * t)
    r1 = -A * L * np.sin(L * t)
    r2 = -A * L * L * np.cos(L * t)
    curv = np.abs(r * r + 2 * r1 * r1 - r * r2) / (r * r + r1 * r1) ** 1.5
    return float(1.0 / np.max(curv))


def batch_2d(n=64, seed=2, sizes=(64, 128, 256, 512, 1024)):
    """Seeded batch of 2D Neumann problems of uneven sizes and shapes.

    Per problem: cells drawn uniformly from ``sizes``, a star r = 0.7 + A cos(L t) with
    L in 3..8 lobes and A ~ U[0.05, 0.2], kappa log-uniform in [50, 2000], sigma = 1 and
    M = 2 cells nodes.  A draw whose smallest radius of curvature is below 2h is drawn again.
    Returns a list of (interface, grid, coeffs).
    """
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        cells = int(rng.choice(sizes))
        L = int(rng.integers(3, 9))
        A = float(rng.uniform(0.05, 0.2))
        kappa = float(np.exp(rng.uniform(np.log(50.0), np.log(2000.0))))
        grid = box(2, cells)
        if _min_curvature_radius(0.7, A, L) < 2.0 * grid.h:
            continue
        out.append((star2d(0.7, A, L, n_nodes=2 * cells), grid, scalar_coeffs(2, 1.0, kappa)))
    return out


def seeded_vector(n, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def grid_points(grid):
    """(N^d, d) coordinates of the interior nodes in [z][y][x] order (input generation only)."""
    c = grid.lo + grid.h * np.arange(1, grid.cells, dtype=np.float64)
    mesh = np.meshgrid(*([c] * grid.dim), indexing="ij")
    return np.stack([m.ravel() for m in reversed(mesh)], axis=1)


def virtual_electrode(grid, anode, cathode, radius=0.25, amplitude=10.0):
    """Stimulus current on the box nodes: +amplitude in a ball about the anode, -amplitude in a
    ball of the same radius about the cathode (the paired electrode of the paper's examples)."""
    pts = grid_points(grid)
    ra = np.sum((pts - np.asarray(anode)[None, :]) ** 2, axis=1)
    rc = np.sum((pts - np.asarray(cathode)[None, :]) ** 2, axis=1)
    return amplitude * (np.where(ra < radius * radius, 1.0, 0.0) - np.where(rc < radius * radius, 1.0, 0.0))


def ball_state(grid, center, radius=0.1):
    """Initial bidomain state: V = 1 inside a ball, 0 elsewhere; q = 0."""
    pts = grid_points(grid)
    r2 = np.sum((pts - np.asarray(center)[None, :]) ** 2, axis=1)
    V = np.where(r2 < radius * radius, 1.0, 0.0)
    return V, np.zeros_like(V)
