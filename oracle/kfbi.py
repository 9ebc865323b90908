"""The kernel-free boundary integral method, step by step (FP64).  Test infrastructure only.

Notation follows the paper: Omega is the tissue ("+" side), its complement in
the box B is the "-" side, n points out of Omega and [w] = w+ - w-
(Sec. 5.1, eq. jump).  Everything is written in the positive form
-div(D grad u) + K u = f (the paper's f is our -f; Sec. 3, eq. bvp).

The pieces, in the order of Algorithm 1:

* density transfer: psi and its surface gradient at intersection points and
  interface nodes.  The paper takes these from local coordinate systems on
  the boundary (Sec. 5.3, Fig. 1 paragraph); here a cubic Lagrange fit in the
  curve parameter (2D: the polar angle, or the spline parameter of a curve
  given by its nodes) or a quadratic least-squares fit over the 10 nearest
  nodes in the tangent plane (3D).
* jump relations of the single-layer interface problem (Sec. 5.1, eq.
  single: [u] = 0, [n.D grad u] = psi, homogeneous equation on both sides).
  For a diagonal D_c the interface conditions give [grad u] = a n with
  a = psi / (n.D n) and [Hess u] = a W + n b^T + b n^T + c n n^T,
  b = (g - 2 a W D n) / (n.D n), c fixed by tr(D [Hess u]) = -[f];
  g = surface gradient of psi, W = shape operator (derived by differentiating
  [u] = 0 twice and the flux jump once along the boundary, and using the PDE
  for the normal-normal part).  For isotropic D = sigma this is
  [grad u] = (psi/sigma) n,
  [Hess u] = (psi/sigma)(W - tr(W) n n^T) + (n g^T + g n^T)/sigma - ([f]/sigma) n n^T.
* right-hand-side correction at irregular nodes (Sec. 5.3, eq. correct):
  for a node p whose arm to the neighbour q crosses the boundary at z,
  rhs_p += s_p (D_a/h^2) ([u] + [u_a] d + 1/2 [u_aa] d^2), d = q_a - z_a,
  s_p = +1 for p in Omega, -1 otherwise (third-order term dropped).
* box solve (``boxsolve``).
* quadratic extrapolation of the "+" limit at each interface node from its
  6 (2D) / 10 (3D) nearest grid nodes, adding the Taylor-expanded jump J_j
  to values on the "-" side (Sec. 5.4, eqs. taylor-i-po, taylor-i-co, ji).
* BIE operator A psi = n.D grad u+ and right-hand side
  g' = g^N - n.D grad u_V+ with u_V the uncorrected box solve of the
  smoothly extended source (Sec. 4, eq. bie; Sec. 5.1, eq. volume).
* the coupled pair's null density (reading, not in the paper): the insulated
  tissue (Sec. 2, eq. bdry cond) fixes both potentials only up to one common
  constant, so the BIE operator of the coupled pair is singular, its null space
  spanned by the density whose single-layer potential is a constant pair in
  Omega.  The potentials are reconstructed from the density with that component
  removed: in Omega this changes them by a constant pair, which the gauge takes
  away, while outside Omega, where the transmembrane potential is also evolved
  (Sec. 5.1), it removes a field that the discrete operator's near-zero
  eigenvalue would otherwise make large and step-dependent.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

from . import boxsolve, geometry
from .geometry import GeometryError
from .gmres import gmres

N_LSQ = 10                       # nodes per 3D least-squares transfer fit
TIE_TOL = 1e-9                   # squared-distance ties (units of h^2) in stencil selection
RANK_TOL = 1e-6                  # relative residual for accepting a stencil node


# ----------------------------------------------------------------------------- density transfer

def _lagrange4(s):
    """Cubic Lagrange weights and s-derivatives at local coordinate s for nodes at -1, 0, 1, 2."""
    w = np.stack([-s * (s - 1) * (s - 2) / 6.0,
                  (s + 1) * (s - 1) * (s - 2) / 2.0,
                  -(s + 1) * s * (s - 2) / 2.0,
                  (s + 1) * s * (s - 1) / 6.0], axis=1)
    dw = np.stack([-(3 * s * s - 6 * s + 2) / 6.0,
                   (3 * s * s - 4 * s - 1) / 2.0,
                   -(3 * s * s - 2 * s - 2) / 2.0,
                   (3 * s * s - 1) / 6.0], axis=1)
    return w, dw


def transfer_2d_points(surf, offset, m, pts):
    """Weights for psi(z) and grad_Gamma psi(z) at boundary points z of one curve.

    The point's curve parameter is its polar angle t*; psi is the cubic through
    the nodes j-1..j+2 with j = floor(t*/dt) (cyclic); d psi/ds = (d psi/dt)/|X'(t*)|.
    """
    dt = 2.0 * math.pi / m
    t = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2.0 * math.pi)
    j = np.minimum(np.floor(t / dt).astype(np.int64), m - 1)
    s = (t - j * dt) / dt
    w, dw = _lagrange4(s)
    idx = offset + np.mod(j[:, None] + np.arange(-1, 3)[None, :], m)
    tau, speed = geometry.curve_tangent(surf, t)
    wg = (dw / (dt * speed[:, None]))[:, :, None] * tau[:, None, :]
    return idx, w, wg


def transfer_2d_nodes(surf, offset, m):
    """Surface-gradient weights at the nodes themselves: 5-point central difference in t."""
    dt = 2.0 * math.pi / m
    j = np.arange(m)
    t = 2.0 * math.pi * j / m
    idx = offset + np.mod(j[:, None] + np.arange(-2, 3)[None, :], m)
    c = np.array([1.0, -8.0, 0.0, 8.0, -1.0]) / (12.0 * dt)
    tau, speed = geometry.curve_tangent(surf, t)
    wg = (c[None, :] / speed[:, None])[:, :, None] * tau[:, None, :]
    return idx, wg


def transfer_spline_points(cv, offset, tpar):
    """Spline curves: the same cubic Lagrange fit, in the spline parameter t* of each point
    (nodes at t = j); d psi/ds = (d psi/dt)/|X'(t*)| along the spline tangent."""
    m = cv.m
    j = np.floor(tpar).astype(np.int64)
    s = tpar - j
    w, dw = _lagrange4(s)
    idx = offset + np.mod(j[:, None] + np.arange(-1, 3)[None, :], m)
    tau, speed = cv.tangent(tpar)
    wg = (dw / speed[:, None])[:, :, None] * tau[:, None, :]
    return idx, w, wg


def transfer_spline_nodes(cv, offset):
    """Spline curves: 5-point central difference in t (unit node spacing) over the speed."""
    m = cv.m
    j = np.arange(m)
    idx = offset + np.mod(j[:, None] + np.arange(-2, 3)[None, :], m)
    c = np.array([1.0, -8.0, 0.0, 8.0, -1.0]) / 12.0
    tau, speed = cv.tangent(j.astype(np.float64))
    wg = (c[None, :] / speed[:, None])[:, :, None] * tau[:, None, :]
    return idx, wg


def tangent_frame(n):
    """tau1 = normalize(e_m x n) with e_m the axis least aligned with n (lowest on ties), tau2 = n x tau1."""
    m = np.argmin(np.abs(n), axis=1)
    e = np.zeros_like(n)
    e[np.arange(len(m)), m] = 1.0
    t1 = np.cross(e, n)
    t1 /= np.sqrt(np.sum(t1 * t1, axis=1))[:, None]
    t2 = np.cross(n, t1)
    return t1, t2


def transfer_3d(xs, offset, pts, nrm, h, k=N_LSQ):
    """Least-squares quadratic fit of psi over the k nearest nodes, in tangent coordinates / h.

    Nearest = smallest squared distance, ties broken by the lower node index.
    Returns node indices (global), weights for psi(z) and for grad_Gamma psi(z).
    """
    tree = cKDTree(xs)
    kq = min(k + 4, xs.shape[0])
    _, cand = tree.query(pts, k=kq)
    diff = xs[cand] - pts[:, None, :]
    d2 = (diff[..., 0] * diff[..., 0] + diff[..., 1] * diff[..., 1]) + diff[..., 2] * diff[..., 2]
    order = np.lexsort((cand, d2), axis=-1)[:, :k]
    sel = np.take_along_axis(cand, order, axis=1)
    diff = xs[sel] - pts[:, None, :]
    t1, t2 = tangent_frame(nrm)
    xi = np.einsum("nkd,nd->nk", diff, t1) / h
    eta = np.einsum("nkd,nd->nk", diff, t2) / h
    V = np.stack([np.ones_like(xi), xi, eta, xi * xi, xi * eta, eta * eta], axis=2)
    pinv = np.linalg.pinv(V)                              # (n, 6, k)
    w0 = pinv[:, 0, :]
    wg = (pinv[:, 1, :, None] * t1[:, None, :] + pinv[:, 2, :, None] * t2[:, None, :]) / h
    return offset + sel, w0, wg


# ----------------------------------------------------------------------------- extrapolation stencils

def quad_basis(r):
    """Quadratic Taylor basis at scaled offsets r (..., d): 1, r_a, r_a^2/2, r_a r_b."""
    d = r.shape[-1]
    one = np.ones(r.shape[:-1])
    if d == 2:
        x, y = r[..., 0], r[..., 1]
        return np.stack([one, x, y, x * x / 2, x * y, y * y / 2], axis=-1)
    x, y, z = r[..., 0], r[..., 1], r[..., 2]
    return np.stack([one, x, y, z, x * x / 2, y * y / 2, z * z / 2, x * y, x * z, y * z], axis=-1)


def select_stencil(grid, q):
    """Grid nodes for the quadratic fit at boundary point q (the paper's 'nearest six/ten').

    Candidates are the 4^d nodes on the four grid lines per axis around q.  They
    are ranked by squared distance (ties within TIE_TOL h^2 by linear index) and
    accepted greedily while they raise the rank of the quadratic Vandermonde rows.
    """
    d, h, lo = grid.dim, grid.h, grid.lo
    S = 6 if d == 2 else 10
    kc = np.floor((q - lo) / h).astype(np.int64)
    rng = [np.arange(kc[a] - 1, kc[a] + 3) for a in range(d)]
    mesh = np.meshgrid(*rng, indexing="ij")
    k = np.stack([m.ravel() for m in mesh], axis=1)                 # grid indices 0..I
    if np.any(k < 1) or np.any(k > grid.cells - 1):
        raise GeometryError("extrapolation stencil reaches the box boundary")
    x = lo + k * h
    r = (x - q[None, :]) / h
    d2 = np.sum(r * r, axis=1)
    lin = geometry.linear_index(grid, k - 1)
    order = np.lexsort((lin, d2))
    # group near-ties and order each group by linear index
    groups, cur = [], [order[0]]
    for i in order[1:]:
        if d2[i] - d2[cur[0]] > TIE_TOL:
            groups.append(cur)
            cur = [i]
        else:
            cur.append(i)
    groups.append(cur)
    ranked = [i for g in groups for i in sorted(g, key=lambda j: lin[j])]
    Q, acc = [], []
    for i in ranked:
        v = quad_basis(r[i])
        w = v.copy()
        for _ in range(2):
            for qv in Q:
                w = w - np.dot(qv, w) * qv
        nw = np.linalg.norm(w)
        if nw > RANK_TOL * np.linalg.norm(v):
            Q.append(w / nw)
            acc.append(i)
            if len(acc) == S:
                break
    if len(acc) < S:
        raise GeometryError("rank-deficient extrapolation stencil")
    acc = np.array(acc)
    V = quad_basis(r[acc])
    Vinv = np.linalg.inv(V)
    wgrad = Vinv[1:1 + d, :].T / h                                   # (S, d)
    return lin[acc], r[acc] * h, wgrad


# ----------------------------------------------------------------------------- the problem

class Problem:
    """Static tables of one KFBI problem (what ``kfbi_setup`` builds)."""

    def __init__(self, iface, grid, coeffs):
        self.iface, self.grid, self.coeffs = iface, grid, coeffs
        d = grid.dim
        if iface.dim != d:
            raise ValueError("interface and grid dimensions differ")
        # diagonal conductivity per component and axis
        self.sigma = [np.asarray(coeffs.D[c][:d], dtype=np.float64) for c in range(coeffs.ncomp)]
        geometry.check_box_clearance(iface, grid)
        self.nodes = geometry.Nodes(iface)
        side = geometry.classify(iface, grid)
        self.cross = geometry.Crossings(iface, grid, side)
        self.inside = self.cross.inside
        self.irregular = geometry.irregular_nodes(grid, self.cross)
        self.M = self.nodes.M
        self._transfer()
        self._stencils()

    # -- transfer weights at crossings and nodes
    def _transfer(self):
        nd, cr, d = self.nodes, self.cross, self.grid.dim
        K = 4 if d == 2 else N_LSQ
        Kn = 5 if d == 2 else N_LSQ
        self.z_idx = np.zeros((cr.count, K), dtype=np.int64)
        self.z_w0 = np.zeros((cr.count, K))
        self.z_wg = np.zeros((cr.count, K, d))
        self.q_idx = np.zeros((self.M, Kn), dtype=np.int64)
        self.q_wg = np.zeros((self.M, Kn, d))
        for s, surf in enumerate(self.iface.surfaces):
            o, m = nd.offsets[s], surf.n_nodes
            msk = cr.surf == s
            if geometry.is_mesh(surf):
                self._transfer_mesh(geometry.trimesh_of(surf), o, m, msk, K, Kn)
            elif geometry.is_spline(surf):
                cv = geometry.curve_of(surf)
                if np.any(msk):
                    self.z_idx[msk], self.z_w0[msk], self.z_wg[msk] = \
                        transfer_spline_points(cv, o, cr.tparam[msk])
                self.q_idx[o:o + m], self.q_wg[o:o + m] = transfer_spline_nodes(cv, o)
            elif d == 2:
                if np.any(msk):
                    self.z_idx[msk], self.z_w0[msk], self.z_wg[msk] = \
                        transfer_2d_points(surf, o, m, cr.z[msk])
                self.q_idx[o:o + m], self.q_wg[o:o + m] = transfer_2d_nodes(surf, o, m)
            else:
                xs = nd.X[o:o + m]
                if np.any(msk):
                    self.z_idx[msk], self.z_w0[msk], self.z_wg[msk] = \
                        transfer_3d(xs, o, cr.z[msk], cr.n[msk], self.grid.h)
                idx, _, wg = transfer_3d(xs, o, xs, nd.n[o:o + m], self.grid.h)
                self.q_idx[o:o + m], self.q_wg[o:o + m] = idx, wg

    def _transfer_mesh(self, tm, o, m, msk, K, Kn):
        """Triangle meshes: the six-point system of the crossing's triangle (slots beyond six
        carry zero weight), and the one-ring fit at each vertex."""
        cr = self.cross
        for c in np.flatnonzero(msk):
            idx, w0, wg = tm.crossing_transfer(int(cr.tparam[c]), cr.z[c])
            self.z_idx[c] = o + idx[0]
            self.z_idx[c, :6] = o + idx
            self.z_w0[c] = 0.0
            self.z_w0[c, :6] = w0
            self.z_wg[c] = 0.0
            self.z_wg[c, :6] = wg
        for j in range(m):
            idx, wg = tm.vertex_transfer(j, Kn)
            k = len(idx)
            self.q_idx[o + j] = o + idx[0]
            self.q_idx[o + j, :k] = o + idx
            self.q_wg[o + j] = 0.0
            self.q_wg[o + j, :k] = wg

    # -- extrapolation stencils
    def _stencils(self):
        S = 6 if self.grid.dim == 2 else 10
        self.st_lin = np.zeros((self.M, S), dtype=np.int64)
        self.st_r = np.zeros((self.M, S, self.grid.dim))
        self.st_wgrad = np.zeros((self.M, S, self.grid.dim))
        for i in range(self.M):
            self.st_lin[i], self.st_r[i], self.st_wgrad[i] = select_stencil(self.grid, self.nodes.X[i])
        self.st_chi = ~self.inside[self.st_lin]                        # stencil node on the "-" side

    # ------------------------------------------------------------------------- jumps
    def node_coord(self, lin, axis):
        N, h = self.grid.n, self.grid.h
        i = (lin // (N ** axis)) % N
        return self.grid.lo + (i + 1) * h

    def jumps_at_crossings(self, psi_c, sigma):
        """[u_a] and [u_aa] at every intersection (a = the arm's axis); [u] = 0."""
        cr = self.cross
        p = np.sum(self.z_w0 * psi_c[self.z_idx], axis=1)
        g = np.einsum("nk,nkd->nd", psi_c[self.z_idx], self.z_wg)
        du, H = jump_relations(p, g, cr.n, cr.W, sigma)
        ar = np.arange(cr.count)
        return np.zeros(cr.count), du[ar, cr.axis], H[ar, cr.axis, cr.axis]

    def jumps_at_nodes(self, psi_c, sigma):
        """[u] (= 0), [grad u] and [Hess u] at every interface node."""
        g = np.einsum("nk,nkd->nd", psi_c[self.q_idx], self.q_wg)
        du, H = jump_relations(psi_c, g, self.nodes.n, self.nodes.W, sigma)
        return np.zeros(self.M), du, H

    # ------------------------------------------------------------------------- correction
    def correction(self, Dc, ju, dua, duua):
        """Right-hand-side increments at irregular nodes from jumps at the intersections."""
        cr, h = self.cross, self.grid.h
        rhs = np.zeros(self.grid.n ** self.grid.dim)
        Da = np.asarray(Dc, dtype=np.float64)[cr.axis] / h ** 2
        zin = np.array([self.node_coord(cr.p_in[i], cr.axis[i]) for i in range(cr.count)]) \
            if cr.count else np.zeros(0)
        zout = np.array([self.node_coord(cr.p_out[i], cr.axis[i]) for i in range(cr.count)]) \
            if cr.count else np.zeros(0)
        za = cr.z[np.arange(cr.count), cr.axis]
        d_in = zout - za            # tissue-side node, neighbour on the "-" side
        d_out = zin - za            # "-"-side node, neighbour in the tissue
        np.add.at(rhs, cr.p_in, Da * (ju + dua * d_in + 0.5 * duua * d_in ** 2))
        np.add.at(rhs, cr.p_out, -Da * (ju + dua * d_out + 0.5 * duua * d_out ** 2))
        return rhs

    # ------------------------------------------------------------------------- extrapolation
    def extrapolate(self, u_c, Dc, ju, du, H):
        """n.D grad u+ at every node: quadratic fit of grid values, jump-corrected on the "-" side."""
        vals = u_c[self.st_lin].copy()
        r = self.st_r
        J = ju[:, None] + np.einsum("nd,nsd->ns", du, r) + 0.5 * np.einsum("nsa,nab,nsb->ns", r, H, r)
        vals = vals + np.where(self.st_chi, J, 0.0)
        grad = np.einsum("nsd,ns->nd", self.st_wgrad, vals)
        Dv = np.asarray(Dc, dtype=np.float64)[: self.grid.dim]
        return np.sum(self.nodes.n * Dv[None, :] * grad, axis=1)

    def extrapolate_smooth(self, u_c, Dc):
        z = np.zeros(self.M)
        d = self.grid.dim
        return self.extrapolate(u_c, Dc, z, np.zeros((self.M, d)), np.zeros((self.M, d, d)))

    # ------------------------------------------------------------------------- operator
    def correction_from_density(self, psi):
        psi = psi.reshape(self.coeffs.ncomp, self.M)
        rhs = np.zeros((self.coeffs.ncomp, self.grid.n ** self.grid.dim))
        for c in range(self.coeffs.ncomp):
            ju, dua, duua = self.jumps_at_crossings(psi[c], self.sigma[c])
            rhs[c] = self.correction(self.coeffs.D[c], ju, dua, duua)
        return rhs

    def apply(self, psi):
        """A psi: corrected box solve of the single-layer problem, then n.D grad u+ at the nodes."""
        psi = np.asarray(psi, dtype=np.float64).reshape(self.coeffs.ncomp, self.M)
        u = boxsolve.box_solve(self.correction_from_density(psi), self.grid, self.coeffs)
        out = np.zeros_like(psi)
        for c in range(self.coeffs.ncomp):
            ju, du, H = self.jumps_at_nodes(psi[c], self.sigma[c])
            out[c] = self.extrapolate(u[c], self.coeffs.D[c], ju, du, H)
        return out

    def bie_rhs(self, g, f):
        """u_V = box solve of the extended source, g' = g - n.D grad u_V+ (Algorithm 1, volume part)."""
        uV = boxsolve.box_solve(np.asarray(f, dtype=np.float64).reshape(self.coeffs.ncomp, -1),
                                self.grid, self.coeffs)
        g = np.asarray(g, dtype=np.float64).reshape(self.coeffs.ncomp, self.M)
        gp = np.stack([g[c] - self.extrapolate_smooth(uV[c], self.coeffs.D[c])
                       for c in range(self.coeffs.ncomp)])
        return gp, uV

    def null_density(self, tol=1e-12, max_iter=6):
        """Coupled pair only: the unit density spanning the (discrete) null space of A, the
        eigenvector of smallest |eigenvalue|, by inverse iteration from the constant density
        (each step one GMRES solve to tol); stops when successive iterates agree to 1e-10 up to
        sign.  Cached."""
        if self.coeffs.ncomp != 2:
            raise ValueError("the null density belongs to the coupled pair")
        if getattr(self, "_null", None) is None:
            x = np.ones(2 * self.M) / math.sqrt(2 * self.M)
            for _ in range(max_iter):
                y, _ = gmres(lambda v: self.apply(v).ravel(), x, np.zeros_like(x), tol, 50, 500)
                y = y / np.linalg.norm(y)
                if np.dot(y, x) < 0:
                    y = -y
                done = np.linalg.norm(y - x) < 1e-10
                x = y
                if done:
                    break
            self._null = x.reshape(2, self.M)
        return self._null

    def remove_null(self, psi):
        """psi minus its component along the null density (coupled pair; unchanged otherwise)."""
        psi = np.asarray(psi, dtype=np.float64).reshape(self.coeffs.ncomp, self.M)
        if self.coeffs.ncomp != 2:
            return psi
        z = self.null_density()
        return psi - np.sum(z * psi) * z

    def reconstruct(self, f, psi):
        """u = box solve of (f + C psi); the coupled pair's density without its null component,
        and the pair gauged to mean_Omega(Phi_e) = 0."""
        psi = self.remove_null(psi)
        rhs = np.asarray(f, dtype=np.float64).reshape(self.coeffs.ncomp, -1) + self.correction_from_density(psi)
        u = boxsolve.box_solve(rhs, self.grid, self.coeffs)
        if self.coeffs.ncomp == 2:
            u = u - np.mean(u[1][self.inside])
        return u

    def solve_neumann(self, g, f, psi0=None, tol=1e-10, restart=50, maxit=500):
        """Neumann BVP: BIE right-hand side, GMRES on A psi = g', then the solution on the grid."""
        gp, _ = self.bie_rhs(g, f)
        x0 = np.zeros(gp.size) if psi0 is None else np.asarray(psi0, dtype=np.float64).ravel()
        psi, info = gmres(lambda v: self.apply(v).ravel(), gp.ravel(), x0, tol, restart, maxit)
        u = self.reconstruct(f, psi)
        return u, psi.reshape(self.coeffs.ncomp, self.M), info


def jump_relations(psi, g, n, W, D, fjump=None):
    """Single-layer jumps from density psi, its surface gradient g, normal n, shape operator W
    and the diagonal conductivity D (a scalar or one value per axis) of the component.

    With [u] = 0 and [n.D grad u] = psi (Sec. 5.1, eq. single):
      [grad u] = a n,  a = psi / (n.D n)   (tangential derivatives of [u] vanish);
      tangential block of [Hess u] = a W    (second tangential derivatives of [u] = 0);
      n.D [Hess u] t = g.t - a t.W D n for tangent t (tangential derivative of the flux jump,
      d n / dt = W t), i.e. the mixed part b = (g - 2 a W D n) / (n.D n);
      tr(D [Hess u]) = -[f]                (the equation on both sides, [u] = 0), which fixes
      the normal-normal part c;
    so [Hess u] = a W + n b^T + b n^T + c n n^T.
    """
    psi = np.asarray(psi, dtype=np.float64)
    d = n.shape[1]
    Dv = np.broadcast_to(np.asarray(D, dtype=np.float64).ravel()[:d] if np.ndim(D) else
                         np.full(d, float(D)), (d,))
    Dn = n * Dv[None, :]
    nDn = np.sum(n * Dn, axis=1)
    a = psi / nDn
    WDn = np.einsum("nij,nj->ni", W, Dn)
    b = (g - 2.0 * a[:, None] * WDn) / nDn[:, None]
    trDW = np.einsum("i,nii->n", Dv, W)
    rhs_c = -a * trDW - 2.0 * np.sum(b * Dn, axis=1)
    if fjump is not None:
        rhs_c = rhs_c - fjump
    c = rhs_c / nDn
    nn = n[:, :, None] * n[:, None, :]
    du = a[:, None] * n
    H = a[:, None, None] * W + n[:, :, None] * b[:, None, :] + b[:, :, None] * n[:, None, :] \
        + c[:, None, None] * nn
    return du, H
