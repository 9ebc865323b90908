"""Closed 3D surfaces given only as triangle meshes (FP64, NumPy).  Test infrastructure only.

In 3D the paper uses nothing but the triangle grid of the boundary and builds local
coordinate systems on it for normals, tangents and curvatures (Sec. 6, the paragraph on
the jumps in 3D, Fig. "six boundary points"; Sec. 7, Example 4).  Here:

* interface nodes are the mesh vertices; at a vertex the height function
  zeta = c1 xi + c2 eta + c3 xi^2 + c4 xi eta + c5 eta^2 over the tangent plane of the
  area-weighted triangle normal is fitted (least squares) to the vertex's one-ring, and n,
  W are those of the graph zeta = w(xi, eta) at the vertex;
* a triangle's local coordinate system uses its six boundary points (its three
  vertices and the three vertices across its edges): the quadratic height function
  through them over the triangle's plane, origin at its centroid;
* a grid node's side is the parity of the mesh crossings beyond it on its grid line
  (lines parallel to x), with a half-open rule on triangle edges so that a line through
  an edge or vertex counts once; a node within 1e-12 of a crossing on any of its three
  grid lines lies on the surface and counts as tissue;
* the crossing of a grid arm is found on the flat triangle it passes through and moved
  onto that triangle's quadratic patch (a quadratic equation along the arm), clamped to
  the arm; n and W at the crossing are the patch's;
* psi and its surface gradient at a crossing come from the same six-point system: the
  quadratic in (xi, eta) through the six values, differentiated along the patch's tangents
  X_xi = t1 + w_xi n0, X_eta = t2 + w_eta n0 (grad_G psi = [X_xi X_eta] g^-1 (psi_xi, psi_eta),
  g the metric); at a vertex, a least-squares quadratic in the vertex frame over the vertex
  and its one-ring (at most 10 points: the nearest neighbours) gives the gradient the same way.

For the graph zeta = w over a frame (t1, t2, n0) with the tissue below it the level set
phi = zeta - w gives n = (-w_xi, -w_eta, 1)/q, q = |grad phi|, and
W = P_n Hess(phi) P_n / q with Hess(phi) = -Hess(w) in the tangent block.
"""
from __future__ import annotations

import numpy as np

SIDE_TOL = 1e-12


class MeshError(ValueError):
    pass


def _frame(n):
    """Orthonormal (t1, t2) completing the unit vector n: t1 = normalize(e_m x n) with e_m the
    axis least aligned with n (lowest index on ties), t2 = n x t1."""
    m = int(np.argmin(np.abs(n)))
    e = np.zeros(3)
    e[m] = 1.0
    t1 = np.cross(e, n)
    t1 /= np.linalg.norm(t1)
    return t1, np.cross(n, t1)


def _graph_geometry(R, c, xi, eta):
    """n and W of the graph zeta = w(xi, eta) = c1 xi + c2 eta + c3 xi^2 + c4 xi eta + c5 eta^2
    (+ c0) in the frame R = [t1 t2 n0] (columns), at the point (xi, eta)."""
    wx = c[1] + 2 * c[3] * xi + c[4] * eta
    wy = c[2] + c[4] * xi + 2 * c[5] * eta
    g = np.array([-wx, -wy, 1.0])
    q = np.linalg.norm(g)
    nf = g / q
    Hf = -np.array([[2 * c[3], c[4], 0.0], [c[4], 2 * c[5], 0.0], [0.0, 0.0, 0.0]])
    P = np.eye(3) - np.outer(nf, nf)
    Wf = P @ Hf @ P / q
    return R @ nf, R @ Wf @ R.T


class TriMesh:
    def __init__(self, surf):
        V = np.asarray(surf.points, dtype=np.float64)
        F = np.asarray(surf.tris, dtype=np.int64)
        if V.ndim != 2 or V.shape[1] != 3 or F.ndim != 2 or F.shape[1] != 3:
            raise MeshError("a mesh needs (n, 3) vertices and (n_tris, 3) triangles")
        if F.size == 0 or F.min() < 0 or F.max() >= V.shape[0]:
            raise MeshError("triangle index out of range")
        self.V, self.F, self.m = V, F, V.shape[0]
        # every edge shared by exactly two triangles that traverse it in opposite directions
        half = {}
        for t, (a, b, c) in enumerate(F):
            for e, (p, q) in enumerate(((a, b), (b, c), (c, a))):
                if (p, q) in half:
                    raise MeshError("mesh is not consistently oriented")
                half[(p, q)] = (t, e)
        self.opp = np.zeros((F.shape[0], 3), dtype=np.int64)     # vertex across each edge
        for (p, q), (t, e) in half.items():
            if (q, p) not in half:
                raise MeshError("mesh is not closed")
            t2, e2 = half[(q, p)]
            self.opp[t, e] = F[t2, (e2 + 2) % 3]
        cr = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
        vol = np.sum(np.einsum("ij,ij->i", V[F[:, 0]], cr)) / 6.0
        self.sigma = float(surf.orient) * (1.0 if vol > 0 else -1.0)
        self.cross = self.sigma * cr                    # area-weighted normals out of the tissue
        self.nT = self.cross / np.linalg.norm(self.cross, axis=1)[:, None]
        nbr = [set() for _ in range(self.m)]
        for a, b, c in F:
            nbr[a] |= {b, c}
            nbr[b] |= {a, c}
            nbr[c] |= {a, b}
        self.nbr = [sorted(s) for s in nbr]
        self._patch = {}
        self._pts = {}

    # -- vertices
    def vertex_geometry(self):
        n = np.zeros((self.m, 3))
        W = np.zeros((self.m, 3, 3))
        acc = np.zeros((self.m, 3))
        for k in range(3):
            np.add.at(acc, self.F[:, k], self.cross)
        for i in range(self.m):
            n0 = acc[i] / np.linalg.norm(acc[i])
            t1, t2 = _frame(n0)
            R = np.stack([t1, t2, n0], axis=1)
            d = self.V[self.nbr[i]] - self.V[i]
            xi, eta, zeta = d @ t1, d @ t2, d @ n0
            A = np.stack([xi, eta, xi * xi, xi * eta, eta * eta], axis=1)
            c = np.linalg.lstsq(A, zeta, rcond=None)[0]
            n[i], W[i] = _graph_geometry(R, np.concatenate([[0.0], c]), 0.0, 0.0)
        return self.V.copy(), n, W

    # -- triangle patches (six boundary points)
    def patch(self, t):
        hit = self._patch.get(t)
        if hit is not None:
            return hit
        idx = list(self.F[t]) + list(self.opp[t])
        n0 = self.nT[t]
        o = self.V[self.F[t]].mean(axis=0)
        e = self.V[self.F[t, 1]] - self.V[self.F[t, 0]]
        t1 = e / np.linalg.norm(e)
        t2 = np.cross(n0, t1)
        R = np.stack([t1, t2, n0], axis=1)
        d = self.V[idx] - o
        L = np.max(np.linalg.norm(d[:3], axis=1))       # coordinates scaled by the triangle size
        xi, eta, zeta = d @ t1 / L, d @ t2 / L, d @ n0
        A = np.stack([np.ones(6), xi, eta, xi * xi, xi * eta, eta * eta], axis=1)
        if np.linalg.cond(A) > 1e10:
            raise MeshError("degenerate six-point local coordinate system")
        c = np.linalg.solve(A, zeta) / np.array([1.0, L, L, L * L, L * L, L * L])
        self._patch[t] = (o, R, c)
        return self._patch[t]

    def onto_patch(self, t, p, axis, s_flat, h):
        """Move the crossing of the line p + s e_axis with triangle t (at s_flat) onto the
        triangle's quadratic patch; s clamped to [0, h].  Returns the point, n and W."""
        o, R, c = self.patch(t)
        q0 = R.T @ (p - o)                              # frame coordinates at s = 0
        dq = R[axis, :]                                 # their change per unit s
        # zeta(s) - w(xi(s), eta(s)) = A2 s^2 + A1 s + A0
        x0, y0, z0 = q0
        dx, dy, dz = dq
        A2 = -(c[3] * dx * dx + c[4] * dx * dy + c[5] * dy * dy)
        A1 = dz - (c[1] * dx + c[2] * dy + 2 * c[3] * x0 * dx + c[4] * (x0 * dy + y0 * dx) + 2 * c[5] * y0 * dy)
        A0 = z0 - (c[0] + c[1] * x0 + c[2] * y0 + c[3] * x0 * x0 + c[4] * x0 * y0 + c[5] * y0 * y0)
        roots = np.roots([A2, A1, A0]) if A2 != 0.0 else (np.array([-A0 / A1]) if A1 != 0.0 else np.array([]))
        roots = np.real(roots[np.abs(np.imag(roots)) <= 1e-12 * max(1.0, np.max(np.abs(roots)))]) \
            if roots.size else roots
        s = s_flat if roots.size == 0 else float(roots[np.argmin(np.abs(roots - s_flat))])
        s = min(h, max(0.0, s))
        z = p.copy()
        z[axis] += s
        qz = R.T @ (z - o)
        n, W = _graph_geometry(R, c, qz[0], qz[1])
        return z, s, n, W

    def _patch_points(self, t):
        """Indices and the inverse of the scaled six-point Vandermonde matrix of triangle t."""
        hit = self._pts.get(t)
        if hit is None:
            o, R, c = self.patch(t)
            idx = np.array(list(self.F[t]) + list(self.opp[t]), dtype=np.int64)
            d = self.V[idx] - o
            L = np.max(np.linalg.norm(d[:3], axis=1))
            xi, eta = d @ R[:, 0] / L, d @ R[:, 1] / L
            A = np.stack([np.ones(6), xi, eta, xi * xi, xi * eta, eta * eta], axis=1)
            hit = (idx, np.linalg.inv(A), L)
            self._pts[t] = hit
        return hit

    def crossing_transfer(self, t, z):
        """Weights carrying the six nodal values of triangle t's local system to psi(z) and
        grad_Gamma psi(z) on its patch: (indices, w0 (6), wg (6, 3))."""
        o, R, c = self.patch(t)
        idx, Ainv, L = self._patch_points(t)
        q = R.T @ (z - o)
        x, y = q[0] / L, q[1] / L
        b = np.array([1.0, x, y, x * x, x * y, y * y])
        bx = np.array([0.0, 1.0, 0.0, 2 * x, y, 0.0]) / L
        by = np.array([0.0, 0.0, 1.0, 0.0, x, 2 * y]) / L
        # psi(q) = b^T a, a = Ainv psi_nodes  ->  weights Ainv^T b
        w0, wx, wy = Ainv.T @ b, Ainv.T @ bx, Ainv.T @ by
        return idx, w0, self._grad_weights(R, c, q[0], q[1], wx, wy)

    @staticmethod
    def _grad_weights(R, c, xi, eta, wx, wy):
        t1, t2, n0 = R[:, 0], R[:, 1], R[:, 2]
        Xx = t1 + (c[1] + 2 * c[3] * xi + c[4] * eta) * n0
        Xy = t2 + (c[2] + c[4] * xi + 2 * c[5] * eta) * n0
        g = np.array([[Xx @ Xx, Xx @ Xy], [Xx @ Xy, Xy @ Xy]])
        gi = np.linalg.inv(g)
        ax = gi[0, 0] * wx + gi[0, 1] * wy
        ay = gi[1, 0] * wx + gi[1, 1] * wy
        return ax[:, None] * Xx[None, :] + ay[:, None] * Xy[None, :]

    def vertex_transfer(self, i, kmax=10):
        """Weights of grad_Gamma psi at vertex i over the vertex and its one-ring (nearest
        kmax - 1 neighbours, ties by index): (indices, wg (k, 3))."""
        acc = self._vacc()[i]
        n0 = acc / np.linalg.norm(acc)
        t1, t2 = _frame(n0)
        R = np.stack([t1, t2, n0], axis=1)
        nb = np.array(self.nbr[i], dtype=np.int64)
        dn = self.V[nb] - self.V[i]
        d2 = np.sum(dn * dn, axis=1)
        nb = nb[np.lexsort((nb, d2))][:kmax - 1]
        d = self.V[nb] - self.V[i]
        xi, eta, zeta = d @ t1, d @ t2, d @ n0
        G = np.stack([xi, eta, xi * xi, xi * eta, eta * eta], axis=1)
        c = np.concatenate([[0.0], np.linalg.lstsq(G, zeta, rcond=None)[0]])
        idx = np.concatenate([[i], nb])
        dd = self.V[idx] - self.V[i]
        L = np.max(np.linalg.norm(dd, axis=1))
        x, y = dd @ t1 / L, dd @ t2 / L
        A = np.stack([np.ones(len(idx)), x, y, x * x, x * y, y * y], axis=1)
        P = np.linalg.pinv(A)
        return idx, self._grad_weights(R, c, 0.0, 0.0, P[1] / L, P[2] / L)

    def _vacc(self):
        if getattr(self, "_acc", None) is None:
            acc = np.zeros((self.m, 3))
            for k in range(3):
                np.add.at(acc, self.F[:, k], self.cross)
            self._acc = acc
        return self._acc

    def patch_geometry(self, t, z):
        """n and W of triangle t's patch over the point z (projected onto its plane)."""
        o, R, c = self.patch(t)
        qz = R.T @ (z - o)
        return _graph_geometry(R, c, qz[0], qz[1])

    # -- grid lines
    def line_hits(self, axis, b_vals, c_vals):
        """Crossings of the grid lines parallel to ``axis``: dict (ib, ic) -> list of
        (coordinate along the axis, triangle), for lines at the other two axes' grid values.

        A triangle is hit when the line's projection lies inside its projection, with the
        half-open rule: a point on an edge belongs to the triangle for which the edge, traversed
        counter-clockwise, points down (or along +b when horizontal)."""
        ax = [a for a in range(3) if a != axis]
        out = {}
        Vb, Vc, Va = self.V[:, ax[0]], self.V[:, ax[1]], self.V[:, axis]
        b0, db = b_vals[0], b_vals[1] - b_vals[0]
        c0, dc = c_vals[0], c_vals[1] - c_vals[0]
        nb, ncv = len(b_vals), len(c_vals)
        for t in range(self.F.shape[0]):
            i, j, k = self.F[t]
            P = [(Vb[i], Vc[i], Va[i]), (Vb[j], Vc[j], Va[j]), (Vb[k], Vc[k], Va[k])]
            s2 = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0])
            if s2 == 0.0:
                continue
            if s2 < 0:
                P = [P[0], P[2], P[1]]
                s2 = -s2
            lo_b, hi_b = min(p[0] for p in P), max(p[0] for p in P)
            lo_c, hi_c = min(p[1] for p in P), max(p[1] for p in P)
            kb0 = max(0, int(np.floor((lo_b - b0) / db)) - 1)
            kb1 = min(nb - 1, int(np.ceil((hi_b - b0) / db)) + 1)
            kc0 = max(0, int(np.floor((lo_c - c0) / dc)) - 1)
            kc1 = min(ncv - 1, int(np.ceil((hi_c - c0) / dc)) + 1)
            for ib in range(kb0, kb1 + 1):
                yb = b_vals[ib]
                if yb < lo_b or yb > hi_b:
                    continue
                for ic in range(kc0, kc1 + 1):
                    yc = c_vals[ic]
                    if yc < lo_c or yc > hi_c:
                        continue
                    lam = []
                    ok = True
                    for e in range(3):
                        A, B = P[(e + 1) % 3], P[(e + 2) % 3]       # edge opposite vertex e
                        eb, ec = B[0] - A[0], B[1] - A[1]
                        E = eb * (yc - A[1]) - ec * (yb - A[0])
                        if E < 0 or (E == 0 and not (ec < 0 or (ec == 0 and eb > 0))):
                            ok = False
                            break
                        lam.append(E)
                    if not ok:
                        continue
                    x = (lam[0] * P[0][2] + lam[1] * P[1][2] + lam[2] * P[2][2]) / s2
                    out.setdefault((ib, ic), []).append((x, t))
        for key in out:
            out[key].sort()
        return out
