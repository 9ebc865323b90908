"""Closed 2D curves given only by their nodes (FP64, NumPy/SciPy).  Test infrastructure only.

In 2D the paper represents the boundary by quasi-uniform nodes and the periodic
cubic spline through them (Sec. 7, the paragraph on the numerical set-up).  The
spline here takes the node index as its parameter, t_j = j, separately for x and
y (scipy's periodic CubicSpline: the C2 closed interpolant).  Everything the
method needs from the boundary is read off this spline:

* normal n (pointing out of the tissue) and shape operator W = sigma k tau tau^T
  with the signed curvature k = (x'y'' - y'x'')/|X'|^3 of the spline, tau = X'/|X'|
  and sigma = +-1 chosen so that n points out of the tissue;
* the side of a grid node: the sign of (x - X(t*)).n(t*) at its closest point
  X(t*) on the curve (tissue where <= 1e-12, as for analytic shapes);
* intersections of a grid line with the curve: the real roots of the cubic
  pieces of one coordinate.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline
from scipy.spatial import cKDTree

SIDE_TOL = 1e-12
SAMPLES = 32            # dense samples per spline piece for the closest-point search


class SplineCurve:
    def __init__(self, surf):
        P = np.asarray(surf.points, dtype=np.float64)
        if P.ndim != 2 or P.shape[1] != 2 or P.shape[0] < 8:
            raise ValueError("a spline curve needs at least 8 points in 2D")
        self.m = m = P.shape[0]
        t = np.arange(m + 1, dtype=np.float64)
        self.cx = CubicSpline(t, np.append(P[:, 0], P[0, 0]), bc_type="periodic")
        self.cy = CubicSpline(t, np.append(P[:, 1], P[0, 1]), bc_type="periodic")
        self.P = P
        # signed area of the node polygon: > 0 for counter-clockwise travel
        area = 0.5 * np.sum(P[:, 0] * np.roll(P[:, 1], -1) - np.roll(P[:, 0], -1) * P[:, 1])
        # the left normal (-y', x') points into a counter-clockwise curve; n = sigma (y', -x')/|X'|
        self.sigma = float(surf.orient) * (1.0 if area > 0 else -1.0)
        self.orient = surf.orient

    # -- evaluation (t taken modulo m)
    def X(self, t, nu=0):
        t = np.mod(np.asarray(t, dtype=np.float64), self.m)
        return np.stack([self.cx(t, nu), self.cy(t, nu)], axis=-1)

    def tangent(self, t):
        X1 = self.X(t, 1)
        speed = np.sqrt(np.sum(X1 * X1, axis=-1))
        return X1 / speed[..., None], speed

    def normal_and_shape(self, t):
        X1, X2 = self.X(t, 1), self.X(t, 2)
        speed = np.sqrt(np.sum(X1 * X1, axis=-1))
        tau = X1 / speed[:, None]
        n = self.sigma * np.stack([X1[:, 1], -X1[:, 0]], axis=1) / speed[:, None]
        k = (X1[:, 0] * X2[:, 1] - X1[:, 1] * X2[:, 0]) / speed ** 3
        W = (self.sigma * k)[:, None, None] * tau[:, :, None] * tau[:, None, :]
        return n, W

    def samples(self, per_piece=SAMPLES):
        t = np.arange(self.m * per_piece, dtype=np.float64) / per_piece
        return t, self.X(t)

    # -- sides
    def signed_distance(self, pts):
        """(x - X(t*)).n(t*) at the closest point X(t*): negative in the tissue."""
        return self.closest(pts)[0]

    def closest(self, pts):
        """Signed distance and the parameter t* of the closest point on the curve."""
        pts = np.asarray(pts, dtype=np.float64)
        ts, xs = self.samples()
        _, k = cKDTree(xs).query(pts)
        t = ts[k]
        for _ in range(30):                     # Newton on (X(t) - x).X'(t) = 0
            X, X1, X2 = self.X(t), self.X(t, 1), self.X(t, 2)
            r = X - pts
            f1 = np.sum(r * X1, axis=1)
            f2 = np.sum(X1 * X1, axis=1) + np.sum(r * X2, axis=1)
            step = np.where(f2 > 0, -f1 / np.where(f2 > 0, f2, 1.0), 0.0)
            step = np.clip(step, -0.5 / SAMPLES, 0.5 / SAMPLES) if _ < 3 else np.clip(step, -0.5, 0.5)
            t = t + step
            if np.all(np.abs(step) < 1e-15):
                break
        t = np.mod(t, self.m)
        n, _ = self.normal_and_shape(t)
        return np.sum((pts - self.X(t)) * n, axis=1), t

    def tissue(self, pts):
        return self.signed_distance(pts) <= SIDE_TOL

    # -- grid lines
    def line_roots(self, coord, c):
        """Parameters t in [0, m) where coordinate ``coord`` (0: x, 1: y) of the curve equals c."""
        cs = self.cx if coord == 0 else self.cy
        r = np.asarray(cs.solve(c, discontinuity=False, extrapolate=False), dtype=np.float64)
        r = np.mod(r[np.isfinite(r)], self.m)
        r = np.sort(r)
        if r.size > 1:                          # a root at a knot is reported by both pieces
            keep = np.concatenate([[True], np.diff(r) > 1e-9])
            r = r[keep]
            if r.size > 1 and r[0] + self.m - r[-1] <= 1e-9:
                r = r[:-1]
        return r
