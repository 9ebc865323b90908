"""Iterative solvers for A psi = g (Sec. 4).  Test infrastructure only.

* ``gmres``: restarted GMRES(m) with modified Gram-Schmidt Arnoldi and Givens
  rotations (the Krylov improvement of the simple iteration named at the end
  of Sec. 4).  Convergence is ||g - A psi||_2 <= tol ||g||_2, judged by the
  Givens residual inside a cycle and by the true residual at each restart.
* ``richardson``: the simple iteration psi <- psi + 2 gamma (g - A psi)
  (Sec. 4, eq. simple iteration; Algorithm 1); for a singular operator (the coupled
  pair) its residual may be measured without the null direction (a reading).
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, x0, tol=1e-10, restart=50, maxit=500):
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = np.linalg.norm(b)
    info = {"iters": 0, "matvecs": 0, "restarts": 0, "rel_resid": 0.0}
    if bnorm == 0.0:
        return np.zeros_like(b), info
    r = b - matvec(x)
    info["matvecs"] += 1
    beta = np.linalg.norm(r)
    its = 0
    while beta > tol * bnorm and its < maxit:
        m = restart
        V = np.zeros((m + 1, b.size))
        Hh = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        gv = np.zeros(m + 1)
        gv[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            w = matvec(V[j])
            info["matvecs"] += 1
            its += 1
            for i in range(j + 1):
                Hh[i, j] = np.dot(w, V[i])
                w = w - Hh[i, j] * V[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            if Hh[j + 1, j] > 0:
                V[j + 1] = w / Hh[j + 1, j]
            for i in range(j):
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = t
            den = np.hypot(Hh[j, j], Hh[j + 1, j])
            cs[j], sn[j] = Hh[j, j] / den, Hh[j + 1, j] / den
            Hh[j, j] = den
            Hh[j + 1, j] = 0.0
            gv[j + 1] = -sn[j] * gv[j]
            gv[j] = cs[j] * gv[j]
            j_end = j + 1
            if abs(gv[j + 1]) <= tol * bnorm or its >= maxit:
                break
        y = np.linalg.solve(np.triu(Hh[:j_end, :j_end]), gv[:j_end])
        x = x + V[:j_end].T @ y
        if abs(gv[j_end]) <= tol * bnorm:
            beta = abs(gv[j_end])
            break
        r = b - matvec(x)
        info["matvecs"] += 1
        info["restarts"] += 1
        beta = np.linalg.norm(r)
    info["iters"] = its
    info["rel_resid"] = beta / bnorm
    return x, info


def richardson(matvec, b, x0, gamma=0.8, tol=1e-8, maxit=500, null=None):
    """The simple iteration.  null (unit vector, optional): the operator's null direction; the
    residual and the right-hand side are then measured without their component along it (the
    part of b no x can match when the operator is singular up to the discretisation), while the
    iterates are unchanged."""
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)

    def norm(v):
        if null is None:
            return np.linalg.norm(v)
        return np.linalg.norm(v - np.dot(null, v) * null)

    bnorm = norm(b)
    info = {"iters": 0, "matvecs": 0, "rel_resid": 0.0}
    if bnorm == 0.0:
        return np.zeros_like(b), info
    for it in range(maxit + 1):
        r = b - matvec(x)
        info["matvecs"] += 1
        rel = norm(r) / bnorm
        info["rel_resid"] = rel
        if rel <= tol or it == maxit:
            break
        x = x + 2.0 * gamma * r
        info["iters"] += 1
    return x, info
