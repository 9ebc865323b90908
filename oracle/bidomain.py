"""Bidomain time step for the oracle (FP64).  Test infrastructure only.

* FitzHugh-Nagumo membrane model (Sec. 7 model paragraph):
  I_ion = H (q - V (V - theta)(1 - V)),  M(V, q) = alpha V - zeta q.
* Second-order Strang splitting (Sec. 3, eqs. ode1, diffusion, ode2):
  reaction for dt/2 by forward Euler, diffusion for dt by the implicit
  midpoint rule, reaction for dt/2 by backward Euler solved with Newton.
* The midpoint rule is a backward-Euler step of length dt/2 for
  w = (V^{n+1} + V^n)/2 followed by V^{n+1} = 2 w - V^n (Sec. 3).  The
  backward-Euler step of length dt/2 is the coupled modified-Helmholtz
  Neumann problem of eq. pde1 with kappa = C_m beta / (dt/2), written in the
  positive form: f = (kappa V, -kappa V + beta I_stim), g^N = 0 (eqs. bvp, BC).
"""
from __future__ import annotations

import numpy as np


def ionic_current(V, q, p):
    return p.H * (q - V * (V - p.theta) * (1.0 - V))


def reaction_forward_euler(V, q, dt_half, p):
    """Step 1 of the splitting: explicit Euler over dt/2."""
    Vn = V + dt_half * (-ionic_current(V, q, p) / p.Cm)
    qn = q + dt_half * (p.alpha * V - p.zeta * q)
    return Vn, qn


def reaction_backward_euler(V, q, dt_half, p):
    """Step 3 of the splitting: implicit Euler over dt/2, q eliminated, Newton on V.

    q' = (q + dt/2 alpha V') / (1 + dt/2 zeta) and
    F(V') = V' - V + (dt/2 / C_m) H (q'(V') - V'(V' - theta)(1 - V')) = 0.
    Newton from V' = V until |F| <= newton_tol, then one more step so that the
    root is resolved to rounding level.
    """
    a = dt_half * p.alpha / (1.0 + dt_half * p.zeta)
    qb = q / (1.0 + dt_half * p.zeta)
    c = dt_half * p.H / p.Cm

    def F(x):
        cub = x * (x - p.theta) * (1.0 - x)
        return x - V + c * (qb + a * x - cub)

    def dF(x):
        dcub = -3.0 * x * x + 2.0 * (1.0 + p.theta) * x - p.theta
        return 1.0 + c * (a - dcub)

    x = np.array(V, dtype=np.float64, copy=True)
    active = np.ones(x.shape, dtype=bool)
    for _ in range(p.newton_maxit):
        fx = F(x)
        conv = np.abs(fx) <= p.newton_tol
        x = x - fx / dF(x)                        # every entry takes the extra step once converged
        active = active & ~conv
        if not np.any(active):
            break
    qn = qb + a * x
    return x, qn


def diffusion_rhs(V, kappa, beta=1.0, I_stim=None):
    """f = (kappa V, -kappa V + beta I_stim) on every box node (the source extended over B)."""
    fe = -kappa * V
    if I_stim is not None:
        fe = fe + beta * I_stim
    return np.stack([kappa * V, fe])


def step(prob, p, V, q, dt, psi0=None, tol=1e-8, restart=50, maxit=500, I_stim=None):
    """One Strang step. prob is a two-component oracle Problem with kappa = 2 C_m beta / dt."""
    dth = 0.5 * dt
    kappa = 2.0 * p.Cm * p.beta / dt
    if abs(prob.coeffs.kappa - kappa) > 1e-12 * kappa:
        raise ValueError("problem kappa does not match 2 C_m beta / dt")
    V1, q1 = reaction_forward_euler(V, q, dth, p)
    f = diffusion_rhs(V1, kappa, p.beta, I_stim)
    g = np.zeros((2, prob.M))
    u, psi, info = prob.solve_neumann(g, f, psi0, tol, restart, maxit)
    V2 = 2.0 * (u[0] - u[1]) - V1
    V3, q3 = reaction_backward_euler(V2, q1, dth, p)
    return V3, q3, u, psi, info


def initial_state(grid, center, radius=0.1):
    """V = 1 inside a ball, 0 elsewhere; q = 0 (the patch stimulus of Sec. 7.4 / Example 4)."""
    from .geometry import grid_points
    pts = grid_points(grid)
    r2 = np.sum((pts - np.asarray(center)[None, :]) ** 2, axis=1)
    V = np.where(r2 < radius * radius, 1.0, 0.0)
    return V, np.zeros_like(V)
