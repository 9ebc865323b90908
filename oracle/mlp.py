"""Warm-start network for the GMRES initial density (FP64).  Test infrastructure only.

Not part of the paper: the paper starts every BIE iteration from psi = 0
(Algorithm 1).  This module restates, in plain NumPy, the small per-node
network the library uses to predict a better initial density, so that the
library's forward / backward / Adam kernels can be checked against it.

The previous solve left A psi^{n-1} = g'^{n-1}, so psi^n - psi^{n-1} =
A^{-1}(g'^n - g'^{n-1}), and A is one half of the identity plus a compact part
(Sec. 4, eq. bie).  The network approximates this change by a *local linear*
map whose coefficients depend on the local geometry only:

    geometry rows  G(i) = (n(i), h tr W(i))                      (static)
    change fields  F_c(i) = ((psi^{n-1} - psi^{n-2})_c / s_d,  (g'^n - g'^{n-1})_c / s_g)
    coefficients   K(i) = net(G(i))   (2 ncomp x ncomp entries used)
    prediction     y_c(i) = sum_f K_{c,f}(i) F_f(i),   psi0 = psi^{n-1} + s_d y

with s_d = max|psi^{n-1} - psi^{n-2}| and s_g = max|g'^n - g'^{n-1}|.  Applying
geometry-dependent weights to the fields' changes keeps the start as smooth as
the fields; a start with node-to-node noise slows GMRES down even when its
residual is small.  Architecture of net: three tanh layers of width 128 and a
linear output layer.  Loss: mean over nodes, components and recorded steps of
(y - target)^2 / 2, target = (psi^n - psi^{n-1}) / s_d.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 128
LAYERS = 3


def geometry_rows(normals, trW, h):
    """Static network inputs per node: the unit normal and h tr W."""
    return np.concatenate([normals, (h * trW)[:, None]], axis=1)


def change_fields(psi1, psi2, gp, gp_prev):
    """Per-node change fields F (M, 2 ncomp) and the scale s_d."""
    psi1, psi2 = np.atleast_2d(psi1), np.atleast_2d(psi2)
    gp, gp_prev = np.atleast_2d(gp), np.atleast_2d(gp_prev)
    dpsi, dg = psi1 - psi2, gp - gp_prev
    sd = np.max(np.abs(dpsi))
    sd = sd if sd > 0 else 1.0
    sg = np.max(np.abs(dg))
    sg = sg if sg > 0 else 1.0
    cols = []
    for c in range(psi1.shape[0]):
        cols += [dpsi[c] / sd, dg[c] / sg]
    return np.stack(cols, axis=1), sd


def combine(K, F, ncomp):
    """y_c = sum_f K[:, c nf + f] F[:, f] with nf = F.shape[1] fields."""
    nf = F.shape[1]
    return np.stack([np.sum(K[:, c * nf:(c + 1) * nf] * F, axis=1) for c in range(ncomp)], axis=1)


def combine_grad(dy, F, n_out):
    """dL/dK from dL/dy (zero in the unused outputs)."""
    nf = F.shape[1]
    dK = np.zeros((F.shape[0], n_out))
    for c in range(dy.shape[1]):
        dK[:, c * nf:(c + 1) * nf] = dy[:, c:c + 1] * F
    return dK


def target(psi, psi1, sd):
    return ((np.atleast_2d(psi) - np.atleast_2d(psi1)) / sd).T


def predict_density(y, psi1, sd):
    return np.atleast_2d(psi1) + sd * y.T


def init_params(n_in, n_out, seed=3, zero_last=True):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases; the output layer starts at
    zero so that the untrained network predicts no change (psi0 = psi^{n-1})."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [HIDDEN] * LAYERS + [n_out]
    params = []
    for i in range(len(dims) - 1):
        b = 1.0 / np.sqrt(dims[i])
        W = rng.uniform(-b, b, size=(dims[i + 1], dims[i]))
        if zero_last and i == len(dims) - 2:
            W[:] = 0.0
        params.append([W, np.zeros(dims[i + 1])])
    return params


def forward(params, x):
    """Returns the output (M, n_out) and the activations needed by ``backward``."""
    acts = [x]
    a = x
    for i, (W, b) in enumerate(params):
        z = a @ W.T + b
        a = np.tanh(z) if i < len(params) - 1 else z
        acts.append(a)
    return a, acts


def backward_from(params, acts, dy):
    """Gradients of sum(dy * output) with respect to every weight and bias."""
    g = dy
    grads = [None] * len(params)
    for i in reversed(range(len(params))):
        W, _ = params[i]
        grads[i] = [g.T @ acts[i], g.sum(axis=0)]
        if i > 0:
            g = (g @ W) * (1.0 - acts[i] ** 2)
    return grads


def loss_and_grad(params, G, samples, ncomp):
    """Mean squared loss over recorded steps [(F, T), ...] and its parameter gradients."""
    K, acts = forward(params, G)
    n = G.shape[0] * ncomp * len(samples)
    dK = np.zeros_like(K)
    loss = 0.0
    for F, T in samples:
        d = combine(K, F, ncomp) - T
        loss += 0.5 * np.sum(d * d) / n
        dK += combine_grad(d / n, F, K.shape[1])
    return loss, backward_from(params, acts, dK)


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); ``state`` holds step count and moments."""
    if not state:
        state["t"] = 0
        state["m"] = [[np.zeros_like(p) for p in layer] for layer in params]
        state["v"] = [[np.zeros_like(p) for p in layer] for layer in params]
    state["t"] += 1
    t = state["t"]
    for i in range(len(params)):
        for j in range(2):
            g = grads[i][j]
            state["m"][i][j] = b1 * state["m"][i][j] + (1 - b1) * g
            state["v"][i][j] = b2 * state["v"][i][j] + (1 - b2) * g * g
            mh = state["m"][i][j] / (1 - b1 ** t)
            vh = state["v"][i][j] / (1 - b2 ** t)
            params[i][j] = params[i][j] - lr * mh / (np.sqrt(vh) + eps)
    return params
