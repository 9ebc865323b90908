"""Warm-start network for the GMRES initial density (FP64).  Test infrastructure only.

Not part of the paper: the paper starts every BIE iteration from psi = 0
(Algorithm 1).  This module restates, in plain NumPy, the small per-node
network the library uses to predict a better initial density, so that the
library's forward / backward / Adam kernels can be checked against it.

Features of interface node i (ncomp components, d dimensions):
    psi^{n-1}_c(i)/s, psi^{n-2}_c(i)/s, g'_c(i)/s_g      for every component c
    n(i) (d entries),  h * tr W(i)
with s = max|psi^{n-1}| and s_g = max|g'| (1 if zero).  The network predicts
y_c(i); the initial density is  2 psi^{n-1} - psi^{n-2} + s y.
Architecture: three tanh layers of width 128 and a linear output layer.
Loss: mean over nodes and outputs of (y - target)^2 / 2.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 128
LAYERS = 3


def n_features(ncomp, dim):
    return 3 * ncomp + dim + 1


def features(psi1, psi2, gp, normals, trW, h):
    """Per-node input rows (M, F) and the density scale s."""
    psi1 = np.atleast_2d(psi1)
    psi2 = np.atleast_2d(psi2)
    gp = np.atleast_2d(gp)
    s = np.max(np.abs(psi1))
    s = s if s > 0 else 1.0
    sg = np.max(np.abs(gp))
    sg = sg if sg > 0 else 1.0
    cols = []
    for c in range(psi1.shape[0]):
        cols += [psi1[c] / s, psi2[c] / s, gp[c] / sg]
    cols += [normals[:, a] for a in range(normals.shape[1])]
    cols += [h * trW]
    return np.stack(cols, axis=1), s


def target(psi, psi1, psi2, s):
    return ((np.atleast_2d(psi) - (2 * np.atleast_2d(psi1) - np.atleast_2d(psi2))) / s).T


def predict_density(y, psi1, psi2, s):
    return 2 * np.atleast_2d(psi1) - np.atleast_2d(psi2) + s * y.T


def init_params(n_in, n_out, seed=3):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [HIDDEN] * LAYERS + [n_out]
    params = []
    for i in range(len(dims) - 1):
        b = 1.0 / np.sqrt(dims[i])
        params.append([rng.uniform(-b, b, size=(dims[i + 1], dims[i])), np.zeros(dims[i + 1])])
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


def loss(y, t):
    return 0.5 * np.mean((y - t) ** 2)


def backward(params, acts, t):
    """Gradients of ``loss`` with respect to every weight and bias."""
    y = acts[-1]
    g = (y - t) / y.size
    grads = [None] * len(params)
    for i in reversed(range(len(params))):
        W, _ = params[i]
        a_in = acts[i]
        grads[i] = [g.T @ a_in, g.sum(axis=0)]
        if i > 0:
            g = (g @ W) * (1.0 - acts[i] ** 2)
    return grads


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
