"""Pins for oracle.gmres, oracle.bidomain and oracle.mlp (CPU only)."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import bidomain, geometry, gmres, kfbi, mlp
from paper_2104_05024_amd import workloads as W


# ----------------------------------------------------------------------------- GMRES / Richardson

def test_gmres_solves_nonsymmetric_system_with_restarts():
    rng = np.random.default_rng(0)
    n = 120
    A = np.eye(n) + 0.3 * rng.normal(size=(n, n)) / math.sqrt(n)
    b = rng.normal(size=n)
    x, info = gmres.gmres(lambda v: A @ v, b, np.zeros(n), tol=1e-12, restart=15, maxit=400)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    assert info["restarts"] >= 1 and info["rel_resid"] <= 1e-12


def test_gmres_warm_start_and_zero_rhs():
    n = 10
    A = np.diag(np.arange(1.0, n + 1))
    b = np.ones(n)
    x0 = np.linalg.solve(A, b)
    x, info = gmres.gmres(lambda v: A @ v, b, x0, tol=1e-10)
    assert info["iters"] == 0 and info["matvecs"] == 1
    x, info = gmres.gmres(lambda v: A @ v, np.zeros(n), np.ones(n), tol=1e-10)
    assert np.all(x == 0)


def test_richardson_converges_for_contraction():
    """The simple iteration with gamma in (0,1) converges when spec(A) lies in (0, 1]."""
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    A = Q @ np.diag(rng.uniform(0.3, 0.9, 30)) @ Q.T
    b = rng.normal(size=30)
    x, info = gmres.richardson(lambda v: A @ v, b, np.zeros(30), gamma=0.8, tol=1e-10)
    assert info["rel_resid"] <= 1e-10
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8)


# ----------------------------------------------------------------------------- FitzHugh-Nagumo

P = W.BidomainParams()


def test_forward_euler_closed_form():
    V = np.array([0.0, 0.2, 0.7, 1.1])
    q = np.array([0.0, 0.05, -0.1, 0.3])
    dt2 = 0.005
    Vn, qn = bidomain.reaction_forward_euler(V, q, dt2, P)
    I = 100.0 * (q - V * (V - 0.13) * (1 - V))
    np.testing.assert_allclose(Vn, V - dt2 * I, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(qn, q + dt2 * (0.25 * V - q), rtol=1e-15, atol=1e-16)


def test_backward_euler_newton_matches_brentq():
    rng = np.random.default_rng(2)
    V = rng.uniform(-0.3, 1.3, 64)
    q = rng.uniform(-0.1, 0.4, 64)
    dt2 = 0.005
    Vn, qn = bidomain.reaction_backward_euler(V, q, dt2, P)
    for i in range(64):
        def F(x):
            qq = (q[i] + dt2 * 0.25 * x) / (1 + dt2)
            return x - V[i] + dt2 * 100.0 * (qq - x * (x - 0.13) * (1 - x))
        r = optimize.brentq(F, -5, 5, xtol=1e-15, rtol=1e-15)
        assert abs(Vn[i] - r) <= 1e-12
        assert abs(qn[i] - (q[i] + dt2 * 0.25 * r) / (1 + dt2)) <= 1e-12
    # implicit-Euler residuals of both equations vanish
    I = 100.0 * (qn - Vn * (Vn - 0.13) * (1 - Vn))
    np.testing.assert_allclose(Vn - V, -dt2 * I, atol=1e-12)
    np.testing.assert_allclose(qn - q, dt2 * (0.25 * Vn - qn), atol=1e-14)


def test_newton_root_is_unique_at_dt_001():
    """F'(V) >= 1 - (dt/2) H max(dcubic) > 0 when dt < 2 C_m / (0.2956 H): monotone, one root."""
    th = 0.13
    max_slope = (1 + th) ** 2 / 3 - th              # max of d/dV V(V-th)(1-V)
    assert 0.01 / 2 * 100 * max_slope < 1


def _small_bidomain(cells=32, M=512, dt=0.01):
    iface = W.ellipsoid(n_nodes=M)
    grid = W.box(3, cells)
    return kfbi.Problem(iface, grid, W.bidomain_coeffs(3, P, dt)), iface, grid


def test_diffusion_step_conserves_tissue_integral_of_V():
    """With the reaction switched off, the midpoint diffusion step keeps int_Omega V (no-flux walls)."""
    prob, iface, grid = _small_bidomain()
    pts = geometry.grid_points(grid)
    V = np.exp(-30 * np.sum((pts - np.array([0.1, 0.0, 0.05])) ** 2, axis=1))
    kappa = prob.coeffs.kappa
    u, _, info = prob.solve_neumann(np.zeros((2, prob.M)), bidomain.diffusion_rhs(V, kappa), tol=1e-12)
    V2 = 2 * (u[0] - u[1]) - V
    s0, s1 = np.sum(V[prob.inside]), np.sum(V2[prob.inside])
    assert abs(s1 - s0) <= 2e-3 * s0
    assert np.max(V2) < np.max(V)                 # diffusion smooths the peak


def test_bidomain_step_gauge_and_midpoint_update():
    prob, iface, grid = _small_bidomain()
    V, q = bidomain.initial_state(grid, W.stimulus_center(iface), radius=0.3)
    V1, q1, u, psi, info = bidomain.step(prob, P, V, q, 0.01, tol=1e-10)
    assert info["rel_resid"] <= 1e-10
    assert abs(np.mean(u[1][prob.inside])) < 1e-13
    # shifting the potentials by a common constant is invisible in V
    kap = prob.coeffs.kappa
    Vh, qh = bidomain.reaction_forward_euler(V, q, 0.005, P)
    u2 = prob.reconstruct(bidomain.diffusion_rhs(Vh, kap), psi.ravel())
    np.testing.assert_allclose(u2, u, atol=1e-13)


# ----------------------------------------------------------------------------- MLP

def test_mlp_gradients_match_central_differences():
    """Parameter gradients of the recorded-steps loss against central differences."""
    rng = np.random.default_rng(5)
    M, ncomp = 23, 2
    G = rng.normal(size=(M, 4))
    samples = [(rng.normal(size=(M, 2 * ncomp)), rng.normal(size=(M, ncomp))) for _ in range(3)]
    params = mlp.init_params(4, 16, seed=3, zero_last=False)
    loss, grads = mlp.loss_and_grad(params, G, samples, ncomp)
    eps = 1e-6
    for li, (W_, b_) in enumerate(params):
        for arr, garr in ((W_, grads[li][0]), (b_, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = garr.reshape(-1)
            for k in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[k]
                flat[k] = old + eps
                lp = mlp.loss_and_grad(params, G, samples, ncomp)[0]
                flat[k] = old - eps
                lm = mlp.loss_and_grad(params, G, samples, ncomp)[0]
                flat[k] = old
                assert abs((lp - lm) / (2 * eps) - gflat[k]) <= 1e-7 * max(1.0, abs(gflat[k]))


def test_untrained_network_predicts_no_change():
    rng = np.random.default_rng(7)
    params = mlp.init_params(4, 16, seed=3)
    K, _ = mlp.forward(params, rng.normal(size=(9, 4)))
    assert np.all(K == 0)


def test_adam_first_step_is_lr_times_sign():
    params = [[np.array([[1.0, -2.0]]), np.array([0.5])]]
    grads = [[np.array([[0.3, -4.0]]), np.array([1e-3])]]
    st = {}
    mlp.adam_step(params, grads, st, lr=0.01)
    np.testing.assert_allclose(params[0][0], [[0.99, -1.99]], atol=1e-7)
    np.testing.assert_allclose(params[0][1], [0.49], atol=1e-5)


def test_change_fields_and_prediction_roundtrip():
    """With K the identity on the density-change field, the prediction is the linear
    extrapolation 2 psi^{n-1} - psi^{n-2}; the target of psi^n inverts the prediction."""
    rng = np.random.default_rng(6)
    M = 40
    psi1, psi2, psi, gp, gq = rng.normal(size=(5, 2, M))
    F, sd = mlp.change_fields(psi1, psi2, gp, gq)
    assert F.shape == (M, 4) and sd == pytest.approx(np.max(np.abs(psi1 - psi2)))
    assert np.max(np.abs(F[:, [0, 2]])) == pytest.approx(1.0)
    K = np.zeros((M, 16))
    K[:, 0] = 1.0                 # comp 0 <- its density change
    K[:, 4 + 2] = 1.0             # comp 1 <- its density change
    y = mlp.combine(K, F, 2)
    np.testing.assert_allclose(mlp.predict_density(y, psi1, sd), 2 * psi1 - psi2, atol=1e-13)
    t = mlp.target(psi, psi1, sd)
    np.testing.assert_allclose(mlp.predict_density(t, psi1, sd), psi, atol=1e-13)
