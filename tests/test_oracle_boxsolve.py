"""Pins for oracle.boxsolve: dense LU of the assembled operator and exact sine eigenvectors."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import boxsolve
from paper_2104_05024_amd import workloads as W


CASES = [
    (2, 8, W.Coeffs(1, [[1.0, 1.0]], 400.0)),
    (2, 16, W.Coeffs(1, [[30.0, 5.0]], 7.0)),
    (2, 16, W.Coeffs(2, [[1.0, 1.0], [2.0, 2.0]], 200.0)),
    (2, 12, W.Coeffs(2, [[30.0, 5.0], [20.0, 10.0]], 50.0)),
    (3, 8, W.Coeffs(1, [[1.0, 1.0, 1.0]], 400.0)),
    (3, 8, W.Coeffs(2, [[1.0, 1.0, 1.0], [2.0, 2.0, 2.0]], 200.0)),
    (3, 6, W.Coeffs(2, [[30.0, 5.0, 5.0], [20.0, 10.0, 10.0]], 3.0)),
]


@pytest.mark.parametrize("dim,cells,coeffs", CASES)
def test_fast_solver_matches_dense_lu(dim, cells, coeffs):
    grid = W.box(dim, cells)
    n = grid.n ** dim
    rhs = np.random.default_rng(cells).normal(size=(coeffs.ncomp, n))
    A = boxsolve.assemble(grid, coeffs)
    ref = spla.splu(A.tocsc()).solve(rhs.ravel()).reshape(coeffs.ncomp, n)
    u = boxsolve.box_solve(rhs, grid, coeffs)
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)
    # and the operator applied to the solution gives back the right-hand side
    assert np.linalg.norm(A @ u.ravel() - rhs.ravel()) <= 1e-11 * np.linalg.norm(rhs)


@pytest.mark.parametrize("dim", [2, 3])
def test_sine_mode_is_exact_eigenvector(dim):
    cells = 16
    grid = W.box(dim, cells)
    N = grid.n
    k = (3, 5, 2)[:dim]
    idx = np.arange(1, N + 1)
    modes = [np.sin(np.pi * k[a] * idx / cells) for a in range(dim)]
    if dim == 2:
        f = modes[1][:, None] * modes[0][None, :]
    else:
        f = modes[2][:, None, None] * modes[1][None, :, None] * modes[0][None, None, :]
    D = [1.3, 0.7, 2.1][:dim]
    kap = 17.0
    lam = sum(D[a] * 4 / grid.h ** 2 * np.sin(np.pi * k[a] / (2 * cells)) ** 2 for a in range(dim)) + kap
    u = boxsolve.box_solve(f.reshape(1, -1), grid, W.Coeffs(1, [D], kap))
    np.testing.assert_allclose(u[0], f.ravel() / lam, atol=1e-13 * np.max(np.abs(f)) / lam)


def test_eigenvalues_closed_form():
    lam = boxsolve.eigenvalues(7, 0.25)
    ref = 4 / 0.25 ** 2 * np.sin(np.arange(1, 8) * np.pi / 16) ** 2
    np.testing.assert_allclose(lam, ref, rtol=1e-15)
