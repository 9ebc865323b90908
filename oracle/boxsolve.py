"""Box operator and its fast solver for the oracle (FP64).  Test infrastructure only.

Sec. 5.2 (eq. FDE): second-order centred differences on the uniform grid of
the box B with I intervals per axis, written here in the positive form

    sum_a D_{c,a} (2 u_p - u_{p+e_a} - u_{p-e_a}) / h^2 + (K u)_p = rhs_p,

with K = kappa for one component and K = kappa [[1, -1], [-1, 1]] for the
coupled intra/extracellular pair (Sec. 3, eq. bvp; the paper's right-hand side
is the negative of ours).  The unknowns are the (I-1)^d interior nodes with
u = 0 on the box boundary (the interface problems of Sec. 5.1 carry v = 0 on
the box boundary).  The sine modes diagonalise each axis, so the solve is a
DST-I per axis, a division by the eigenvalues (a 2x2 solve per mode for the
coupled pair) and an inverse DST-I (end of Sec. 5.3).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft
import scipy.sparse as sp

# the FFTs use every host core the process may run on (independent 1D transforms: the result does
# not depend on the count)
WORKERS = len(os.sched_getaffinity(0))


def eigenvalues(N, h):
    """lambda_k = (4/h^2) sin^2(k pi / (2(N+1))), k = 1..N: eigenvalues of -D2 with zero ends."""
    k = np.arange(1, N + 1, dtype=np.float64)
    return 4.0 / h ** 2 * np.sin(k * np.pi / (2.0 * (N + 1))) ** 2


def _mode_sums(dim, N, h, Dc):
    lam = eigenvalues(N, h)
    if dim == 2:
        return Dc[1] * lam[:, None] + Dc[0] * lam[None, :]                 # [ky][kx]
    return (Dc[2] * lam[:, None, None] + Dc[1] * lam[None, :, None]
            + Dc[0] * lam[None, None, :])                                   # [kz][ky][kx]


def box_solve(rhs, grid, coeffs):
    """Solve the box system for rhs of shape (ncomp, N^d) (x fastest); returns the same shape."""
    d, N, h = grid.dim, grid.n, grid.h
    shape = (N,) * d
    f = rhs.reshape((coeffs.ncomp,) + shape)
    fh = np.stack([scipy.fft.dstn(f[c], type=1, workers=WORKERS) for c in range(coeffs.ncomp)])
    kap = coeffs.kappa
    if coeffs.ncomp == 1:
        uh = fh / (_mode_sums(d, N, h, coeffs.D[0]) + kap)[None]
    else:
        ai = _mode_sums(d, N, h, coeffs.D[0])
        ae = _mode_sums(d, N, h, coeffs.D[1])
        det = (ai + kap) * (ae + kap) - kap * kap
        ui = ((ae + kap) * fh[0] + kap * fh[1]) / det
        ue = (kap * fh[0] + (ai + kap) * fh[1]) / det
        uh = np.stack([ui, ue])
    u = np.stack([scipy.fft.idstn(uh[c], type=1, workers=WORKERS) for c in range(coeffs.ncomp)])
    return u.reshape(coeffs.ncomp, -1)


def assemble(grid, coeffs):
    """Sparse matrix of the box operator (pin for the fast solver on tiny grids)."""
    d, N, h = grid.dim, grid.n, grid.h
    I1 = sp.identity(N, format="csr")
    T = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1], format="csr") / h ** 2
    blocks = []
    for c in range(coeffs.ncomp):
        Dc = coeffs.D[c]
        if d == 2:
            A = Dc[0] * sp.kron(I1, T) + Dc[1] * sp.kron(T, I1)
        else:
            A = (Dc[0] * sp.kron(sp.kron(I1, I1), T) + Dc[1] * sp.kron(sp.kron(I1, T), I1)
                 + Dc[2] * sp.kron(sp.kron(T, I1), I1))
        blocks.append(A)
    n = N ** d
    Id = sp.identity(n, format="csr")
    k = coeffs.kappa
    if coeffs.ncomp == 1:
        return (blocks[0] + k * Id).tocsr()
    return sp.bmat([[blocks[0] + k * Id, -k * Id], [-k * Id, blocks[1] + k * Id]]).tocsr()
