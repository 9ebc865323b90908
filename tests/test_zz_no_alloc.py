"""kfbi_box_solve_noalloc (the box solve that allocates nothing) against kfbi_box_solve.

Calls in a row through the C ABI share the static scratch array: a coupled 128^3 FP64 field (the
largest case the 36 MiB array holds), then smaller 2D and 3D problems; each is compared element by
element with kfbi_box_solve of a problem set up on the same grid and coefficients and with the
oracle's box solve: FP64 to 1e-12; FP32 to 1e-6 against kfbi_box_solve (its tables are rounded
from FP64 values computed on the device rather than on the host) and to 5e-6 against the FP64
oracle (u32 = 6e-8 per DST stage over 2 log2(cells) stages and two axes).  A grid beyond the array's
size is rejected before any GPU work."""
import sys

import numpy as np
import pytest

from oracle import boxsolve as obs
from paper_2104_05024_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_05024_amd import kfbi as K  # noqa: E402

DEV = torch.device("cuda:0")


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def err(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


CASES = [
    ("coupled 128^3 FP64", W.ellipsoid(n_nodes=1024), W.box(3, 128), W.bidomain_coeffs(3, W.BidomainParams(), 0.01),
     torch.float64, 1e-12, 1e-12),
    ("2D 64^2 FP64", W.star2d(n_nodes=128), W.box(2, 64), W.scalar_coeffs(2, 1.0, 400.0), torch.float64, 1e-12,
     1e-12),
    ("anisotropic coupled 2D 256^2 FP32", W.circle2d(0.5, n_nodes=256), W.box(2, 256),
     W.Coeffs(2, [[3.0, 0.5], [2.0, 1.0]], 200.0), torch.float32, 1e-6, 5e-6),
    ("3D 32^3 FP64", W.ellipsoid(n_nodes=512), W.box(3, 32), W.scalar_coeffs(3, 1.0, 50.0), torch.float64, 1e-12,
     1e-12),
]


def test_noalloc_box_solve_matches_box_solve():
    for name, iface, grid, co, dt, tol, tol_oracle in CASES:
        say(f"[noalloc] {name}")
        f = np.random.default_rng(grid.cells).normal(size=(co.ncomp, grid.n ** grid.dim))
        ft = torch.tensor(f, dtype=dt, device=DEV)
        u = K.box_solve_noalloc(grid, co, ft).double().cpu().numpy()
        p = K.Problem(iface, grid, co)
        ref = p.box_solve(ft).double().cpu().numpy()
        p.close()
        e, eo = err(u, ref), err(u, obs.box_solve(f, grid, co))
        say(f"    vs kfbi_box_solve {e:.2e}, vs the oracle {eo:.2e}")
        assert e < tol and eo < tol_oracle
        # in place (f and u alias), as kfbi_box_solve allows
        K.box_solve_noalloc(grid, co, ft, out=ft)
        assert err(ft.double().cpu().numpy(), ref) < tol


def test_noalloc_rejects_grids_beyond_its_scratch():
    grid, co = W.box(3, 256), W.bidomain_coeffs(3, W.BidomainParams(), 0.01)
    f = torch.zeros(1, dtype=torch.float64, device=DEV)
    g, c = K.grid_desc(grid), K.coeffs_desc(co)
    import ctypes as C
    rc = K.lib().kfbi_box_solve_noalloc(C.byref(g), C.byref(c), C.c_void_p(f.data_ptr()), C.c_void_p(f.data_ptr()),
                                        K.KFBI_F64, None)
    assert rc == K.KFBI_EINVAL
    assert b"36 MiB" in K.lib().kfbi_last_error()
