"""Python binding of libkfbi.so (ctypes).  Argument marshalling only: every step of the
method runs inside the HIP library.  Device buffers are torch tensors (HIP memory);
the binding passes their raw pointers and the current HIP stream.

The library must be built (``python -m paper_2104_05024_amd.build``); loading fails
loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkfbi.so")

KFBI_OK, KFBI_EINVAL, KFBI_EGEOM, KFBI_ENOCONV, KFBI_EHIP, KFBI_ENOMEM, KFBI_ENODEV = 0, -1, -2, -3, -4, -5, -6
KFBI_F64, KFBI_F32 = 0, 1
MAX_TERMS = 16

EXPORTED = [
    "kfbi_setup", "kfbi_destroy", "kfbi_query", "kfbi_table", "kfbi_apply", "kfbi_box_solve", "kfbi_solve_neumann",
    "bidomain_create", "bidomain_destroy", "bidomain_step", "bidomain_mlp_init", "bidomain_train",
    "bidomain_mlp_params", "bidomain_mlp_eval", "kfbi_strerror", "kfbi_last_error", "kfbi_kernel_time",
    "kfbi_batch_setup", "kfbi_batch_destroy", "kfbi_batch_query", "kfbi_batch_apply", "kfbi_batch_solve_neumann",
    "kfbi_batch_graph", "kfbi_get_tiles", "kfbi_set_tiles", "kfbi_use_graph", "bidomain_use_graph",
    "kfbi_profile", "bidomain_reset", "kfbi_box_solve_noalloc", "bidomain_true_resid", "kfbi_batch_merge",
]


class KfbiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kfbi error {code}: {msg}")
        self.code = code


class Surface(C.Structure):
    _fields_ = [("axes", C.c_double * 3), ("orient", C.c_int32), ("n_terms", C.c_int32), ("n_nodes", C.c_int64),
                ("coef", C.c_double * MAX_TERMS), ("exps", (C.c_int32 * 3) * MAX_TERMS),
                ("kind", C.c_int32), ("pad_", C.c_int32), ("points", C.c_void_p), ("tris", C.c_void_p),
                ("n_tris", C.c_int64)]


class Interface(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_surfaces", C.c_int32), ("surf", Surface * 2)]


class GridDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("cells", C.c_int32), ("lo", C.c_double), ("hi", C.c_double)]


class CoeffsDesc(C.Structure):
    _fields_ = [("ncomp", C.c_int32), ("pad_", C.c_int32), ("D", (C.c_double * 3) * 2), ("kappa", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iters", C.c_int32), ("precision", C.c_int32),
                ("x0", C.c_int32), ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("method", C.c_int32),
                ("gamma", C.c_double), ("true_resid", C.c_int32), ("pad_", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer", C.c_int32), ("matvecs_fp64", C.c_int32),
                ("matvecs_fp32", C.c_int32), ("rel_resid", C.c_double), ("gp_norm", C.c_double),
                ("warm_start_used", C.c_int32), ("pad_", C.c_int32), ("start_resid", C.c_double),
                ("true_resid", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class BidomainParamsDesc(C.Structure):
    _fields_ = [("Cm", C.c_double), ("beta", C.c_double), ("H", C.c_double), ("theta", C.c_double),
                ("alpha", C.c_double), ("zeta", C.c_double), ("newton_tol", C.c_double),
                ("newton_maxit", C.c_int32), ("warm_start", C.c_int32), ("solve", SolveOpts)]


class BidomainState(C.Structure):
    _fields_ = [("V", C.c_void_p), ("q", C.c_void_p), ("phi", C.c_void_p), ("psi_hist", C.c_void_p),
                ("I_stim", C.c_void_p)]


_lib = None


def lib():
    """Load libkfbi.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_05024_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64p, dp = C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_double
    L.kfbi_setup.argtypes = [C.POINTER(Interface), C.POINTER(GridDesc), C.POINTER(CoeffsDesc), C.c_uint32,
                             C.POINTER(vp)]
    L.kfbi_destroy.argtypes = [vp]
    L.kfbi_destroy.restype = None
    L.kfbi_query.argtypes = [vp, i64p, i64p, i64p, i64p]
    L.kfbi_table.argtypes = [vp, C.c_char_p, vp, i64p, C.POINTER(C.c_int32)]
    L.kfbi_apply.argtypes = [vp, vp, vp, i32, vp]
    L.kfbi_box_solve.argtypes = [vp, vp, vp, i32, vp]
    L.kfbi_solve_neumann.argtypes = [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    L.bidomain_create.argtypes = [vp, C.POINTER(BidomainParamsDesc), C.POINTER(vp)]
    L.bidomain_destroy.argtypes = [vp]
    L.bidomain_destroy.restype = None
    L.bidomain_step.argtypes = [vp, C.POINTER(BidomainState), dp, C.POINTER(SolveInfo), vp]
    L.bidomain_mlp_init.argtypes = [vp, i32, C.c_uint64]
    L.bidomain_train.argtypes = [vp, i32, dp, C.POINTER(dp), vp]
    L.bidomain_mlp_params.argtypes = [vp, C.POINTER(C.c_float), i64p]
    L.bidomain_mlp_eval.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp]
    L.kfbi_strerror.argtypes = [C.c_int]
    L.kfbi_strerror.restype = C.c_char_p
    L.kfbi_last_error.restype = C.c_char_p
    L.kfbi_kernel_time.argtypes = [vp, C.c_char_p, C.POINTER(dp), i64p]
    L.kfbi_profile.argtypes = [vp, i32]
    L.kfbi_get_tiles.argtypes = [vp, i32, C.POINTER(C.c_int32)]
    L.kfbi_use_graph.argtypes = [vp, i32]
    L.bidomain_use_graph.argtypes = [vp, i32]
    L.bidomain_reset.argtypes = [vp]
    L.bidomain_true_resid.argtypes = [vp, i32]
    L.kfbi_box_solve_noalloc.argtypes = [C.POINTER(GridDesc), C.POINTER(CoeffsDesc), vp, vp, i32, vp]
    L.kfbi_set_tiles.argtypes = [vp, i32, C.POINTER(C.c_int32)]
    L.kfbi_batch_setup.argtypes = [i32, C.POINTER(Interface), C.POINTER(GridDesc), C.POINTER(CoeffsDesc),
                                   C.POINTER(vp)]
    L.kfbi_batch_destroy.argtypes = [vp]
    L.kfbi_batch_destroy.restype = None
    L.kfbi_batch_query.argtypes = [vp, i32, i64p, i64p, i64p, i64p]
    L.kfbi_batch_apply.argtypes = [vp, vp, vp, i32, vp]
    L.kfbi_batch_solve_neumann.argtypes = [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    L.kfbi_batch_graph.argtypes = [vp, i32]
    L.kfbi_batch_merge.argtypes = [vp, i32]
    _lib = L
    return L


def _check(rc, allow=()):
    if rc != KFBI_OK and rc not in allow:
        L = lib()
        raise KfbiError(rc, f"{L.kfbi_strerror(rc).decode()}: {L.kfbi_last_error().decode()}")
    return rc


# ----------------------------------------------------------------------------- descriptors

SURF_KINDS = {"analytic": 0, "spline": 1, "mesh": 2}


def interface_desc(iface) -> Interface:
    """ctypes descriptor of an interface; node and triangle arrays stay referenced by the
    descriptor (attribute ``keep``) for as long as it lives."""
    d = Interface()
    d.dim = iface.dim
    d.n_surfaces = len(iface.surfaces)
    d.keep = []
    for s, surf in enumerate(iface.surfaces):
        cs = d.surf[s]
        kind = getattr(surf, "kind", "analytic")
        cs.kind = SURF_KINDS[kind]
        if kind != "analytic":
            pts = np.ascontiguousarray(surf.points, dtype=np.float64)
            if pts.shape != (surf.n_nodes, iface.dim):
                raise ValueError("points must have shape (n_nodes, dim)")
            d.keep.append(pts)
            cs.points = pts.ctypes.data
            if kind == "mesh":
                tris = np.ascontiguousarray(surf.tris, dtype=np.int32)
                d.keep.append(tris)
                cs.tris = tris.ctypes.data
                cs.n_tris = tris.shape[0]
        for a in range(iface.dim):
            cs.axes[a] = surf.axes[a]
        cs.orient = surf.orient
        cs.n_nodes = surf.n_nodes
        if len(surf.terms) > MAX_TERMS:
            raise ValueError("too many polynomial terms")
        cs.n_terms = len(surf.terms)
        for t, (coef, e) in enumerate(surf.terms):
            cs.coef[t] = coef
            for a in range(len(e)):
                cs.exps[t][a] = int(e[a])
    return d


def grid_desc(grid) -> GridDesc:
    return GridDesc(grid.dim, grid.cells, grid.lo, grid.hi)


def coeffs_desc(co) -> CoeffsDesc:
    d = CoeffsDesc()
    d.ncomp = co.ncomp
    for c in range(co.ncomp):
        for a in range(len(co.D[c])):
            d.D[c][a] = co.D[c][a]
        for a in range(len(co.D[c]), 3):
            d.D[c][a] = co.D[c][0]
    d.kappa = co.kappa
    return d


def box_solve_noalloc(grid, coeffs, f, out=None):
    """kfbi_box_solve_noalloc: u = S f for a grid and coefficients without a problem handle and
    without any allocation in the library (its work field lives in a static device array)."""
    import torch
    if out is None:
        out = torch.empty_like(f)
    dt = {torch.float64: KFBI_F64, torch.float32: KFBI_F32}[f.dtype]
    assert f.is_contiguous() and out.is_contiguous() and f.numel() == coeffs.ncomp * grid.n ** grid.dim
    g, c = grid_desc(grid), coeffs_desc(coeffs)
    _check(lib().kfbi_box_solve_noalloc(C.byref(g), C.byref(c), _ptr(f), _ptr(out), dt, _stream()))
    return out


def solve_opts(tol=1e-10, restart=50, max_iters=500, precision=0, x0=0, inner_tol=1e-4, max_outer=20,
               method=0, gamma=0.8, true_resid=0) -> SolveOpts:
    return SolveOpts(tol, restart, max_iters, precision, x0, inner_tol, max_outer, method, gamma,
                     1 if true_resid else 0, 0)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


# ----------------------------------------------------------------------------- problem

class Problem:
    """A KFBI problem: static tables on the host and (unless host_only) on the GPU."""

    def __init__(self, iface, grid, coeffs, host_only=False):
        self._h = C.c_void_p()
        self.dim, self.ncomp = grid.dim, coeffs.ncomp
        self._descs = (interface_desc(iface), grid_desc(grid), coeffs_desc(coeffs))
        _check(lib().kfbi_setup(C.byref(self._descs[0]), C.byref(self._descs[1]), C.byref(self._descs[2]),
                                1 if host_only else 0, C.byref(self._h)))
        M, N, nc, ni = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().kfbi_query(self._h, C.byref(M), C.byref(N), C.byref(nc), C.byref(ni)))
        self.M, self.N, self.n_crossings, self.n_irregular = M.value, N.value, nc.value, ni.value

    def close(self):
        if self._h:
            lib().kfbi_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def table(self, name):
        n, eb = C.c_int64(), C.c_int32()
        _check(lib().kfbi_table(self._h, name.encode(), None, C.byref(n), C.byref(eb)))
        dt = {1: np.int8, 8: np.int64 if name in _INT_TABLES else np.float64}[eb.value]
        out = np.zeros(n.value, dtype=dt)
        _check(lib().kfbi_table(self._h, name.encode(), out.ctypes.data_as(C.c_void_p), C.byref(n), C.byref(eb)))
        return out

    def apply(self, psi, out=None):
        """out = A psi on the GPU; psi is a (ncomp, M) torch tensor (float64 or float32)."""
        import torch
        if out is None:
            out = torch.empty_like(psi)
        dt = {torch.float64: KFBI_F64, torch.float32: KFBI_F32}[psi.dtype]
        assert psi.is_contiguous() and out.is_contiguous() and psi.numel() == self.ncomp * self.M
        _check(lib().kfbi_apply(self._h, _ptr(psi), _ptr(out), dt, _stream()))
        return out

    def box_solve(self, f, out=None):
        """u = S f (the DST-I box solve alone); f is a (ncomp, N^d) torch tensor."""
        import torch
        if out is None:
            out = torch.empty_like(f)
        dt = {torch.float64: KFBI_F64, torch.float32: KFBI_F32}[f.dtype]
        assert f.is_contiguous() and out.is_contiguous() and f.numel() == self.ncomp * self.N ** self.dim
        _check(lib().kfbi_box_solve(self._h, _ptr(f), _ptr(out), dt, _stream()))
        return out

    def solve_neumann(self, g, f, psi=None, u=None, allow_noconv=False, **opts):
        """Solve the Neumann problem; g (ncomp, M) or None, f (ncomp, N^d) float64 tensors."""
        import torch
        dev = f.device
        if u is None:
            u = torch.empty_like(f)
        if psi is None:
            psi = torch.zeros(self.ncomp, self.M, dtype=torch.float64, device=dev)
            opts.setdefault("x0", 0)
        else:
            opts.setdefault("x0", 1)
        o = solve_opts(**opts)
        info = SolveInfo()
        rc = lib().kfbi_solve_neumann(self._h, _ptr(g), _ptr(f), _ptr(u), _ptr(psi), C.byref(o), C.byref(info),
                                      _stream())
        _check(rc, allow=(KFBI_ENOCONV,) if allow_noconv else ())
        return u, psi, info.as_dict()

    def profile(self, enable=True):
        _check(lib().kfbi_profile(self._h, 1 if enable else 0))

    def use_graph(self, enable=True):
        _check(lib().kfbi_use_graph(self._h, 1 if enable else 0))

    def tiles(self, dtype=KFBI_F64):
        """Autotuned DST tile widths (x, y, last-axis pass) for KFBI_F64 / KFBI_F32."""
        w = (C.c_int32 * 3)()
        _check(lib().kfbi_get_tiles(self._h, dtype, w))
        return tuple(w)

    def set_tiles(self, widths, dtype=KFBI_F64):
        w = (C.c_int32 * 3)(*widths)
        _check(lib().kfbi_set_tiles(self._h, dtype, w))

    def kernel_time(self, name):
        us, n = C.c_double(), C.c_int64()
        _check(lib().kfbi_kernel_time(self._h, name.encode(), C.byref(us), C.byref(n)))
        return us.value, n.value


class Batch:
    """Many 2D one-component Neumann problems solved together (size-grouped DST launches,
    work-list interface kernels, lockstep GMRES with a captured Arnoldi step)."""

    def __init__(self, problems):
        """problems: list of (interface, grid, coeffs) with dim 2 and one component."""
        n = len(problems)
        self.n = n
        self._if_keep = [interface_desc(p[0]) for p in problems]     # owns the node arrays
        self._ifs = (Interface * n)(*self._if_keep)
        self._grs = (GridDesc * n)(*[grid_desc(p[1]) for p in problems])
        self._cos = (CoeffsDesc * n)(*[coeffs_desc(p[2]) for p in problems])
        self._h = C.c_void_p()
        _check(lib().kfbi_batch_setup(n, self._ifs, self._grs, self._cos, C.byref(self._h)))
        self.M, self.N, self.ioff, self.goff = [], [], [], []
        for i in range(n):
            M, N, io, go = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
            _check(lib().kfbi_batch_query(self._h, i, C.byref(M), C.byref(N), C.byref(io), C.byref(go)))
            self.M.append(M.value)
            self.N.append(N.value)
            self.ioff.append(io.value)
            self.goff.append(go.value)
        L, G = C.c_int64(), C.c_int64()
        _check(lib().kfbi_batch_query(self._h, -1, None, None, C.byref(L), C.byref(G)))
        self.L, self.G = L.value, G.value

    def close(self):
        if self._h:
            lib().kfbi_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def graph(self, enable=True):
        _check(lib().kfbi_batch_graph(self._h, 1 if enable else 0))

    def merge(self, enable=True):
        """One DST launch per pass over all size groups (default) or one per group and pass."""
        _check(lib().kfbi_batch_merge(self._h, 1 if enable else 0))

    def apply(self, psi, out=None):
        """A psi for every problem; psi is a concatenated (L,) torch tensor (float64 / float32)."""
        import torch
        if out is None:
            out = torch.empty_like(psi)
        dt = {torch.float64: KFBI_F64, torch.float32: KFBI_F32}[psi.dtype]
        assert psi.is_contiguous() and out.is_contiguous() and psi.numel() == self.L
        _check(lib().kfbi_batch_apply(self._h, _ptr(psi), _ptr(out), dt, _stream()))
        return out

    def solve_neumann(self, g, f, psi=None, u=None, allow_noconv=False, **opts):
        """g: (L,) or None, f: (G,) concatenated float64 tensors; returns u, psi, [info per problem]."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        if psi is None:
            psi = torch.zeros(self.L, dtype=torch.float64, device=f.device)
            opts.setdefault("x0", 0)
        else:
            opts.setdefault("x0", 1)
        assert f.numel() == self.G and psi.numel() == self.L
        o = solve_opts(**opts)
        infos = (SolveInfo * self.n)()
        rc = lib().kfbi_batch_solve_neumann(self._h, _ptr(g), _ptr(f), _ptr(u), _ptr(psi), C.byref(o), infos,
                                            _stream())
        _check(rc, allow=(KFBI_ENOCONV,) if allow_noconv else ())
        return u, psi, [i.as_dict() for i in infos]


_INT_TABLES = {"cross_axis", "cross_surf", "cross_pin", "cross_pout", "z_idx", "q_idx", "st_lin", "irregular"}


def bidomain_params(p, tol=1e-8, precision=0, warm_start=0, restart=50, max_iters=500, inner_tol=1e-4,
                    max_outer=20, method=0, gamma=0.8, true_resid=0):
    d = BidomainParamsDesc()
    d.Cm, d.beta, d.H, d.theta, d.alpha, d.zeta = p.Cm, p.beta, p.H, p.theta, p.alpha, p.zeta
    d.newton_tol, d.newton_maxit = p.newton_tol, p.newton_maxit
    d.warm_start = warm_start
    d.solve = solve_opts(tol=tol, restart=restart, max_iters=max_iters, precision=precision, x0=1,
                         inner_tol=inner_tol, max_outer=max_outer, method=method, gamma=gamma,
                         true_resid=true_resid)
    return d


class Bidomain:
    """Strang-split FitzHugh-Nagumo bidomain stepper on a two-component Problem."""

    def __init__(self, problem: Problem, params, **kw):
        self.problem = problem
        self._params = bidomain_params(params, **kw)
        self._h = C.c_void_p()
        _check(lib().bidomain_create(problem.handle, C.byref(self._params), C.byref(self._h)))

    def close(self):
        if self._h:
            lib().bidomain_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, V, q, psi_hist, dt, phi=None, allow_noconv=False, I_stim=None):
        """One Strang step; I_stim (optional) is a stimulus current on the box nodes."""
        st = BidomainState(V.data_ptr(), q.data_ptr(), phi.data_ptr() if phi is not None else None,
                           psi_hist.data_ptr(), I_stim.data_ptr() if I_stim is not None else None)
        info = SolveInfo()
        rc = lib().bidomain_step(self._h, C.byref(st), dt, C.byref(info), _stream())
        _check(rc, allow=(KFBI_ENOCONV,) if allow_noconv else ())
        return info.as_dict()

    def use_graph(self, enable=True):
        _check(lib().bidomain_use_graph(self._h, 1 if enable else 0))

    def reset(self):
        _check(lib().bidomain_reset(self._h))

    def true_resid(self, enable=True):
        """Report the FP64 residual of every following solve from an explicit product."""
        _check(lib().bidomain_true_resid(self._h, 1 if enable else 0))

    def mlp_init(self, capacity=256, seed=3):
        _check(lib().bidomain_mlp_init(self._h, capacity, seed))

    def train(self, epochs, lr=1e-3):
        loss = C.c_double()
        _check(lib().bidomain_train(self._h, epochs, lr, C.byref(loss), _stream()))
        return loss.value

    def mlp_eval(self, X, dY=None):
        """Network outputs on host rows X [R][16]; with dY [R][16] also the parameter gradients
        of sum(dY * outputs), in mlp_params order."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        R = X.shape[0]
        Y = np.zeros((R, 16), dtype=np.float32)
        grad = None
        dYp = None
        if dY is not None:
            dYp = np.ascontiguousarray(dY, dtype=np.float32)
            grad = np.zeros(self.mlp_params().size, dtype=np.float32)
        _check(lib().bidomain_mlp_eval(self._h, X.ctypes.data_as(C.c_void_p), R, Y.ctypes.data_as(C.c_void_p),
                                       dYp.ctypes.data_as(C.c_void_p) if dYp is not None else None,
                                       grad.ctypes.data_as(C.c_void_p) if grad is not None else None, _stream()))
        return Y, grad

    def mlp_params(self):
        n = C.c_int64()
        _check(lib().bidomain_mlp_params(self._h, None, C.byref(n)))
        out = np.zeros(n.value, dtype=np.float32)
        _check(lib().bidomain_mlp_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), C.byref(n)))
        return out
