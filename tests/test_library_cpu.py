"""CPU checks of the HIP library: it loads, exports every declared symbol, and its host-side
setup tables (built by C++ in kfbi_setup, host-only mode) agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import kfbi as ok
from paper_2104_05024_amd import kfbi as K
from paper_2104_05024_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kfbi.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = K.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(K.EXPORTED) <= set(names)


def test_error_codes_without_gpu():
    L = K.lib()
    assert L.kfbi_strerror(K.KFBI_EGEOM) == b"geometry outside the method's assumptions"
    # interface closer than 3h to the box
    with pytest.raises(K.KfbiError) as e:
        K.Problem(W.circle2d(1.15, 64), W.box(2, 32), W.scalar_coeffs(2), host_only=True)
    assert e.value.code == K.KFBI_EGEOM
    # conductivities must be positive on every axis (anisotropic ones are accepted)
    with pytest.raises(K.KfbiError) as e:
        K.Problem(W.star2d(n_nodes=64), W.box(2, 32), W.Coeffs(1, [[30.0, -5.0]], 1.0), host_only=True)
    assert e.value.code == K.KFBI_EINVAL
    K.Problem(W.star2d(n_nodes=64), W.box(2, 32), W.Coeffs(1, [[30.0, 5.0]], 1.0), host_only=True).close()
    # node-given boundaries: a mesh with a hole, a spline in 3D
    V, F = W.icosphere(2)
    with pytest.raises(K.KfbiError) as e:
        K.Problem(W.Interface(3, [W.mesh_surface(0.5 * V, F[:-1])]), W.box(3, 32), W.scalar_coeffs(3), host_only=True)
    assert e.value.code == K.KFBI_EGEOM
    with pytest.raises(K.KfbiError) as e:
        K.Problem(W.Interface(3, [W.mesh_surface(0.5 * V, F)]), W.box(2, 32), W.scalar_coeffs(2), host_only=True)
    assert e.value.code == K.KFBI_EINVAL
    # a host-only problem refuses device calls before touching the GPU
    p = K.Problem(W.star2d(n_nodes=64), W.box(2, 32), W.scalar_coeffs(2), host_only=True)
    rc = L.kfbi_apply(p.handle, ctypes.c_void_p(8), ctypes.c_void_p(8), 0, None)
    assert rc == K.KFBI_ENODEV
    p.close()


CASES = {
    "star2d_64": (W.star2d(n_nodes=128), W.box(2, 64), W.scalar_coeffs(2)),
    "ellipsoid_32": (W.ellipsoid(n_nodes=1024), W.box(3, 32), W.scalar_coeffs(3)),
    "ellipsoid_64_tip_on_grid": (W.ellipsoid(n_nodes=2048), W.box(3, 64), W.scalar_coeffs(3)),
    "psphere_32": (W.perturbed_sphere(n_nodes=1500), W.box(3, 32), W.scalar_coeffs(3)),
    "shell_64": (W.thick_shell(n_nodes=3000), W.box(3, 64), W.Coeffs(2, [[1.0] * 3, [2.0] * 3], 200.0)),
    "heart_spline_128": (W.heart2d(256), W.box(2, 128), W.scalar_coeffs(2)),
    "circle_spline_cw_64": (W.spline_circle(0.55, 100, clockwise=True), W.box(2, 64), W.scalar_coeffs(2)),
    # an interface node on a grid node: the circle's node j = 0 is the grid node (x_24, y_16)
    "circle_spline_node_on_grid_32": (W.spline_star(-1.2 + 24 * (2.4 / 32), 0.0, 5, 64), W.box(2, 32),
                                      W.scalar_coeffs(2)),
    "mesh_sphere_32": (W.mesh_sphere(0.5, 3), W.box(3, 32), W.scalar_coeffs(3)),
    "mesh_ellipsoid_flipped_32": (W.mesh_ellipsoid(level=3, flip=True), W.box(3, 32), W.scalar_coeffs(3)),
    "mesh_shell_64": (W.mesh_shell(level_out=4, level_in=3), W.box(3, 64),
                      W.Coeffs(2, [[1.0] * 3, [2.0] * 3], 200.0)),
    "mesh_vertex_on_grid_32": (None, W.box(3, 32), W.scalar_coeffs(3)),
}


def _vertex_on_grid(grid):
    """The level-3 mesh sphere with the vertex nearest a grid node moved onto that node."""
    s = W.mesh_sphere(0.5, 3).surfaces[0]
    P = s.points.copy()
    c = grid.lo + grid.h * np.arange(1, grid.cells)
    node = c[np.argmin(np.abs(c[:, None, None] - P[None]), axis=0)]     # nearest grid coordinates
    j = int(np.argmin(np.sum((node - P) ** 2, axis=1)))
    P[j] = node[j]
    return W.Interface(3, [W.mesh_surface(P, s.tris)])


@pytest.mark.parametrize("name", list(CASES))
def test_setup_tables_match_oracle(name):
    iface, grid, co = CASES[name]
    if iface is None:
        iface = _vertex_on_grid(grid)
    P = K.Problem(iface, grid, co, host_only=True)
    O = ok.Problem(iface, grid, co)
    assert (P.M, P.n_crossings, P.n_irregular) == (O.M, O.cross.count, len(O.irregular))
    exact = {"inside": O.inside.astype(np.int8), "cross_axis": O.cross.axis, "cross_pin": O.cross.p_in,
             "cross_pout": O.cross.p_out, "z_idx": O.z_idx, "q_idx": O.q_idx, "st_lin": O.st_lin,
             "irregular": O.irregular}
    for k, v in exact.items():
        np.testing.assert_array_equal(P.table(k), np.asarray(v).ravel(), err_msg=k)
    close = {"nodes_X": O.nodes.X, "nodes_n": O.nodes.n, "nodes_W": O.nodes.W, "cross_z": O.cross.z,
             "cross_n": O.cross.n, "cross_W": O.cross.W,
             "z_w0": O.z_w0, "z_wg": O.z_wg, "q_wg": O.q_wg, "st_r": O.st_r, "st_wgrad": O.st_wgrad}
    if iface.surfaces[0].kind == "mesh":        # the triangle of each crossing
        np.testing.assert_array_equal(P.table("cross_t"), O.cross.tparam)
    if iface.surfaces[0].kind == "spline":      # the spline parameter, compared on the circle of length m
        m = iface.surfaces[0].n_nodes
        dt = np.mod(P.table("cross_t") - O.cross.tparam + m / 2, m) - m / 2
        assert np.max(np.abs(dt)) < 1e-10
    for k, v in close.items():
        v = np.asarray(v).ravel()
        scale = max(1.0, np.max(np.abs(v)))
        np.testing.assert_allclose(P.table(k), v, rtol=0, atol=1e-12 * scale, err_msg=k)
    P.close()
