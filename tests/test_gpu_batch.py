"""Batched 2D Neumann problems on the GPU: 64 seeded problems of grid sizes 64..1024 and
star shapes with 3-8 lobes, one batch.  Parity against the FP64 oracle (element by element) on
small problems and on a 512^2 and a 1024^2 member, against the single-problem GPU path on all,
manufactured-solution accuracy on all, the mixed-precision batch against the FP64 batch, the
captured Arnoldi step against direct launches, and the merged DST launches against one launch per
size group."""
import sys
import time

import numpy as np
import pytest

from oracle import geometry as ogeo
from oracle import kfbi as ok
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
    """Largest element-wise difference relative to the largest reference magnitude."""
    a, b = np.ravel(a), np.ravel(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def T(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def mms(iface, grid, kappa):
    """u = e^x sin(pi y): source on the grid, Neumann data at the oracle's interface nodes."""
    pts = ogeo.grid_points(grid)
    ue = np.exp(pts[:, 0]) * np.sin(np.pi * pts[:, 1])
    nodes = ogeo.Nodes(iface)
    X, n = nodes.X, nodes.n
    grad = np.stack([np.exp(X[:, 0]) * np.sin(np.pi * X[:, 1]),
                     np.pi * np.exp(X[:, 0]) * np.cos(np.pi * X[:, 1])], 1)
    return (np.pi ** 2 - 1 + kappa) * ue, np.sum(n * grad, 1), ue


@pytest.fixture(scope="module")
def batch():
    probs = W.batch_2d()
    say(f"[setup] batch of {len(probs)}: cells {[g.cells for _, g, _ in probs]}")
    t0 = time.perf_counter()
    b = K.Batch(probs)
    say(f"    setup {time.perf_counter() - t0:.1f} s, {b.L} nodes, {b.G} grid unknowns")
    f, g, ue = [], [], []
    for iface, grid, co in probs:
        fi, gi, ui = mms(iface, grid, co.kappa)
        f.append(fi)
        g.append(gi)
        ue.append(ui)
    yield b, probs, np.concatenate(f), np.concatenate(g), ue
    b.close()


def seg(v, b, i):
    return v[b.ioff[i]:b.ioff[i] + b.M[i]]


def gseg(v, b, i):
    return v[b.goff[i]:b.goff[i] + b.N[i] ** 2]


def _members(probs):
    """Indices compared with the oracle: up to four small problems and the first problem of the
    512^2 and of the 1024^2 size groups."""
    small = [i for i, (_, g, _) in enumerate(probs) if g.cells <= 128][:4]
    big = [next(i for i, (_, g, _) in enumerate(probs) if g.cells == c) for c in (512, 1024)]
    return small + big


_ORACLE = {}


def oracle_problem(probs, i):
    if i not in _ORACLE:
        iface, grid, co = probs[i]
        say(f"    [oracle setup] problem {i} (cells {grid.cells})")
        _ORACLE[i] = ok.Problem(iface, grid, co)
    return _ORACLE[i]


def test_batch_apply_matches_oracle(batch):
    """The batched product against the oracle's, element by element, on small problems and on a
    512^2 and a 1024^2 member (whose DST passes are their own size groups' launches)."""
    b, probs, _, _, _ = batch
    psi = np.random.default_rng(4).uniform(-1, 1, size=b.L)
    say("[batch apply f64]")
    out = b.apply(T(psi)).cpu().numpy()
    out32 = b.apply(T(psi).float()).double().cpu().numpy()
    for i in _members(probs):
        o = oracle_problem(probs, i)
        ref = o.apply(seg(psi, b, i)[None])[0]
        e, e32 = err(seg(out, b, i), ref), err(seg(out32, b, i), ref)
        say(f"    problem {i} (cells {probs[i][1].cells}): FP64 err {e:.2e}, FP32 err {e32:.2e}")
        assert e < 1e-12
        assert e32 < 1e-5


def test_batch_apply_matches_single_problem_path(batch):
    """Every problem of the batch, including the 512^2 and 1024^2 ones, against its own
    kfbi_apply (same kernels, one problem per launch), in FP64 and FP32."""
    b, probs, _, _, _ = batch
    psi = np.random.default_rng(5).uniform(-1, 1, size=b.L)
    out64 = b.apply(T(psi)).cpu().numpy()
    out32 = b.apply(T(psi).float()).double().cpu().numpy()
    worst64 = worst32 = 0.0
    for i, (iface, grid, co) in enumerate(probs):
        p = K.Problem(iface, grid, co)
        s = T(seg(psi, b, i)[None])
        worst64 = max(worst64, err(seg(out64, b, i), p.apply(s).cpu().numpy()))
        worst32 = max(worst32, err(seg(out32, b, i), p.apply(s).cpu().numpy()))
        p.close()
    say(f"    batch vs single: FP64 worst {worst64:.2e}, FP32 batch vs FP64 single worst {worst32:.2e}")
    # element-wise: the FP32 grid side loses about u32 = 6e-8 per DST stage, and the extrapolated
    # gradient (differences of grid values over h) magnifies it at the finest grids (1024^2)
    assert worst64 < 1e-12
    assert worst32 < 5e-5


@pytest.mark.timeout(900)
def test_batch_solve_f64_parity_and_accuracy(batch):
    b, probs, f, g, ue = batch
    say("[batch solve f64]")
    t0 = time.perf_counter()
    u, psi, infos = b.solve_neumann(T(g), T(f), tol=1e-12)
    torch.cuda.synchronize()
    say(f"    {time.perf_counter() - t0:.2f} s; iterations {[i['iters'] for i in infos]}")
    u = u.cpu().numpy()
    psi = psi.cpu().numpy()
    assert all(i["rel_resid"] <= 1e-12 for i in infos)
    worst = 0.0
    for i, (iface, grid, co) in enumerate(probs):
        o_inside = ogeo.classify(iface, grid).all(axis=0)
        e_exact = np.max(np.abs(gseg(u, b, i) - ue[i])[o_inside])
        # second order: the 128^2 star of the 2D parity case has max error 0.57 h^2; allow 10x
        worst = max(worst, e_exact / grid.h ** 2)
        assert e_exact < 6.0 * grid.h ** 2, (i, grid.cells, e_exact)
    say(f"    worst max-norm error / h^2 = {worst:.2f}")
    for i in _members(probs):
        iface, grid, co = probs[i]
        o = oracle_problem(probs, i)
        fi, gi, _ = mms(iface, grid, co.kappa)
        uo, psio, infoo = o.solve_neumann(gi[None], fi[None], tol=1e-13)
        gp, _ = o.bie_rhs(gi[None], fi[None])
        e = err(gseg(u, b, i)[o.inside], uo[0][o.inside])
        ep = err(seg(psi, b, i), psio[0])
        # both densities solve A psi = g' to their tolerances, so A maps their difference to at most
        # the sum of the two residual bounds plus the difference of the two right-hand sides.  g' =
        # g - dn u_V is formed with cancellation (|g - g'| / |g'| = cg, up to 8e4 at 1024^2 here) from
        # a one-sided derivative (weights of order 1/h) of the box solution, so the two FP64 box
        # solves' rounding reaches g' amplified by both: bounded here by 4 times the derivative
        # that the extrapolation takes of the measured difference of the two solutions.  Element
        # by element the densities can differ more at the finest grids, where a node-to-node
        # oscillation of psi (node spacing about h) is nearly invisible to A.
        ea = np.linalg.norm(o.apply(seg(psi, b, i)[None] - psio)) / np.linalg.norm(gp)
        cg = np.linalg.norm(gi[None] - gp) / np.linalg.norm(gp)
        du = np.linalg.norm(o.extrapolate_smooth(gseg(u, b, i) - uo[0], co.D[0])) / np.linalg.norm(gp)
        say(f"    problem {i} (cells {grid.cells}): u err vs oracle {e:.2e}, psi err {ep:.2e}, "
            f"|A (psi - psi_oracle)| / |g'| {ea:.2e} (cancellation in g' {cg:.0f}, derivative of the u "
            f"difference {du:.1e}), iters {infos[i]['iters']} / {infoo['iters']}")
        assert e < 1e-10
        assert ea <= 1.2e-12 + 4.0 * du
        if grid.cells <= 512:
            assert ep < 1e-9


def test_batch_solve_mixed_precision(batch):
    b, probs, f, g, _ = batch
    say("[batch solve mixed]")
    u64, _, _ = b.solve_neumann(T(g), T(f), tol=1e-10)
    u32, _, infos = b.solve_neumann(T(g), T(f), tol=1e-10, precision=1, inner_tol=1e-4)
    u64, u32 = u64.cpu().numpy(), u32.cpu().numpy()
    say(f"    outer {[i['outer'] for i in infos]}")
    assert all(i["rel_resid"] <= 1e-10 for i in infos)
    assert all(i["matvecs_fp32"] > 0 for i in infos)
    worst = max(err(gseg(u32, b, i), gseg(u64, b, i)) for i in range(b.n))
    say(f"    worst u difference mixed vs FP64 {worst:.2e}")
    assert worst < 1e-8


def test_batch_graph_replay_matches_direct_launches(batch):
    """The captured Arnoldi step replayed every iteration gives the same solves as launching
    its kernels directly (same kernels in the same order: identical results)."""
    b, probs, f, g, _ = batch
    b.graph(True)
    u1, p1, i1 = b.solve_neumann(T(g), T(f), tol=1e-10)
    b.graph(False)
    u2, p2, i2 = b.solve_neumann(T(g), T(f), tol=1e-10)
    b.graph(True)
    u3, p3, i3 = b.solve_neumann(T(g), T(f), tol=1e-10)
    assert [x["iters"] for x in i1] == [x["iters"] for x in i2] == [x["iters"] for x in i3]
    assert torch.equal(u1, u2) and torch.equal(p1, p2)
    assert torch.equal(u1, u3) and torch.equal(p1, p3)


def test_batch_merged_launches_match_grouped_launches(batch):
    """Each DST pass as one launch over all size groups (the default) against one launch per
    group and pass: the same arithmetic for every pencil, so identical products (FP64 and FP32)
    and identical FP64 and mixed-precision solves."""
    b, probs, f, g, _ = batch
    rng = np.random.default_rng(17)
    psi = rng.uniform(-1, 1, size=b.L)
    out = {}
    for merged in (True, False):
        b.merge(merged)
        a64 = b.apply(T(psi))
        a32 = b.apply(torch.tensor(psi, dtype=torch.float32, device=DEV))
        s64 = b.solve_neumann(T(g), T(f), tol=1e-10)
        smx = b.solve_neumann(T(g), T(f), tol=1e-10, precision=1, inner_tol=1e-4)
        out[merged] = (a64, a32, s64, smx)
    b.merge(True)
    (a64, a32, s64, smx), (b64, b32, t64, tmx) = out[True], out[False]
    assert torch.equal(a64, b64) and torch.equal(a32, b32)
    for x, y in ((s64, t64), (smx, tmx)):
        assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1])
        assert [i["iters"] for i in x[2]] == [i["iters"] for i in y[2]]
    say(f"    merged == grouped: products and solves identical ({b.n} problems)")


def test_batch_with_spline_boundaries_matches_single_problems():
    """A batch mixing analytic stars and node-given spline curves (heart, clockwise circle)
    of three grid sizes: every problem's product equals its own single-problem product."""
    probs = [(W.heart2d(256), W.box(2, 128), W.scalar_coeffs(2, 1.0, 300.0)),
             (W.star2d(n_nodes=128), W.box(2, 64), W.scalar_coeffs(2, 1.0, 100.0)),
             (W.spline_circle(0.55, 100, clockwise=True), W.box(2, 64), W.scalar_coeffs(2, 1.0, 900.0)),
             (W.heart2d(512, seed=7), W.box(2, 256), W.scalar_coeffs(2, 1.0, 50.0))]
    say("[batch with splines]")
    b = K.Batch(probs)
    psi = np.random.default_rng(9).uniform(-1, 1, size=b.L)
    out = b.apply(T(psi)).cpu().numpy()
    for i, (iface, grid, co) in enumerate(probs):
        p = K.Problem(iface, grid, co)
        ref = p.apply(T(seg(psi, b, i)[None])).cpu().numpy()
        e = err(seg(out, b, i), ref)
        say(f"    problem {i}: rel diff {e:.2e}")
        assert e < 1e-13
        p.close()
    b.close()
