"""The paper's own parameter regime on the GPU (Sec. 7): anisotropic conductivities
D_i = diag(30, 5[, 5]), D_e = diag(20, 10[, 10]), C_m = 1, beta = 1000, dt = h, the virtual
electrode, FitzHugh-Nagumo with theta = 0.25.

* Example 1 (2D circle given by spline nodes): oracle parity of the first steps, second-order
  convergence of V in space and time together (dt = h) over 64^2 .. 1024^2, and the
  GMRES iterations per step (the paper reports 7-10 at relative tolerance 1e-8).
* Example 3 (3D sphere): GMRES beside the simple (Richardson) iteration with gamma = 0.8 (the
  paper: 18-21 iterations), with the virtual electrode and with a stimulus ball.

The radius of the circle and sphere and the box are not stated in the paper; the readings are
those of workloads.paper_circle_example / paper_sphere_example, so the paper's error values are
not expected, only their behaviour."""
import sys
import time

import numpy as np
import pytest

from oracle import bidomain as obd
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


def T(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def run(example, cells, t_end, tol=1e-8, times=(), ball=False, allow_noconv=False, **kw):
    """Steps of a paper example from rest to t_end (dt = h); V at the requested times (host), the
    solve infos and the wall time of the stepping.  ball: no stimulus current, V = 1 in a seeded ball
    at t = 0 instead (the initial condition of the paper's Example 4)."""
    iface, grid, co, p, dt, stim = example(cells)
    prob = K.Problem(iface, grid, co)
    bd = K.Bidomain(prob, p, tol=tol, **kw)
    n = grid.n ** grid.dim
    if ball:
        V0, _ = W.ball_state(grid, W.stimulus_center(iface), radius=0.25)
        V, Is = T(V0), None
    else:
        V, Is = T(np.zeros(n)), T(stim)
    q = T(np.zeros(n))
    hist = torch.zeros(2, 2, prob.M, dtype=torch.float64, device=DEV)
    nsteps = int(round(t_end / dt))
    marks = {int(round(t / dt)): t for t in times}
    snaps, infos = {}, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(1, nsteps + 1):
        infos.append(bd.step(V, q, hist, dt, I_stim=Is, allow_noconv=allow_noconv))
        if s in marks:
            snaps[marks[s]] = V.cpu().numpy()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    inside = prob.table("inside").astype(bool)
    bd.close()
    prob.close()
    return snaps, infos, wall, grid, inside


def test_example1_circle_matches_oracle():
    """The first steps of Example 1 at 64^2 against the oracle's steps (tolerance 1e-12)."""
    iface, grid, co, p, dt, stim = W.paper_circle_example(64)
    g = K.Problem(iface, grid, co)
    o = ok.Problem(iface, grid, co)
    bd = K.Bidomain(g, p, tol=1e-12)
    n = grid.n ** 2
    V, q = T(np.zeros(n)), T(np.zeros(n))
    hist = torch.zeros(2, 2, g.M, dtype=torch.float64, device=DEV)
    Vo, qo, psi = np.zeros(n), np.zeros(n), None
    Is = T(stim)
    for s in range(6):
        info = bd.step(V, q, hist, dt, I_stim=Is)
        Vo, qo, _, psi, io = obd.step(o, p, Vo, qo, dt, psi0=psi, tol=1e-12, I_stim=stim)
        e = np.max(np.abs(V.cpu().numpy() - Vo)) / np.max(np.abs(Vo))
        say(f"[example 1, 64^2] step {s}: V err {e:.2e}, iterations {info['iters']} / {io['iters']}, "
            f"max V {Vo.max():.3f}")
        assert info["rel_resid"] <= 1e-12 and e < 1e-9
    bd.close()
    g.close()


def test_example1_circle_second_order_and_gmres_iterations():
    """V at t = 0.5, 1 and 2 on 64^2 .. 1024^2 (the sizes of the paper's Tables 1-4): the
    differences of consecutive grids at the coarser grid's tissue nodes (scaled l2 and max norm,
    the norms of the paper's tables) fall at second order (dt = h, so space and time together);
    V stays bounded at every size; GMRES iterations per step at tolerance 1e-8 stay near the
    paper's 7-10 and do not grow with refinement.  (Before the coupled pair's null density was
    removed from the reconstruction, 1024^2 blew up within 16 steps in the oracle and on the GPU
    alike: the null component's exterior field fed back through the extended source.)"""
    times = (0.5, 1.0, 2.0)
    sizes = (64, 128, 256, 512, 1024)
    runs = {}
    for cells in sizes:
        snaps, infos, wall, grid, inside = run(W.paper_circle_example, cells, 2.0, times=times)
        assert all(i["rel_resid"] <= 1e-8 for i in infos)
        its = float(np.mean([i["iters"] for i in infos]))
        runs[cells] = (snaps, inside, its)
        vmax = max(float(np.max(np.abs(v))) for v in snaps.values())
        say(f"[example 1] {cells}^2: {len(infos)} steps in {wall:.2f} s, GMRES {its:.2f} per step, "
            f"max V at t=2 {snaps[2.0].max():.3f}, max |V| {vmax:.3f}")
        assert vmax < 1.2
    for t in times:
        d = []
        for c in sizes[:-1]:
            idx = np.arange(1, c) * 2 - 1
            e = (runs[c][0][t].reshape(c - 1, c - 1) - runs[2 * c][0][t].reshape(2 * c - 1, 2 * c - 1)[np.ix_(idx, idx)]).ravel()
            e = e[runs[c][1]]
            d.append((float(np.sqrt(np.mean(e * e))), float(np.max(np.abs(e)))))
        o2 = [np.log2(d[i][0] / d[i + 1][0]) for i in range(len(d) - 1)]
        oi = [np.log2(d[i][1] / d[i + 1][1]) for i in range(len(d) - 1)]
        say(f"[example 1] t={t}: differences l2 {[f'{x[0]:.3e}' for x in d]} (orders {[f'{o:.2f}' for o in o2]}), "
            f"max {[f'{x[1]:.3e}' for x in d]} (orders {[f'{o:.2f}' for o in oi]})")
        assert min(o2[-2:]) > 1.7 and np.mean(o2) > 1.7
    its = [runs[c][2] for c in sizes]
    assert max(its) <= 16 and its[-1] <= its[0] + 3


def test_example3_sphere_gmres_and_the_simple_iteration():
    """Example 3 on the sphere at 64^3 and 128^3 (dt = h) to t = 0.25, tolerance 1e-8, from the
    virtual electrode and from a stimulus ball (no stimulus current).  GMRES and the simple
    iteration (gamma = 0.8) both converge every step and give the same V; iterations per step are
    reported beside the paper's (the simple iteration: 19 at 64^3, 21 at 128^3).  The coupled
    pair's operator is singular up to the discretisation (one eigenvalue near zero, along the null
    density), so the simple iteration's residual is measured without its component along the null
    density: measured in full it stalls at the part of g' that no density can match (8e-3 at 64^3,
    5e-4 at 128^3 from the electrode), reached within 25 iterations."""
    for cells in (64, 128):
        for ball in (False, True):
            tag = "ball" if ball else "electrode"
            sg, ig, wg, _, inside = run(W.paper_sphere_example, cells, 0.25, times=(0.25,), ball=ball)
            sr, ir, wr, _, _ = run(W.paper_sphere_example, cells, 0.25, times=(0.25,), ball=ball, method=1,
                                   gamma=0.8, max_iters=500)
            assert all(i["rel_resid"] <= 1e-8 for i in ig + ir)
            its_g = float(np.mean([i["iters"] for i in ig]))
            its_r = float(np.mean([i["iters"] for i in ir]))
            d = np.max(np.abs(sr[0.25] - sg[0.25])) / np.max(np.abs(sg[0.25]))
            di = np.max(np.abs(sr[0.25] - sg[0.25])[inside]) / np.max(np.abs(sg[0.25]))
            say(f"[example 3, {tag}] {cells}^3, {len(ig)} steps: GMRES {its_g:.2f} iterations per step "
                f"({len(ig) / wg:.1f} steps/s), simple iteration {its_r:.2f} ({len(ir) / wr:.1f} steps/s); "
                f"V difference {d:.1e} (tissue {di:.1e})")
            assert its_g <= 40 and its_r <= 120
            assert d < 1e-5
