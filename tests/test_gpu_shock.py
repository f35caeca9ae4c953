"""The wall-bounded shock problems of Sec. 4.2 on the GPU, through the C
ABI: boundary faces (fp_apply_bcs), global Lax-Friedrichs splitting and the
boundary-driven RK3 (fp_solve_bcs) against the FP64 oracle, then the double
Mach reflection (961 x 241, 5% and 20% random grids, t = 0.2, CFL 0.6) and the Mach 2
cylinder (61 x 81, 20% random grid) at full size.  The paper shows these
only as contour plots, so the full-size checks are physical: positivity and
bounded density, the incident shock where the exact solution puts it, the
state ahead of the shocks left uniform by the free-stream preserving scheme
(not by the standard one), and the cylinder's stagnation pressure against
the Rayleigh pitot formula."""
import math
import time

import numpy as np
import pytest
import torch

import oracle as O
from paper_2101_05886_amd import fp
from paper_2101_05886_amd import inputs as I
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need the MI355X"
    fp.lib()
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return max(np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(a.shape[0]))


def interior(a, g, ndim):
    return a[(slice(None),) + (slice(g, -g),) * ndim]


def bcs_pair(spec, nodes):
    """the same faces for the oracle (host arrays) and the library (device)"""
    ob = O.Bcs(spec["kind"], mask=spec.get("mask"), nodes=nodes, pre=spec.get("pre"), post=spec.get("post"),
               normal=spec.get("normal", (1, 0, 0)), offset=spec.get("offset", 0.0), speed=spec.get("speed", 0.0))
    dmask = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in (spec.get("mask") or {}).items()}
    fb = fp.Bcs(spec["kind"], mask=dmask, nodes=dev(nodes), pre=spec.get("pre"), post=spec.get("post"),
                normal=spec.get("normal", (1, 0, 0)), offset=spec.get("offset", 0.0), speed=spec.get("speed", 0.0))
    return ob, fb


def dmr_case(nx, ny, rand, g=3, Y=6, seed=11):
    xyz = I.dmr_grid(nx, ny, rand, g, Y, seed)
    nodes = I.state_nodes(xyz, g, Y)
    og, fg = O.Grid(2, (nx, ny), g, bc=[1, 1]), fp.Grid(2, (nx, ny), g, bc=[1, 1])
    met = O.metrics(og, Y, xyz)
    q = I.dmr_state(nodes, g)
    ob, fb = bcs_pair(I.dmr_faces(nodes, g), nodes)
    return og, fg, met, q, nodes, ob, fb


def cylinder_case(imax, jmax, rand, g=3, Y=6, seed=5):
    xyz = I.cylinder_grid(imax, jmax, rand, g, Y, seed)
    nodes = I.state_nodes(xyz, g, Y)
    og, fg = O.Grid(2, (imax, jmax), g, bc=[1, 1]), fp.Grid(2, (imax, jmax), g, bc=[1, 1])
    met = O.metrics(og, Y, xyz)
    q = I.cylinder_state((imax, jmax), g)
    ob, fb = bcs_pair(I.cylinder_faces(), nodes)
    return og, fg, met, q, nodes, ob, fb


def test_apply_bcs_matches_the_oracle():
    og, fg, met, q, nodes, ob, fb = dmr_case(121, 31, 0.05)
    rng = np.random.default_rng(1)
    q = np.ascontiguousarray(q * (1 + 0.01 * rng.standard_normal(q.shape)))
    ref = O.apply_bcs(og, ob, met, q, 0.013)
    got = host(fp.apply_bcs(fg, fb, dev(met), dev(q), 0.013))
    assert relerr(got, ref) <= 1e-15
    og, fg, met, q, nodes, ob, fb = cylinder_case(31, 41, 0.2)
    q = np.ascontiguousarray(q * (1 + 0.01 * rng.standard_normal(q.shape)))
    ref = O.apply_bcs(og, ob, met, q, 0.0)
    got = host(fp.apply_bcs(fg, fb, dev(met), dev(q), 0.0))
    assert relerr(got, ref) <= 1e-15
    # a 3D block with walls on a rotated grid and extrapolated faces
    n, g, Y = (14, 12, 10), 3, 6
    a = 0.4
    A = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1.0]])
    xyz = I.affine_grid(3, n, g, Y, A)
    og, fg = O.Grid(3, n, g, bc=[1, 1, 0]), fp.Grid(3, n, g, bc=[1, 1, 0])
    met = O.metrics(og, Y, xyz)
    q = np.ascontiguousarray(I.uniform_state(3, n, g, 1.1, [0.3, 0.2, -0.1], 1.0)
                             * (1 + 0.05 * rng.standard_normal(I.state_shape(3, n, g))))
    spec = dict(kind=[[2, 1], [1, 2], [0, 0]])
    ob, fb = bcs_pair(spec, I.state_nodes(xyz, g, Y))
    ref = O.apply_bcs(og, ob, met, q, 0.0)
    got = host(fp.apply_bcs(fg, fb, dev(met), dev(q), 0.0))
    # the wall normal's normalisation rounds differently (contracted
    # multiply-adds on the GPU): a few ulps of the momenta
    assert relerr(got, ref) <= 1e-14


@pytest.mark.parametrize("recon,Y,g", [("weno5", 6, 3), ("linup5", 6, 3), ("weno7", 8, 4), ("wenocu6", 6, 3)])
@pytest.mark.parametrize("ndim", [2, 3])
def test_glf_rk3_step_matches_the_oracle(recon, Y, g, ndim):
    n = (40, 33) if ndim == 2 else (20, 17, 14)
    case = G.periodic_case(ndim, n, Y, g=g, state="noisy", seed=51)
    og, fg = O.Grid(ndim, n, g), fp.Grid(ndim, n, g)
    met = O.metrics(og, Y, case["xyz"])
    osc = O.Scheme(recon, Y, True, splitting="glf")
    fsc = fp.Scheme(recon, Y, True, splitting="glf")
    dt = 0.5 * O.max_dt(og, osc, met, case["q"], 1.0)
    ref = O.rk3_step(og, osc, met, case["q"], dt)
    qg = dev(case["q"])
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.rk3_step(fg, fsc, dev(met), qg, work, dt)
    assert relerr(interior(host(qg), g, ndim), interior(ref, g, ndim)) <= 1e-12
    # the third stage's speed set (the workspace tail's set 2: doubles
    # 96 + 16 d .. 98 + 16 d) holds the oracle's global speeds of that
    # stage's input (the second stage register), to rounding
    w = host(work)
    vol = case["q"].size
    B = w[vol:2 * vol].reshape(case["q"].shape)
    for d in range(ndim):
        want = O.glf_speeds(og, osc, met, B, d)
        got = w[3 * vol + 96 + 16 * d: 3 * vol + 99 + 16 * d]
        assert np.abs(got - want).max() <= 1e-13 * want.max(), (d, got, want)
    if recon == "weno5" and ndim == 3:
        fsc_m = fp.Scheme(recon, Y, True, precision="mixed", splitting="glf")
        qm = dev(case["q"])
        work.zero_()
        fp.rk3_step(fg, fsc_m, dev(met), qm, work, dt)
        assert relerr(interior(host(qm), g, ndim), interior(ref, g, ndim)) <= 1e-6


def test_solve_bcs_3d_walls_and_glf_match_the_oracle():
    """A 3D block with slip walls and extrapolated faces on a rotated grid
    (the third axis periodic), global LF speeds: the boundary-face kernel,
    the GLF reduction of frozen 3D axes and the captured step graph against
    the oracle, over two calls."""
    n, g, Y = (18, 14, 10), 3, 6
    a = 0.4
    A = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1.0]])
    xyz = I.affine_grid(3, n, g, Y, A)
    og, fg = O.Grid(3, n, g, bc=[1, 1, 0]), fp.Grid(3, n, g, bc=[1, 1, 0])
    met = O.metrics(og, Y, xyz)
    rng = np.random.default_rng(81)
    q = np.ascontiguousarray(I.uniform_state(3, n, g, 1.4, [0.3, -0.2, 0.1], 1.0)
                             * (1 + 0.05 * rng.standard_normal(I.state_shape(3, n, g))))
    ob, fb = bcs_pair(dict(kind=[[2, 1], [1, 2], [0, 0]]), I.state_nodes(xyz, g, Y))
    osc = O.Scheme("weno5", Y, True, splitting="glf")
    dt = 0.3 * O.max_dt(og, osc, met, q, 1.0)
    ref = O.solve_bcs(og, osc, ob, met, q, 0.0, dt, 5)
    qg = dev(q)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fsc = fp.Scheme("weno5", Y, True, splitting="glf")
    fp.solve_bcs(fg, fsc, fb, dev(met), qg, work, 0.0, dt, 2)
    fp.solve_bcs(fg, fsc, fb, dev(met), qg, work, 2 * dt, dt, 3)
    assert relerr(interior(host(qg), g, 3), interior(ref, g, 3)) <= 1e-11


def test_glf_is_rejected_where_there_is_no_workspace():
    case = G.periodic_case(2, (20, 20), 6)
    fg = fp.Grid(2, (20, 20), 3)
    sc = fp.Scheme("weno5", 6, True, splitting="glf")
    met = fp.metrics(fg, 6, dev(case["xyz"]))
    with pytest.raises(fp.FPError):
        fp.residual(fg, sc, met, dev(case["q"]))
    with pytest.raises(fp.FPError):
        fp.Batch(sc, 2)


def test_solve_bcs_matches_the_oracle():
    for mk, steps, dt in ((dmr_case, 8, 1.0e-4), (cylinder_case, 8, 0.004)):
        for recon, Y, g in (("weno5", 6, 3), ("weno7", 8, 4)):
            args = (121, 31, 0.05) if mk is dmr_case else (31, 41, 0.2)
            og, fg, met, q, nodes, ob, fb = mk(*args, g=g, Y=Y)
            for split in ("glf", "llf"):
                osc = O.Scheme(recon, Y, True, splitting=split)
                ref = O.solve_bcs(og, osc, ob, met, q, 0.0, dt, steps)
                qg = dev(q)
                work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
                # two calls: the second replays the captured step graph from t = 3 dt
                fsc = fp.Scheme(recon, Y, True, splitting=split)
                fp.solve_bcs(fg, fsc, fb, dev(met), qg, work, 0.0, dt, 3)
                fp.solve_bcs(fg, fsc, fb, dev(met), qg, work, 3 * dt, dt, steps - 3)
                assert relerr(interior(host(qg), g, 2), interior(ref, g, 2)) <= 1e-11, (recon, split)


@pytest.mark.parametrize("rand", [0.05, 0.2])
def test_double_mach_reflection_full_size_steps_match_the_oracle(rand):
    """The benchmarked double Mach reflection (961 x 241, WENO5-M6, global
    LF, boundary faces every stage, dt at CFL 0.6 from the initial state)
    through the captured step graph of fp_solve_bcs: 20 steps against the
    oracle's, at the bar of the small boundary-driven runs."""
    og, fg, met, q, nodes, ob, fb = dmr_case(961, 241, rand)
    osc = O.Scheme("weno5", 6, True, splitting="glf")
    fsc = fp.Scheme("weno5", 6, True, splitting="glf")
    dt = O.max_dt(og, osc, met, q, 0.6)
    ref = O.solve_bcs(og, osc, ob, met, q, 0.0, dt, 20)
    qg = dev(q)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.solve_bcs(fg, fsc, fb, dev(met), qg, work, 0.0, dt, 20)
    err = relerr(interior(host(qg), 3, 2), interior(ref, 3, 2))
    print(f"DMR {rand:.0%} grid, 20 steps at dt {dt:.4e}: {err:.2e} of the oracle", flush=True)
    assert err <= 1e-11


def test_supersonic_cylinder_full_size_steps_match_the_oracle():
    """The 61 x 81 cylinder grid with 20% randomness at its full size and
    dt = 0.005: 20 steps of fp_solve_bcs against the oracle's."""
    og, fg, met, q, nodes, ob, fb = cylinder_case(61, 81, 0.2)
    osc = O.Scheme("weno5", 6, True, splitting="glf")
    fsc = fp.Scheme("weno5", 6, True, splitting="glf")
    ref = O.solve_bcs(og, osc, ob, met, q, 0.0, 0.005, 20)
    qg = dev(q)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.solve_bcs(fg, fsc, fb, dev(met), qg, work, 0.0, 0.005, 20)
    err = relerr(interior(host(qg), 3, 2), interior(ref, 3, 2))
    print(f"cylinder, 20 steps: {err:.2e} of the oracle", flush=True)
    assert err <= 1e-11


def prim(q):
    rho = q[0]
    u, v = q[1] / rho, q[2] / rho
    p = 0.4 * (q[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def run_to(fg, sc, fb, met, q, t_end, cfl, every=10):
    """fp_solve_bcs in chunks of `every` steps at the CFL-limited dt of the
    chunk's start, the last chunk shortened to end at t_end"""
    qg, mg = dev(q), dev(met)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    t, steps = 0.0, 0
    while t < t_end - 1e-14:
        dt = float(fp.max_dt(fg, sc, mg, qg, cfl).item())
        if not (math.isfinite(dt) and dt > 0.0):
            break  # the state has diverged (the standard scheme on a rough grid)
        k = every
        if t + k * dt > t_end:
            k = max(1, int(math.ceil((t_end - t) / dt)))
            dt = (t_end - t) / k
        fp.solve_bcs(fg, sc, fb, mg, qg, work, t, dt, k)
        t += k * dt
        steps += k
    return host(qg), steps


# The 5% grid with every scheme the paper shows on it, and the 20% grid,
# which the paper says leaves the preserving schemes' results unchanged
DMR_CASES = [("weno5", 6, 3, 0.05), ("wenocu6", 6, 3, 0.05), ("weno7", 6, 4, 0.05), ("weno7", 8, 4, 0.05),
             ("weno5", 6, 3, 0.2), ("weno7", 8, 4, 0.2)]


@pytest.mark.parametrize("recon,Y,g,rand", DMR_CASES)
def test_double_mach_reflection_full_size(recon, Y, g, rand):
    og, fg, met, q, nodes, ob, fb = dmr_case(961, 241, rand, g=g, Y=Y)
    x, y = I.interior(nodes, g)
    res = {}
    for reform in (True, False):
        sc = fp.Scheme(recon, Y, reform, splitting="glf")
        t0 = time.time()
        out, steps = run_to(fg, sc, fb, met, q, 0.2, 0.6)
        wall = time.time() - t0
        rho, u, v, p = prim(I.interior(out, g))
        # right of every shock: the incident shock leans forward, so its top
        # point leads (the Mach stem trails it)
        ahead = x > I.dmr_shock_x(0.2, 1.0) + 0.1
        dev_ahead = max(np.abs(rho[ahead] - 1.4).max(), np.abs(u[ahead]).max(), np.abs(v[ahead]).max(),
                        np.abs(p[ahead] - 1.0).max())
        res[reform] = dev_ahead if np.isfinite(out).all() else math.inf
        print(f"DMR {rand:.0%} grid {recon}-M{Y} reform={reform}: {steps} steps in {wall:.2f} s; rho [{rho.min():.3f}, "
              f"{rho.max():.3f}], p min {p.min():.3f}, deviation ahead of the shock {dev_ahead:.3e}", flush=True)
        if reform:
            assert np.isfinite(out).all() and rho.min() > 0 and p.min() > 0
            assert 1.0 < rho.max() < 25.0
            # the incident shock on the top row sits where the exact solution puts it
            top = rho[-1]
            xs = x[-1][np.argmax(top < 0.5 * (1.4 + 8.0))]
            assert abs(xs - I.dmr_shock_x(0.2, 1.0)) < 4 * (4.0 / 960)
    assert res[True] < 1e-9 and res[False] > 1e-3


def test_supersonic_cylinder_full_size():
    og, fg, met, q, nodes, ob, fb = cylinder_case(61, 81, 0.2)
    x, y = I.interior(nodes, 3)
    res = {}
    for reform in (True, False):
        sc = fp.Scheme("weno5", 6, reform, splitting="glf")
        qg, mg = dev(q), dev(met)
        work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
        dt, t = 0.005, 0.0
        fp.solve_bcs(fg, sc, fb, mg, qg, work, t, dt, 3000)
        mid = host(qg).copy()
        fp.solve_bcs(fg, sc, fb, mg, qg, work, t + 3000 * dt, dt, 400)
        out = host(qg)
        rho, u, v, p = prim(I.interior(out, 3))
        change = np.abs(I.interior(out, 3) - I.interior(mid, 3)).max()
        pwall = p[-1]
        ahead = x > 2.7
        dev_ahead = np.abs(p[ahead] - 1.0).max()
        res[reform] = dev_ahead if np.isfinite(out).all() else math.inf
        print(f"cylinder reform={reform}: wall p max {pwall.max():.4f} (pitot 5.640), p range [{p.min():.3f}, "
              f"{p.max():.3f}], change over the last 2.0 time units {change:.2e}, "
              f"deviation ahead of the bow shock {dev_ahead:.3e}", flush=True)
        if reform:
            assert np.isfinite(out).all() and p.min() > 0 and rho.min() > 0
            # Rayleigh pitot: p02/p1 = ((g+1)^2 M^2 / (4 g M^2 - 2 (g-1)))^(g/(g-1)) (1 - g + 2 g M^2)/(g+1)
            gm, M = 1.4, 2.0
            pitot = ((gm + 1) ** 2 * M * M / (4 * gm * M * M - 2 * (gm - 1))) ** (gm / (gm - 1)) \
                * (1 - gm + 2 * gm * M * M) / (gm + 1)
            assert abs(pwall.max() / pitot - 1) < 0.03
    # the standard scheme diverges on this grid; the preserving one keeps the
    # free stream ahead of the bow shock (measured 1.7e-8)
    assert res[True] < 1e-6 and res[False] > 1e-4
