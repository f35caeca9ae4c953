"""GPU parity of the viscous fluxes (Sec. 2.1 eqs. NSv1-NSv3; sixth-order
central differences, Sec. 2.2) against the FP64 oracle through the C ABI:
the Navier-Stokes residual and RK3 steps on periodic curvilinear grids (2D
and 3D, FP64, FP32-mixed characteristic part, local and global LF), and a
shear wave whose amplitude decays as exp(-nu k^2 t)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2101_05886_amd import fp
from paper_2101_05886_amd import inputs as I
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu

MU, PR = 0.02, 0.72


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


@pytest.mark.parametrize("ndim,n,Y", [(2, (40, 33), 6), (2, (30, 26), 4), (3, (20, 17, 14), 6),
                                      # the smallest 3D block (every axis at 7..9 nodes: the
                                      # marching kernels' tiles and halos wrap several times)
                                      (3, (7, 8, 9), 6),
                                      # more than one tile and k-run along every axis
                                      (3, (70, 12, 40), 4)])
def test_viscous_residual_matches_the_oracle(ndim, n, Y):
    case = G.periodic_case(ndim, n, Y, state="noisy", seed=61)
    og, fg = O.Grid(ndim, n, 3), fp.Grid(ndim, n, 3)
    met = O.metrics(og, Y, case["xyz"])
    ref = O.residual(og, O.Scheme("weno5", Y, True, mu=MU, prandtl=PR), met, case["q"])
    vw = fp.viscous_work(fg)
    got = host(fp.viscous_residual(fg, fp.Scheme("weno5", Y, True, mu=MU, prandtl=PR), dev(met),
                                   dev(case["q"]), vw))
    assert relerr(interior(got, 3, ndim), interior(ref, 3, ndim)) <= 1e-11
    # the viscous part itself (the residual less the inviscid one) to the same bar
    inv = O.residual(og, O.Scheme("weno5", Y, True), met, case["q"])
    got_inv = host(fp.residual(fg, fp.Scheme("weno5", Y, True), dev(met), dev(case["q"])))
    vis_ref = interior(ref - inv, 3, ndim)[1:]
    vis_got = interior(got - got_inv, 3, ndim)[1:]
    assert relerr(vis_got, vis_ref) <= 1e-9
    if ndim == 3:
        gm = host(fp.viscous_residual(fg, fp.Scheme("weno5", Y, True, precision="mixed", mu=MU, prandtl=PR),
                                      dev(met), dev(case["q"]), vw))
        assert relerr(interior(gm, 3, ndim), interior(ref, 3, ndim)) <= 1e-4


@pytest.mark.parametrize("split", ["llf", "glf"])
def test_solve_ns_matches_the_oracle(split):
    n, Y = (36, 30), 6
    case = G.periodic_case(2, n, Y, state="vortex", seed=62)
    og, fg = O.Grid(2, n, 3), fp.Grid(2, n, 3)
    met = O.metrics(og, Y, case["xyz"])
    osc = O.Scheme("weno5", Y, True, splitting=split, mu=MU, prandtl=PR)
    dt = 0.5 * O.max_dt(og, osc, met, case["q"], 1.0)
    ref = O.solve(og, osc, met, case["q"], dt, 5)
    qg = dev(case["q"])
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.solve_ns(fg, fp.Scheme("weno5", Y, True, splitting=split, mu=MU, prandtl=PR), dev(met), qg, work,
                fp.viscous_work(fg), dt, 5)
    assert relerr(interior(host(qg), 3, 2), interior(ref, 3, 2)) <= 1e-12


def test_shear_wave_decays_at_the_viscous_rate():
    # u = A sin(k y) at rest otherwise, rho = 1, p = 1 (Mach 0.008): the
    # momentum equation reduces to u_t = nu u_yy, so A(t) = A exp(-nu k^2 t)
    n, g, Y, L, A, mu = 48, 3, 6, 12.0, 0.01, 0.05
    k = 2 * math.pi / L
    xyz = I.wavy_grid(2, (n, n), L, g, Y, amp=0.1)
    nodes = I.state_nodes(xyz, g, Y)
    u = A * np.sin(k * nodes[1])
    q = np.ascontiguousarray(I.primitive_to_conserved(np.ones_like(u), [u, 0 * u], np.ones_like(u)))
    fg = fp.Grid(2, n, g)
    met = fp.metrics(fg, Y, dev(xyz))
    sc = fp.Scheme("weno5", Y, True, mu=mu, prandtl=PR)
    T, steps = 20.0, 400
    qg = dev(q)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.solve_ns(fg, sc, met, qg, work, fp.viscous_work(fg), T / steps, steps)
    out = interior(host(qg), g, 2)
    yi = I.interior(nodes, g)[1]
    s = np.sin(k * yi)
    amp = float((out[1] / out[0] * s).sum() / (s * s).sum())
    want = A * math.exp(-mu * k * k * T)
    print(f"shear wave: amplitude {amp:.6e}, exp(-nu k^2 t) gives {want:.6e}", flush=True)
    assert abs(amp / want - 1) < 2e-3


def test_viscous_schemes_are_rejected_elsewhere():
    case = G.periodic_case(2, (20, 20), 6)
    fg = fp.Grid(2, (20, 20), 3)
    sc = fp.Scheme("weno5", 6, True, mu=0.01)
    met = fp.metrics(fg, 6, dev(case["xyz"]))
    with pytest.raises(fp.FPError):
        fp.residual(fg, sc, met, dev(case["q"]))
    with pytest.raises(fp.FPError):
        fp.Batch(sc, 2)
    fz = fp.Grid(2, (20, 20), 3, bc=[1, 0])
    with pytest.raises(fp.FPError):
        fp.viscous_residual(fz, sc, met, dev(case["q"]), fp.viscous_work(fg))
