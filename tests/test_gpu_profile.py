"""fp_profile_step: the instrumented step is the step (bitwise fp_rk3_step,
and one step of fp_solve_bcs / fp_solve_ns), with one timed entry per
launch in launch order."""
import numpy as np
import pytest
import torch

from paper_2101_05886_amd import fp
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need the MI355X"
    fp.lib()
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def kinds(prof):
    return [k for k, _ in prof]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_profiled_step_is_the_step_3d_periodic(prec):
    case = G.periodic_case(3, (24, 20, 18), 6, state="noisy", seed=71)
    fg = fp.Grid(3, case["n"], 3)
    sc = fp.Scheme("weno5", 6, True, precision=prec)
    met = fp.metrics(fg, 6, dev(case["xyz"]))
    q1, q2 = dev(case["q"]), dev(case["q"])
    w1 = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    w2 = torch.zeros_like(w1)
    fp.rk3_step(fg, sc, met, q1, w1, 1e-3)
    prof = fp.profile_step(fg, sc, met, q2, w2, 1e-3)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)
    assert kinds(prof) == [0, 1, 2] * 3
    assert all(ms > 0.0 for _, ms in prof)


def test_profiled_step_with_boundary_faces_and_glf():
    from tests.test_gpu_shock import dmr_case
    og, fg, met, q, nodes, ob, fb = dmr_case(121, 31, 0.05)
    sc = fp.Scheme("weno5", 6, True, splitting="glf")
    mg = dev(met)
    q1, q2 = dev(q), dev(q)
    w1 = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    w2 = torch.zeros_like(w1)
    dt = 1e-4
    fp.solve_bcs(fg, sc, fb, mg, q1, w1, 0.0, dt, 1)
    prof = fp.profile_step(fg, sc, mg, q2, w2, dt, bcs=fb, t=0.0)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)
    assert kinds(prof) == [3, 9] + [6, 5, 0, 1] * 3


def test_profiled_step_navier_stokes():
    case = G.periodic_case(3, (20, 17, 14), 6, state="noisy", seed=72)
    fg = fp.Grid(3, case["n"], 3)
    sc = fp.Scheme("weno5", 6, True, mu=1e-3, prandtl=0.72)
    met = fp.metrics(fg, 6, dev(case["xyz"]))
    q1, q2 = dev(case["q"]), dev(case["q"])
    w1 = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    w2 = torch.zeros_like(w1)
    v1, v2 = fp.viscous_work(fg), fp.viscous_work(fg)
    fp.solve_ns(fg, sc, met, q1, w1, v1, 1e-3, 1)
    prof = fp.profile_step(fg, sc, met, q2, w2, 1e-3, vwork=v2)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)
    assert kinds(prof) == [7, 8, 0, 1, 2] * 3


def test_profile_step_rejects_bad_arguments():
    case = G.periodic_case(3, (16, 14, 12), 6)
    fg = fp.Grid(3, case["n"], 3)
    met = fp.metrics(fg, 6, dev(case["xyz"]))
    q = dev(case["q"])
    w = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(fp.FPError):
        fp.profile_step(fg, fp.Scheme("weno5", 6, True), met, q, w, -1.0)
    with pytest.raises(fp.FPError):  # viscous without its workspace
        fp.profile_step(fg, fp.Scheme("weno5", 6, True, mu=1e-3), met, q, w, 1e-3)
