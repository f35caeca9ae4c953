"""fp_rk3_step_noalloc (the RK3 step whose workspace is the library's static
per-GPU array) against fp_rk3_step with a caller-allocated workspace: two
calls in a row, the second on a smaller grid, each bitwise equal to the
allocating entry point on the same inputs (both run the same kernels)."""
import numpy as np
import pytest
import torch

from paper_2101_05886_amd import fp
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def step_both(case, scheme):
    grid = fp.Grid(case["ndim"], case["n"], case["g"], bc=case["bc"])
    met = fp.metrics(grid, case["Y"], dev(case["xyz"]))
    q_ref = dev(case["q"])
    dt = float(fp.max_dt(grid, scheme, met, q_ref, 0.5).item())
    work = torch.zeros(grid.work_shape(), dtype=torch.float64, device="cuda")
    fp.rk3_step(grid, scheme, met, q_ref, work, dt)
    q = dev(case["q"])
    fp.rk3_step_noalloc(grid, scheme, met, q, dt)
    torch.cuda.synchronize()
    return q, q_ref


def test_noalloc_step_equals_allocating_step_twice_then_smaller():
    print("no-alloc step: 3D periodic 40x36x30 WENO5-M6 FP64, then a 24x20x12 frozen block "
          "LU5-M6 mixed with global LF speeds, then a 2D 50x37 WENO5", flush=True)
    big = G.periodic_case(3, (40, 36, 30), 6, state="noisy", seed=61)
    q, ref = step_both(big, fp.Scheme("weno5", 6, True))
    assert torch.equal(q, ref)
    small = G.frozen_case((24, 20, 12), 6, perturb=0.05, seed=62)
    q, ref = step_both(small, fp.Scheme("linup5", 6, True, precision="mixed", splitting="glf"))
    assert torch.equal(q, ref)
    # a third, 2D, call: the array keeps the last call's contents, which
    # the step never reads before writing
    flat = G.periodic_case(2, (50, 37), 6, state="vortex", seed=63)
    q, ref = step_both(flat, fp.Scheme("weno5", 6, True))
    assert torch.equal(q, ref)


def test_noalloc_step_rejects_a_grid_beyond_the_workspace():
    grid = fp.Grid(3, (80, 80, 80), 3)
    met = torch.zeros(grid.metric_shape(), dtype=torch.float64, device="cuda")
    q = torch.ones(grid.state_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(fp.FPError) as e:
        fp.rk3_step_noalloc(grid, fp.Scheme("weno5", 6, True), met, q, 0.1)
    assert e.value.status == fp.FP_EINVAL
    assert torch.equal(q, torch.ones_like(q))  # nothing was enqueued
