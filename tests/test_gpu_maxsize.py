"""The largest block the kernels take: 800^3 interior nodes, (800 + 6)^3 =
5.2e8 nodes with the ghost layers, 98% of the 2^29 the 32-bit indices of the
kernels allow, and 4.2 GB per variable array: past 2^31 bytes, so the byte
offsets and buffer extents use the full unsigned 32-bit range.

On the periodic wavy grid (WENO5-JS, sixth-order metrics): the metrics and
the residual of a smoothly perturbed state at sampled nodes (the eight
corners, i.e. the largest indices, and random interior nodes) against the
oracle evaluated node by node from the coordinates, with the bars of the
256^3 sampled test; and the residual of the uniform flow, which must vanish
to round-off at every node (free-stream preservation at full size): within
10 unit roundoffs of max|x|/h, the rounding of metrics that are differences of coordinate
products."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2101_05886_amd import fp
from paper_2101_05886_amd import inputs as I
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


def test_largest_block_sampled_residual_and_free_stream():
    n, g, Y, L = 800, 3, 6, 12.0
    assert (n + 2 * g) ** 3 < 1 << 29
    print(f"{n}^3 block: {(n + 2 * g) ** 3:.3e} nodes with ghosts", flush=True)
    xyz = I.wavy_grid(3, n, L, g, Y, amp=0.1)
    q = G.smooth_periodic_state(n, g)
    og, fg = O.Grid(3, n, g), fp.Grid(3, n, g)
    sc = fp.Scheme("weno5", Y, True)
    xg = torch.from_numpy(xyz).cuda()
    mg = fp.metrics(fg, Y, xg)
    del xg
    torch.cuda.empty_cache()
    pts = G.sample_nodes([n] * 3, 3, 40, seed=17)
    ii = [torch.as_tensor(pts[:, d] + g, device="cuda") for d in range(3)]
    xmax = float(np.abs(xyz).max())
    tol = 1e-13 * xmax / (L / n)
    # metrics at the sampled nodes
    got_m = mg[:, ii[2], ii[1], ii[0]].T.cpu().numpy()
    ref_m = O.metrics_at(og, Y, xyz, pts)
    for d in range(3):
        sc_d = np.abs(ref_m[:, 3 * d:3 * d + 3]).max()
        assert np.abs(got_m[:, 3 * d:3 * d + 3] - ref_m[:, 3 * d:3 * d + 3]).max() <= tol * sc_d
    assert np.abs(got_m[:, 9] - ref_m[:, 9]).max() <= tol * np.abs(ref_m[:, 9]).max()
    # the perturbed state's residual at the sampled nodes
    qg = torch.from_numpy(q).cuda()
    r = fp.residual(fg, sc, mg, qg)
    got = r[:, ii[2], ii[1], ii[0]].T.cpu().numpy()
    del r
    torch.cuda.empty_cache()
    ref = O.residual_at_xyz(og, O.Scheme("weno5", Y, True), xyz, q, pts)
    speed = 0.0
    for p, m in zip(pts, ref_m):
        Qp = q[:, g + p[2], g + p[1], g + p[0]]
        u = Qp[1:4] / Qp[0]
        c = math.sqrt(1.4 * 0.4 * (Qp[4] - 0.5 * Qp[0] * u @ u) / Qp[0])
        speed = max(speed, sum(abs(m[3 * d:3 * d + 3] @ u) + c * np.linalg.norm(m[3 * d:3 * d + 3])
                               for d in range(3)) / m[9])
    dt = 0.5 / speed
    qscale = np.abs(q.reshape(5, -1)).max(axis=1)
    err = (dt * np.abs(got - ref).max(axis=0) / qscale).max()
    print(f"sampled residual vs oracle: dt*|diff|/max|Q| = {err:.2e} (bar {max(1e-12, 20 * tol):.1e})", flush=True)
    assert err <= max(1e-12, 20 * tol)
    del q, xyz
    # the uniform flow: zero residual at every node, to round-off
    vel = I.mach_velocity(0.5, I.direction_3d())
    qu = torch.from_numpy(I.uniform_state(3, 1, 0, 1.4, vel, 1.0).reshape(5)).cuda()
    for v in range(5):
        qg[v].fill_(float(qu[v]))
    r = fp.residual(fg, sc, mg, qg)
    worst = max(float(r[v, g:-g, g:-g, g:-g].abs().max()) * dt / abs(float(qu[v])) if float(qu[v]) else
                float(r[v, g:-g, g:-g, g:-g].abs().max()) * dt for v in range(5))
    # round-off bar: the metrics come from differences of coordinate
    # products (size |x| h) of size h^2, so their rounding is some ulps of
    # |x|/h relative, and so is the surface-conservation defect that the
    # uniform flow's residual reflects: 10 u max|x|/h with u the unit
    # roundoff (4.5e-13 here)
    fs_bar = 10 * np.finfo(np.float64).eps / 2 * xmax / (L / n)
    print(f"uniform flow: dt*max|residual|/|Q| = {worst:.2e} (bar {fs_bar:.1e})", flush=True)
    assert worst <= fs_bar
