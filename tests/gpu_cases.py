"""Seeded workloads shared by the GPU parity tests (inputs only: grids and
states from paper_2101_05886_amd.inputs; no arithmetic of the method)."""
import math

import numpy as np

from paper_2101_05886_amd import inputs as I

GAMMA = 1.4


def periodic_case(ndim, n, Y, g=None, state="vortex", jitter=0.05, seed=1, L=12.0, mach=0.5):
    """Jittered periodic wavy grid with a vortex (or uniform flow, or a
    vortex plus random noise) on it."""
    g = g or max(3, Y // 2)
    xyz = I.wavy_grid(ndim, n, L, g, Y, amp=0.1, jitter=jitter, seed=seed)
    per = I.wavy_periods(ndim, n, L)
    d = I.direction_3d() if ndim == 3 else np.array([math.cos(math.radians(20)), math.sin(math.radians(20))])
    vel = I.mach_velocity(mach, d)
    if state == "uniform":
        q = I.uniform_state(ndim, n, g, GAMMA, vel, 1.0)
    else:
        v3 = tuple(vel) + (0.0,) * (3 - len(vel))
        q = I.Vortex(vel_inf=v3).state(I.state_nodes(xyz, g, Y), period=per[:2])
        if state == "noisy":
            rng = np.random.Generator(np.random.PCG64(seed + 100))
            q = q * (1.0 + 0.02 * rng.standard_normal(q.shape))
    bc = [0, 0, 0]
    return dict(ndim=ndim, n=I._n3(ndim, n), g=g, Y=Y, bc=bc, xyz=xyz, q=np.ascontiguousarray(q))


def frozen_case(n, Y, g=None, mach=3.0, seed=3, perturb=0.0):
    """One O-grid sector block with frozen free-stream ghosts on every axis."""
    g = g or max(3, Y // 2)
    xyz = I.ogrid_sector_block(n, g, Y, sector=2.0, skew_deg=20.0, rotation=0.7)
    q = I.uniform_state(3, n, g, GAMMA, I.mach_velocity(mach, [1.0, 0.0, 0.0]), 1.0)
    if perturb:
        rng = np.random.Generator(np.random.PCG64(seed))
        nodes = I.state_nodes(xyz, g, Y)
        bump = perturb * np.exp(-((nodes[0] - 1.5) ** 2 + nodes[1] ** 2) / 0.3)
        q = q * (1.0 + bump[None]) * (1.0 + 1e-3 * rng.standard_normal(q.shape))
    return dict(ndim=3, n=list(n), g=g, Y=Y, bc=[1, 1, 1], xyz=xyz, q=np.ascontiguousarray(q))


def sample_nodes(n, ndim, count, seed=0):
    """Interior nodes to sample: the eight corners plus random ones."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = []
    for c in range(1 << ndim):
        pts.append([(n[d] - 1) if (c >> d) & 1 else 0 for d in range(ndim)] + [0] * (3 - ndim))
    for _ in range(count):
        pts.append([int(rng.integers(0, n[d])) for d in range(ndim)] + [0] * (3 - ndim))
    return np.array(pts, dtype=np.int32)


def smooth_periodic_state(n, g, mach=0.5, eps=0.01, gamma=GAMMA):
    """Uniform 3D flow (Mach `mach` along the 3D direction of the workloads,
    p = 1) whose density carries the periodic perturbation
    1 + eps*s(i)*s(j)*s(k), s(i) = sin(2*pi*(i + 1/2)/n) over the node index
    (ghost nodes take their periodic image's value); the pressure stays 1.
    Separable, so it is cheap at any size."""
    idx = np.arange(-g, n + g) % n
    s = np.sin(2.0 * math.pi * (idx + 0.5) / n)
    rho = gamma * (1.0 + eps * s[:, None, None] * s[None, :, None] * s[None, None, :])
    vel = I.mach_velocity(mach, I.direction_3d())
    return np.ascontiguousarray(I.primitive_to_conserved(rho, [float(v) for v in vel], 1.0, gamma))
