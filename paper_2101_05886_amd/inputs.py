"""Seeded synthetic inputs: curvilinear grids and initial states.

This module holds no arithmetic of the numerical method.  It only produces
node coordinates (with ghost images) and conserved states, in the array
layout every entry point uses:

* state ``q``: ``(nv, Nk, Nj, Ni)`` in 3D or ``(nv, Nj, Ni)`` in 2D, float64,
  C order (i fastest), ``N_d = n_d + 2*g``; ``nv`` = 5 (3D) or 4 (2D),
  variables (rho, rho*u, rho*v[, rho*w], rho*E);
* metrics: ``(nmet, ...)`` with the state extents, ``nmet`` = 10 in 3D
  (xi_x, xi_y, xi_z, eta_x, ..., zeta_z, all divided by J, then 1/J) and 5 in
  2D (xi_x, xi_y, eta_x, eta_y divided by J, then 1/J);
* coordinates: ``(ndim, ...)`` with extents ``n_d + 2*(g + Y/2)``, where Y is
  the metric order; ghost nodes hold the periodic image (shifted by the period)
  or the analytic mapping evaluated out of range.  ``g + Y/2`` ghost
  coordinates are what the symmetric conservative metrics need at the
  outermost state ghost node.

The grid recipes follow the test problems of Sec. 4.1 of the paper (wavy and
randomly perturbed grids, uniform flow, isentropic vortex) and the synthetic
workloads derived from them.  Random numbers come from numpy's PCG64 with an
explicit seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 1.4


def coord_ghost(g: int, Y: int) -> int:
    """Ghost width of coordinate arrays: state ghost width plus half the
    metric order (the reach of one central derivative of order Y)."""
    return g + Y // 2


def state_shape(ndim: int, n, g: int, nv: int | None = None):
    n = _n3(ndim, n)
    if nv is None:
        nv = ndim + 2
    if ndim == 2:
        return (nv, n[1] + 2 * g, n[0] + 2 * g)
    return (nv, n[2] + 2 * g, n[1] + 2 * g, n[0] + 2 * g)


def metric_shape(ndim: int, n, g: int):
    return state_shape(ndim, n, g, nv=10 if ndim == 3 else 5)


def coord_shape(ndim: int, n, g: int, Y: int):
    n = _n3(ndim, n)
    gc = coord_ghost(g, Y)
    if ndim == 2:
        return (2, n[1] + 2 * gc, n[0] + 2 * gc)
    return (3, n[2] + 2 * gc, n[1] + 2 * gc, n[0] + 2 * gc)


def _n3(ndim, n):
    if np.isscalar(n):
        n = [int(n)] * ndim
    n = [int(v) for v in n]
    if ndim == 2:
        return [n[0], n[1], 1]
    return n


def _jitter_field(ndim, n, frac, spacing, rng):
    """Displacement of fixed magnitude ``frac*spacing`` in a uniformly random
    direction, one per unique node; shape (ndim, [nk,] nj, ni)."""
    shape = tuple(reversed(n[:ndim]))
    if frac == 0.0:
        return np.zeros((ndim,) + shape)
    if ndim == 2:
        th = rng.uniform(0.0, 2.0 * math.pi, size=shape)
        d = np.stack([np.cos(th), np.sin(th)])
    else:
        v = rng.standard_normal(size=(3,) + shape)
        d = v / np.linalg.norm(v, axis=0, keepdims=True)
    return d * (frac * spacing)


def _periodic_take(field, ndim, n, gc):
    """Evaluate a per-unique-node field at indices -gc..n+gc-1 by periodicity."""
    idx = [np.arange(-gc, n[d] + gc) % n[d] for d in range(ndim)]
    if ndim == 2:
        return field[:, idx[1][:, None], idx[0][None, :]]
    return field[:, idx[2][:, None, None], idx[1][None, :, None], idx[0][None, None, :]]


def wavy_grid(ndim: int, n, L: float, g: int, Y: int, amp: float = 0.1,
              jitter: float = 0.0, seed: int = 0) -> np.ndarray:
    """Periodic wavy grid with node spacing h = L/n[0] on every axis, axis d
    of length L_d = n[d]*h, centred on the origin.

    2D: ``x = xi + A*s0(xi)*s1(eta)``, ``y = eta + A*s0(xi)*s1(eta)``;
    3D: ``x = xi + P``, ``y = eta + P``, ``z = zeta + P`` with
    ``P = A*s0(xi)*s1(eta)*s2(zeta)``, ``s_d(t) = sin(2*pi*(t + L_d/2)/L_d)`` and
    ``A = amp*min_d L_d`` (for amp = 0.1 the mapping keeps J >= 1 - 0.2*pi in
    2D and 1 - 0.2*pi*2/sqrt(3) in 3D on any axis lengths).  Optional jitter: ``jitter*h`` in a random direction per
    unique node, carried to ghost images (periodic).  Ghost nodes are the
    mapping evaluated out of range plus the image's jitter, so
    ``x(i + n) = x(i) + L_d``.
    """
    n3 = _n3(ndim, n)
    gc = coord_ghost(g, Y)
    h = L / n3[0]
    Ld = [h * n3[d] for d in range(ndim)]
    ax = [-Ld[d] / 2 + np.arange(-gc, n3[d] + gc) * h for d in range(ndim)]
    s = [np.sin(2.0 * math.pi * (ax[d] + Ld[d] / 2) / Ld[d]) for d in range(ndim)]
    A = amp * min(Ld)
    if ndim == 2:
        eta, xi = np.meshgrid(ax[1], ax[0], indexing="ij")
        P = A * s[1][:, None] * s[0][None, :]
        xyz = np.stack([xi + P, eta + P])
    else:
        zeta, eta, xi = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        P = A * s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]
        xyz = np.stack([xi + P, eta + P, zeta + P])
    if jitter:
        rng = np.random.Generator(np.random.PCG64(seed))
        jf = _jitter_field(ndim, n3, jitter, h, rng)
        xyz = xyz + _periodic_take(jf, ndim, n3, gc)
    return np.ascontiguousarray(xyz)


def wavy_periods(ndim: int, n, L: float):
    """Physical period of each axis of ``wavy_grid(ndim, n, L, ...)``."""
    n3 = _n3(ndim, n)
    return tuple(L / n3[0] * n3[d] for d in range(ndim))


def paper_wavy_grid_2d(n: int, g: int, Y: int, L: float = 20.0, A: float = 0.6,
                       waves: int = 4) -> np.ndarray:
    """The 2D wavy grid of the free-stream test (Sec. 4.1.1): the x
    coordinate is displaced by ``A*sin(2*pi*waves*(eta - ymin)/L)`` and the y
    coordinate by ``A*sin(2*pi*waves*(xi - xmin)/L)``; ``n`` unique nodes per
    axis (the paper's 21 points include the periodic duplicate, so n = 20)."""
    gc = coord_ghost(g, Y)
    a = -L / 2 + np.arange(-gc, n + gc) * (L / n)
    eta, xi = np.meshgrid(a, a, indexing="ij")
    x = xi + A * np.sin(2.0 * math.pi * waves * (eta + L / 2) / L)
    y = eta + A * np.sin(2.0 * math.pi * waves * (xi + L / 2) / L)
    return np.ascontiguousarray(np.stack([x, y]))


def paper_random_displacement(shape, frac: float, rng) -> np.ndarray:
    """The paper's random grid displacement (the law its Sec. 4.2.2 prints for
    the cylinder grid: xi = i + frac*phi, eta = j + frac*sqrt(1 - phi^2),
    phi ~ U(0, 1)): a displacement of ``frac`` node spacings in a random
    direction of the first quadrant, in index units; shape (2, *shape)."""
    phi = rng.uniform(0.0, 1.0, size=shape)
    return frac * np.stack([phi, np.sqrt(1.0 - phi * phi)])


def random_grid_2d(n: int, g: int, Y: int, L: float = 20.0, frac: float = 0.2,
                   seed: int = 0) -> np.ndarray:
    """Periodic Cartesian grid on [-L/2, L/2)^2 with every unique node moved
    by ``frac`` of the spacing in a random direction (the random grid of
    Sec. 4.1.1, with the displacement law of paper_random_displacement);
    ghost nodes are the periodic images shifted by the period."""
    gc = coord_ghost(g, Y)
    h = L / n
    ax = -L / 2 + np.arange(-gc, n + gc) * h
    eta, xi = np.meshgrid(ax, ax, indexing="ij")
    rng = np.random.Generator(np.random.PCG64(seed))
    d = paper_random_displacement((n, n), frac, rng) * h
    return np.ascontiguousarray(np.stack([xi, eta]) + _periodic_take(d, 2, [n, n], gc))


def cartesian_grid(ndim: int, n, g: int, Y: int, spacing=1.0, origin=0.0) -> np.ndarray:
    """Uniform Cartesian grid (possibly anisotropic spacing per axis)."""
    n3 = _n3(ndim, n)
    gc = coord_ghost(g, Y)
    sp = [spacing] * ndim if np.isscalar(spacing) else list(spacing)
    ax = [origin + np.arange(-gc, n3[d] + gc) * sp[d] for d in range(ndim)]
    if ndim == 2:
        eta, xi = np.meshgrid(ax[1], ax[0], indexing="ij")
        return np.ascontiguousarray(np.stack([xi, eta]))
    zeta, eta, xi = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.ascontiguousarray(np.stack([xi, eta, zeta]))


def affine_grid(ndim: int, n, g: int, Y: int, A: np.ndarray, b=None) -> np.ndarray:
    """x = A @ (i, j[, k]) + b evaluated at every coordinate node."""
    n3 = _n3(ndim, n)
    gc = coord_ghost(g, Y)
    ax = [np.arange(-gc, n3[d] + gc, dtype=np.float64) for d in range(ndim)]
    A = np.asarray(A, dtype=np.float64)
    b = np.zeros(ndim) if b is None else np.asarray(b, dtype=np.float64)
    if ndim == 2:
        J, I = np.meshgrid(ax[1], ax[0], indexing="ij")
        comp = [I, J]
    else:
        K, J, I = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        comp = [I, J, K]
    out = np.stack([sum(A[c, e] * comp[e] for e in range(ndim)) + b[c] for c in range(ndim)])
    return np.ascontiguousarray(out)


def ogrid_sector_block(n, g: int, Y: int, sector: float, skew_deg: float = 0.0,
                       rotation: float = 0.0, r_wall: float = 1.0, dr0: float = 0.01,
                       ratio: float = 1.1, cap: int = 48) -> np.ndarray:
    """One block of an O-grid around a cylinder of radius ``r_wall``: index i
    runs along the (decreasing) polar angle over ``sector`` radians, j outward
    from the wall with first spacing ``dr0`` growing by ``ratio`` per cell
    (constant after ``cap`` cells; ghosts inside the wall keep ``dr0``), k
    along the axis with spacing ``r_wall*dtheta``.  The angle is skewed by
    ``tan(skew)*(r - r_wall)/r`` and the block is rotated by ``rotation``
    about the axis.  Ghost coordinates are the mapping evaluated out of range
    (a block with frozen ghost layers on every axis)."""
    nt, nr, nz = (int(v) for v in n)
    gc = coord_ghost(g, Y)
    i = np.arange(-gc, nt + gc, dtype=np.float64)
    jj = np.arange(-gc, nr + gc)
    k = np.arange(-gc, nz + gc, dtype=np.float64)
    dth = sector / nt
    steps = dr0 * ratio ** np.minimum(np.arange(nr + gc), cap)
    r = np.empty(jj.shape)
    pos = jj >= 0
    r[pos] = r_wall + np.concatenate([[0.0], np.cumsum(steps)])[jj[pos]]
    r[~pos] = r_wall + jj[~pos] * dr0
    th0 = 0.5 * sector
    K, J, Ii = np.meshgrid(k, r, i, indexing="ij")
    theta = th0 - Ii * dth + math.tan(math.radians(skew_deg)) * (J - r_wall) / J
    x = J * np.cos(theta + rotation)
    y = J * np.sin(theta + rotation)
    z = K * (r_wall * dth)
    return np.ascontiguousarray(np.stack([x, y, z]))


@dataclass
class BlockSpec:
    n: tuple
    sector: float
    skew_deg: float
    rotation: float


def multiblock_specs(nblocks: int = 48, seed: int = 4):
    """Seeded uneven O-grid sector blocks: n_theta ~ U{32..192},
    n_r ~ U{32..128}, n_z ~ U{16..64}, sector ~ U(pi/3, pi),
    skew ~ U(0, 30) degrees, rotation ~ U(0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(nblocks):
        n = (int(rng.integers(32, 193)), int(rng.integers(32, 129)), int(rng.integers(16, 65)))
        out.append(BlockSpec(n, float(rng.uniform(math.pi / 3, math.pi)),
                             float(rng.uniform(0.0, 30.0)), float(rng.uniform(0.0, 2 * math.pi))))
    return out


def state_nodes(xyz: np.ndarray, g: int, Y: int) -> np.ndarray:
    """Coordinates of the state nodes (interior plus g ghosts) cut out of a
    coordinate array."""
    ndim = xyz.shape[0]
    h = Y // 2
    sl = (slice(None),) + (slice(h, -h),) * ndim
    return np.ascontiguousarray(xyz[sl])


# ----------------------------------------------------------------------------
# states
# ----------------------------------------------------------------------------

def primitive_to_conserved(rho, vel, p, gamma=GAMMA):
    """(rho, velocity components, p) -> conserved (rho, rho*u_k, rho*E)."""
    ke = 0.5 * sum(v * v for v in vel)
    E = p / ((gamma - 1.0) * rho) + ke
    return np.stack([rho] + [rho * v for v in vel] + [rho * E])


def uniform_state(ndim: int, n, g: int, rho: float, vel, p: float, gamma=GAMMA) -> np.ndarray:
    shape = state_shape(ndim, n, g)[1:]
    vel = list(vel)[:ndim]
    out = primitive_to_conserved(np.full(shape, rho), [np.full(shape, v) for v in vel],
                                 np.full(shape, p), gamma)
    return np.ascontiguousarray(out)


def mach_velocity(mach: float, direction, rho=GAMMA, p=1.0, gamma=GAMMA):
    c = math.sqrt(gamma * p / rho)
    d = np.asarray(direction, dtype=np.float64)
    return mach * c * d / np.linalg.norm(d)


def direction_3d(theta_deg=20.0, phi_deg=10.0):
    t, f = math.radians(theta_deg), math.radians(phi_deg)
    return np.array([math.cos(t) * math.cos(f), math.sin(t) * math.cos(f), math.sin(f)])


@dataclass
class Vortex:
    """Isentropic vortex of Sec. 4.1.2: velocity perturbation
    ``eps*tau*exp(alpha*(1-tau^2))*(sin th, -cos th)`` and temperature drop
    ``-(gamma-1)*eps^2/(4*alpha*gamma)*exp(2*alpha*(1-tau^2))`` with
    ``tau = r/rc``, zero entropy change, on a uniform background
    (rho_inf, vel_inf, p_inf).  In 3D the vortex is a column along z."""
    eps: float = 5.0 / (2.0 * math.pi)
    alpha: float = 0.5
    rc: float = 1.0
    center: tuple = (0.0, 0.0)
    rho_inf: float = GAMMA
    p_inf: float = 1.0
    vel_inf: tuple = (0.5, 0.0, 0.0)
    gamma: float = GAMMA

    def primitives(self, x, y, t=0.0, period=None):
        """(rho, u, v, p) at points (x, y) and time t (centre translated by
        the background velocity; nearest periodic image if ``period``, a
        scalar or the (x, y) periods)."""
        g = self.gamma
        cx = self.center[0] + self.vel_inf[0] * t
        cy = self.center[1] + self.vel_inf[1] * t
        dx = x - cx
        dy = y - cy
        if period is not None:
            px, py = (period, period) if np.isscalar(period) else (period[0], period[1])
            dx = dx - px * np.round(dx / px)
            dy = dy - py * np.round(dy / py)
        r = np.sqrt(dx * dx + dy * dy)
        tau = r / self.rc
        ex = np.exp(self.alpha * (1.0 - tau * tau))
        # tau*(sin th, -cos th) = (dy, -dx)/rc
        du = self.eps * ex * dy / self.rc
        dv = -self.eps * ex * dx / self.rc
        dT = -(g - 1.0) * self.eps ** 2 / (4.0 * self.alpha * g) * ex * ex
        Tinf = self.p_inf / self.rho_inf
        T = Tinf + dT
        rho = self.rho_inf * (T / Tinf) ** (1.0 / (g - 1.0))
        p = rho * T
        return rho, self.vel_inf[0] + du, self.vel_inf[1] + dv, p

    def state(self, nodes: np.ndarray, t=0.0, period=None) -> np.ndarray:
        """Conserved state at node coordinates ``nodes`` (ndim, ...)."""
        ndim = nodes.shape[0]
        rho, u, v, p = self.primitives(nodes[0], nodes[1], t, period)
        vel = [u, v] if ndim == 2 else [u, v, np.full_like(u, self.vel_inf[2])]
        return np.ascontiguousarray(primitive_to_conserved(rho, vel, p, self.gamma))


def interior(a: np.ndarray, g: int) -> np.ndarray:
    """View of the interior nodes of a state-like array (leading variable axis)."""
    nd = a.ndim - 1
    return a[(slice(None),) + (slice(g, -g),) * nd]


# ----------------------------------------------------------------------------
# wall-bounded shock problems (Sec. 4.2): double Mach reflection and the
# supersonic cylinder.  Grids, initial states and which face is what; the
# boundary treatment itself belongs to the solver.
# ----------------------------------------------------------------------------

def _point_reflect(X, idx_ghost, idx_bnd, idx_src):
    """X[..., ghost] = 2 X[..., boundary] - X[..., source] along the last axes"""
    X[idx_ghost] = 2.0 * X[idx_bnd] - X[idx_src]


def dmr_grid(nx: int = 961, ny: int = 241, rand: float = 0.05, g: int = 3, Y: int = 6, seed: int = 0,
             Lx: float = 4.0, Ly: float = 1.0) -> np.ndarray:
    """Grid of the double Mach reflection on [0, Lx] x [0, Ly] with nx x ny
    nodes, every node moved by ``rand`` of the spacing in a random direction
    (the displacement law of paper_random_displacement, as the random grid of
    Sec. 4.1.1); nodes on the boundary lines keep the component along the
    line only and the corners stay.  Ghost layers: the mirror image of the
    interior about the bottom wall y = 0, point reflections through the
    boundary nodes on the other sides."""
    gc = coord_ghost(g, Y)
    assert nx > gc and ny > gc
    hx, hy = Lx / (nx - 1), Ly / (ny - 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = i * hx
    y = j * hy
    d = paper_random_displacement(x.shape, rand, rng)
    dx = hx * d[0]
    dy = hy * d[1]
    inner_i = (i > 0) & (i < nx - 1)
    inner_j = (j > 0) & (j < ny - 1)
    x = x + np.where(inner_i, dx, 0.0)
    y = y + np.where(inner_j, dy, 0.0)
    X = np.zeros((2, ny + 2 * gc, nx + 2 * gc))
    X[:, gc:gc + ny, gc:gc + nx] = np.stack([x, y])
    rows = slice(gc, gc + ny)
    for l in range(1, gc + 1):  # left and right: point reflection
        _point_reflect(X, (slice(None), rows, gc - l), (slice(None), rows, gc), (slice(None), rows, gc + l))
        r = gc + nx - 1
        _point_reflect(X, (slice(None), rows, r + l), (slice(None), rows, r), (slice(None), rows, r - l))
    for l in range(1, gc + 1):  # bottom: mirror about y = 0; top: point reflection
        X[0, gc - l, :] = X[0, gc + l, :]
        X[1, gc - l, :] = -X[1, gc + l, :]
        t = gc + ny - 1
        _point_reflect(X, (slice(None), t + l, slice(None)), (slice(None), t, slice(None)),
                       (slice(None), t - l, slice(None)))
    return np.ascontiguousarray(X)


DMR_PRE = (1.4, 0.0, 0.0, 1.0)                  # rho, u, v, p ahead of the shock
DMR_POST = (8.0, 7.1447, -4.125, 116.5)         # behind it (Mach 10, 60 degrees)
DMR_X0 = 1.0 / 6.0                               # where the shock meets the wall at t = 0
DMR_NORMAL = (math.cos(math.pi / 6), -math.sin(math.pi / 6), 0.0)
DMR_SPEED = 10.0


def dmr_state(nodes: np.ndarray, g: int, gamma=GAMMA) -> np.ndarray:
    """Initial state at the state nodes (ghosts included): post-shock where
    x - y tan(pi/6) < 1/6, pre-shock elsewhere; the ghost layers below the
    bottom boundary left of x = 1/6 (its inflow part) hold the post-shock
    state."""
    x, y = nodes[0], nodes[1]
    post = x - y * math.tan(math.pi / 6) < DMR_X0
    post[:g, :] = nodes[0][:g, :] < DMR_X0
    rho = np.where(post, DMR_POST[0], DMR_PRE[0])
    u = np.where(post, DMR_POST[1], DMR_PRE[1])
    v = np.where(post, DMR_POST[2], DMR_PRE[2])
    p = np.where(post, DMR_POST[3], DMR_PRE[3])
    return np.ascontiguousarray(primitive_to_conserved(rho, [u, v], p, gamma))


def dmr_faces(nodes: np.ndarray, g: int, gamma=GAMMA) -> dict:
    """What each face of the double Mach reflection is: left post-shock
    inflow (held), right outflow (extrapolated), bottom a slip wall from
    x = 1/6 on (held post-shock inflow before), top the exact moving shock
    (plane normal . x = cos(pi/6)/6 + 10 t).  mask: one byte per bottom
    boundary node."""
    bottom_x = nodes[0][g, g:-g]
    def cons(s):
        return [float(a) for a in primitive_to_conserved(np.array(s[0]), [np.array(s[1]), np.array(s[2])],
                                                          np.array(s[3]), gamma)]
    return dict(kind=[[0, 1], [2, 3]], mask={(1, 0): (bottom_x >= DMR_X0).astype(np.uint8)},
                pre=cons(DMR_PRE), post=cons(DMR_POST), normal=DMR_NORMAL,
                offset=DMR_NORMAL[0] * DMR_X0, speed=DMR_SPEED)


def dmr_shock_x(t: float, y: float = 1.0) -> float:
    """x of the incident shock at height y and time t"""
    return DMR_X0 + y * math.tan(math.pi / 6) + DMR_SPEED * t / math.cos(math.pi / 6)


def cylinder_grid(imax: int = 61, jmax: int = 81, rand: float = 0.2, g: int = 3, Y: int = 6, seed: int = 0,
                  Rx: float = 3.0, Ry: float = 6.0, theta: float = 5.0 * math.pi / 12.0) -> np.ndarray:
    """Grid of the supersonic cylinder (Sec. 4.2.2): node (i, j) at
    x = (Rx - (Rx-1) eta') cos(theta (2 xi' - 1)),
    y = (Ry - (Ry-1) eta') sin(theta (2 xi' - 1)), xi' = xi/(imax-1),
    eta' = eta/(jmax-1) with xi = i + rand phi, eta = j + rand sqrt(1 - phi^2),
    phi ~ U(0, 1) drawn per interior node (boundary nodes unmoved).  Index i
    runs along the body (axis 0), j from the outer boundary (j = 0) to the
    cylinder wall r = 1 (j = jmax-1, axis 1).  Ghost layers: the mapping
    continued, except beyond the wall, where they are the mirror image of the
    interior about the wall's tangent at each wall node."""
    gc = coord_ghost(g, Y)
    assert imax > gc and jmax > gc
    rng = np.random.Generator(np.random.PCG64(seed))
    jj, ii = np.meshgrid(np.arange(-gc, jmax + gc, dtype=np.float64), np.arange(-gc, imax + gc, dtype=np.float64),
                         indexing="ij")
    phi = rng.uniform(0.0, 1.0, ii.shape)
    inner = (ii > 0) & (ii < imax - 1) & (jj > 0) & (jj < jmax - 1)
    xi = ii + np.where(inner, rand * phi, 0.0)
    eta = jj + np.where(inner, rand * np.sqrt(1.0 - phi * phi), 0.0)
    xp, ep = xi / (imax - 1), eta / (jmax - 1)
    X = np.stack([(Rx - (Rx - 1.0) * ep) * np.cos(theta * (2.0 * xp - 1.0)),
                  (Ry - (Ry - 1.0) * ep) * np.sin(theta * (2.0 * xp - 1.0))])
    w = gc + jmax - 1  # the wall row
    for l in range(1, gc + 1):
        xw = X[:, w, :]
        nrm = xw / np.linalg.norm(xw, axis=0)
        d = X[:, w - l, :] - xw
        X[:, w + l, :] = xw + d - 2.0 * (nrm * d).sum(axis=0) * nrm
    return np.ascontiguousarray(X)


CYL_MACH = 2.0


def cylinder_state(ndim_n, g: int, gamma=GAMMA) -> np.ndarray:
    """Uniform Mach 2 free stream towards -x with p = 1, rho = gamma (c = 1)."""
    return uniform_state(2, ndim_n, g, gamma, [-CYL_MACH, 0.0], 1.0, gamma)


def cylinder_faces() -> dict:
    """outflow (extrapolated) along the two rays, held free-stream inflow at
    the outer boundary, slip wall on the cylinder"""
    return dict(kind=[[1, 1], [0, 2]])
