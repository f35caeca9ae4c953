"""Pins of two oracle parts that no paper value fixes (CPU only).

The time step (reading of the CFL rule used by the paper's runs): on an affine
grid x = A xi + b the contravariant metrics are exact, so the stable step is
CFL over the largest sum of index-space characteristic speeds,
sum_d (|grad(xi_d) . u| + c |grad(xi_d)|), with grad(xi_d) the rows of the
inverse of A.  That is the textbook CFL condition in index space; it uses no
metric array and no 1/J, so a dropped 1/J, a max over directions instead of
a sum, or a transposed metric index fails it.

The tangent basis of the 3D characteristic system (Sec. 2.2 leaves it open):
t1 = normalize(n x e_a) with a the axis of the smallest |n_k|, components
within 1e-10 counting as tied and the lowest k winning; t2 = n x t1.  The
shear rows of R are (0, t, u.t), so the basis can be read off R.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2101_05886_amd import inputs as I

GAMMA = 1.4


def index_speed_dt(Ainv, u, c, cfl):
    """CFL / sum_d (|grad xi_d . u| + c |grad xi_d|) at one state."""
    lam = sum(abs(Ainv[d] @ u) + c * np.linalg.norm(Ainv[d]) for d in range(len(u)))
    return cfl / lam


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("Y", [2, 6])
def test_max_dt_uniform_flow_affine_grid(ndim, Y):
    rng = np.random.default_rng(40 + ndim + Y)
    A = np.eye(ndim) * 0.7 + 0.25 * rng.standard_normal((ndim, ndim))
    n = [9, 8, 7][:ndim]
    g = 3
    gr = O.Grid(ndim, n, g, bc=[1] * ndim)
    met = O.metrics(gr, Y, I.affine_grid(ndim, n, g, Y, A, b=[0.5] * ndim))
    vel = I.mach_velocity(0.8, rng.standard_normal(ndim))
    q = I.uniform_state(ndim, n, g, GAMMA, vel, 1.0)
    got = O.max_dt(gr, O.Scheme("weno5", Y, True), met, q, 0.5)
    want = index_speed_dt(np.linalg.inv(A), vel, 1.0, 0.5)  # c = 1 for rho = gamma, p = 1
    assert got == pytest.approx(want, rel=1e-12)


def test_max_dt_cartesian_textbook():
    # x = diag(h) xi: dt = CFL / sum_d (|u_d| + c) / h_d
    h = np.array([0.5, 0.25, 2.0])
    n, g, Y = [6, 7, 8], 3, 4
    gr = O.Grid(3, n, g, bc=[1, 1, 1])
    met = O.metrics(gr, Y, I.affine_grid(3, n, g, Y, np.diag(h)))
    u = np.array([0.3, -0.2, 0.1])
    q = I.uniform_state(3, n, g, GAMMA, u, 1.0)
    got = O.max_dt(gr, O.Scheme("weno5", Y, True), met, q, 0.9)
    assert got == pytest.approx(0.9 / np.sum((np.abs(u) + 1.0) / h), rel=1e-13)


def test_max_dt_takes_the_fastest_node():
    # a varying state on a sheared grid: the step is set by the node with
    # the largest index-space speed sum (found here from A^-1 and the
    # primitive variables, node by node)
    A = np.array([[1.1, 0.3, 0.0], [-0.2, 0.8, 0.1], [0.05, 0.0, 0.6]])
    n, g, Y = [8, 7, 6], 3, 6
    gr = O.Grid(3, n, g, bc=[1, 1, 1])
    met = O.metrics(gr, Y, I.affine_grid(3, n, g, Y, A))
    rng = np.random.default_rng(5)
    shape = I.state_shape(3, n, g)[1:]
    rho = rng.uniform(0.8, 1.6, shape)
    u = [rng.uniform(-0.7, 0.7, shape) for _ in range(3)]
    p = rng.uniform(0.6, 1.8, shape)
    q = I.primitive_to_conserved(rho, u, p, GAMMA)
    got = O.max_dt(gr, O.Scheme("weno5", Y, True), met, q, 0.5)
    Ainv = np.linalg.inv(A)
    best = math.inf
    for k in range(g, g + n[2]):
        for j in range(g, g + n[1]):
            for i in range(g, g + n[0]):
                uu = np.array([u[c][k, j, i] for c in range(3)])
                c = math.sqrt(GAMMA * p[k, j, i] / rho[k, j, i])
                best = min(best, index_speed_dt(Ainv, uu, c, 0.5))
    assert got == pytest.approx(best, rel=1e-12)


def shear_tangents(R):
    """t1, t2 from the shear columns of R (rows 1..3 of columns 2 and 3)."""
    return R[1:4, 2], R[1:4, 3]


def state(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.concatenate([[rho], rho * u, [p / (GAMMA - 1) + 0.5 * rho * u @ u]])


@pytest.mark.parametrize("delta", [0.0, 1e-15, -1e-15, 3e-11, -3e-11])
def test_tangent_tie_lowest_axis_wins(delta):
    # n = (0.8, 0.6 cos45, 0.6 sin45): |n_y| = |n_z| analytically, both
    # smaller than |n_x|; perturbations below the tie width keep a = y, so
    # t1 = normalize(n x e_y) has no y component
    qL = state(1.2, [0.3, -0.1, 0.2], 1.1)
    qR = state(1.0, [0.2, 0.1, -0.3], 0.9)
    s = 0.6 / math.sqrt(2.0)
    sf = np.array([0.8, s, s * (1.0 + delta)]) * 2.5
    _, R, _ = O.eigensystem(3, GAMMA, qL, qR, sf, 1.3)
    n = sf / np.linalg.norm(sf)
    t1, t2 = shear_tangents(R)
    ey = np.array([0.0, 1.0, 0.0])
    want = np.cross(n, ey)
    want /= np.linalg.norm(want)
    assert np.abs(t1 - want).max() < 1e-14
    assert np.abs(t2 - np.cross(n, want)).max() < 1e-14


@pytest.mark.parametrize("sf,axis", [((0.2, 0.7, 0.5), 0), ((0.7, 0.2, 0.5), 1), ((0.7, 0.5, 0.2), 2),
                                     ((-0.7, 0.5, -0.2), 2), ((0.5, 0.5, 0.5), 0),
                                     ((0.5, -0.3, 0.3 + 2e-10), 1)])
def test_tangent_axis_is_smallest_normal_component(sf, axis):
    # outside the tie width the strictly smallest |n_k| picks the axis (the
    # last case: 2e-10 apart, not tied); a full tie picks axis 0
    qL = state(1.0, [0.1, 0.2, 0.3], 1.0)
    sf = np.asarray(sf, dtype=float)
    _, R, _ = O.eigensystem(3, GAMMA, qL, qL, sf, 1.0)
    n = sf / np.linalg.norm(sf)
    e = np.zeros(3)
    e[axis] = 1.0
    want = np.cross(n, e)
    want /= np.linalg.norm(want)
    t1, t2 = shear_tangents(R)
    assert abs(t1 @ e) < 1e-14
    assert np.abs(t1 - want).max() < 1e-14
    # orthonormal and right-handed with n
    assert abs(t1 @ n) < 1e-14 and abs(t2 @ n) < 1e-14 and abs(t1 @ t2) < 1e-14
    assert np.abs(np.cross(t1, t2) - n).max() < 1e-14
