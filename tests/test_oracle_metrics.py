"""Pins of the oracle's symmetric conservative metrics (Sec. 2.1, eqs. JBabc
and JB, with D_Y of eq. metric_discret) against closed forms (CPU only)."""
import numpy as np
import pytest

import oracle as O
from paper_2101_05886_amd import inputs as I

TEXTBOOK = {
    2: np.array([-1, 0, 1]) / 2.0,
    4: np.array([1, -8, 0, 8, -1]) / 12.0,
    6: np.array([-1, 9, -45, 0, 45, -9, 1]) / 60.0,
    8: np.array([3, -32, 168, -672, 0, 672, -168, 32, -3]) / 840.0,
}


def central_diff(f, Y, axis, g):
    """Textbook central derivative of order Y along ``axis`` (array axis of a
    field without the variable axis), evaluated on the interior."""
    c = TEXTBOOK[Y]
    h = Y // 2
    out = 0.0
    nd = f.ndim
    for k, ck in enumerate(c):
        if ck == 0:
            continue
        sl = []
        for a in range(nd):
            n = f.shape[a] - 2 * g
            if a == axis:
                sl.append(slice(g + k - h, g + k - h + n))
            else:
                sl.append(slice(g, g + n))
        out = out + ck * f[tuple(sl)]
    return out


def analytic_cofactors(A):
    return np.linalg.det(A) * np.linalg.inv(A)  # adj(A): row d = s_d


@pytest.mark.parametrize("Y", [2, 4, 6, 8])
def test_affine_grid_metrics_are_cofactors_3d(Y):
    rng = np.random.default_rng(Y)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    g = max(3, Y // 2)
    n = [7, 6, 5]
    gr = O.Grid(3, n, g, bc=[1, 1, 1])
    xyz = I.affine_grid(3, n, g, Y, A, b=[0.3, -1.0, 2.0])
    met = O.metrics(gr, Y, xyz)
    adj = analytic_cofactors(A)
    for d in range(3):
        for c in range(3):
            assert np.allclose(met[3 * d + c], adj[d, c], rtol=0, atol=1e-12)
    assert np.allclose(met[9], np.linalg.det(A), rtol=1e-12, atol=0)


@pytest.mark.parametrize("Y", [2, 4, 6, 8])
def test_affine_grid_metrics_are_cofactors_2d(Y):
    A = np.array([[1.3, 0.4], [-0.2, 0.9]])
    g = max(3, Y // 2)
    n = [9, 8]
    gr = O.Grid(2, n, g, bc=[1, 1])
    met = O.metrics(gr, Y, I.affine_grid(2, n, g, Y, A))
    adj = analytic_cofactors(A)
    for d in range(2):
        for c in range(2):
            assert np.allclose(met[2 * d + c], adj[d, c], rtol=0, atol=1e-13)
    assert np.allclose(met[4], np.linalg.det(A), rtol=1e-13, atol=0)


def _wavy3_analytic(n, L, amp, g):
    """Analytic metrics of the 3D wavy mapping at the state nodes."""
    h = L / n
    a = -L / 2 + np.arange(-g, n + g) * h
    Z, Yy, X = np.meshgrid(a, a, a, indexing="ij")
    k = 2 * np.pi / L
    s = lambda t: np.sin(k * (t + L / 2))
    cs = lambda t: np.cos(k * (t + L / 2))
    A = amp * L
    grad = np.stack([A * k * cs(X) * s(Yy) * s(Z), A * k * s(X) * cs(Yy) * s(Z),
                     A * k * s(X) * s(Yy) * cs(Z)])
    # dx_c/dxi_e (index units) = h*(delta_ce + grad_e)
    Jm = h * (np.eye(3)[:, :, None, None, None] + grad[None, :, ...])
    Jm = np.moveaxis(Jm, (0, 1), (-2, -1))
    det = np.linalg.det(Jm)
    adj = det[..., None, None] * np.linalg.inv(Jm)
    return adj, det


@pytest.mark.parametrize("Y", [2, 4])
def test_metric_order_of_accuracy_3d(Y):
    errs = []
    for n in (12, 24):
        g = 3
        xyz = I.wavy_grid(3, n, 12.0, g, Y, amp=0.05)
        met = O.metrics(O.Grid(3, n, g), Y, xyz)
        adj, det = _wavy3_analytic(n, 12.0, 0.05, g)
        h = 12.0 / n
        e = max(np.abs(met[3 * d + c] - adj[..., d, c]).max() / h ** 2 for d in range(3) for c in range(3))
        errs.append(max(e, np.abs(met[9] - det).max() / h ** 3))
    assert np.log2(errs[0] / errs[1]) == pytest.approx(Y, abs=0.6)


@pytest.mark.parametrize("Y", [2, 4, 6])
def test_metric_order_of_accuracy_2d(Y):
    errs = []
    for n in (16, 32):
        g = 3
        L = 10.0
        xyz = I.wavy_grid(2, n, L, g, Y, amp=0.05)
        met = O.metrics(O.Grid(2, n, g), Y, xyz)
        h = L / n
        a = -L / 2 + np.arange(-g, n + g) * h
        E, X = np.meshgrid(a, a, indexing="ij")
        k = 2 * np.pi / L
        A = 0.05 * L
        sx, sy = np.sin(k * (X + L / 2)), np.sin(k * (E + L / 2))
        cx, cy = np.cos(k * (X + L / 2)), np.cos(k * (E + L / 2))
        x_xi, x_eta = h * (1 + A * k * cx * sy), h * (A * k * sx * cy)
        y_xi, y_eta = h * (A * k * cx * sy), h * (1 + A * k * sx * cy)
        exact = [y_eta, -x_eta, -y_xi, x_xi, x_xi * y_eta - x_eta * y_xi]
        e = max(np.abs(met[c] - exact[c]).max() / (h if c < 4 else h * h) for c in range(5))
        errs.append(e)
    assert np.log2(errs[0] / errs[1]) == pytest.approx(Y, abs=0.5)


@pytest.mark.parametrize("Y", [2, 4, 6, 8])
def test_surface_conservation_law_3d(Y):
    # eq. (SCL): sum_d D_Y,d (s_{d,c}) = 0 to round-off on a jittered grid
    g = max(3, Y // 2)
    n = 10
    xyz = I.wavy_grid(3, n, 10.0, g, Y, amp=0.1, jitter=0.1, seed=5)
    met = O.metrics(O.Grid(3, n, g), Y, xyz)
    scale = np.abs(met[:9]).max()
    for c in range(3):
        # array axes of a field: (k, j, i) -> direction d is array axis 2-d
        Ic = sum(central_diff(met[3 * d + c], Y, 2 - d, g) for d in range(3))
        assert np.abs(Ic).max() < 1e-14 * scale * 10
    # the identity needs the derivative of the metric order: a sixth-order
    # derivative of second-order metrics leaves an O(h^2) residue
    if Y == 2:
        Ic = sum(central_diff(met[3 * d], 6, 2 - d, g) for d in range(3))
        assert np.abs(Ic).max() > 1e-6 * scale


@pytest.mark.parametrize("Y", [2, 6, 8])
def test_surface_conservation_law_2d(Y):
    g = max(3, Y // 2)
    n = 24
    xyz = I.wavy_grid(2, n, 20.0, g, Y, amp=0.1, jitter=0.2, seed=3)
    met = O.metrics(O.Grid(2, n, g), Y, xyz)
    scale = np.abs(met[:4]).max()
    for c in range(2):
        Ic = sum(central_diff(met[2 * d + c], Y, 1 - d, g) for d in range(2))
        assert np.abs(Ic).max() < 1e-14 * scale * 10


def test_periodic_ghost_metrics_match_computed_values():
    # periodic ghosts are copies of the image; evaluating the formulas at a
    # ghost node from the shifted coordinates gives the same value
    Y, g, n = 6, 3, 10
    xyz = I.wavy_grid(3, n, 10.0, g, Y, amp=0.1, jitter=0.05, seed=2)
    gr = O.Grid(3, n, g)
    met = O.metrics(gr, Y, xyz)
    pts = np.array([[-1, 0, 0], [n + 2, 3, 4], [2, -3, n + 1], [-2, -2, -2]])
    vals = O.metrics_at(gr, Y, xyz, pts)
    for p, v in zip(pts, vals):
        stored = met[:, p[2] + g, p[1] + g, p[0] + g]
        assert np.allclose(v, stored, rtol=0, atol=1e-13 * np.abs(met).max())


def test_metrics_3d_of_extruded_2d_grid_reduce_to_2d():
    Y, g, n = 4, 3, 12
    xy = I.wavy_grid(2, n, 12.0, g, Y, amp=0.1, jitter=0.1, seed=9)
    m2 = O.metrics(O.Grid(2, n, g), Y, xy)
    gc = I.coord_ghost(g, Y)
    nk = 6
    hz = 0.75
    z = (np.arange(-gc, nk + gc) * hz)[:, None, None] * np.ones_like(xy[0])[None]
    xyz = np.stack([np.broadcast_to(xy[0], z.shape), np.broadcast_to(xy[1], z.shape), z])
    m3 = O.metrics(O.Grid(3, [n, n, nk], g), Y, xyz)
    k = g + 2
    pairs = [(0, 0), (1, 1), (3, 2), (4, 3)]
    for c3, c2 in pairs:
        assert np.allclose(m3[c3, k] / hz, m2[c2], rtol=0, atol=1e-13)
    for c3 in (2, 5, 6, 7):
        assert np.abs(m3[c3, k]).max() < 1e-13
    assert np.allclose(m3[8, k], m2[4], rtol=1e-13, atol=1e-14)
    assert np.allclose(m3[9, k] / hz, m2[4], rtol=1e-13, atol=1e-14)


def test_folded_grid_is_rejected():
    # x = xi + A sin(2 pi xi / n) with A 2 pi / n > 1 folds the grid (x_xi < 0)
    n, g, Y = 16, 3, 2
    xyz = I.cartesian_grid(2, n, g, Y)
    xyz[0] = xyz[0] + 4.0 * np.sin(2 * np.pi * xyz[0] / n)
    with pytest.raises(ValueError):
        O.metrics(O.Grid(2, n, g), Y, xyz)
