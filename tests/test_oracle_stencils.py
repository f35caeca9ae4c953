"""Pins of the oracle's building blocks against closed forms (CPU only).

* face interpolation I_Y and derivative D_Y (Sec. 3, eq. metric_discret)
  against the textbook central first derivatives of order Y;
* WENO5-JS (Sec. 2.2, eqs. weno and weno_wights) on hand-computed inputs,
  its invariances and its fifth-order convergence on cell averages;
* the fifth-order linear upwind scheme (eq. linear_upwind) as WENO5 with the
  optimal weights, and its split into a sixth-order central part plus the
  fifth difference (eq. Linear_upwind_standard).
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle as O

# textbook central first-derivative stencils of order 2, 4, 6, 8 on nodes
# i-Y/2 .. i+Y/2
TEXTBOOK = {
    2: [Fr(-1, 2), 0, Fr(1, 2)],
    4: [Fr(1, 12), Fr(-8, 12), 0, Fr(8, 12), Fr(-1, 12)],
    6: [Fr(-1, 60), Fr(9, 60), Fr(-45, 60), 0, Fr(45, 60), Fr(-9, 60), Fr(1, 60)],
    8: [Fr(3, 840), Fr(-32, 840), Fr(168, 840), Fr(-672, 840), 0, Fr(672, 840),
        Fr(-168, 840), Fr(32, 840), Fr(-3, 840)],
}


def deriv(Y, w):
    """D_Y from samples w[0..Y] via two oracle face interpolations."""
    return O.face_interp(Y, w[1:]) - O.face_interp(Y, w[:-1])


@pytest.mark.parametrize("Y", [2, 4, 6, 8])
def test_derivative_is_textbook_central_difference(Y):
    for k in range(Y + 1):
        e = np.zeros(Y + 1)
        e[k] = 1.0
        assert deriv(Y, e) == pytest.approx(float(TEXTBOOK[Y][k]), abs=1e-15)


@pytest.mark.parametrize("Y", [2, 4, 6, 8])
def test_interp_exact_on_polynomials_and_partition_of_unity(Y):
    # conservative FD view: if the node values are cell averages of p over
    # [m-1/2, m+1/2], I_Y returns p at the face exactly for deg p < Y
    h = Y // 2
    x = np.arange(-h + 1, h + 1, dtype=float)  # nodes i-Y/2+1 .. i+Y/2, face at 0.5
    for deg in range(Y):
        w = ((x + 0.5) ** (deg + 1) - (x - 0.5) ** (deg + 1)) / (deg + 1)
        assert O.face_interp(Y, w) == pytest.approx(0.5 ** deg, rel=1e-13, abs=1e-13)
    assert O.face_interp(Y, np.ones(Y)) == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("Y", [2, 4, 6])
def test_derivative_order_of_accuracy(Y):
    errs = []
    for hstep in (0.2, 0.1):
        x = 0.3 + hstep * np.arange(-Y // 2, Y // 2 + 1)
        errs.append(abs(deriv(Y, np.sin(x)) / hstep - np.cos(0.3)))
    rate = np.log2(errs[0] / errs[1])
    assert rate == pytest.approx(Y, abs=0.3)


def test_weno5_hand_values():
    # constant data: every candidate equals the constant
    assert O.weno5([3.0] * 5) == pytest.approx(3.0, rel=1e-15)
    # linear data (0,1,2,3,4): beta = (1,1,1), weights = optimal, W = 2.5
    assert O.weno5([0, 1, 2, 3, 4]) == pytest.approx(2.5, rel=1e-14)
    # step (0,0,0,1,1): beta = (0, 4/3, 10/3); the smooth left candidate
    # (q0 = 0) takes almost all the weight
    C = np.array([0.1, 0.6, 0.3])
    beta = np.array([0.0, 4.0 / 3.0, 10.0 / 3.0])
    a = C / (beta + 1e-6) ** 2
    w = a / a.sum()
    q = np.array([0.0, 1.0 / 3.0, 2.0 / 3.0])
    assert O.weno5([0, 0, 0, 1, 1]) == pytest.approx(float(w @ q), rel=1e-12)
    assert O.weno5([0, 0, 0, 1, 1]) < 2e-12


def test_weno5_invariances():
    rng = np.random.default_rng(0)
    for _ in range(50):
        v = rng.standard_normal(5)
        c = rng.standard_normal()
        assert O.weno5(v + c) == pytest.approx(O.weno5(v) + c, rel=1e-12, abs=1e-12)
        assert O.weno5(-v) == pytest.approx(-O.weno5(v), rel=1e-13, abs=1e-15)


def test_weno5_fifth_order_on_cell_averages():
    # v_m = cell averages of h = cos over [m-1/2, m+1/2]*dx: W approximates h(x_{i+1/2})
    errs = []
    for dx in (0.1, 0.05, 0.025):
        xf = 0.4
        m = np.arange(-2, 3)
        lo = xf + (m - 1) * dx
        hi = xf + m * dx
        v = (np.sin(hi) - np.sin(lo)) / dx
        errs.append(abs(O.weno5(v, 1e-40) - np.cos(xf)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 4.5


def test_linear_upwind_is_weno_with_optimal_weights():
    # sum_k C_k q_k with the q_k of eq. (weno) (q0 = 1/3,-7/6,11/6) gives
    # (2,-13,47,27,-3)/60 of eq. (linear_upwind)
    q = [[Fr(1, 3), Fr(-7, 6), Fr(11, 6), 0, 0],
         [0, Fr(-1, 6), Fr(5, 6), Fr(1, 3), 0],
         [0, 0, Fr(1, 3), Fr(5, 6), Fr(-1, 6)]]
    C = [Fr(1, 10), Fr(3, 5), Fr(3, 10)]
    lin = [sum(C[k] * q[k][j] for k in range(3)) for j in range(5)]
    assert lin == [Fr(2, 60), Fr(-13, 60), Fr(47, 60), Fr(27, 60), Fr(-3, 60)]
    for j in range(5):
        e = np.zeros(5)
        e[j] = 1.0
        assert O.linear_upwind5(e) == pytest.approx(float(lin[j]), abs=1e-16)
    # a WENO input whose smoothness indicators are all equal takes the
    # optimal weights, so W equals the linear scheme there
    v = np.array([0.0, 1.0, 2.0, 3.0, 4.0]) * 0.7 + 1.3
    assert O.weno5(v) == pytest.approx(O.linear_upwind5(v), rel=1e-14)


def test_linear_upwind_central_plus_fifth_difference():
    # F+ from nodes i-2..i+2 and F- mirrored from i+3..i-1: half their sum is
    # the sixth-order central interpolation (1,-8,37,37,-8,1)/60 and half
    # their difference is (1,-5,10,-10,5,-1)/60 (eq. Linear_upwind_standard)
    for j in range(6):
        e = np.zeros(6)
        e[j] = 1.0
        plus = O.linear_upwind5(e[0:5])
        minus = O.linear_upwind5(e[::-1][0:5])
        cen = [1, -8, 37, 37, -8, 1][j] / 60.0
        d5 = [1, -5, 10, -10, 5, -1][j] / 60.0
        assert 0.5 * (plus + minus) == pytest.approx(cen, abs=1e-16)
        assert 0.5 * (plus - minus) == pytest.approx(d5, abs=1e-16)
        assert O.face_interp(6, e) == pytest.approx(cen, abs=1e-16)
