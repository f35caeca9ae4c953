"""Pins of the oracle's WENO7-JS (the seventh-order WENO that Remark 2
extends the method to) and of the scheme built on it (CPU only).

* Each candidate face value q_k is the face value of the cubic whose cell
  averages are the stencil values, and each smoothness indicator beta_k is
  240 x the Jiang-Shu measure sum_{l=1..3} int_cell (p_k^(l))^2 dx of that
  cubic (the integer quadratic forms, used without the 1/240: the reading
  that reproduces Table 2's WENO7 rows): both computed here in exact
  rational arithmetic from the definitions.
* With the optimal weights the scheme is the seventh-order upwind
  interpolation: exact on cell averages of polynomials of degree <= 6, and
  its split halves sum to the eighth-order central interpolation I_8.
* Hand values, invariances and seventh-order convergence of the nonlinear
  scheme on smooth data.
* The free-stream scheme with WENO7: Table 1 (round-off for WENO7-M6/M8 on
  the wavy and random grids, the standard WENO7 within a factor of two on
  the wavy grid) and Table 2 (WENO7-M4/M8 vortex errors on the coarse
  grids).
"""
import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle as O
from paper_2101_05886_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
C7 = [Fr(1, 35), Fr(12, 35), Fr(18, 35), Fr(4, 35)]


def cubic_from_cell_averages(vals, cells):
    """coefficients (ascending) of the polynomial whose averages over
    [c-1/2, c+1/2] are vals, exact rationals"""
    n = len(vals)
    A = []
    for c in cells:
        row = []
        for k in range(n):
            lo, hi = Fr(c) - Fr(1, 2), Fr(c) + Fr(1, 2)
            row.append((hi ** (k + 1) - lo ** (k + 1)) / (k + 1))
        A.append(row)
    # Gaussian elimination over the rationals
    M = [r + [Fr(v)] for r, v in zip(A, vals)]
    for i in range(n):
        piv = next(r for r in range(i, n) if M[r][i] != 0)
        M[i], M[piv] = M[piv], M[i]
        for r in range(n):
            if r != i and M[r][i] != 0:
                f = M[r][i] / M[i][i]
                M[r] = [a - f * b for a, b in zip(M[r], M[i])]
    return [M[i][n] / M[i][i] for i in range(n)]


def poly_eval(c, x):
    return sum(ck * x ** k for k, ck in enumerate(c))


def poly_deriv(c):
    return [k * c[k] for k in range(1, len(c))]


def poly_int_sq(c, lo, hi):
    """int_lo^hi p(x)^2 dx"""
    sq = [Fr(0)] * (2 * len(c) - 1) if c else [Fr(0)]
    for i, a in enumerate(c):
        for j, b in enumerate(c):
            sq[i + j] += a * b
    return sum(s * (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k, s in enumerate(sq))


def beta_definition(c):
    tot = Fr(0)
    d = c
    for _ in range(3):
        d = poly_deriv(d)
        tot += poly_int_sq(d, Fr(-1, 2), Fr(1, 2))
    return tot


@pytest.mark.parametrize("seed", range(6))
def test_candidates_and_smoothness_from_definition(seed):
    rng = np.random.default_rng(seed)
    v = [Fr(int(rng.integers(-50, 50)), int(rng.integers(1, 9))) for _ in range(7)]  # f_{i-3..i+3}
    q, beta = O.weno7_parts(np.array([float(x) for x in v]))
    for k in range(4):
        cells = [k - 3 + j for j in range(4)]  # stencil k: nodes i-3+k .. i+k, node i at cell 0
        c = cubic_from_cell_averages(v[k:k + 4], cells)
        assert q[k] == pytest.approx(float(poly_eval(c, Fr(1, 2))), rel=1e-13, abs=1e-12)
        assert beta[k] == pytest.approx(float(240 * beta_definition(c)), rel=1e-12, abs=1e-8)


def linear7(v):
    """the optimal-weight combination in exact arithmetic"""
    q = [(-3 * v[0] + 13 * v[1] - 23 * v[2] + 25 * v[3]) / 12, (v[1] - 5 * v[2] + 13 * v[3] + 3 * v[4]) / 12,
         (-v[2] + 7 * v[3] + 7 * v[4] - v[5]) / 12, (3 * v[3] + 13 * v[4] - 5 * v[5] + v[6]) / 12]
    return sum(ck * qk for ck, qk in zip(C7, q))


def test_optimal_weights_are_seventh_order_upwind_and_split_to_central8():
    # exact on cell averages of x^d, d <= 6 (the face at x = 1/2)
    for d in range(7):
        v = [(Fr(c) + Fr(1, 2)) ** (d + 1) / (d + 1) - (Fr(c) - Fr(1, 2)) ** (d + 1) / (d + 1) for c in range(-3, 4)]
        assert linear7(v) == Fr(1, 2) ** d
        # the nonlinear scheme with a huge epsilon has the optimal weights
        assert O.weno7(np.array([float(x) for x in v]), 1e30) == pytest.approx(float(Fr(1, 2) ** d), abs=1e-13)
    # the "+" and mirrored "-" halves (nodes i-3..i+3 and i+4..i-2) average to I_8
    coef = []
    for m in range(8):  # node i-3+m
        e = [Fr(0)] * 8
        e[m] = Fr(1)
        coef.append((linear7(e[0:7]) + linear7(e[7:0:-1])) / 2)
    assert coef == [Fr(-3, 840), Fr(29, 840), Fr(-139, 840), Fr(533, 840), Fr(533, 840),
                    Fr(-139, 840), Fr(29, 840), Fr(-3, 840)]


def test_hand_values_and_invariances():
    assert O.weno7(np.ones(7)) == pytest.approx(1.0, abs=1e-15)
    assert O.weno7(np.arange(7.0)) == pytest.approx(3.5, abs=1e-14)  # linear: the exact face value
    assert abs(O.weno7(np.array([0, 0, 0, 0, 1, 1, 1.0]))) < 1e-10  # step after the face node
    rng = np.random.default_rng(3)
    for _ in range(20):
        v = rng.standard_normal(7)
        assert O.weno7(v + 2.5) == pytest.approx(O.weno7(v) + 2.5, abs=1e-12)
        assert O.weno7(-v) == pytest.approx(-O.weno7(v), abs=1e-14)


def test_seventh_order_convergence_on_smooth_cell_averages():
    errs = []
    for h in (0.2, 0.1, 0.05):
        x0 = 0.37
        cells = x0 + h * np.arange(-3, 4)
        v = (np.cos(cells - h / 2) - np.cos(cells + h / 2)) / h  # cell averages of sin
        errs.append(abs(O.weno7(v, 1e-40) - np.sin(x0 + h / 2)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 6.3


def run_table1(grid, scheme, Y):
    g = 4
    n = 20
    xyz = I.paper_wavy_grid_2d(n, g, Y) if grid == "wavy" else I.random_grid_2d(n, g, Y, seed=7)
    gr = O.Grid(2, n, g)
    met = O.metrics(gr, Y, xyz)
    q = I.uniform_state(2, n, g, 1.4, [0.5, 0.0], 1.0)
    out = O.solve(gr, scheme, met, q, 0.2, 100)
    v = I.interior(out, g)[2] / I.interior(out, g)[0]
    return math.sqrt(float(np.mean(v * v))), float(np.abs(v).max())


@pytest.mark.parametrize("grid", ["wavy", "random"])
@pytest.mark.parametrize("name,Y", [("WENO7-M6", 6), ("WENO7-M8", 8)])
def test_table1_weno7_free_stream_at_round_off(grid, name, Y):
    paper = GOLD["table1"][grid][name]
    l2, li = run_table1(grid, O.Scheme("weno7", Y, True), Y)
    assert l2 < 10 * paper["L2"] and li < 10 * paper["Linf"]


def test_table1_standard_weno7():
    paper = GOLD["table1"]["wavy"]["WENO7"]
    l2, li = run_table1("wavy", O.Scheme("weno7", 8, False), 8)
    assert 0.5 < l2 / paper["L2"] < 2.0
    assert 0.5 < li / paper["Linf"] < 2.0
    paper = GOLD["table1"]["random"]["WENO7"]
    l2, li = run_table1("random", O.Scheme("weno7", 8, False), 8)
    assert 0.5 < l2 / paper["L2"] < 2.0
    assert 0.5 < li / paper["Linf"] < 2.0


def run_vortex(Y, n):
    g = 4
    vx = I.Vortex(eps=0.02, alpha=0.204, rc=1.0, vel_inf=(0.5, 0.0, 0.0))
    xyz = I.paper_wavy_grid_2d(n, g, Y)
    gr = O.Grid(2, n, g)
    met = O.metrics(gr, Y, xyz)
    nodes = I.state_nodes(xyz, g, Y)
    q = vx.state(nodes, 0.0, period=20.0)
    sc = O.Scheme("weno7", Y, True)
    T = 40.0
    nsteps = int(math.ceil(T / O.max_dt(gr, sc, met, q, 0.5)))
    out = O.solve(gr, sc, met, q, T / nsteps, nsteps)
    qe = I.interior(vx.state(nodes, T, period=20.0), g)
    qi = I.interior(out, g)
    e = qi[2] / qi[0] - qe[2] / qe[0]
    return math.sqrt(float(np.mean(e * e))), float(np.abs(e).max())


@pytest.mark.parametrize("name,Y", [("WENO7-M4", 4), ("WENO7-M8", 8)])
def test_table2_weno7_coarse_grids(name, Y):
    for npts in (21, 41):
        l2, li = run_vortex(Y, npts - 1)
        p2, pi = GOLD["table2"][name][str(npts)]
        assert 0.5 < l2 / p2 < 2.0, (npts, l2, p2)
        assert 0.5 < li / pi < 2.0, (npts, li, pi)


@pytest.mark.slow
def test_table2_weno7_m8_rate_41_to_81():
    # at 41^2 the oracle's error is 0.62x the printed one (Table 2 gives no
    # time step; this run takes CFL 0.5), so the observed rate is lower than
    # the printed 6.59: it must still show the high order, and the 81^2
    # error must match within a factor of two
    e41, e81 = run_vortex(8, 40), run_vortex(8, 80)
    p81 = GOLD["table2"]["WENO7-M8"]["81"]
    assert 0.5 < e81[0] / p81[0] < 2.0 and 0.5 < e81[1] / p81[1] < 2.0
    assert math.log2(e41[0] / e81[0]) > 5.5


@pytest.mark.parametrize("Y", [6, 8])
def test_weno7_3d_free_stream_jittered_grid(Y):
    n, g = (12, 10, 9), 4
    xyz = I.wavy_grid(3, n, 12.0, g, Y, amp=0.1, jitter=0.05, seed=9)
    gr = O.Grid(3, n, g)
    met = O.metrics(gr, Y, xyz)
    vel = I.mach_velocity(0.8, I.direction_3d())
    q = I.uniform_state(3, n, g, 1.4, vel, 1.0)
    r = O.residual(gr, O.Scheme("weno7", Y, True), met, q)
    assert np.abs(I.interior(r, g)).max() < 1e-12
    r0 = O.residual(gr, O.Scheme("weno7", Y, False), met, q)
    assert np.abs(I.interior(r0, g)).max() > 1e-6


def test_weno7_needs_four_ghosts():
    gr = O.Grid(2, 16, 3)
    with pytest.raises(ValueError):
        O.residual(gr, O.Scheme("weno7", 6, True), np.zeros(gr.metric_shape()), np.ones(gr.state_shape()))
