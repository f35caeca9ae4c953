"""The oracle against the values the paper prints (tests/golden/paper_tables.json).

Table 1 (Sec. 4.1.1): free stream on the 21x21 wavy and random grids, dt 0.2,
100 steps.  Table 2 (Sec. 4.1.2): isentropic-vortex errors and rates on the
wavy grid.  The paper does not print every detail of its runs (its random
grid realisation, its exact time steps), so the comparison is by magnitude:
round-off level for the free-stream-preserving schemes, within a factor of
two for the errors that carry digits, and the observed rate within 0.8.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2101_05886_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def v_errors(q, g, v_exact=0.0):
    qi = I.interior(q, g)
    v = qi[2] / qi[0]
    e = v - v_exact
    return math.sqrt(float(np.mean(e * e))), float(np.abs(e).max())


def run_table1(grid, scheme, Y):
    g = max(3, Y // 2)
    n = 20  # 21 points including the periodic duplicate
    xyz = I.paper_wavy_grid_2d(n, g, Y) if grid == "wavy" else I.random_grid_2d(n, g, Y, seed=7)
    gr = O.Grid(2, n, g)
    met = O.metrics(gr, Y, xyz)
    q = I.uniform_state(2, n, g, 1.4, [0.5, 0.0], 1.0)
    out = O.solve(gr, scheme, met, q, 0.2, 100)
    return v_errors(out, g)


def test_table1_wavy_standard_weno5():
    paper = GOLD["table1"]["wavy"]["WENO5"]
    l2, li = run_table1("wavy", O.Scheme("weno5", 6, False), 6)
    assert 0.5 < l2 / paper["L2"] < 2.0
    assert 0.5 < li / paper["Linf"] < 2.0


@pytest.mark.parametrize("grid", ["wavy", "random"])
@pytest.mark.parametrize("Y", [2, 6, 8])
def test_table1_free_stream_preserving_at_round_off(grid, Y):
    paper = GOLD["table1"][grid]["WENO5-M6"]
    l2, li = run_table1(grid, O.Scheme("weno5", Y, True), Y)
    assert l2 < 10 * paper["L2"] and li < 10 * paper["Linf"]


def test_table1_random_standard_weno5():
    # the random grid with the paper's displacement law (the one it prints
    # for the cylinder grid): the standard scheme's errors within 2x of
    # Table 1 (ours 1.80e-2 / 5.97e-2 against 1.29e-2 / 4.41e-2; a uniformly
    # random direction gives 5.6e-2 / 2.1e-1, four to five times the paper)
    paper = GOLD["table1"]["random"]["WENO5"]
    l2, li = run_table1("random", O.Scheme("weno5", 6, False), 6)
    assert 0.5 < l2 / paper["L2"] < 2.0
    assert 0.5 < li / paper["Linf"] < 2.0


def run_vortex(recon, Y, n):
    g = 3
    vx = I.Vortex(eps=0.02, alpha=0.204, rc=1.0, vel_inf=(0.5, 0.0, 0.0))
    xyz = I.paper_wavy_grid_2d(n, g, Y)
    gr = O.Grid(2, n, g)
    met = O.metrics(gr, Y, xyz)
    nodes = I.state_nodes(xyz, g, Y)
    q = vx.state(nodes, 0.0, period=20.0)
    sc = O.Scheme(recon, Y, True)
    T = 40.0
    nsteps = int(math.ceil(T / O.max_dt(gr, sc, met, q, 0.5)))
    out = O.solve(gr, sc, met, q, T / nsteps, nsteps)
    qe = I.interior(vx.state(nodes, T, period=20.0), g)
    return v_errors(out, g, qe[2] / qe[0])


CASES = [("Linear-Upwind5-M6", "linup5", 6), ("WENO5-M2", "weno5", 2),
         ("WENO5-M4", "weno5", 4), ("WENO5-M6", "weno5", 6)]


@pytest.mark.parametrize("name,recon,Y", CASES)
def test_table2_coarse_grids(name, recon, Y):
    for npts in (21, 41):
        l2, li = run_vortex(recon, Y, npts - 1)
        p2, pi = GOLD["table2"][name][str(npts)]
        assert 0.5 < l2 / p2 < 2.0, (npts, l2, p2)
        assert 0.5 < li / pi < 2.0, (npts, li, pi)


@pytest.mark.slow
@pytest.mark.parametrize("name,recon,Y", [CASES[0]])
def test_table2_rate_41_to_81(name, recon, Y):
    e41 = run_vortex(recon, Y, 40)
    e81 = run_vortex(recon, Y, 80)
    p41, p81 = GOLD["table2"][name]["41"], GOLD["table2"][name]["81"]
    assert 0.5 < e81[0] / p81[0] < 2.0
    rate = math.log2(e41[0] / e81[0])
    paper_rate = math.log2(p41[0] / p81[0])
    assert abs(rate - paper_rate) < 0.8
