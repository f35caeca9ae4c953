"""bench.py's host logic (CPU only): the algorithmic flop count, the
roofline record and its counter tables, the repeat statistics, and the
single-GPU contract."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_flops_per_face(bench):
    # the figures the design notes and the roofline records quote
    assert bench.alg_flops_per_face("weno5", 3, 6) == 1897
    assert bench.alg_flops_per_face("linup5", 3, 6) == 906
    assert bench.alg_flops_per_face("weno7", 3, 8) == 3169
    assert bench.alg_flops_per_face("wenocu6", 3, 6) == 2847
    assert bench.alg_flops_per_face("weno5", 2, 6) == 1407
    # only the face reference state depends on the metric order: 2 (1 + D)
    # + 3 nv flops per interpolation point
    for D in (2, 3):
        nv = D + 2
        assert (bench.alg_flops_per_face("weno5", D, 8) - bench.alg_flops_per_face("weno5", D, 6)
                == 2 * (2 * (1 + D) + 3 * nv))


def test_faces_along(bench):
    assert bench.faces_along([4, 5, 6], 0) == 5 * 5 * 6
    assert bench.faces_along([4, 5, 6], 2) == 4 * 5 * 7
    assert bench.faces_along([9, 7], 1) == 9 * 8


def test_alu_peak(bench):
    assert bench.PEAK_ALU_TFLOPS == pytest.approx(78.6432)
    assert bench.VALU_ISSUE_PER_S == pytest.approx(1024 * 2.4e9 / 4)


def test_roofline_record(bench):
    n = 256
    faces = bench.faces_along([n] * 3, 2)
    r = bench.roofline("weno5", 3, 6, "mixed", "k_sweep_wg<zeta>", 1.0, faces, n ** 3, "c3m/k_sweep_wg<zeta>")
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in r
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(1897 * faces / 1e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    # the counter tables count only while they were taken on these sources
    _, current = bench.counter_table(bench.TRAFFIC_FILE)
    assert (r["traffic"] is not None) == current
    if current:
        clk = r["clock"]
        assert clk["live_ghz"] == pytest.approx(clk["active_cycles"] / 1e-3 / 1e9)
    # an unknown launch has no counters
    assert bench.roofline("weno5", 3, 6, "mixed", "x", 1.0, faces, n ** 3, "nope/x")["traffic"] is None


def test_median_rate(bench):
    m = bench.median_rate([2.0, 1.0, 4.0], 1000.0)
    assert m == {"n": 3, "median": 1000.0 / 2e-3, "min": 1000.0 / 4e-3, "max": 1000.0 / 1e-3}


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
