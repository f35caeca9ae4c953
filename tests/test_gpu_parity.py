"""GPU parity: the gfx950 library (through its C ABI) against the FP64 oracle
on the same seeded inputs.

Bar (FP64 path): per variable, max |gpu - oracle| / max |oracle| <= 1e-12 for
face fluxes, residuals and one RK3 step; metrics <= 1e-13.  The mixed path is
checked against the oracle by the free-stream residual (round-off) and by a
bound on the relative difference of the residual.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2101_05886_amd import fp
from paper_2101_05886_amd import inputs as I
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need the MI355X"
    fp.lib()  # the HIP library must be built and loadable
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def grids(case):
    og = O.Grid(case["ndim"], case["n"], case["g"], bc=case["bc"])
    fg = fp.Grid(case["ndim"], case["n"], case["g"], bc=case["bc"])
    return og, fg


def relerr(a, b):
    """per-variable max |a-b| / max |b|, maximised over variables"""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return max(np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(a.shape[0]))


def interior(a, g, ndim):
    return a[(slice(None),) + (slice(g, -g),) * ndim]


METRIC_CASES = [(2, (70, 45), 2), (2, (70, 45), 4), (2, (33, 64), 6), (2, (40, 40), 8),
                (3, (21, 18, 16), 2), (3, (17, 20, 13), 6), (3, (16, 16, 16), 8)]


@pytest.mark.parametrize("ndim,n,Y", METRIC_CASES)
def test_metrics_periodic(ndim, n, Y):
    case = G.periodic_case(ndim, n, Y)
    og, fg = grids(case)
    ref = O.metrics(og, Y, case["xyz"])
    got = host(fp.metrics(fg, Y, dev(case["xyz"])))
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("Y", [2, 6, 8])
def test_metrics_frozen_ogrid(Y):
    case = G.frozen_case((37, 26, 11), Y)
    og, fg = grids(case)
    ref = O.metrics(og, Y, case["xyz"])
    got = host(fp.metrics(fg, Y, dev(case["xyz"])))
    # per direction, relative to that direction's metric vector (some
    # components of an extruded block vanish analytically)
    for d in range(3):
        scale = np.abs(ref[3 * d:3 * d + 3]).max()
        for c in range(3 * d, 3 * d + 3):
            assert np.abs(got[c] - ref[c]).max() <= 1e-12 * scale, c
    assert np.abs(got[9] - ref[9]).max() <= 1e-12 * np.abs(ref[9]).max()


FLUX_CASES = [
    # ndim, n, Y, recon, reform, state
    (2, (70, 45), 2, "weno5", 1, "vortex"),
    (2, (70, 45), 6, "linup5", 1, "vortex"),
    (2, (33, 64), 4, "weno5", 0, "noisy"),
    (2, (40, 40), 8, "weno5", 1, "noisy"),
    (3, (21, 18, 16), 2, "weno5", 1, "vortex"),
    (3, (17, 20, 13), 6, "linup5", 1, "noisy"),
    (3, (16, 16, 16), 8, "weno5", 1, "vortex"),
    (3, (19, 16, 15), 4, "weno5", 0, "noisy"),
    (3, (18, 17, 15), 4, "linup5", 1, "noisy"),
]


def _ids(c):
    return f"{c[0]}d-{'x'.join(map(str, c[1]))}-M{c[2]}-{c[3]}-{'fp' if c[4] else 'std'}-{c[5]}"


@pytest.mark.parametrize("ndim,n,Y,recon,reform,state", FLUX_CASES, ids=[_ids(c) for c in FLUX_CASES])
def test_face_fluxes_and_residual(ndim, n, Y, recon, reform, state):
    case = G.periodic_case(ndim, n, Y, state=state)
    og, fg = grids(case)
    met = O.metrics(og, Y, case["xyz"])
    osc = O.Scheme(recon, Y, bool(reform))
    fsc = fp.Scheme(recon, Y, bool(reform))
    mg, qg = dev(met), dev(case["q"])
    for d in range(ndim):
        ref = O.face_fluxes(og, osc, met, case["q"], d)
        got = host(fp.face_fluxes(fg, fsc, mg, qg, d))
        assert relerr(got, ref) <= 1e-12, f"direction {d}"
    ref = O.residual(og, osc, met, case["q"])
    got = host(fp.residual(fg, fsc, mg, qg))
    g = case["g"]
    assert relerr(interior(got, g, ndim), interior(ref, g, ndim)) <= 1e-11


# Uniform Cartesian grids (anisotropic spacing): every face normal is a
# coordinate axis, so in 3D its two other components tie exactly at zero
# and the tangent basis takes the lowest of them; with the background at
# rest the normal velocity changes sign across many faces.  Remark 1: on
# such grids the reformulated scheme equals the standard one.
CART_CASES = [(2, (40, 36), (0.5, 0.8)), (3, (20, 18, 16), (0.3, 0.45, 0.35))]


def relerr_vec(a, b, ndim):
    """relerr with the momentum components measured against the momentum
    vector's scale and every variable against at least 1e-6 of the largest
    one: a component that vanishes analytically (the z-momentum of a vortex
    column at rest, its mass and energy fluxes across the z faces) is
    rounding noise on both sides"""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    top = np.abs(b).max()
    mom = np.abs(b[1:1 + ndim]).max()
    return max(np.abs(a[v] - b[v]).max() / max(mom if 1 <= v <= ndim else np.abs(b[v]).max(), 1e-6 * top)
               for v in range(a.shape[0]))


@pytest.mark.parametrize("vel", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.1)], ids=["at-rest", "moving"])
@pytest.mark.parametrize("recon", ["weno5", "linup5", "wenocu6"])
@pytest.mark.parametrize("ndim,n,h", CART_CASES, ids=["2d", "3d"])
def test_cartesian_grid_matches_oracle_and_recovers_standard_scheme(ndim, n, h, recon, vel):
    g, Y = 3, 6
    xyz = I.cartesian_grid(ndim, n, g, Y, spacing=h)
    per = [n[d] * h[d] for d in range(ndim)]
    q = np.ascontiguousarray(I.Vortex(vel_inf=vel).state(I.state_nodes(xyz, g, Y), period=per[:2]))
    og, fg = O.Grid(ndim, n, g), fp.Grid(ndim, n, g)
    met = O.metrics(og, Y, xyz)
    osc, fsc = O.Scheme(recon, Y, True), fp.Scheme(recon, Y, True)
    mg, qg = dev(met), dev(q)
    for d in range(ndim):
        ref = O.face_fluxes(og, osc, met, q, d)
        got = host(fp.face_fluxes(fg, fsc, mg, qg, d))
        assert relerr_vec(got, ref, ndim) <= 1e-12, f"direction {d}"
    dt = 0.5 * O.max_dt(og, osc, met, q, 1.0)
    ref = O.rk3_step(og, osc, met, q, dt)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.rk3_step(fg, fsc, mg, qg, work, dt)
    assert relerr_vec(interior(host(qg), g, ndim), interior(ref, g, ndim), ndim) <= 1e-12
    qg = dev(q)
    r1 = interior(host(fp.residual(fg, fsc, mg, qg)), g, ndim)
    r0 = interior(host(fp.residual(fg, fp.Scheme(recon, Y, False), mg, qg)), g, ndim)
    # the residual bar: a difference of fluxes about 100 times larger
    assert np.abs(r1 - r0).max() <= 1e-11 * np.abs(r0).max()
    # the FP32-mixed form: exactly tied normal components tie in FP32 too
    rm = interior(host(fp.residual(fg, fp.Scheme(recon, Y, True, precision="mixed"), mg, qg)), g, ndim)
    ro = interior(O.residual(og, osc, met, q), g, ndim)
    assert relerr_vec(rm, ro, ndim) <= 1e-4


# Short xi lines: the xi sweep packs the faces of consecutive lines into
# items of at most 64, as many as the staged window holds (88 entries for the
# FP32-mixed six-point stencils and FP64 LU5, 128 for the others), so lines of a few nodes
# give items of many short lines and lines under 30 nodes items of fewer than
# 64 faces.  Every xi difference of the sweep is the difference of the
# face-flux kernel's fluxes (the same face code, one lane per face), and the
# residual meets the oracle bar of its precision.
SHORT_X = [(3, 4, 5), (5, 3, 7), (13, 6, 4), (29, 5, 3), (30, 4, 4), (67, 3, 3),
           (3, 5), (13, 4), (29, 6), (67, 3)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("recon", ["weno5", "linup5", "wenocu6"])
@pytest.mark.parametrize("n", SHORT_X, ids=["x".join(map(str, n)) for n in SHORT_X])
def test_xi_sweep_short_lines(n, recon, prec):
    nd = len(n)
    case = G.periodic_case(nd, n, 6)
    og, fg = grids(case)
    met = O.metrics(og, 6, case["xyz"])
    fsc = fp.Scheme(recon, 6, True, precision=prec)
    mg, qg = dev(met), dev(case["q"])
    F = host(fp.face_fluxes(fg, fsc, mg, qg, 0))
    acc = torch.zeros_like(qg)
    got = interior(host(fp.residual_dir(fg, fsc, mg, qg, 0, acc)), 3, nd)
    assert relerr(got, -(F[..., 1:] - F[..., :-1])) <= 1e-9
    ref = O.residual(og, O.Scheme(recon, 6, True), met, case["q"])
    res = host(fp.residual(fg, fsc, mg, qg))
    assert relerr(interior(res, 3, nd), interior(ref, 3, nd)) <= (1e-11 if prec == "fp64" else 1e-4)


# Linear upwind with fourth-order metrics: its xi sweep takes the same
# three-wave, 88-entry path as with sixth-order metrics in both precisions.
SHORT_X_M4 = [(3, 4, 5), (29, 5, 3), (30, 4, 4), (67, 3, 3), (13, 4), (67, 3)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n", SHORT_X_M4, ids=["x".join(map(str, n)) for n in SHORT_X_M4])
def test_xi_sweep_short_lines_lu5_m4(n, prec):
    nd = len(n)
    case = G.periodic_case(nd, n, 4, state="noisy")
    og, fg = grids(case)
    met = O.metrics(og, 4, case["xyz"])
    fsc = fp.Scheme("linup5", 4, True, precision=prec)
    mg, qg = dev(met), dev(case["q"])
    F = host(fp.face_fluxes(fg, fsc, mg, qg, 0))
    got = interior(host(fp.residual_dir(fg, fsc, mg, qg, 0, torch.zeros_like(qg))), 3, nd)
    assert relerr(got, -(F[..., 1:] - F[..., :-1])) <= 1e-9
    ref = O.residual(og, O.Scheme("linup5", 4, True), met, case["q"])
    res = host(fp.residual(fg, fsc, mg, qg))
    assert relerr(interior(res, 3, nd), interior(ref, 3, nd)) <= (1e-11 if prec == "fp64" else 1e-4)
    if prec == "fp64":
        dt = 0.5 * O.max_dt(og, O.Scheme("linup5", 4, True), met, case["q"], 1.0)
        refq = O.rk3_step(og, O.Scheme("linup5", 4, True), met, case["q"], dt)
        work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
        fp.rk3_step(fg, fsc, mg, qg, work, dt)
        assert relerr(interior(host(qg), 3, nd), interior(refq, 3, nd)) <= 1e-12


# The same for the wide stencils (WENO7, eighth-order metrics; ghost 4),
# whose sweeps stage 128 entries in both precisions.
SHORT_X_WIDE = [(4, 5, 6), (13, 4, 4), (29, 5, 4), (61, 4, 4), (4, 5), (29, 6), (67, 4)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("recon,Y", [("weno7", 8), ("weno7", 6), ("weno5", 8)])
@pytest.mark.parametrize("n", SHORT_X_WIDE, ids=["x".join(map(str, n)) for n in SHORT_X_WIDE])
def test_xi_sweep_short_lines_wide(n, recon, Y, prec):
    nd = len(n)
    case = G.periodic_case(nd, n, Y, g=4)
    og, fg = grids(case)
    met = O.metrics(og, Y, case["xyz"])
    fsc = fp.Scheme(recon, Y, True, precision=prec)
    mg, qg = dev(met), dev(case["q"])
    F = host(fp.face_fluxes(fg, fsc, mg, qg, 0))
    acc = torch.zeros_like(qg)
    got = interior(host(fp.residual_dir(fg, fsc, mg, qg, 0, acc)), 4, nd)
    assert relerr(got, -(F[..., 1:] - F[..., :-1])) <= 1e-9
    ref = O.residual(og, O.Scheme(recon, Y, True), met, case["q"])
    res = host(fp.residual(fg, fsc, mg, qg))
    assert relerr(interior(res, 4, nd), interior(ref, 4, nd)) <= (1e-11 if prec == "fp64" else 1e-4)


# Accumulating direction residuals: with accumulate set, each direction adds
# its flux difference to what the array holds (the xi sweep then runs its
# accumulating kernel variant), so the result is the held values plus the
# direction's own residual, and the ghost layers keep theirs.
ACC_CASES = [(2, (5, 7)), (2, (40, 33)), (3, (3, 4, 5)), (3, (29, 5, 3)), (3, (24, 20, 18))]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("ndim,n", ACC_CASES, ids=[f"{c[0]}d-{'x'.join(map(str, c[1]))}" for c in ACC_CASES])
def test_residual_dir_accumulates(ndim, n, prec):
    case = G.periodic_case(ndim, n, 6)
    og, fg = grids(case)
    met = O.metrics(og, 6, case["xyz"])
    fsc = fp.Scheme("weno5", 6, True, precision=prec)
    mg, qg = dev(met), dev(case["q"])
    acc0 = np.random.Generator(np.random.PCG64(7)).standard_normal(case["q"].shape)
    ghost = np.ones(acc0.shape[1:], dtype=bool)
    ghost[(slice(3, -3),) * ndim] = False
    for d in range(ndim):
        own = host(fp.residual_dir(fg, fsc, mg, qg, d, torch.zeros_like(qg)))
        got = host(fp.residual_dir(fg, fsc, mg, qg, d, dev(acc0), accumulate=True))
        want = interior(acc0, 3, ndim) + interior(own, 3, ndim)
        assert np.abs(interior(got, 3, ndim) - want).max() <= 1e-14 * np.abs(want).max(), f"direction {d}"
        assert np.array_equal(got[:, ghost], acc0[:, ghost]), f"direction {d}"


RK_CASES = [(2, (70, 45), 2, "weno5"), (2, (64, 64), 6, "linup5"), (3, (21, 18, 16), 6, "weno5"),
            (3, (20, 20, 20), 2, "linup5"), (3, (20, 18, 16), 4, "linup5")]


@pytest.mark.parametrize("ndim,n,Y,recon", RK_CASES)
def test_rk3_step(ndim, n, Y, recon):
    case = G.periodic_case(ndim, n, Y)
    og, fg = grids(case)
    met = O.metrics(og, Y, case["xyz"])
    osc, fsc = O.Scheme(recon, Y, True), fp.Scheme(recon, Y, True)
    dt = 0.5 * O.max_dt(og, osc, met, case["q"], 1.0)
    ref = O.rk3_step(og, osc, met, case["q"], dt)
    qg = dev(case["q"])
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.rk3_step(fg, fsc, dev(met), qg, work, dt)
    got = host(qg)
    g = case["g"]
    assert relerr(interior(got, g, ndim), interior(ref, g, ndim)) <= 1e-12
    # only the interior is written
    assert np.array_equal(got[:, :g], case["q"][:, :g])


def test_solve_graph_matches_steps_and_oracle():
    case = G.periodic_case(2, (48, 40), 4)
    og, fg = grids(case)
    met = O.metrics(og, 4, case["xyz"])
    osc, fsc = O.Scheme("weno5", 4, True), fp.Scheme("weno5", 4, True)
    dt = 0.5 * O.max_dt(og, osc, met, case["q"], 1.0)
    mg = dev(met)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    q1 = dev(case["q"])
    for _ in range(6):
        fp.rk3_step(fg, fsc, mg, q1, work, dt)
    q2 = dev(case["q"])
    fp.solve(fg, fsc, mg, q2, work, dt, 4)   # captures the step graph
    fp.solve(fg, fsc, mg, q2, work, dt, 2)   # replays it
    a, b = host(q1), host(q2)
    assert np.array_equal(a, b)
    ref = O.solve(og, osc, met, case["q"], dt, 6)
    assert relerr(interior(a, 3, 2), interior(ref, 3, 2)) <= 1e-11


def test_frozen_block_residual_and_step():
    case = G.frozen_case((41, 29, 12), 6, perturb=0.05)
    og, fg = grids(case)
    met = O.metrics(og, 6, case["xyz"])
    osc, fsc = O.Scheme("weno5", 6, True), fp.Scheme("weno5", 6, True)
    mg, qg = dev(met), dev(case["q"])
    ref = O.residual(og, osc, met, case["q"])
    got = host(fp.residual(fg, fsc, mg, qg))
    assert relerr(interior(got, 3, 3), interior(ref, 3, 3)) <= 1e-11
    dt = 0.5 * O.max_dt(og, osc, met, case["q"], 1.0)
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.rk3_step(fg, fsc, mg, qg, work, dt)
    refq = O.rk3_step(og, osc, met, case["q"], dt)
    gotq = host(qg)
    assert relerr(interior(gotq, 3, 3), interior(refq, 3, 3)) <= 1e-12
    # frozen ghost layers are never written
    assert np.array_equal(gotq[:, :3], case["q"][:, :3])
    assert np.array_equal(gotq[:, :, :, -3:], case["q"][:, :, :, -3:])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("recon", ["weno5", "linup5"])
def test_free_stream_preserved_on_gpu(prec, recon):
    # C1 shape: 64^2 wavy grid, 5% jitter, second-order metrics, 100 RK3 steps
    case = G.periodic_case(2, 64, 2, state="uniform", L=20.0)
    og, fg = grids(case)
    met = O.metrics(og, 2, case["xyz"])
    osc = O.Scheme(recon, 2, True)
    dt = O.max_dt(og, osc, met, case["q"], 0.5)
    mg, qg = dev(met), dev(case["q"])
    work = torch.zeros(fg.work_shape(), dtype=torch.float64, device="cuda")
    fp.solve(fg, fp.Scheme(recon, 2, True, precision=prec), mg, qg, work, dt, 100)
    out = host(qg)
    dev_ = np.abs(interior(out, 3, 2) - interior(case["q"], 3, 2)).max() / np.abs(case["q"]).max()
    assert dev_ < 1e-13
    # the standard scheme departs from the free stream
    q0 = dev(case["q"])
    fp.solve(fg, fp.Scheme(recon, 2, False, precision=prec), mg, q0, work, dt, 100)
    out0 = host(q0)
    assert np.abs(interior(out0, 3, 2) - interior(case["q"], 3, 2)).max() > 1e-5


def test_free_stream_frozen_ogrid_mixed_and_fp64():
    case = G.frozen_case((64, 48, 24), 6)
    og, fg = grids(case)
    mg = fp.metrics(fg, 6, dev(case["xyz"]))
    qg = dev(case["q"])
    for prec in ("fp64", "mixed"):
        r = host(fp.residual(fg, fp.Scheme("weno5", 6, True, precision=prec), mg, qg))
        met = host(mg)
        scale = np.abs(case["q"]).max() * np.abs(met[:9]).max() / interior(met, 3, 3)[9].min()
        assert np.abs(interior(r, 3, 3)).max() < 1e-14 * scale, prec


def test_mixed_precision_residual_close_to_fp64_oracle():
    case = G.periodic_case(3, (24, 20, 18), 6)
    og, fg = grids(case)
    met = O.metrics(og, 6, case["xyz"])
    ref = O.residual(og, O.Scheme("weno5", 6, True), met, case["q"])
    got = host(fp.residual(fg, fp.Scheme("weno5", 6, True, precision="mixed"), dev(met),
                           dev(case["q"])))
    err = relerr(interior(got, 3, 3), interior(ref, 3, 3))
    assert err < 1e-4


def test_deterministic_bitwise():
    case = G.periodic_case(3, (20, 18, 16), 6, state="noisy")
    og, fg = grids(case)
    mg = fp.metrics(fg, 6, dev(case["xyz"]))
    qg = dev(case["q"])
    sc = fp.Scheme("weno5", 6, True)
    a = host(fp.residual(fg, sc, mg, qg))
    b = host(fp.residual(fg, sc, mg, qg))
    assert np.array_equal(a, b)


def test_tangent_tie_faces_match_oracle():
    """A grid symmetric under the swap of y and z (the unjittered wavy
    mapping with n_eta = n_zeta): on the xi-lines with j = k the xi-face
    normals have |n_y| = |n_z| analytically, the two smallest components, so
    the tangent basis is decided by the tie rule (lowest axis wins within
    1e-10), not by rounding.  A different choice rotates the shear fields and
    changes the WENO fluxes far above the bar, so FP64 parity on a
    non-uniform state shows that both sides take the same basis.  The mixed
    path decides on FP32 normals, where 1e-10 is below one ulp: analytic ties
    round to equal FP32 values and take the same axis."""
    case = G.periodic_case(3, (20, 16, 16), 6, state="noisy", jitter=0.0, seed=9)
    og, fg = grids(case)
    met = O.metrics(og, 6, case["xyz"])
    # xi-face metrics by the sixth-order face interpolation, on the j = k lines
    w = np.array([1, -8, 37, 37, -8, 1]) / 60.0
    g = case["g"]
    s = met[0:3]
    sf = sum(w[r] * s[..., r:r + s.shape[-1] - 5] for r in range(6))  # faces i-1/2 .. over the x extent
    j = np.arange(16)
    ny, nz = np.abs(sf[1, g + j, g + j]), np.abs(sf[2, g + j, g + j])
    nx = np.abs(sf[0, g + j, g + j])
    assert np.all(np.minimum(ny, nz) < nx)
    gap = np.abs(ny - nz) / np.sqrt(sf[0, g + j, g + j] ** 2 + ny ** 2 + nz ** 2)
    assert np.all(gap < 1e-13)
    mg, qg = dev(met), dev(case["q"])
    ref = O.face_fluxes(og, O.Scheme("weno5", 6, True), met, case["q"], 0)
    got = host(fp.face_fluxes(fg, fp.Scheme("weno5", 6, True), mg, qg, 0))
    assert relerr(got, ref) <= 1e-12
    diag = (slice(None), j, j)  # the flux arrays hold interior lines only
    assert relerr(got[diag], ref[diag]) <= 1e-12
    mixed = host(fp.face_fluxes(fg, fp.Scheme("weno5", 6, True, precision="mixed"), mg, qg, 0))
    assert relerr(mixed[diag], ref[diag]) <= 1e-5


def test_max_dt_and_check_state():
    case = G.periodic_case(3, (20, 18, 16), 4)
    og, fg = grids(case)
    met = O.metrics(og, 4, case["xyz"])
    ref = O.max_dt(og, O.Scheme("weno5", 4, True), met, case["q"], 0.5)
    got = float(host(fp.max_dt(fg, fp.Scheme("weno5", 4, True), dev(met), dev(case["q"]), 0.5))[0])
    assert got == pytest.approx(ref, rel=1e-13)
    sc = fp.Scheme("weno5", 4, True)
    assert int(host(fp.check_state(fg, sc, dev(case["q"])))[0]) == 0
    bad = case["q"].copy()
    bad[4, 3 + 5, 3 + 6, 3 + 7] = -1.0  # negative energy -> negative pressure
    assert int(host(fp.check_state(fg, sc, dev(bad)))[0]) == 1
    bad = case["q"].copy()
    bad[1, 3 + 2, 3 + 2, 3 + 2] = np.nan
    assert int(host(fp.check_state(fg, sc, dev(bad)))[0]) == 1


@pytest.mark.parametrize("ndim,n", [(2, (3, 3)), (2, (200, 3)), (3, (3, 4, 5)), (3, (65, 3, 7))])
def test_small_and_ragged_grids(ndim, n):
    case = G.periodic_case(ndim, n, 2, state="noisy")
    og, fg = grids(case)
    met = O.metrics(og, 2, case["xyz"])
    assert np.abs(host(fp.metrics(fg, 2, dev(case["xyz"]))) - met).max() <= 1e-13 * np.abs(met).max()
    ref = O.residual(og, O.Scheme("weno5", 2, True), met, case["q"])
    got = host(fp.residual(fg, fp.Scheme("weno5", 2, True), dev(met), dev(case["q"])))
    assert relerr(interior(got, 3, ndim), interior(ref, 3, ndim)) <= 1e-11


def test_invalid_arguments_enqueue_nothing():
    fg = fp.Grid(3, (8, 8, 8), 3)
    q = torch.zeros(fg.state_shape(), dtype=torch.float64, device="cuda")
    met = torch.zeros(fg.metric_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(fp.FPError) as e:
        fp.residual(fg, fp.Scheme("weno5", 3, True), met, q)
    assert e.value.status == fp.FP_EUNSUPPORTED
    with pytest.raises(fp.FPError) as e:
        fp.residual(fp.Grid(3, (8, 8, 8), 3), fp.Scheme("weno5", 8, True), met, q)
    assert e.value.status == fp.FP_EINVAL
    with pytest.raises(fp.FPError):
        fp.residual(fg, fp.Scheme("weno5", 6, True), met, q[:, :2].contiguous())
