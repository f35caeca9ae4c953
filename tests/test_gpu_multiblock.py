"""Multi-block interfaces (fp_batch_set_links) on the GPU: a periodic grid
cut into sub-blocks joined by links must advance exactly as the single
block does, bitwise: every face flux on a shared face sees the same stencil
values (the neighbour's stage register through the exchange) and the same
metrics (the neighbour's interior metrics, copied once), so the sub-blocks
reproduce the single-block arithmetic node for node.  That also makes the
scheme conservative across the interfaces."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2101_05886_amd import fp
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu

FROZEN, PERIODIC = fp.FP_BC_FROZEN, fp.FP_BC_PERIODIC


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need the MI355X"
    fp.lib()
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def decompose(case, cuts, Y, recon, prec, steps):
    """single block vs its decomposition into cuts[d] pieces along the
    first two axes (the other axes stay whole and periodic)"""
    ndim, n, g = case["ndim"], list(case["n"][:case["ndim"]]), case["g"]
    sc = fp.Scheme(recon, Y, True, precision=prec)
    gc = g + Y // 2
    # the single block
    G1 = fp.Grid(ndim, n, g)
    met1 = fp.metrics(G1, Y, dev(case["xyz"]))
    q1 = dev(case["q"])
    w1 = torch.zeros(G1.work_shape(), dtype=torch.float64, device="cuda")
    dt = float(fp.max_dt(G1, sc, met1, q1, 0.5).item())
    fp.solve(G1, sc, met1, q1, w1, dt, steps)
    # the pieces
    sizes = [n[d] // cuts[d] if d < 2 else n[d] for d in range(ndim)]
    pieces, index = [], {}
    grid_cuts = [cuts[d] if d < 2 else 1 for d in range(ndim)]
    for c in np.ndindex(*grid_cuts):
        lo = [c[d] * sizes[d] for d in range(ndim)]
        sl_x = (slice(None),) + tuple(slice(lo[d], lo[d] + sizes[d] + 2 * gc) for d in reversed(range(ndim)))
        sl_q = (slice(None),) + tuple(slice(lo[d], lo[d] + sizes[d] + 2 * g) for d in reversed(range(ndim)))
        bc = [FROZEN if d < 2 else PERIODIC for d in range(ndim)]
        Gp = fp.Grid(ndim, sizes, g, bc=bc)
        met = fp.metrics(Gp, Y, dev(case["xyz"][sl_x]))
        q = dev(case["q"][sl_q])
        work = torch.zeros(Gp.work_shape(), dtype=torch.float64, device="cuda")
        index[c] = len(pieces)
        pieces.append((Gp, met, q, work, dt, lo))
    links = []
    for c, i in index.items():
        for d in range(2):
            for side in (0, 1):
                nb = list(c)
                nb[d] = (c[d] + (1 if side else -1)) % grid_cuts[d]
                links.append((i, d, side, index[tuple(nb)]))
    b = fp.Batch(sc, len(pieces))
    b.set([p[:5] for p in pieces])
    b.set_links(links)
    # one instrumented step first: the exchange runs before every stage
    kinds = [k for _, k, _ in b.profile_step()]
    assert kinds.count(4) == 3
    b.solve(steps - 1)
    torch.cuda.synchronize()
    full = q1.cpu().numpy()
    for Gp, met, q, work, dt, lo in pieces:
        got = q.cpu().numpy()[(slice(None),) + (slice(g, -g),) * ndim]
        ref = full[(slice(None),) + tuple(slice(g + lo[d], g + lo[d] + sizes[d]) for d in reversed(range(ndim)))]
        assert np.array_equal(got, ref), f"piece at {lo}: max diff {np.abs(got - ref).max():.3e}"
    b.close()
    return pieces


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_3d_periodic_grid_cut_2x2_is_bitwise_the_single_block(prec):
    case = G.periodic_case(3, (48, 40, 24), 6, state="noisy", seed=41)
    decompose(case, (2, 2), 6, "weno5", prec, 3)


def test_2d_grid_cut_3x2_lu5():
    case = G.periodic_case(2, (66, 40), 4, state="vortex", seed=42)
    decompose(case, (3, 2), 4, "linup5", "fp64", 4)


def test_weno7_m8_cut_2x1():
    case = G.periodic_case(3, (40, 28, 20), 8, g=4, state="noisy", seed=43)
    decompose(case, (2, 1), 8, "weno7", "mixed", 2)


@pytest.mark.parametrize("ndim,n,cuts,Y,recon", [(3, (48, 40, 24), (2, 2), 6, "weno5"),
                                                 (2, (66, 40), (3, 2), 4, "linup5")])
def test_linked_blocks_match_oracle_on_undivided_grid(ndim, n, cuts, Y, recon):
    """The linked pieces against the FP64 oracle advancing the undivided
    periodic grid.  Each piece takes its slice of the oracle's metrics of the
    whole grid (its ghost layers are then the neighbours' interior metrics,
    which the link setup copies in), so both sides start from identical
    inputs: FP64 within 1e-12 per variable after one RK3 step and 3e-12
    after three; FP32-mixed within 1e-4 of the increment after one step."""
    case = G.periodic_case(ndim, n, Y, state="noisy", seed=44)
    g = case["g"]
    og = O.Grid(ndim, n, g)
    met = O.metrics(og, Y, case["xyz"])
    osc = O.Scheme(recon, Y, True)
    dt = 0.5 * O.max_dt(og, osc, met, case["q"], 1.0)
    ref1 = O.rk3_step(og, osc, met, case["q"], dt)
    ref3 = O.solve(og, osc, met, case["q"], dt, 3)
    sizes = [n[d] // cuts[d] if d < 2 else n[d] for d in range(ndim)]
    grid_cuts = [cuts[d] if d < 2 else 1 for d in range(ndim)]
    for prec, steps, ref in (("fp64", 1, ref1), ("fp64", 3, ref3), ("mixed", 1, ref1)):
        sc = fp.Scheme(recon, Y, True, precision=prec)
        pieces, index = [], {}
        for c in np.ndindex(*grid_cuts):
            lo = [c[d] * sizes[d] for d in range(ndim)]
            sl = (slice(None),) + tuple(slice(lo[d], lo[d] + sizes[d] + 2 * g) for d in reversed(range(ndim)))
            bc = [FROZEN if d < 2 else PERIODIC for d in range(ndim)]
            Gp = fp.Grid(ndim, sizes, g, bc=bc)
            index[c] = len(pieces)
            pieces.append((Gp, dev(met[sl]), dev(case["q"][sl]),
                           torch.zeros(Gp.work_shape(), dtype=torch.float64, device="cuda"), dt, lo))
        links = []
        for c, i in index.items():
            for d in range(2):
                for side in (0, 1):
                    nb = list(c)
                    nb[d] = (c[d] + (1 if side else -1)) % grid_cuts[d]
                    links.append((i, d, side, index[tuple(nb)]))
        b = fp.Batch(sc, len(pieces))
        b.set([p[:5] for p in pieces])
        b.set_links(links)
        b.solve(steps)
        torch.cuda.synchronize()
        for Gp, mp, qp, work, _, lo in pieces:
            sl = (slice(None),) + tuple(slice(g + lo[d], g + lo[d] + sizes[d]) for d in reversed(range(ndim)))
            got = qp.cpu().numpy()[(slice(None),) + (slice(g, -g),) * ndim].reshape(len(ref), -1)
            want = ref[sl].reshape(len(ref), -1)
            base = want if prec == "fp64" else want - case["q"][sl].reshape(len(ref), -1)
            bar = 1e-12 * steps if prec == "fp64" else 1e-4
            for v in range(len(ref)):
                err = np.abs(got[v] - want[v]).max() / np.abs(base[v]).max()
                assert err <= bar, f"{prec} {steps} steps, piece at {lo}, variable {v}: {err:.3e}"
        b.close()


def test_links_are_validated():
    sc = fp.Scheme("weno5", 6, True)
    a = fp.Grid(3, (16, 12, 10), 3, bc=[FROZEN, FROZEN, PERIODIC])
    c = fp.Grid(3, (16, 13, 10), 3, bc=[FROZEN, FROZEN, PERIODIC])
    ents = []
    for grid in (a, a, c):
        met = torch.zeros(grid.metric_shape(), dtype=torch.float64, device="cuda")
        q = torch.ones(grid.state_shape(), dtype=torch.float64, device="cuda")
        ents.append((grid, met, q, torch.zeros(grid.work_shape(), dtype=torch.float64, device="cuda"), 0.1))
    b = fp.Batch(sc, 4)
    b.set(ents)
    for bad in ([(0, 0, 1, 5)], [(0, 3, 1, 1)], [(0, 0, 2, 1)], [(0, 2, 1, 1)],  # range, axis, side, periodic axis
                [(0, 0, 1, 2)],  # extents differ along y
                [(0, 0, 1, 1), (0, 0, 1, 1)]):  # a face linked twice
        with pytest.raises(fp.FPError):
            b.set_links(bad)
    b.set_links([(0, 0, 1, 1), (1, 0, 0, 0)])
    b.set_links([])
    b.close()
