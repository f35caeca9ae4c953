"""Batched multi-block RK3 (fp_batch_*) on the GPU.

Every block of a batch must come out bitwise equal to the same block
advanced alone by fp_rk3_step (same kernels' arithmetic, only the work
distribution differs), whatever the mix of 2D/3D, periodic/frozen blocks,
after a change of the block set, through the captured step graph, and after
the autotuner changes the tile shape.  The single-block path is held to the
FP64 oracle by the parity tests; one block here is also checked against the
oracle directly.  At the full 48-block O-grid workload the batch must also
keep the uniform Mach-3 free stream to round-off in FP64 and FP32-mixed.
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
    fp.lib()
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mixed_cases():
    """uneven blocks: 3D periodic and frozen, 2D periodic"""
    return [G.periodic_case(3, (20, 17, 13), 6, state="noisy", seed=11),
            G.frozen_case((40, 24, 16), 6, perturb=0.05, seed=12),
            G.periodic_case(2, (50, 37), 6, state="noisy", seed=13),
            G.frozen_case((33, 20, 18), 6, perturb=0.03, seed=14),
            G.periodic_case(3, (70, 9, 11), 6, state="vortex", seed=15),
            G.periodic_case(2, (19, 64), 6, state="vortex", seed=16)]


class Block:
    def __init__(self, case, scheme, cfl=0.5):
        self.case = case
        self.grid = fp.Grid(case["ndim"], case["n"], case["g"], bc=case["bc"])
        self.met = fp.metrics(self.grid, case["Y"], dev(case["xyz"]))
        self.q0 = dev(case["q"])
        self.q = self.q0.clone()
        self.work = torch.zeros(self.grid.work_shape(), dtype=torch.float64, device="cuda")
        self.dt = float(fp.max_dt(self.grid, scheme, self.met, self.q0, cfl).item())

    def entry(self):
        return (self.grid, self.met, self.q, self.work, self.dt)

    def alone(self, scheme, steps):
        q = self.q0.clone()
        w = torch.zeros_like(self.work)
        for _ in range(steps):
            fp.rk3_step(self.grid, scheme, self.met, q, w, self.dt)
        return q


SCHEMES = [("weno5", "fp64"), ("linup5", "fp64"), ("weno5", "mixed")]


@pytest.mark.parametrize("recon,prec", SCHEMES)
def test_batch_step_bitwise_equals_blocks_alone(recon, prec):
    sc = fp.Scheme(recon, 6, True, precision=prec)
    blocks = [Block(c, sc) for c in mixed_cases()]
    b = fp.Batch(sc, 16)
    b.set([k.entry() for k in blocks])
    b.rk3_step()
    torch.cuda.synchronize()
    for i, k in enumerate(blocks):
        ref = k.alone(sc, 1)
        assert torch.equal(k.q, ref), f"block {i}: batched step differs from the block alone"
    b.close()


def test_batch_block_matches_oracle():
    sc = fp.Scheme("weno5", 6, True)
    cases = mixed_cases()
    blocks = [Block(c, sc) for c in cases]
    b = fp.Batch(sc, 8)
    b.set([k.entry() for k in blocks])
    b.rk3_step()
    torch.cuda.synchronize()
    for i in (1, 2):  # a frozen 3D block and a periodic 2D block
        c, k = cases[i], blocks[i]
        og = O.Grid(c["ndim"], c["n"], c["g"], bc=c["bc"])
        met = k.met.cpu().numpy()
        ref = O.rk3_step(og, O.Scheme("weno5", 6, True), met, c["q"], k.dt)
        got = k.q.cpu().numpy()
        sl = (slice(None),) + (slice(c["g"], -c["g"]),) * c["ndim"]
        for v in range(got.shape[0]):
            err = np.abs(got[sl][v] - ref[sl][v]).max() / np.abs(ref[sl][v]).max()
            assert err <= 1e-12, f"block {i} variable {v}: {err:.3e}"
    b.close()


def test_batch_graph_survives_set_changes():
    sc = fp.Scheme("weno5", 6, True)
    blocks = [Block(c, sc) for c in mixed_cases()]
    b = fp.Batch(sc, 8)
    # all blocks, graph replay of 3 steps
    b.set([k.entry() for k in blocks])
    b.solve(3)
    torch.cuda.synchronize()
    for i, k in enumerate(blocks):
        assert torch.equal(k.q, k.alone(sc, 3)), f"block {i} after 3 graph steps"
    # a different subset (3D only, then 2D only, then all again): the work
    # list changes under the captured graphs
    subsets = [[0, 1, 4], [2, 5], [5, 3, 0, 2]]
    for sub in subsets:
        for i in sub:
            blocks[i].q.copy_(blocks[i].q0)
            blocks[i].dt *= 0.9
        b.set([blocks[i].entry() for i in sub])
        b.solve(2)
        torch.cuda.synchronize()
        for i in sub:
            assert torch.equal(blocks[i].q, blocks[i].alone(sc, 2)), f"subset {sub}: block {i}"
    b.set([])
    b.solve(1)  # an empty batch is a no-op
    b.close()


def test_batch_autotune_keeps_results():
    sc = fp.Scheme("linup5", 6, True)
    blocks = [Block(c, sc) for c in mixed_cases()]
    b = fp.Batch(sc, 8)
    b.set([k.entry() for k in blocks])
    seg = b.autotune()
    targets = (15, 23, 31, 47, 63, 95, 127)
    tiles = b.tiles()
    assert seg == tiles["seg_eta"] and seg in targets and tiles["seg_zeta"] in targets
    for k in blocks:
        assert torch.equal(k.q, k.q0), "the autotuner must not touch q"
    b.solve(2)
    torch.cuda.synchronize()
    for i, k in enumerate(blocks):
        assert torch.equal(k.q, k.alone(sc, 2)), f"block {i} after autotune"
    # a second batch of the same size class reuses the cached choice
    for k in blocks:
        k.q.copy_(k.q0)
    b2 = fp.Batch(sc, 8)
    b2.set([k.entry() for k in blocks])
    b2.autotune()
    t2 = b2.tiles()
    assert t2["from_cache"] and (t2["seg_eta"], t2["seg_zeta"]) == (tiles["seg_eta"], tiles["seg_zeta"])
    b2.solve(1)
    torch.cuda.synchronize()
    for i, k in enumerate(blocks):
        assert torch.equal(k.q, k.alone(sc, 1)), f"block {i} after the cached autotune"
    b.close()
    b2.close()


def test_batch_rejects_bad_blocks():
    sc = fp.Scheme("weno5", 6, True)
    k = Block(G.periodic_case(3, (12, 12, 12), 6), sc)
    b = fp.Batch(sc, 2)
    with pytest.raises(fp.FPError):
        b.set([k.entry()] * 3)  # more than max_blocks
    bad = list(k.entry())
    bad[4] = -1.0
    with pytest.raises(fp.FPError):
        b.set([tuple(bad)])
    g2 = fp.Grid(3, (12, 12, 12), 2)  # ghost too small for 6th-order metrics
    with pytest.raises(fp.FPError):
        b.set([(g2, k.met, k.q, k.work, k.dt)])
    b.close()


def c4_blocks(scheme, perturb=False):
    out = []
    for i, spec in enumerate(I.multiblock_specs(48, seed=4)):
        g, Y = 3, 6
        xyz = I.ogrid_sector_block(spec.n, g, Y, spec.sector, spec.skew_deg, spec.rotation)
        q = I.uniform_state(3, spec.n, g, G.GAMMA, I.mach_velocity(3.0, [1.0, 0.0, 0.0]), 1.0)
        out.append(Block(dict(ndim=3, n=list(spec.n), g=g, Y=Y, bc=[1, 1, 1], xyz=xyz, q=q), scheme))
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c4_free_stream_and_bitwise(prec):
    sc = fp.Scheme("weno5", 6, True, precision=prec)
    blocks = c4_blocks(sc)
    nodes = sum(int(np.prod(k.grid.n)) for k in blocks)
    print(f"C4: 48 O-grid blocks, {nodes} nodes, {prec}", flush=True)
    b = fp.Batch(sc, 48)
    b.set([k.entry() for k in blocks])
    b.solve(5)
    torch.cuda.synchronize()
    worst = 0.0
    for k in blocks:
        g = k.grid.ghost
        d = (k.q - k.q0)[:, g:-g, g:-g, g:-g].abs().amax(dim=(1, 2, 3))
        # per variable, relative to its free-stream size; the momentum
        # components (zero for the ones normal to the flow) to rho |u|
        scale = k.q0[:, g:-g, g:-g, g:-g].abs().amax(dim=(1, 2, 3))
        scale[1:4] = scale[1:4].max()
        worst = max(worst, float((d / scale).max()))
    print(f"C4 free-stream deviation after 5 steps: {worst:.3e}", flush=True)
    assert worst < 1e-13
    for i in (0, 17, 47):
        assert torch.equal(blocks[i].q, blocks[i].alone(sc, 5)), f"block {i}"
    b.close()


def test_batch_profile_step_is_a_step():
    sc = fp.Scheme("weno5", 6, True, precision="mixed")
    blocks = [Block(c, sc) for c in mixed_cases()]
    b = fp.Batch(sc, 8)
    b.set([k.entry() for k in blocks])
    prof = b.profile_step()
    # 2D part: ghost copy + 3 stages x 2 sweeps; 3D part: ghost copy + 3 x 3
    assert [(d, k) for d, k, _ in prof] == ([(2, 3)] + [(2, k) for _ in range(3) for k in (0, 1)]
                                            + [(3, 3)] + [(3, k) for _ in range(3) for k in (0, 1, 2)])
    assert all(t > 0.0 for _, _, t in prof)
    for i, k in enumerate(blocks):
        assert torch.equal(k.q, k.alone(sc, 1)), f"block {i}"
    b.close()


def test_c4_full_size_blocks_match_oracle():
    """The 48-block workload at full size with a perturbed (non-uniform)
    state: after one batched step, two blocks (the largest and a small one)
    against the FP64 oracle stepping the same block from the GPU's metrics."""
    sc = fp.Scheme("weno5", 6, True)
    specs = I.multiblock_specs(48, seed=4)
    blocks = []
    for i, spec in enumerate(specs):
        g, Y = 3, 6
        xyz = I.ogrid_sector_block(spec.n, g, Y, spec.sector, spec.skew_deg, spec.rotation)
        q = I.uniform_state(3, spec.n, g, G.GAMMA, I.mach_velocity(3.0, [1.0, 0.0, 0.0]), 1.0)
        rng = np.random.Generator(np.random.PCG64(100 + i))
        q = np.ascontiguousarray(q * (1.0 + 0.01 * rng.standard_normal(q.shape)))
        blocks.append(Block(dict(ndim=3, n=list(spec.n), g=g, Y=Y, bc=[1, 1, 1], xyz=xyz, q=q), sc))
    b = fp.Batch(sc, 48)
    b.set([k.entry() for k in blocks])
    b.rk3_step()
    torch.cuda.synchronize()
    sizes = [int(np.prod(k.grid.n)) for k in blocks]
    for i in (int(np.argmax(sizes)), int(np.argmin(sizes))):
        k = blocks[i]
        c = k.case
        og = O.Grid(3, c["n"], c["g"], bc=[1, 1, 1])
        ref = O.rk3_step(og, O.Scheme("weno5", 6, True), k.met.cpu().numpy(), c["q"], k.dt)
        got = k.q.cpu().numpy()
        sl = (slice(None),) + (slice(c["g"], -c["g"]),) * 3
        for v in range(5):
            err = np.abs(got[sl][v] - ref[sl][v]).max() / np.abs(ref[sl][v]).max()
            print(f"C4 block {i} {c['n']} variable {v}: {err:.2e}", flush=True)
            assert err <= 1e-12
    b.close()


def test_c4_full_size_every_block_fp64_and_mixed_vs_oracle():
    """All 48 blocks of the benchmarked workload with a non-uniform state (a
    smooth 5% density-and-energy bump near the cylinder plus 0.1% noise), one
    batched RK3 step in each precision from identical inputs, against the
    FP64 oracle stepping every block from the same metrics: FP64 within
    1e-12 per variable, FP32-mixed within 1e-4 of the step's increment."""
    specs = I.multiblock_specs(48, seed=4)
    cases = []
    for i, spec in enumerate(specs):
        g, Y = 3, 6
        xyz = I.ogrid_sector_block(spec.n, g, Y, spec.sector, spec.skew_deg, spec.rotation)
        q = I.uniform_state(3, spec.n, g, G.GAMMA, I.mach_velocity(3.0, [1.0, 0.0, 0.0]), 1.0)
        x = I.state_nodes(xyz, g, Y)
        bump = 0.05 * np.exp(-((x[0] - 1.3) ** 2 + (x[1] - 0.4) ** 2) / 0.2)
        rng = np.random.Generator(np.random.PCG64(200 + i))
        q = q * (1.0 + bump[None]) * (1.0 + 1e-3 * rng.standard_normal(q.shape))
        cases.append(dict(ndim=3, n=list(spec.n), g=g, Y=Y, bc=[1, 1, 1], xyz=xyz, q=np.ascontiguousarray(q)))
    worst = {"fp64": 0.0, "mixed": 0.0}
    sc64 = fp.Scheme("weno5", 6, True)
    blocks = [Block(c, sc64) for c in cases]
    refs = []
    for k in blocks:
        c = k.case
        og = O.Grid(3, c["n"], c["g"], bc=[1, 1, 1])
        refs.append(O.rk3_step(og, O.Scheme("weno5", 6, True), k.met.cpu().numpy(), c["q"], k.dt))
    for prec in ("fp64", "mixed"):
        for k in blocks:
            k.q.copy_(k.q0)
        b = fp.Batch(fp.Scheme("weno5", 6, True, precision=prec), 48)
        b.set([k.entry() for k in blocks])
        b.rk3_step()
        torch.cuda.synchronize()
        for i, (k, ref) in enumerate(zip(blocks, refs)):
            c = k.case
            sl = (slice(None),) + (slice(c["g"], -c["g"]),) * 3
            got = k.q.cpu().numpy()[sl].reshape(5, -1)
            want = ref[sl].reshape(5, -1)
            base = want if prec == "fp64" else want - c["q"][sl].reshape(5, -1)
            for v in range(5):
                err = np.abs(got[v] - want[v]).max() / np.abs(base[v]).max()
                worst[prec] = max(worst[prec], float(err))
                assert err <= (1e-12 if prec == "fp64" else 1e-4), f"{prec} block {i} variable {v}: {err:.3e}"
        b.close()
    print(f"C4 48 blocks vs oracle: FP64 {worst['fp64']:.2e} (of the state), "
          f"mixed {worst['mixed']:.2e} (of the increment)", flush=True)


def test_batch_solve_copies_frozen_ghosts_once_per_call():
    # fp_batch_solve copies the frozen ghost layers at the start of each call;
    # ghost values the caller changes between calls take effect at the next
    # call, exactly as with per-step fp_rk3_step (which copies every step)
    sc = fp.Scheme("weno5", 6, True, precision="mixed")
    case = G.frozen_case((30, 22, 14), 6, perturb=0.04, seed=21)
    blk = Block(case, sc)
    ref_q, ref_w = blk.q.clone(), torch.zeros_like(blk.work)
    b = fp.Batch(sc, 2)
    b.set([blk.entry()])
    b.solve(3)
    for _ in range(3):
        fp.rk3_step(blk.grid, sc, blk.met, ref_q, ref_w, blk.dt)
    torch.cuda.synchronize()
    assert torch.equal(blk.q, ref_q)
    g = case["g"]
    for q in (blk.q, ref_q):  # a new inflow state on the low xi face's ghosts
        q[:, :, :, :g] *= 1.01
    b.solve(2)
    for _ in range(2):
        fp.rk3_step(blk.grid, sc, blk.met, ref_q, ref_w, blk.dt)
    torch.cuda.synchronize()
    assert torch.equal(blk.q, ref_q)
    b.close()


def test_solve_copies_frozen_ghosts_once_per_call():
    # the single-block fp_solve follows the same rule as the batch
    sc = fp.Scheme("weno5", 6, True)
    case = G.frozen_case((26, 20, 12), 6, perturb=0.04, seed=22)
    blk = Block(case, sc)
    ref_q, ref_w = blk.q.clone(), torch.zeros_like(blk.work)
    fp.solve(blk.grid, sc, blk.met, blk.q, blk.work, blk.dt, 3)
    for _ in range(3):
        fp.rk3_step(blk.grid, sc, blk.met, ref_q, ref_w, blk.dt)
    torch.cuda.synchronize()
    assert torch.equal(blk.q, ref_q)
    g = case["g"]
    for q in (blk.q, ref_q):
        q[:, :, :, :g] *= 1.01
    fp.solve(blk.grid, sc, blk.met, blk.q, blk.work, blk.dt, 2)
    for _ in range(2):
        fp.rk3_step(blk.grid, sc, blk.met, ref_q, ref_w, blk.dt)
    torch.cuda.synchronize()
    assert torch.equal(blk.q, ref_q)
