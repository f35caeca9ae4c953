"""The serving loop on the GPU: requests of different grids, kinds and Mach
numbers arrive while others run, are admitted into the running batch and
share its launches; each result must equal the same request solved alone
(fp_rk3_step, one block), bitwise: the per-block arithmetic of the batched
kernels is that of the single-block ones, so the stated tolerance is 0."""
import pytest
import torch

from paper_2101_05886_amd import fp
from paper_2101_05886_amd import serve as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need the MI355X"
    fp.lib()
    yield


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_alone_equals_in_the_mix(prec):
    sc = fp.Scheme("weno5", 6, True, precision=prec)
    reqs = S.make_requests(12, seed=21, rate=400.0, nodes_range=(64 ** 2, 28 ** 3), steps=1)
    for i, r in enumerate(reqs):
        r.steps = 6 + (5 * i) % 17  # uneven, not multiples of the round length
    be = S.GpuBackend(sc, 16, workers=4)
    st, results = S.Scheduler(be, 8 << 30, 16, round_steps=4).run(reqs)
    torch.cuda.synchronize()
    be.close()
    print(st.summary(), flush=True)
    assert st.peak_active > 1, "requests should have shared rounds"
    assert sorted(results) == [r.rid for r in reqs]
    for r in reqs:
        alone = S.run_alone(r, sc)
        assert torch.equal(results[r.rid], alone), f"request {r.rid} ({r.kind} {r.n}) differs"


def test_small_slot_count_still_serves_everything():
    sc = fp.Scheme("weno5", 6, True, precision="mixed")
    reqs = S.make_requests(9, seed=22, rate=None, nodes_range=(64 ** 2, 24 ** 3), steps=5)
    be = S.GpuBackend(sc, 2, workers=2)
    st, results = S.Scheduler(be, 8 << 30, 2, round_steps=3).run(reqs)
    torch.cuda.synchronize()
    be.close()
    assert st.peak_active == 2 and sorted(results) == [r.rid for r in reqs]
    for r in reqs[:3]:
        assert torch.equal(results[r.rid], S.run_alone(r, sc))
