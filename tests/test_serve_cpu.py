"""Host logic of the serving loop, driven by a simulated backend (no GPU):
the request stream, admission by HBM footprint and slots (first fit in
arrival order), continuous batching (requests join a running set), exact
step accounting and the latency statistics."""
import math

import numpy as np
import pytest

from paper_2101_05886_amd import serve as S


class SimBackend:
    """Simulated device: a round of k steps costs k * (launch + per-node
    time x active nodes) seconds of simulated time."""

    def __init__(self, per_node=1e-9, launch=1e-4):
        self.t = 0.0
        self.per_node, self.launch = per_node, launch
        self.active = []
        self.steps = {}
        self.allocated = 0
        self.peak = 0
        self.admit_time = {}
        self.finish_time = {}
        self.retired = []
        self.prefetched = set()

    def footprint(self, r):
        return r.nodes * (30 if r.ndim == 3 else 24) * 8

    def prefetch(self, reqs):
        self.prefetched.update(r.rid for r in reqs)

    def admit(self, r):
        self.allocated += self.footprint(r)
        self.peak = max(self.peak, self.allocated)
        self.steps[r.rid] = 0
        self.admit_time[r.rid] = self.t
        return r

    def set_active(self, handles):
        self.active = list(handles)

    def advance(self, k):
        self.t += k * (self.launch + self.per_node * sum(r.nodes for r in self.active))
        for r in self.active:
            self.steps[r.rid] += k

    def retire(self, r):
        self.allocated -= self.footprint(r)
        self.retired.append(r.rid)
        self.finish_time[r.rid] = self.t
        return ("result", r.rid, self.steps[r.rid])

    def round_end(self):
        return self.t

    def completion(self, tok):
        return tok

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


def test_request_stream_is_seeded_and_shaped():
    a = S.make_requests(500, seed=5, rate=4.0)
    b = S.make_requests(500, seed=5, rate=4.0)
    assert a == b
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 0.25) < 0.25 * 0.15  # Poisson at 4 per second
    nodes = np.array([r.nodes for r in a])
    assert nodes.min() >= 0.9 * 64 ** 2 and nodes.max() <= 1.1 * 160 ** 3
    # log-uniform: the median node count is near the geometric mean of the range
    assert abs(math.log(np.median(nodes)) - 0.5 * math.log(64 ** 2 * 160 ** 3)) < 0.5
    assert {r.kind for r in a} == {"wavy2d", "wavy3d", "ogrid3d"}
    assert all(0.3 <= r.mach <= 2.0 and 0.0 <= r.angle_deg <= 10.0 and r.steps == 200 for r in a)
    closed = S.make_requests(10, seed=5, rate=None)
    assert all(r.arrival == 0.0 for r in closed)


def test_shapes():
    assert S.request_shape("wavy2d", 64 ** 2) == (64, 64)
    assert S.request_shape("wavy3d", 160 ** 3) == (160, 160, 160)
    nt, nr, nz = S.request_shape("ogrid3d", 64 ** 3)
    assert (nt, nr, nz) == (128, 64, 32)


def run(reqs, budget=10 ** 12, slots=64, round_steps=10, **kw):
    be = SimBackend(**kw)
    st, res = S.Scheduler(be, budget, slots, round_steps).run(reqs)
    return be, st, res


def test_every_request_gets_exactly_its_steps():
    reqs = S.make_requests(60, seed=7, rate=50.0, nodes_range=(1000, 200000), steps=37)
    for i, r in enumerate(reqs):
        r.steps = 5 + (i * 7) % 41  # uneven step counts, not multiples of the round
    be, st, res = run(reqs, round_steps=8)
    assert sorted(be.retired) == [r.rid for r in reqs]
    for r in reqs:
        assert be.steps[r.rid] == r.steps
        assert res[r.rid] == ("result", r.rid, r.steps)
    assert set(st.latency) == {r.rid for r in reqs}


def test_budget_and_slots_are_respected():
    reqs = S.make_requests(80, seed=8, rate=None, nodes_range=(20000, 400000), steps=20)
    budget = 120 * 10 ** 6
    be, st, _ = run(reqs, budget=budget, slots=6)
    assert be.peak <= budget
    assert st.peak_bytes <= budget and st.peak_active <= 6
    assert be.allocated == 0


def test_first_fit_in_arrival_order():
    running = S.Request(0, 0.0, "wavy3d", (60, 60, 60), 0.5, 0.0, 30)
    big = S.Request(1, 0.0, "wavy3d", (100, 100, 100), 0.5, 0.0, 10)
    small = [S.Request(i, 0.0, "wavy2d", (20, 20), 0.5, 0.0, 10) for i in (2, 3)]
    be = SimBackend()
    budget = be.footprint(big) + 1000  # room for the big one alone, not beside the running one
    S.Scheduler(be, budget, 8, 10).run([running, big] + small)
    # the big request does not fit next to the running one; the small ones
    # behind it do and are admitted at once; the big one waits for room
    assert be.admit_time[0] == be.admit_time[2] == be.admit_time[3] == 0.0
    assert be.admit_time[1] >= be.finish_time[0]


def test_arrivals_join_a_running_set():
    long = S.Request(0, 0.0, "wavy3d", (80, 80, 80), 0.5, 0.0, 200)
    late = S.Request(1, 0.01, "wavy2d", (64, 64), 0.5, 0.0, 20)
    be, st, _ = run([long, late])
    assert be.admit_time[1] < be.finish_time[0]  # admitted while the long one runs
    assert be.finish_time[1] < be.finish_time[0]  # and done before it
    assert st.peak_active == 2


def test_latency_statistics():
    reqs = S.make_requests(40, seed=9, rate=20.0, nodes_range=(4096, 100000), steps=30)
    be, st, _ = run(reqs)
    for r in reqs:
        assert st.latency[r.rid] >= st.wait[r.rid] >= 0.0
        assert math.isclose(st.latency[r.rid], be.finish_time[r.rid] - r.arrival)
    s = st.summary()
    assert s["requests"] == 40 and s["p50_latency_s"] <= s["p99_latency_s"]
    assert s["makespan_s"] == pytest.approx(max(be.finish_time.values()))
    assert s["cell_stage_per_s"] == pytest.approx(sum(3 * r.steps * r.nodes for r in reqs) / s["makespan_s"])


def test_oversized_request_is_an_error():
    r = S.Request(0, 0.0, "wavy3d", (100, 100, 100), 0.5, 0.0, 10)
    with pytest.raises(ValueError):
        run([r], budget=1000)


class HeldBackend(SimBackend):
    """Device memory as the GPU backend holds it: a retired request's
    buffers stay allocated while the batch still references them, i.e.
    until the next set_active that leaves them out."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.held = set()

    def set_active(self, handles):
        keep = {r.rid for r in handles}
        for rid in list(self.held):
            if rid not in keep:
                self.held.discard(rid)
                self.allocated -= self.fp[rid]
        super().set_active(handles)

    def admit(self, r):
        self.fp = getattr(self, "fp", {})
        self.fp[r.rid] = self.footprint(r)
        return super().admit(r)

    def retire(self, r):
        out = super().retire(r)
        self.allocated += self.footprint(r)  # not freed yet
        self.held.add(r.rid)
        return out


def test_retired_buffers_are_released_before_admission():
    # a tight budget and a steady stream: every admission follows a
    # retirement, so device use would exceed the budget if the batch still
    # held the retired requests' buffers when new ones are allocated
    reqs = S.make_requests(60, seed=12, rate=None, nodes_range=(30000, 300000), steps=25)
    for i, r in enumerate(reqs):
        r.steps = 10 + (i * 13) % 37
    budget = 150 * 10 ** 6
    be = HeldBackend()
    st, res = S.Scheduler(be, budget, 8, 10).run(reqs)
    assert len(res) == len(reqs)
    assert be.peak <= budget
    for r in reqs:
        assert be.steps[r.rid] == r.steps
