"""Serving loop: a stream of solve requests with continuous batching.

Each request asks for `steps` RK3 steps of the free-stream-preserving scheme
on its own grid (2D or 3D periodic wavy grid with a vortex in a uniform
flow, or a 3D O-grid sector block in a uniform flow with frozen ghosts) at
its own Mach number and flow angle.  The scheduler keeps every admitted
request's state on the device and advances all of them together, a round
of a few RK steps at a time, through one batch of the library (fp_batch_*):
every sweep of every RK stage is one shared launch over all active
requests.  Between rounds it retires finished requests (result copied to
pinned host memory), frees their memory and admits waiting requests, first
fit in arrival order, while their HBM footprint fits the budget and a batch
slot is free.  So requests that arrive while others run join the running
set at the next round boundary and their work shares launches with the
others'.

The scheduler is host logic over a small backend interface; `GpuBackend`
drives the library, tests drive the scheduler with a simulated backend.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I

GAMMA = 1.4


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    kind: str  # "wavy2d", "wavy3d" or "ogrid3d"
    n: tuple  # interior nodes per axis
    mach: float
    angle_deg: float  # flow angle in the x-y plane
    steps: int

    @property
    def ndim(self):
        return 2 if self.kind == "wavy2d" else 3

    @property
    def nodes(self):
        return int(np.prod(self.n))


def request_shape(kind: str, nodes: float):
    """Interior extents for about `nodes` nodes: square/cubic wavy grids,
    O-grid blocks with n_theta : n_r : n_z = 2 : 1 : 1/2."""
    if kind == "wavy2d":
        m = max(8, int(round(math.sqrt(nodes))))
        return (m, m)
    if kind == "wavy3d":
        m = max(8, int(round(nodes ** (1.0 / 3.0))))
        return (m, m, m)
    m = max(16, int(round(nodes ** (1.0 / 3.0))))
    return (2 * m, m, max(8, m // 2))


def make_requests(count=500, seed=5, rate=1.0, nodes_range=(64 ** 2, 160 ** 3), steps=200,
                  kinds=("wavy2d", "wavy3d", "ogrid3d"), mach_range=(0.3, 2.0), angle_range=(0.0, 10.0)):
    """Seeded request stream: Poisson arrivals at `rate` per second (rate
    None: all at t = 0, the closed-loop case), grid kind uniform over
    `kinds`, node count log-uniform over `nodes_range`, Mach and angle
    uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for rid in range(count):
        if rate:
            t += float(rng.exponential(1.0 / rate))
        kind = kinds[int(rng.integers(0, len(kinds)))]
        nodes = math.exp(rng.uniform(math.log(nodes_range[0]), math.log(nodes_range[1])))
        mach = float(rng.uniform(*mach_range))
        ang = float(rng.uniform(*angle_range))
        out.append(Request(rid, t if rate else 0.0, kind, request_shape(kind, nodes), mach, ang, steps))
    return out


def request_inputs(req: Request, g=3, Y=6, L=12.0):
    """(bc, xyz, q) host arrays of a request (seeded by its id)."""
    a = math.radians(req.angle_deg)
    if req.kind == "ogrid3d":
        rng = np.random.Generator(np.random.PCG64(1000 + req.rid))
        xyz = I.ogrid_sector_block(req.n, g, Y, sector=float(rng.uniform(math.pi / 3, math.pi)),
                                   skew_deg=float(rng.uniform(0.0, 30.0)),
                                   rotation=float(rng.uniform(0.0, 2 * math.pi)))
        vel = I.mach_velocity(req.mach, [math.cos(a), math.sin(a), 0.0])
        q = I.uniform_state(3, req.n, g, GAMMA, vel, 1.0)
        return [1, 1, 1], xyz, q
    ndim = req.ndim
    xyz = I.wavy_grid(ndim, req.n, L, g, Y, amp=0.1, jitter=0.0, seed=1000 + req.rid)
    per = I.wavy_periods(ndim, req.n, L)
    d = [math.cos(a), math.sin(a)] + ([0.0] if ndim == 3 else [])
    vel = I.mach_velocity(req.mach, d)
    v3 = tuple(vel) + (0.0,) * (3 - len(vel))
    q = I.Vortex(vel_inf=v3).state(I.state_nodes(xyz, g, Y), period=per[:2])
    return [0] * ndim, xyz, np.ascontiguousarray(q)


@dataclass
class Slot:
    req: Request
    handle: object
    footprint: int
    remaining: int
    admitted: float = 0.0


@dataclass
class ServeStats:
    latency: dict = field(default_factory=dict)  # rid -> seconds, arrival to result on the host
    wait: dict = field(default_factory=dict)  # rid -> seconds, arrival to admission
    makespan: float = 0.0
    cell_stages: float = 0.0
    rounds: int = 0
    peak_bytes: int = 0
    peak_active: int = 0

    def percentile(self, p):
        v = np.array(sorted(self.latency.values()))
        return float(np.percentile(v, p)) if len(v) else float("nan")

    def summary(self):
        n = len(self.latency)
        return {"requests": n, "p50_latency_s": self.percentile(50), "p99_latency_s": self.percentile(99),
                "mean_queue_wait_s": float(np.mean(list(self.wait.values()))) if n else float("nan"),
                "requests_per_s": n / self.makespan if self.makespan else float("nan"),
                "cell_stage_per_s": self.cell_stages / self.makespan if self.makespan else float("nan"),
                "makespan_s": self.makespan, "rounds": self.rounds, "peak_active": self.peak_active,
                "peak_bytes": self.peak_bytes}


class Scheduler:
    """Continuous batching over a backend with this interface:

    footprint(req) -> bytes the request holds on the device while active
    prefetch(reqs)  start preparing host inputs of requests soon admitted
    admit(req) -> handle           allocate and set up (metrics, dt)
    set_active(handles)            the batch's blocks for the next rounds
    advance(nsteps) -> token       enqueue nsteps RK3 steps of the batch
    retire(handle) -> result       enqueue the copy of the result to the
                                   host and release the device memory
    completion(token) -> seconds   wait for a token; its completion time
                                   since start() on the backend's clock
    start() -> None, now() -> seconds, sleep_until(seconds)
    """

    def __init__(self, backend, budget_bytes, max_active, round_steps=10, prefetch=8):
        self.b = backend
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.round_steps = int(round_steps)
        self.prefetch = int(prefetch)

    def run(self, requests):
        b = self.b
        st = ServeStats()
        results = {}
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue = []
        active = []
        used = 0
        inflight = None  # (token, finished slots) of the last enqueued round
        changed = True
        released = False  # finished requests the batch may still reference
        b.start()
        while pending or queue or active:
            now = b.now()
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            b.prefetch(queue[: self.prefetch])
            if released:
                # the batch drops its references to the retired requests'
                # buffers before new ones are allocated, so device use stays
                # within the budget that `used` accounts for
                b.set_active([s.handle for s in active])
                released = False
                changed = False
            # admission: first fit, in arrival order, by footprint and slots
            i = 0
            while i < len(queue) and len(active) < self.max_active:
                r = queue[i]
                fpb = b.footprint(r)
                if fpb > self.budget:
                    raise ValueError(f"request {r.rid} needs {fpb} B, more than the budget {self.budget} B")
                if used + fpb <= self.budget:
                    queue.pop(i)
                    active.append(Slot(r, b.admit(r), fpb, r.steps, admitted=b.now()))
                    st.wait[r.rid] = active[-1].admitted - r.arrival
                    used += fpb
                    changed = True
                else:
                    i += 1
            st.peak_bytes = max(st.peak_bytes, used)
            st.peak_active = max(st.peak_active, len(active))
            if not active:
                if inflight is not None:
                    self._finish(inflight, st, results)
                    inflight = None
                    continue
                if pending:
                    b.sleep_until(pending[0].arrival)
                    continue
                break
            k = min(self.round_steps, min(s.remaining for s in active))
            if changed:
                b.set_active([s.handle for s in active])
                changed = False
            for s in active:
                s.remaining -= k
                st.cell_stages += 3.0 * k * s.req.nodes
            done = [s for s in active if s.remaining == 0]
            if done:
                active = [s for s in active if s.remaining > 0]
                changed = True
            # the round's work, then the copies of finished results
            b.advance(k)
            for s in done:
                results[s.req.rid] = b.retire(s.handle)
                used -= s.footprint
                released = True
            token = b.round_end()
            st.rounds += 1
            if inflight is not None:
                self._finish(inflight, st, results)
            inflight = (token, done)
        if inflight is not None:
            self._finish(inflight, st, results)
        st.makespan = max((st.latency[r.rid] + r.arrival for r in requests if r.rid in st.latency),
                          default=0.0)
        return st, results

    def _finish(self, inflight, st, results):
        token, done = inflight
        t = self.b.completion(token)
        for s in done:
            st.latency[s.req.rid] = t - s.req.arrival


class GpuBackend:
    """The library's batch on the current GPU.  Host inputs are prepared by
    a thread pool ahead of admission; metrics and dt are computed on a side
    stream; rounds, result copies and completion events run on the main
    stream."""

    def __init__(self, scheme, max_active, g=3, workers=8):
        import torch

        from . import fp
        self.torch, self.fp = torch, fp
        self.scheme = scheme
        self.g, self.Y = g, scheme.metric_order
        self.batch = fp.Batch(scheme, max_active)
        self.pool = cf.ThreadPoolExecutor(workers)
        self.futures = {}
        self.side = torch.cuda.Stream()
        self.main = torch.cuda.current_stream()
        self.t0_host = 0.0
        self.ev0 = None

    def close(self):
        self.batch.close()
        self.pool.shutdown(wait=True)

    def _grid(self, req, bc):
        return self.fp.Grid(req.ndim, list(req.n), self.g, bc=bc)

    def footprint(self, req):
        fp = self.fp
        bc = [1, 1, 1] if req.kind == "ogrid3d" else [0] * req.ndim
        G = self._grid(req, bc)
        return fp.state_bytes(G) + fp.metric_bytes(G) + fp.work_bytes(G)

    def prefetch(self, reqs):
        for r in reqs:
            if r.rid not in self.futures:
                self.futures[r.rid] = self.pool.submit(request_inputs, r, self.g, self.Y)

    def admit(self, req):
        torch, fp = self.torch, self.fp
        if req.rid not in self.futures:
            self.prefetch([req])
        bc, xyz, q = self.futures.pop(req.rid).result()
        G = self._grid(req, bc)
        with torch.cuda.stream(self.side):
            met = fp.metrics(G, self.Y, torch.from_numpy(xyz).cuda())
            qd = torch.from_numpy(q).cuda()
            work = torch.zeros(G.work_shape(), dtype=torch.float64, device="cuda")
            dt = float(fp.max_dt(G, self.scheme, met, qd, 0.5).item())
        self.main.wait_stream(self.side)
        for t in (met, qd, work):
            t.record_stream(self.main)
        return dict(grid=G, met=met, q=qd, work=work, dt=dt, req=req)

    def set_active(self, handles):
        self.batch.set([(h["grid"], h["met"], h["q"], h["work"], h["dt"]) for h in handles])

    def advance(self, nsteps):
        self.batch.solve(nsteps)

    def retire(self, h):
        g, nd = self.g, h["req"].ndim
        src = h["q"][(slice(None),) + (slice(g, -g),) * nd]
        out = self.torch.empty(src.shape, dtype=self.torch.float64, pin_memory=True)
        out.copy_(src, non_blocking=True)
        h["met"] = h["q"] = h["work"] = None  # device memory returns to torch's cache in stream order
        return out

    def round_end(self):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.main)
        return ev

    def completion(self, ev):
        ev.synchronize()
        return self.ev0.elapsed_time(ev) * 1e-3

    def start(self):
        self.torch.cuda.synchronize()
        self.ev0 = self.torch.cuda.Event(enable_timing=True)
        self.ev0.record(self.main)
        self.t0_host = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0_host

    def sleep_until(self, t):
        d = t - self.now()
        if d > 0:
            time.sleep(d)


def run_alone(req, scheme, g=3):
    """The request advanced by itself with fp_rk3_step (the reference of the
    alone-versus-mix check); returns the interior of its final state."""
    import torch

    from . import fp
    bc, xyz, q = request_inputs(req, g, scheme.metric_order)
    G = fp.Grid(req.ndim, list(req.n), g, bc=bc)
    met = fp.metrics(G, scheme.metric_order, torch.from_numpy(xyz).cuda())
    qd = torch.from_numpy(q).cuda()
    work = torch.zeros(G.work_shape(), dtype=torch.float64, device="cuda")
    dt = float(fp.max_dt(G, scheme, met, qd, 0.5).item())
    for _ in range(req.steps):
        fp.rk3_step(G, scheme, met, qd, work, dt)
    return qd[(slice(None),) + (slice(g, -g),) * req.ndim].cpu()
