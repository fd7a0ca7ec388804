"""Continuous-batching serving loop for ensemble and regional solves.

Requests (a box mesh, an order N, an initial perturbation, K steps, and
optionally the five-stage integrator and a filter) arrive over time.  The
server keeps every admitted state resident in device memory, admits requests
first-come-first-served while their memory footprint fits a budget, groups the
active requests by order and integrator and advances each group by one step
per iteration in batched launches (numa_step_batch: one element launch and one
finish launch per stage for all members, then each filtered member's filter),
replaying a HIP graph of that step while the group's membership is unchanged.  A request that has run
its K steps retires at the end of the iteration, its memory is released and
waiting requests are admitted.  Latency is completion time minus arrival time.

The scheduling logic talks to an executor; GpuExecutor drives libnuma, and the
tests substitute a host-only executor to check admission, ordering and
release without a GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    workload: dict          # inputs.box_workload(...)
    noise_seed: int
    steps: int = 50
    integrator: int = 0     # numa.RK_SSP33 or numa.RK_SSP53
    filter: tuple = None    # (filter order p, cutoff) applied after every step, or None
    # filled by the server
    admitted: float = -1.0
    done: float = -1.0
    state: object = None    # final state (executor-specific), if kept

    @property
    def key(self):
        """Requests with equal keys share one geometry (and its step settings)."""
        m = self.workload["mesh"]
        return (tuple(m["ne"]), m["N"], tuple(m["periodic"]), tuple(m["extent"]), m["h0"], self.integrator,
                self.filter)

    @property
    def order(self):
        return self.workload["mesh"]["N"]

    @property
    def group(self):
        """Requests batched together: one order and one integrator per launch."""
        return (self.order, self.integrator)

    @property
    def stages(self):
        return 5 if self.integrator == 1 else 3


@dataclass
class Slot:
    req: Request
    geom: object
    handle: object
    bytes: int = 0
    steps_done: int = 0


class GpuExecutor:
    """libnuma on one GPU: geometry per mesh shape (shared, read-only), and per
    request a state and private scratch in device memory.  Box meshes run with
    the metric recomputed every stage unless metric says otherwise."""

    def __init__(self, prec=0, device="cuda:0", use_graphs=True, metric=None):
        import torch
        from . import numa
        self.torch, self.numa = torch, numa
        self.prec = prec
        self.metric = numa.METRIC_RECOMPUTE if metric is None else metric
        self.device = device
        self.use_graphs = use_graphs
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self._geoms = {}
        self._graphs = {}

    def geometry(self, req: Request):
        g = self._geoms.get(req.key)
        if g is None:
            with self.torch.cuda.stream(self.stream):
                g = self.numa.Mesh(req.workload["mesh"], req.workload["phys"], prec_mask=1 | (2 if self.prec else 0),
                                   device=self.device, stream=self.stream)
                if req.workload["mesh"]["kind"] == self.numa.MESH_BOX:
                    g.set_metric(self.metric)
                g.set_integrator(req.integrator)
                if req.filter is not None:
                    g.set_filter(*req.filter)
            self._geoms[req.key] = g
        return g

    def geometry_bytes(self, req: Request) -> int:
        g = self._geoms.get(req.key)
        return g.workspace_bytes if g is not None else 0

    def request_bytes(self, req: Request, geom) -> int:
        return 40 * geom.n_unique + self.numa.step_scratch_bytes(geom, self.prec) + 512

    def start(self, req: Request, geom):
        from . import inputs
        with self.torch.cuda.stream(self.stream):
            noise = inputs.device_noise(geom.n_unique, req.noise_seed, device=self.device)
            q = geom.init_state(req.workload["ic"], noise, stream=self.stream)
            scratch = self.numa.alloc_scratch(geom, self.prec)
        # noise was allocated on self.stream, so the caching allocator reuses its
        # memory only for later work on the same stream: safe to drop here
        return (q, scratch)

    def step_group(self, group, slots, dt: float):
        items = [(s.geom, s.handle[0], s.handle[1], dt) for s in slots]
        key = (group, tuple(s.req.id for s in slots))
        if not self.use_graphs:
            self.numa.step_batch(items, 1, self.prec, stream=self.stream)
            return
        g = self._graphs.get(group)
        if g is None or g[0] != key:
            if g is not None:
                g[1].close()
            g = (key, self.numa.Graph(items, 1, self.prec, self.stream))
            self._graphs[group] = g
        g[1].launch(self.stream)

    def sync(self):
        self.stream.synchronize()

    def finish(self, slot: Slot, keep: bool):
        return slot.handle[0].clone() if keep else None

    def release(self, slot: Slot):
        slot.handle = None

    def drop_graphs(self):
        for k, g in list(self._graphs.items()):
            g[1].close()
        self._graphs.clear()


@dataclass
class ServeStats:
    latencies: list = field(default_factory=list)
    wall: float = 0.0
    updates: float = 0.0      # grid-point RHS updates (unique nodes x stages x steps)
    iterations: int = 0
    max_active: int = 0
    peak_bytes: int = 0

    def percentile(self, p):
        xs = sorted(self.latencies)
        if not xs:
            return float("nan")
        i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
        return xs[i]


class Server:
    def __init__(self, executor, budget_bytes: int, dt: float = 0.05, keep_states: bool = False,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = budget_bytes
        self.dt = dt
        self.keep = keep_states
        self.clock = clock
        self.sleep = sleep
        self.used = 0

    def prewarm(self, requests):
        """Build the geometry of every mesh shape the requests use (the
        serving equivalent of loading a model before taking traffic)."""
        for r in requests:
            self.ex.geometry(r)
        self.ex.sync()

    def run(self, requests, realtime: bool = True) -> ServeStats:
        """Serve the requests (arrival times relative to the start).  With
        realtime=False every request is available at once (back-to-back)."""
        future = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        waiting = collections.deque()
        active = collections.OrderedDict()  # request id -> Slot
        st = ServeStats()
        t0 = self.clock()
        while future or waiting or active:
            now = self.clock() - t0
            while future and (not realtime or future[0].arrival <= now):
                waiting.append(future.popleft())
            # first come, first served: stop at the first request that does not fit
            while waiting:
                req = waiting[0]
                geom = self.ex.geometry(req)
                need = self.ex.request_bytes(req, geom)
                if need > self.budget:
                    raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.id, need))
                if self.used + need > self.budget:
                    break
                waiting.popleft()
                self.used += need
                st.peak_bytes = max(st.peak_bytes, self.used)
                req.admitted = self.clock() - t0
                active[req.id] = Slot(req, geom, self.ex.start(req, geom), bytes=need)
            if not active:
                if future:
                    self.sleep(max(0.0, min(1e-3, future[0].arrival - (self.clock() - t0))))
                continue
            st.max_active = max(st.max_active, len(active))
            groups = collections.defaultdict(list)
            for s in active.values():
                groups[s.req.group].append(s)
            for grp in sorted(groups):
                self.ex.step_group(grp, groups[grp], self.dt)
            self.ex.sync()
            st.iterations += 1
            now = self.clock() - t0
            for rid in list(active):
                s = active[rid]
                s.steps_done += 1
                st.updates += s.req.stages * s.geom.n_unique
                if s.steps_done >= s.req.steps:
                    s.req.done = now
                    s.req.state = self.ex.finish(s, self.keep)
                    st.latencies.append(now - s.req.arrival if realtime else now)
                    self.ex.release(s)
                    self.used -= s.bytes
                    del active[rid]
        st.wall = self.clock() - t0
        return st
