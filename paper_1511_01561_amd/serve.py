"""Continuous-batching serving loop for ensemble and regional solves.

Requests (a box mesh, an order N, an initial perturbation, K steps, and
optionally the five-stage integrator and a filter) arrive over time.  The
server keeps every admitted state resident in device memory, admits requests
first-come-first-served while their memory footprint fits a budget, groups the
active requests by order and integrator and advances each group by one step
per iteration in batched launches (numa_step_batch: one element launch and one
finish launch per stage for all members, then each filtered member's filter),
replaying a HIP graph of that step while the group's membership is unchanged.

The budget covers everything the server holds on the device: every request's
state, scratch and flag, and every geometry (the mesh workspaces, shared by
the requests of one mesh shape).  A geometry no active request uses is
evicted, least recently used first, when a request would not fit otherwise.

The host does not wait for an iteration before it enqueues the next: it
waits for iteration i - 1 after enqueueing iteration i.  A request that has
run its K steps leaves the launches at once and is retired (its result
taken, its memory released, its latency recorded) when that wait returns.
Every stage sets a per-request flag when it writes a non-finite value into
the request's state; such a request is retired at the same point as failed,
alone: the others' states are untouched.

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
    failed: bool = False    # retired because its state became non-finite
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
    request a state, private scratch and a non-finite flag in device memory.
    Box meshes run with the metric recomputed every stage unless metric says
    otherwise.  All device work goes to one non-default stream."""

    def __init__(self, prec=0, device="cuda:0", use_graphs=True, metric=None, max_slots=4096):
        import torch
        from . import numa
        self.torch, self.numa = torch, numa
        self.prec = prec
        self.metric = numa.METRIC_RECOMPUTE if metric is None else metric
        self.device = device
        self.use_graphs = use_graphs
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self._geoms = {}
        self._sizes = {}
        self._graphs = {}
        # non-finite flags: one int32 per slot on the device, copied to one of
        # two pinned host buffers after every iteration
        self.flags = torch.zeros(max_slots, dtype=torch.int32, device=device)
        self._host = [torch.zeros(max_slots, dtype=torch.int32, pin_memory=True) for _ in range(2)]
        self._turn = 0
        self._free = list(range(max_slots - 1, -1, -1))

    def _prec_mask(self, req: Request):
        """the workspace a request's geometry needs: lean (no per-node metric,
        gather map or mesh scratch) for boxes stepped with the recomputed
        metric and no filter, which only the batched steps touch"""
        m = 1 | (2 if self.prec else 0)
        if (req.workload["mesh"]["kind"] == self.numa.MESH_BOX and self.metric == self.numa.METRIC_RECOMPUTE
                and req.filter is None):
            m |= self.numa.WS_LEAN
        return m

    def sizes(self, req: Request):
        """(geometry workspace bytes, request bytes) of a request, on the host."""
        z = self._sizes.get(req.key)
        if z is None:
            ws, nu, scr = self.numa.mesh_sizes(req.workload["mesh"], self._prec_mask(req), self.prec)
            z = (ws + 256, 40 * nu + 256 + scr + 256)
            self._sizes[req.key] = z
        return z

    def has_geometry(self, key) -> bool:
        return key in self._geoms

    def geometry(self, req: Request):
        g = self._geoms.get(req.key)
        if g is None:
            with self.torch.cuda.stream(self.stream):
                g = self.numa.Mesh(req.workload["mesh"], req.workload["phys"], prec_mask=self._prec_mask(req),
                                   device=self.device, stream=self.stream)
                if req.workload["mesh"]["kind"] == self.numa.MESH_BOX:
                    g.set_metric(self.metric)
                g.set_integrator(req.integrator)
                if req.filter is not None:
                    g.set_filter(*req.filter)
            self._geoms[req.key] = g
        return g

    def drop_geometry(self, key):
        """Free a geometry no request uses any more (its graphs are gone with
        the groups that held it)."""
        g = self._geoms.pop(key, None)
        if g is not None:
            g.close()
            with self.torch.cuda.stream(self.stream):
                del g  # the workspace tensor goes back to the allocator on the serving stream

    def request_bytes(self, req: Request, geom=None) -> int:
        return self.sizes(req)[1]

    def start(self, req: Request, geom):
        from . import inputs
        idx = self._free.pop()
        with self.torch.cuda.stream(self.stream):
            noise = inputs.device_noise(geom.n_unique, req.noise_seed, device=self.device)
            q = geom.init_state(req.workload["ic"], noise, stream=self.stream)
            scratch = self.numa.alloc_scratch(geom, self.prec)
            self.flags[idx].zero_()
        # noise was allocated on self.stream, so the caching allocator reuses its
        # memory only for later work on the same stream: safe to drop here
        return (q, scratch, idx)

    def step_group(self, group, slots, dt: float):
        items = [(s.geom, s.handle[0], s.handle[1], dt, self.flags[s.handle[2]:s.handle[2] + 1]) for s in slots]
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

    def mark(self):
        """After an iteration's launches: copy the flags to a pinned buffer and
        record an event; wait(token) returns the flags once it has passed."""
        host = self._host[self._turn]
        self._turn ^= 1
        with self.torch.cuda.stream(self.stream):
            host.copy_(self.flags, non_blocking=True)
            ev = self.torch.cuda.Event()
            ev.record(self.stream)
        return (ev, host)

    def wait(self, token):
        ev, host = token
        ev.synchronize()
        return host

    def failed(self, flags, slot: Slot) -> bool:
        return bool(flags[slot.handle[2]].item())

    def sync(self):
        self.stream.synchronize()

    def finish(self, slot: Slot, keep: bool):
        if not keep:
            return None
        with self.torch.cuda.stream(self.stream):  # ordered after the slot's last step
            return slot.handle[0].clone()

    def release(self, slot: Slot):
        self._free.append(slot.handle[2])
        slot.handle = None  # freed on the serving stream, after its last use there

    def drop_graphs(self):
        for k, g in list(self._graphs.items()):
            g[1].close()
        self._graphs.clear()


@dataclass
class ServeStats:
    latencies: list = field(default_factory=list)
    failed: int = 0           # requests retired because their state became non-finite
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
        self.used = 0                                 # bytes of admitted requests
        self.geoms = collections.OrderedDict()        # geometry key -> bytes, least recently used first
        self.refs = collections.Counter()             # geometry key -> requests holding it

    @property
    def geom_bytes(self) -> int:
        return sum(self.geoms.values())

    def _sizes(self, req):
        """(geometry bytes, request bytes); executors without sizes() hold
        geometry outside the budget"""
        if hasattr(self.ex, "sizes"):
            return self.ex.sizes(req)
        return 0, self.ex.request_bytes(req, self.ex.geometry(req))

    def _build(self, req):
        g = self.ex.geometry(req)
        if req.key not in self.geoms:
            self.geoms[req.key] = self._sizes(req)[0]
        self.geoms.move_to_end(req.key)
        return g

    def _make_room(self, need, keep_key) -> bool:
        """Evict idle geometries (least recently used first) until need more
        bytes fit the budget."""
        while self.used + self.geom_bytes + need > self.budget:
            idle = [k for k in self.geoms if self.refs[k] == 0 and k != keep_key]
            if not idle:
                return False
            k = idle[0]
            del self.geoms[k]
            if hasattr(self.ex, "drop_geometry"):
                self.ex.drop_geometry(k)
        return True

    def prewarm(self, requests, fraction: float = 0.5):
        """Build the geometry of the mesh shapes the requests use, in order of
        first use, while the geometries fit `fraction` of the budget (the
        serving equivalent of loading models before taking traffic); the rest
        are built when first needed."""
        for r in requests:
            if r.key in self.geoms:
                continue
            gb = self._sizes(r)[0]
            if self.geom_bytes + gb > fraction * self.budget:
                continue
            self._build(r)
        self.ex.sync()

    def run(self, requests, realtime: bool = True) -> ServeStats:
        """Serve the requests (arrival times relative to the start).  With
        realtime=False every request is available at once (back-to-back)."""
        future = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        waiting = collections.deque()
        active = collections.OrderedDict()  # request id -> Slot (still stepping)
        pending = None                      # the last iteration: (token, its slots, slots that finished in it)
        st = ServeStats()
        t0 = self.clock()
        mark = getattr(self.ex, "mark", None)

        def retire(s, failed):
            now = self.clock() - t0
            s.req.done = now
            s.req.failed = failed
            s.req.state = self.ex.finish(s, self.keep)
            if failed:
                st.failed += 1
            else:
                st.latencies.append(now - s.req.arrival if realtime else now)
            self.ex.release(s)
            self.used -= s.bytes
            self.refs[s.req.key] -= 1

        def settle(p):
            """wait for iteration p and retire what finished or failed in it"""
            token, launched, finished = p
            flags = self.ex.wait(token) if mark else None
            fin = {id(s) for s in finished}
            for s in launched:
                if s.handle is None:  # retired by the previous wait (failed there)
                    continue
                bad = flags is not None and self.ex.failed(flags, s)
                if id(s) in fin:
                    retire(s, bad)
                elif bad and s.req.id in active:
                    del active[s.req.id]
                    retire(s, True)

        while future or waiting or active or pending:
            now = self.clock() - t0
            while future and (not realtime or future[0].arrival <= now):
                waiting.append(future.popleft())
            # first come, first served: stop at the first request that does not fit
            while waiting:
                req = waiting[0]
                gb, need = self._sizes(req)
                gneed = 0 if req.key in self.geoms else gb
                if gneed + need > self.budget:
                    raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.id, gneed + need))
                if not self._make_room(gneed + need, req.key):
                    break
                waiting.popleft()
                geom = self._build(req)
                self.used += need
                self.refs[req.key] += 1
                st.peak_bytes = max(st.peak_bytes, self.used + self.geom_bytes)
                req.admitted = self.clock() - t0
                active[req.id] = Slot(req, geom, self.ex.start(req, geom), bytes=need)
            if not active:
                if pending:
                    settle(pending)
                    pending = None
                elif future:
                    self.sleep(max(0.0, min(1e-3, future[0].arrival - (self.clock() - t0))))
                continue
            st.max_active = max(st.max_active, len(active))
            groups = collections.defaultdict(list)
            for s in active.values():
                groups[s.req.group].append(s)
            for grp in sorted(groups):
                self.ex.step_group(grp, groups[grp], self.dt)
            token = mark() if mark else None
            st.iterations += 1
            launched, finished = list(active.values()), []
            for s in launched:
                s.steps_done += 1
                st.updates += s.req.stages * s.geom.n_unique
                if s.steps_done >= s.req.steps:
                    finished.append(s)
                    del active[s.req.id]
            if not mark:
                self.ex.sync()
            if pending:
                settle(pending)
            pending = (token, launched, finished)
            if not mark:
                settle(pending)
                pending = None
        st.wall = self.clock() - t0
        return st
