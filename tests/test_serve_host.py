"""Scheduling logic of the serving loop on the host (no GPU): admission by
memory footprint, first-come-first-served order, one batched step per order
group and iteration, completion after exactly K steps, memory release."""
import pytest

from paper_1511_01561_amd.serve import Request, Server


class FakeGeom:
    def __init__(self, n_unique):
        self.n_unique = n_unique


class FakeExecutor:
    """Counts steps per request; every step_group call advances a fake clock."""

    def __init__(self, clock):
        self.clock = clock
        self.log = []
        self.geoms = {}
        self.live = 0

    def geometry(self, req):
        return self.geoms.setdefault(req.key, FakeGeom(req.workload["mesh"]["ne"][0] ** 3))

    def request_bytes(self, req, geom):
        return 100 * geom.n_unique

    def start(self, req, geom):
        self.live += 1
        return {"steps": 0}

    def step_group(self, group, slots, dt):
        assert len({s.req.group for s in slots}) == 1 and slots[0].req.group == group
        self.log.append((self.clock.t, group, tuple(s.req.id for s in slots)))
        for s in slots:
            s.handle["steps"] += 1
        self.clock.t += 0.001 * len(slots)

    def sync(self):
        pass

    def finish(self, slot, keep):
        return slot.handle["steps"]

    def release(self, slot):
        self.live -= 1


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 1e-4)


def req(i, arrival, n=8, order=4, steps=5):
    wl = dict(mesh=dict(kind=0, N=order, ne=(n, n, n), periodic=(1, 1, 0), extent=(1., 1., 1.), h0=0.0),
              phys={}, ic={})
    return Request(id=i, arrival=arrival, workload=wl, noise_seed=i, steps=steps)


def test_every_request_completes_after_exactly_k_steps_and_memory_is_released():
    clk = Clock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=10 ** 9, clock=clk, sleep=clk.sleep, keep_states=True)
    reqs = [req(i, 0.002 * i, n=4 + (i % 3), order=3 + (i % 2), steps=3 + i % 4) for i in range(12)]
    st = srv.run(reqs)
    assert len(st.latencies) == 12
    for r in reqs:
        assert r.state == r.steps and r.done >= r.admitted >= r.arrival
    assert srv.used == 0 and ex.live == 0


def test_admission_by_footprint_is_fifo_and_never_exceeds_budget():
    clk = Clock()
    ex = FakeExecutor(clk)
    budget = 100 * (8 ** 3) * 2 + 10          # room for two 8^3 requests at a time
    srv = Server(ex, budget_bytes=budget, clock=clk, sleep=clk.sleep)
    reqs = [req(i, 0.0, n=8, steps=4) for i in range(6)]
    st = srv.run(reqs)
    assert st.peak_bytes <= budget and st.max_active == 2
    admitted = sorted(reqs, key=lambda r: r.admitted)
    assert [r.id for r in admitted] == list(range(6))
    # a waiting request is admitted in the iteration after a slot frees up
    for a, b in zip(reqs[:-2], reqs[2:]):
        assert b.admitted >= a.done


def test_groups_by_order_and_continuous_batching():
    clk = Clock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=10 ** 9, clock=clk, sleep=clk.sleep)
    reqs = [req(0, 0.0, order=4, steps=10), req(1, 0.0, order=5, steps=10), req(2, 0.0035, order=4, steps=3)]
    srv.run(reqs)
    groups = [g for g in ex.log]
    # orders never mix in one launch; request 2 joins request 0's batch while 0 is running
    assert all(len(set(reqs[i].order for i in ids)) == 1 for _, _, ids in groups)
    assert any(ids == (0, 2) for _, g, ids in groups if g == (4, 0))
    assert reqs[2].done < reqs[0].done


def test_integrators_never_share_a_launch_and_updates_count_stages():
    clk = Clock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=10 ** 9, clock=clk, sleep=clk.sleep)
    reqs = [req(0, 0.0, order=4, steps=4), req(1, 0.0, order=4, steps=4), req(2, 0.0, order=4, steps=4)]
    reqs[1].integrator = 1
    reqs[2].filter = (16.0, 1)
    st = srv.run(reqs, realtime=False)
    launches = [(g, ids) for _, g, ids in ex.log]
    assert all(ids == (0, 2) for g, ids in launches if g == (4, 0))      # a filter does not split a group
    assert all(ids == (1,) for g, ids in launches if g == (4, 1))
    assert len({r.key for r in reqs}) == 3                              # but it needs its own geometry
    n = reqs[0].workload["mesh"]["ne"][0] ** 3
    assert st.updates == 4 * n * (3 + 5 + 3)


def test_request_larger_than_budget_is_refused():
    clk = Clock()
    srv = Server(FakeExecutor(clk), budget_bytes=1000, clock=clk, sleep=clk.sleep)
    with pytest.raises(ValueError):
        srv.run([req(0, 0.0, n=8)])


def test_back_to_back_mode_ignores_arrival_times():
    clk = Clock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget_bytes=10 ** 9, clock=clk, sleep=clk.sleep)
    reqs = [req(i, 100.0 + i, steps=2) for i in range(4)]
    st = srv.run(reqs, realtime=False)
    assert st.wall < 1.0 and len(st.latencies) == 4
