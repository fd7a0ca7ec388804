"""numa_step's time loop as a captured HIP graph (Code example 1: the loop of
stages and filter, replayed per step) against direct launches of the same
kernels: bitwise equal, across replays of a kept capture, re-captures after a
change of dt, state or settings, and inside a caller's own stream capture."""
import pytest

from paper_1511_01561_amd import inputs
from test_gpu_parity import small_box_terrain, small_shell, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def pair(wl, seed=0):
    from paper_1511_01561_amd import numa
    a = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=3)
    b = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=3)
    b.set_step_graph(False)
    q = a.init_state(wl["ic"], inputs.device_noise(a.n_unique, seed))
    return a, b, q


def both(a, b, setting):
    setting(a)
    setting(b)


CASES = {
    "box-gather": (lambda: inputs.small_box(), lambda m: None),
    "box-terrain-recompute": (lambda: small_box_terrain(4), lambda m: m.set_metric(1)),
    "box-block": (lambda: inputs.box_workload(8, 4, 3, 4, 5e4, 2.5e4, 6e3, terrain=300.0,
                                              bubble_centre=(2e4, 1e4, 3e3), bubble_radius=4e3),
                  lambda m: (m.set_metric(1), m.set_stage(1))),
    "box-colour": (lambda: inputs.box_workload(4, 4, 2, 3, 2.5e4, 2.5e4, 4e3, terrain=300.0,
                                               bubble_centre=(1e4, 1e4, 2e3), bubble_radius=4e3),
                   lambda m: (m.set_metric(1), m.set_stage(2))),
    "box-ssp53-filter": (lambda: inputs.small_box(), lambda m: (m.set_integrator(1), m.set_filter(16, 1))),
    "shell": (lambda: small_shell(), lambda m: m.set_metric(1)),
}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_step_graph_equals_direct(torch_cuda, case, prec):
    torch = torch_cuda
    make, setting = CASES[case]
    a, b, q0 = pair(make())
    both(a, b, setting)
    qa, qb = q0.clone(), q0.clone()
    for rep, (dt, n) in enumerate([(0.05, 3), (0.05, 2), (0.05, 1), (0.04, 2)]):
        print("%s prec %d: call %d, dt %g, %d steps" % (case, prec, rep, dt, n), flush=True)
        a.step(qa, dt, n, prec=prec)
        b.step(qb, dt, n, prec=prec)
        junk = torch.randn(1 << 16, device="cuda:0", dtype=torch.float64).sum()  # eager work between
        torch.cuda.synchronize()
        assert torch.equal(qa, qb), rep
    assert not torch.equal(qa, q0)
    assert torch.isfinite(junk)
    # another state (re-capture), then the first again
    qc, qd = q0.clone(), q0.clone()
    a.step(qc, 0.05, 2, prec=prec)
    b.step(qd, 0.05, 2, prec=prec)
    a.step(qa, 0.05, 1, prec=prec)
    b.step(qb, 0.05, 1, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(qc, qd) and torch.equal(qa, qb)


def test_step_graph_follows_setting_changes(torch_cuda):
    """a kept capture is not replayed after the metric, the integrator or the
    filter changed"""
    torch = torch_cuda
    a, b, q0 = pair(small_box_terrain(4))
    qa, qb = q0.clone(), q0.clone()
    steps = [lambda m: m.set_metric(1), lambda m: m.set_integrator(1), lambda m: m.set_filter(12, 2),
             lambda m: m.set_filter(None), lambda m: m.set_metric(0), lambda m: m.set_integrator(0)]
    for k, change in enumerate(steps):
        a.step(qa, 0.05, 1)
        b.step(qb, 0.05, 1)
        both(a, b, change)
        a.step(qa, 0.05, 2)
        b.step(qb, 0.05, 2)
        torch.cuda.synchronize()
        assert torch.equal(qa, qb), k


def test_numa_step_inside_a_callers_capture(torch_cuda):
    """a caller capturing its stream records numa_step's direct launches;
    replays match eager steps"""
    torch = torch_cuda
    a, b, q0 = pair(small_box_terrain(4))
    a.set_metric(1)
    b.set_metric(1)
    qg, qe = q0.clone(), q0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        a.step(q0.clone(), 0.05, 1, stream=s)  # warm-up outside the capture
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            a.step(qg, 0.05, 2, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        b.step(qe, 0.05, 2)
        torch.cuda.synchronize()
        assert torch.equal(qg, qe), rep
