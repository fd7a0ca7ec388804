"""The Boyd-Vandeven filter (numa_filter) against the FP64 oracle's filter:
element filter matrix, J w weighting, DSS / M and the wall projection, FP64
within 1e-12 relative max-norm per variable group."""
import numpy as np
import pytest

from paper_1511_01561_amd import inputs
from test_gpu_parity import TOL64, Pair, assert_groups, small_shell

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def terrain_box(N, ne=(4, 3, 3), perz=False):
    return inputs.box_workload(*ne, N, 12e3, 9e3, 6e3, terrain=400.0, bubble_centre=(6e3, 4.5e3, 2e3),
                               bubble_radius=2.5e3, periodic_z=perz)


def filter_pair(p, q, order, cutoff, what):
    qg = p.dev(q)
    p.g.filter(qg, order, cutoff)
    qo = p.o.filter(q, order, cutoff)
    assert_groups(p.host(qg), qo, TOL64, what)
    return qo


@pytest.mark.parametrize("metric", [0, 1])
@pytest.mark.parametrize("N", range(1, 9))
def test_filter_parity_all_orders(torch_cuda, oracle_mod, N, metric):
    """Stored J w and J w from the column factors of the recomputed metric."""
    # 4 x 3 x 3 = 36 elements: a ragged last block for every elements-per-block count above 1
    p = Pair(terrain_box(N), oracle_mod)
    p.g.set_metric(metric)
    q = inputs.random_state(p.nu, seed=70 + N)
    cutoff = max(0, N // 2 - 1)
    qo = filter_pair(p, q, 12.0, cutoff, "filter N=%d cutoff=%d metric=%d" % (N, cutoff, metric))
    assert np.abs(qo - q).max() > 0


@pytest.mark.parametrize("order,cutoff", [(2.0, 0), (8.0, 1), (36.0, 2), (16.0, 3)])
def test_filter_parity_parameters(torch_cuda, oracle_mod, order, cutoff):
    p = Pair(terrain_box(4, perz=cutoff == 3), oracle_mod)
    filter_pair(p, inputs.random_state(p.nu, seed=80 + cutoff), order, cutoff,
                "filter p=%g s=%d" % (order, cutoff))


@pytest.mark.parametrize("N", [3, 4, 6])
def test_filter_parity_shell(torch_cuda, oracle_mod, N):
    p = Pair(small_shell(N), oracle_mod)
    q = p.o.init_state(p.wl["ic"], None)
    q[0] += inputs.random_state(p.nu, seed=90 + N)[0]
    filter_pair(p, q, 12.0, N // 2, "shell filter N=%d" % N)


@pytest.mark.parametrize("metric", [0, 1])
@pytest.mark.parametrize("N,ne", [(4, (5, 3, 2)), (6, (3, 2, 2)), (7, (3, 3, 1))])
def test_filter_parity_generic_box_path(torch_cuda, oracle_mod, N, ne, metric):
    """x extents that the box finish segments do not divide: element-major
    contributions and the generic DSS."""
    p = Pair(terrain_box(N, ne=ne), oracle_mod)
    p.g.set_metric(metric)
    filter_pair(p, inputs.random_state(p.nu, seed=60 + N), 12.0, 1, "generic-path filter N=%d ne=%s" % (N, ne))


def test_filter_full_cutoff_is_identity(torch_cuda, oracle_mod):
    """cutoff >= N: F = I, and the DSS of J w q / M returns the continuous
    state (its wall velocity already tangential) up to rounding."""
    p = Pair(terrain_box(5), oracle_mod)
    q = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 5))
    qg = p.dev(q)
    p.g.filter(qg, 12.0, 5)
    assert_groups(p.host(qg), q, 1e-14, "identity filter")


def test_filter_after_steps(torch_cuda, oracle_mod):
    """The time loop with the filter after every step (stages, then filter,
    then DSS), three steps, on the stored and the recomputed metric."""
    from paper_1511_01561_amd import numa
    p = Pair(terrain_box(4), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 6))
    qo = q0.copy()
    for _ in range(3):
        qo = p.o.filter(p.o.step(qo, 0.05, 1), 10.0, 1)
    for mode in (numa.METRIC_STORED, numa.METRIC_RECOMPUTE):
        p.g.set_metric(mode)
        qg = p.dev(q0)
        for _ in range(3):
            p.g.step(qg, 0.05, 1)
            p.g.filter(qg, 10.0, 1)
        assert_groups(p.host(qg), qo, TOL64, "step+filter x3 metric=%d" % mode)


def test_filter_on_side_stream(torch_cuda, oracle_mod):
    p = Pair(terrain_box(3), oracle_mod)
    q = inputs.random_state(p.nu, seed=95)
    s = torch_cuda.cuda.Stream()
    qg = p.dev(q)
    torch_cuda.cuda.synchronize()
    with torch_cuda.cuda.stream(s):
        p.g.filter(qg, 12.0, 1, stream=s)
    s.synchronize()
    assert_groups(qg.cpu().numpy(), p.o.filter(q, 12.0, 1), TOL64, "filter on a side stream")


def test_filter_rejects_bad_parameters(torch_cuda, oracle_mod):
    from paper_1511_01561_amd import numa
    p = Pair(terrain_box(2), oracle_mod)
    q = p.dev(inputs.random_state(p.nu, seed=96))
    before = q.clone()
    for order, cutoff in ((0.0, 1), (-3.0, 1), (float("nan"), 1), (12.0, -2)):
        with pytest.raises(numa.NumaError):
            p.g.filter(q, order, cutoff)
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(q, before)


def test_filter_full_size(torch_cuda, oracle_mod):
    """64 x 64 x 16 elements, N = 4, terrain 500 m: the whole filtered state,
    with the stored and the recomputed metric (the bench's mode)."""
    from paper_1511_01561_amd import numa
    p = Pair(inputs.gpu_box(), oracle_mod)
    q = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 7))
    q[0] += 1e-3 * inputs.random_state(p.nu, seed=97)[0]
    qo = p.o.filter(q, 16.0, 1)
    for mode in (numa.METRIC_STORED, numa.METRIC_RECOMPUTE):
        p.g.set_metric(mode)
        qg = p.dev(q)
        p.g.filter(qg, 16.0, 1)
        assert_groups(p.host(qg), qo, TOL64, "full-size filter metric=%d" % mode)


@pytest.mark.parametrize("which", ["box", "generic", "shell"])
def test_step_with_mesh_filter_is_step_then_filter(torch_cuda, oracle_mod, which):
    """numa_mesh_set_filter: every step of numa_step ends with the filter, the
    same kernels as calling numa_filter after each step (bitwise), and the
    oracle's stages-then-filter loop within the FP64 tolerance."""
    wl = {"box": terrain_box(4), "generic": terrain_box(4, ne=(5, 3, 2)), "shell": small_shell(4)}[which]
    p = Pair(wl, oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 8) if which != "shell" else None)
    a, b = p.dev(q0), p.dev(q0)
    p.g.set_filter(16.0, 1)
    p.g.step(a, 0.05, 3)
    p.g.set_filter(None)
    for _ in range(3):
        p.g.step(b, 0.05, 1)
        p.g.filter(b, 16.0, 1)
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(a, b)
    qo = q0.copy()
    for _ in range(3):
        qo = p.o.filter(p.o.step(qo, 0.05, 1), 16.0, 1)
    assert_groups(p.host(a), qo, TOL64, "%s step with mesh filter" % which)
    c = p.dev(q0)                        # the filter switched off again
    p.g.step(c, 0.05, 1)
    assert_groups(p.host(c), p.o.step(q0, 0.05, 1), TOL64, "%s step after the filter is off" % which)


def _box_item(n, N, seed, nz):
    Lx, H = n * 6250.0, nz * 1250.0
    return inputs.box_workload(n, n, nz, N, Lx, Lx, H, terrain=500.0, bubble_centre=(Lx / 3, Lx / 2, H / 2))


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_with_filter_equals_alone_bitwise(torch_cuda, prec):
    """Two items on one filtered mesh and one unfiltered item: each batched
    result is bitwise its result alone."""
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    wa, wb = _box_item(8, 4, 1, 4), _box_item(4, 4, 2, 3)
    ga = numa.Mesh(wa["mesh"], wa["phys"], prec_mask=3)
    gb = numa.Mesh(wb["mesh"], wb["phys"], prec_mask=3)
    ga.set_filter(12.0, 1)
    qs = [ga.init_state(wa["ic"], inputs.device_noise(ga.n_unique, 1)),
          ga.init_state(wa["ic"], inputs.device_noise(ga.n_unique, 2)),
          gb.init_state(wb["ic"], inputs.device_noise(gb.n_unique, 3))]
    meshes = [ga, ga, gb]
    ref = [q.clone() for q in qs]
    numa.step_batch([(g, q, numa.alloc_scratch(g, prec), 0.05) for g, q in zip(meshes, qs)], 3, prec)
    for g, r in zip(meshes, ref):
        g.step(r, 0.05, 3, prec=prec)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(qs, ref))
    # the filtered items differ from an unfiltered run
    ga.set_filter(None)
    u = ga.init_state(wa["ic"], inputs.device_noise(ga.n_unique, 1))
    ga.step(u, 0.05, 3, prec=prec)
    torch.cuda.synchronize()
    assert not torch.equal(u, qs[0])


def test_graph_with_filter_replays_match_eager(torch_cuda):
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    wa = _box_item(8, 4, 4, 4)
    g = numa.Mesh(wa["mesh"], wa["phys"], prec_mask=1)
    g.set_filter(10.0, 2)
    q = g.init_state(wa["ic"], inputs.device_noise(g.n_unique, 4))
    e = q.clone()
    s = torch.cuda.Stream()
    sg, se = numa.alloc_scratch(g, 0), numa.alloc_scratch(g, 0)
    graph = numa.Graph([(g, q, sg, 0.05)], 2, 0, s)
    for rep in range(3):
        graph.launch(s)
        s.synchronize()
        numa.step_batch([(g, e, se, 0.05)], 2, 0)
        junk = torch.randn(1 << 18, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert torch.equal(q, e), rep
    graph.close()
    del junk
