"""The recomputed box metric (NUMA_METRIC_RECOMPUTE) against the FP64 oracle,
whose metric is the stored isoparametric one: same tolerances as the stored
path (FP64 1e-12 per variable group, mixed 1e-5)."""
import numpy as np
import pytest

from paper_1511_01561_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, Pair, assert_groups, group_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def terrain_box(N, ne=(4, 3, 3), perz=False, h0=400.0):
    return inputs.box_workload(*ne, N, 12e3, 9e3, 6e3, terrain=h0, bubble_centre=(6e3, 4.5e3, 2e3),
                               bubble_radius=2.5e3, periodic_z=perz)


def recompute_pair(wl, oracle_mod):
    from paper_1511_01561_amd import numa
    p = Pair(wl, oracle_mod)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    return p


@pytest.mark.parametrize("N", range(1, 9))
def test_rhs_parity_recomputed_metric(torch_cuda, oracle_mod, N):
    p = recompute_pair(terrain_box(N), oracle_mod)
    q = inputs.random_state(p.nu, seed=40 + N)
    Co = p.o.rhs(q)
    assert_groups(p.host(p.g.rhs(p.dev(q))), Co, TOL64, "recomputed rhs N=%d" % N)


@pytest.mark.parametrize("N", [3, 4, 6, 8])
def test_rhs_mixed_recomputed_metric(torch_cuda, oracle_mod, N):
    from paper_1511_01561_amd import numa
    p = recompute_pair(terrain_box(N), oracle_mod)
    q = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 2))
    Co = p.o.rhs(q)
    assert_groups(p.host(p.g.rhs(p.dev(q), prec=numa.PREC_MIXED)), Co, TOLMIX, "recomputed mixed rhs N=%d" % N)


def test_undeformed_box_recomputed_metric(torch_cuda, oracle_mod):
    p = recompute_pair(inputs.small_box(), oracle_mod)
    q = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    assert_groups(p.host(p.g.rhs(p.dev(q))), p.o.rhs(q), TOL64, "undeformed recomputed rhs")
    # rest state stays exactly at rest
    assert np.all(p.host(p.g.rhs(p.dev(np.zeros((5, p.nu))))) == 0.0)


@pytest.mark.parametrize("N,ne,perz", [(2, (8, 4, 3), False), (4, (8, 4, 2), True), (5, (4, 3, 2), False),
                                       (4, (6, 4, 3), False)])
def test_step_parity_recomputed_metric(torch_cuda, oracle_mod, N, ne, perz):
    p = recompute_pair(terrain_box(N, ne, perz), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, N))
    qo = p.o.step(q0, 0.05, 3)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 3)
    assert_groups(p.host(qg), qo, TOL64, "recomputed step N=%d ne=%s" % (N, ne))


def test_full_size_recomputed_metric(torch_cuda, oracle_mod):
    p = recompute_pair(inputs.gpu_box(), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    assert_groups(p.host(p.g.rhs(p.dev(q0))), p.o.rhs(q0), TOL64, "full recomputed rhs")
    qo = p.o.step(q0, 0.05, 2)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    assert_groups(p.host(qg), qo, TOL64, "full recomputed 2-step state")


def test_recomputed_batch_equals_alone(torch_cuda):
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    objs = []
    for k, (n, nz) in enumerate(((8, 4), (4, 3), (12, 2))):
        wl = inputs.box_workload(n, n, nz, 4, n * 6250.0, n * 6250.0, nz * 1250.0, terrain=500.0,
                                 bubble_centre=(n * 3000.0, n * 3000.0, nz * 600.0))
        g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=1)
        g.set_metric(numa.METRIC_RECOMPUTE)
        q = g.init_state(wl["ic"], inputs.device_noise(g.n_unique, k))
        objs.append((g, q, numa.alloc_scratch(g, 0)))
    alone = [q.clone() for _, q, _ in objs]
    numa.step_batch([(g, q, s, 0.05) for g, q, s in objs], 2, 0)
    for (g, _, _), a in zip(objs, alone):
        g.step(a, 0.05, 2)
    torch.cuda.synchronize()
    assert all(torch.equal(q, a) for (_, q, _), a in zip(objs, alone))


# ------------------------------------------------------------------- shell
def shell_pair(N, oracle_mod, ne=3, nz=2):
    from paper_1511_01561_amd import numa
    from test_gpu_parity import Pair
    p = Pair(inputs.shell_workload(ne=ne, nz=nz, N=N, seed=0), oracle_mod)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    return p


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
def test_shell_rhs_parity_recomputed_metric(torch_cuda, oracle_mod, N):
    """The shell's metric and gravity formed every stage from the column and
    layer factors: FP64 RHS against the oracle (stored isoparametric metric)
    with an arbitrary non-tangential wind."""
    p = shell_pair(N, oracle_mod, ne=2 if N > 5 else 3)
    q = p.o.init_state(p.wl["ic"], None)
    q[1:4] += 0.5 * inputs.noise(p.nu, 7)
    assert_groups(p.host(p.g.rhs(p.dev(q))), p.o.rhs(q), TOL64, "shell recomputed rhs N=%d" % N)


def test_shell_rest_state_exactly_zero_recomputed_metric(torch_cuda, oracle_mod):
    p = shell_pair(4, oracle_mod)
    assert np.all(p.host(p.g.rhs(p.dev(np.zeros((5, p.nu))))) == 0.0)


def test_shell_mixed_rhs_recomputed_metric(torch_cuda, oracle_mod):
    """Mixed precision on the balanced jet, against the term scale (the
    rho' and theta' increments are nearly cancelled sums)."""
    from paper_1511_01561_amd import numa
    from test_gpu_parity import scale_err
    p = shell_pair(4, oracle_mod)
    q = p.o.init_state(p.wl["ic"], None)
    Co = p.o.rhs(q)
    Cg = p.host(p.g.rhs(p.dev(q), prec=numa.PREC_MIXED))
    e = scale_err(Cg, Co, p.o.rhs_scale(q))
    print("shell recomputed mixed rhs, term-scale norm", {k: "%.2e" % v for k, v in e.items()})
    assert max(e.values()) <= TOLMIX
    assert group_err(Cg, Co)["u"] <= TOLMIX


@pytest.mark.parametrize("N", [3, 4])
def test_shell_step_parity_recomputed_metric(torch_cuda, oracle_mod, N):
    p = shell_pair(N, oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], None)
    qo = p.o.step(q0, 0.5, 5)
    qg = p.dev(q0)
    p.g.step(qg, 0.5, 5)
    assert_groups(p.host(qg), qo, TOL64, "shell recomputed step N=%d" % N)


def test_shell_full_size_recomputed_metric(torch_cuda, oracle_mod):
    """The 6x32x32x10, N = 4 shell: one FP64 step of the recomputed-metric
    path against the oracle."""
    from test_gpu_parity import Pair
    from paper_1511_01561_amd import numa
    p = Pair(inputs.shell_workload(32, 10, 4, seed=0), oracle_mod)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    q0 = p.o.init_state(p.wl["ic"], None)
    qo = p.o.step(q0, 0.5, 1)
    qg = p.dev(q0)
    p.g.step(qg, 0.5, 1)
    assert_groups(p.host(qg), qo, TOL64, "full shell recomputed step")


@pytest.mark.parametrize("N,ne,perz", [(1, (4, 3, 3), 0), (2, (8, 3, 2), 0), (3, (4, 3, 3), 1), (4, (4, 3, 3), 0),
                                       (5, (4, 5, 1), 0), (6, (4, 3, 2), 1), (7, (2, 3, 2), 0), (8, (2, 2, 2), 0)])
def test_step_parity_all_orders_recomputed_metric(torch_cuda, oracle_mod, N, ne, perz):
    """Every order through the recomputed-metric stage kernels (several
    elements per workgroup, element counts that leave the last workgroup of
    the mesh partly empty), FP64 against the oracle and the mixed path within
    the mixed tolerance of it."""
    from paper_1511_01561_amd import numa
    p = recompute_pair(terrain_box(N, ne, perz), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, N))
    qo = p.o.step(q0, 0.05, 2)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    assert_groups(p.host(qg), qo, TOL64, "recomputed step N=%d ne=%s" % (N, ne))
    qm = p.dev(q0)
    p.g.step(qm, 0.05, 2, prec=numa.PREC_MIXED)
    e = group_err(p.host(qm) - q0, qo - q0)
    print("recomputed mixed 2-step increment", {k: "%.1e" % v for k, v in e.items()})
    assert max(e.values()) <= TOLMIX


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("N", [3, 4, 6])
def test_recomputed_batch_equals_alone_ragged(torch_cuda, prec, N):
    """Items whose element counts are not multiples of the elements per
    workgroup, batched: bitwise the same as each alone, both precisions."""
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    objs = []
    for k, ne in enumerate(((4, 3, 3), (8, 5, 1), (4, 3, 1))):
        wl = inputs.box_workload(*ne, N, ne[0] * 6250.0, ne[1] * 6250.0, ne[2] * 1250.0, terrain=500.0,
                                 bubble_centre=(ne[0] * 3000.0, ne[1] * 3000.0, ne[2] * 600.0))
        g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=3)
        g.set_metric(numa.METRIC_RECOMPUTE)
        q = g.init_state(wl["ic"], inputs.device_noise(g.n_unique, 30 + k))
        objs.append((g, q, numa.alloc_scratch(g, prec)))
    alone = [q.clone() for _, q, _ in objs]
    numa.step_batch([(g, q, s, 0.05) for g, q, s in objs], 2, prec)
    for (g, _, _), a in zip(objs, alone):
        g.step(a, 0.05, 2, prec=prec)
    torch.cuda.synchronize()
    assert all(torch.equal(q, a) for (_, q, _), a in zip(objs, alone))


def test_full_size_largest_order(torch_cuda, oracle_mod):
    """The largest configuration of the order sweep, 64x64x16 at N = 8
    (33.8 M unique nodes), in the launch configuration the benchmark times:
    one FP64 step against the oracle, and the mixed step within the mixed
    tolerance of it."""
    from paper_1511_01561_amd import numa
    p = recompute_pair(inputs.gpu_box(8), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    qo = p.o.step(q0, 0.05, 1)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 1)
    assert_groups(p.host(qg), qo, TOL64, "N=8 full-size step")
    qm = p.dev(q0)
    p.g.step(qm, 0.05, 1, prec=numa.PREC_MIXED)
    e = group_err(p.host(qm) - q0, qo - q0)
    print("N=8 full-size mixed increment", {k: "%.1e" % v for k, v in e.items()})
    assert max(e.values()) <= TOLMIX


@pytest.mark.parametrize("which", ["box4", "box8", "shell4"])
def test_folded_stages_keep_the_state_at_zero_dt(torch_cuda, which):
    """FP64 stages fold q_s into the contributions (J w (q_s + cdt R)); with
    dt = 0 a step returns M^-1 sum(J w q_s), which is q_s to rounding only if
    the mass is formed from the same J w as the contributions.  With the
    recomputed metric that is J w from the column (and layer) factors, not
    the stored isoparametric J w, which differs from it by ~1e-14 and would
    scale the state by that much at every stage (60 stages here: 1e-13 at
    N = 4, 2e-13 at N = 8 against ~3e-15 with the consistent mass)."""
    from paper_1511_01561_amd import numa
    from test_gpu_parity import small_shell
    wl = {"box4": terrain_box(4), "box8": terrain_box(8), "shell4": small_shell(4)}[which]
    for metric in (numa.METRIC_STORED, numa.METRIC_RECOMPUTE):
        g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=1)
        g.set_metric(metric)
        q = g.init_state(wl["ic"], inputs.device_noise(g.n_unique, 5) if which != "shell4" else None)
        q0 = q.clone()
        g.step(q, 0.0, 20)
        a, b = q.cpu().numpy(), q0.cpu().numpy()
        e = group_err(a, b)
        print(which, "metric", metric, {k: "%.1e" % v for k, v in e.items()}, flush=True)
        assert max(e.values()) <= 2e-14, (which, metric, e)
