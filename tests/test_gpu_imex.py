"""The 1D-IMEX leap-frog step (numa_imex_step) against the oracle's, on the box
and the shell: the explicit leap-frog stage, the per-line vertical solve (the
library eliminates rho' and theta' and solves a band system for the vertical
velocity; the oracle solves each line's full system densely) and the
Robert-Asselin filter.  FP64 states within 1e-12 relative
max-norm per variable group; the mixed-precision explicit stage within 1e-5
of the increment."""
import numpy as np
import pytest

from paper_1511_01561_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, Pair, assert_groups, group_err, small_shell

pytestmark = pytest.mark.gpu


def Pair_(wl, oracle_mod):
    """Oracle and library mesh; the workspace holds the IMEX line factors."""
    return Pair(wl, oracle_mod, prec_mask=7)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def terrain_box(N, ne=(4, 3, 3), perz=False):
    return inputs.box_workload(*ne, N, 12e3, 9e3, 6e3, terrain=400.0, bubble_centre=(6e3, 4.5e3, 2e3),
                               bubble_radius=2.5e3, periodic_z=perz)


def imex_case(p, dt, ra, nsteps, seed, prec=0):
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, seed))
    qm = p.o.step(q0, -dt, 1)                    # the level one step back
    oa, ob = p.o.imex_step(qm, q0, dt, ra, nsteps)
    ga, gb = p.dev(qm), p.dev(q0)
    p.g.imex_step(ga, gb, dt, ra, nsteps, prec=prec)
    return q0, (oa, ob), (p.host(ga), p.host(gb))


@pytest.mark.parametrize("metric", [0, 1])
@pytest.mark.parametrize("N", range(1, 9))
def test_imex_parity_all_orders(torch_cuda, oracle_mod, N, metric):
    p = Pair_(terrain_box(N), oracle_mod)
    p.g.set_metric(metric)
    _, (oa, ob), (ga, gb) = imex_case(p, 0.1, 0.05, 3, 10 + N)
    assert_groups(gb, ob, TOL64, "imex q^{n+1} N=%d metric=%d" % (N, metric))
    assert_groups(ga, oa, TOL64, "imex filtered q^n N=%d metric=%d" % (N, metric))


@pytest.mark.parametrize("ne", [(5, 3, 2), (3, 2, 4)])
def test_imex_parity_generic_box_path(torch_cuda, oracle_mod, ne):
    """x extents that the box finish segments do not divide: the explicit
    stage runs through the general kernels."""
    p = Pair_(terrain_box(4, ne=ne), oracle_mod)
    _, (oa, ob), (ga, gb) = imex_case(p, 0.1, 0.1, 2, 20)
    assert_groups(gb, ob, TOL64, "imex generic ne=%s" % (ne,))
    assert_groups(ga, oa, TOL64, "imex generic filtered ne=%s" % (ne,))


def test_imex_forward_start_and_no_filter(torch_cuda, oracle_mod):
    """qprev = qcur (a forward first step), ra = 0."""
    p = Pair_(inputs.small_box(), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 3))
    oa, ob = p.o.imex_step(q0, q0, 0.2, 0.0, 4)
    ga, gb = p.dev(q0), p.dev(q0)
    p.g.imex_step(ga, gb, 0.2, 0.0, 4)
    assert_groups(p.host(gb), ob, TOL64, "imex forward start")
    assert_groups(p.host(ga), oa, TOL64, "imex forward start, previous level")


def test_imex_mixed_precision_explicit_stage(torch_cuda, oracle_mod):
    from paper_1511_01561_amd import numa
    p = Pair_(terrain_box(4), oracle_mod)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    q0, (_, ob), (_, gb) = imex_case(p, 0.1, 0.05, 2, 30, prec=numa.PREC_MIXED)
    e = group_err(gb - q0, ob - q0)
    print("imex mixed increment", {k: "%.1e" % v for k, v in e.items()}, flush=True)
    assert max(e.values()) <= TOLMIX


def test_imex_stable_beyond_the_vertical_acoustic_limit(torch_cuda, oracle_mod):
    """Vertical spacing 8x finer than horizontal, dt = 2 s (explicit SSP-RK3
    blows up at 0.5 s on this mesh): 20 steps bounded and equal to the oracle."""
    wl = inputs.box_workload(4, 4, 8, 4, 40e3, 40e3, 5e3, terrain=0.0, bubble_centre=(20e3, 20e3, 2e3),
                             bubble_radius=2e3)
    p = Pair_(wl, oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    oa, ob = p.o.imex_step(q0, q0, 2.0, 0.05, 20)
    ga, gb = p.dev(q0), p.dev(q0)
    p.g.imex_step(ga, gb, 2.0, 0.05, 20)
    gb = p.host(gb)
    assert np.all(np.isfinite(gb))
    assert_groups(gb, ob, 1e-11, "imex 20 steps at dt = 2 s")


@pytest.mark.parametrize("N", [2, 3, 4, 6])
def test_imex_parity_shell(torch_cuda, oracle_mod, N):
    """Radial lines of the cubed-sphere shell: the radial velocity component
    is corrected, r^2 enters the radial divergence."""
    p = Pair_(small_shell(N), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], None)
    qm = p.o.step(q0, -2.0, 1)
    oa, ob = p.o.imex_step(qm, q0, 2.0, 0.05, 3)
    ga, gb = p.dev(qm), p.dev(q0)
    p.g.imex_step(ga, gb, 2.0, 0.05, 3)
    assert_groups(p.host(gb), ob, TOL64, "shell imex q^{n+1} N=%d" % N)
    assert_groups(p.host(ga), oa, TOL64, "shell imex filtered q^n N=%d" % N)


def test_imex_shell_thin_layers_large_dt(torch_cuda, oracle_mod):
    """1.25 km layers under ~840 km horizontal spacing, dt = 20 s (explicit
    SSP-RK3 blows up at 2 s): 10 steps equal to the oracle."""
    p = Pair_(inputs.shell_workload(ne=3, nz=8, N=4, seed=0, H=10e3), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], None)
    oa, ob = p.o.imex_step(q0, q0, 20.0, 0.05, 10)
    ga, gb = p.dev(q0), p.dev(q0)
    p.g.imex_step(ga, gb, 20.0, 0.05, 10)
    gb = p.host(gb)
    assert np.all(np.isfinite(gb))
    assert_groups(gb, ob, 1e-11, "shell imex 10 steps at dt = 20 s")


def test_imex_refusals(torch_cuda, oracle_mod):
    from paper_1511_01561_amd import numa
    cases = [Pair_(terrain_box(3, perz=True), oracle_mod)]
    for p in cases:
        q = p.dev(np.zeros((5, p.nu)))
        r = p.dev(np.zeros((5, p.nu)))
        with pytest.raises(numa.NumaError, match="walls"):
            p.g.imex_step(q, r, 0.1, 0.0, 1)
    p = Pair_(terrain_box(2), oracle_mod)
    q = p.dev(np.zeros((5, p.nu)))
    r = p.dev(np.zeros((5, p.nu)))
    for dt, ra in ((0.1, -0.1), (0.1, 1.0), (float("nan"), 0.0)):
        with pytest.raises(numa.NumaError):
            p.g.imex_step(q, r, dt, ra, 1)
    with pytest.raises(numa.NumaError):
        p.g.imex_step(q, q, 0.1, 0.0, 1)
    # a workspace without the line factors
    p3 = Pair(terrain_box(2), oracle_mod, prec_mask=3)
    with pytest.raises(numa.NumaError, match="NUMA_WS_IMEX"):
        p3.g.imex_step(p3.dev(np.zeros((5, p3.nu))), p3.dev(np.zeros((5, p3.nu))), 0.1, 0.0, 1)
    # 161 levels at N = 8 need more than 64 KB of LDS per line
    wl = inputs.box_workload(2, 2, 20, 8, 4e3, 4e3, 20e3)
    g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=5)
    z = g.init_state(wl["ic"], None)
    with pytest.raises(numa.NumaError, match="LDS"):
        g.imex_step(z.clone(), z, 0.1, 0.0, 1)


def test_imex_full_size_sampled_lines(torch_cuda, oracle_mod):
    """64 x 64 x 16 elements, N = 4, terrain 500 m, recomputed metric: one step;
    the oracle solves about 100 sampled vertical lines, some through the warm
    bubble so that every variable group is populated."""
    from paper_1511_01561_amd import numa
    p = Pair_(inputs.gpu_box(), oracle_mod)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 1))
    rng = np.random.default_rng(5)
    nh = p.o.n_horiz
    ni = int(round(np.sqrt(nh)))
    through_bubble = [gi + ni * gj for gi in range(116, 141, 4) for gj in range(116, 141, 6)]   # (200, 200) km
    lines = np.unique(np.concatenate([rng.integers(0, nh, 60), [0, 1, 255, 256, nh - 1], through_bubble]))
    oa, ob = p.o.imex_step(q0, q0, 0.2, 0.05, 1, lines=lines)
    ga, gb = p.dev(q0), p.dev(q0)
    p.g.imex_step(ga, gb, 0.2, 0.05, 1)
    ga, gb = p.host(ga), p.host(gb)
    idx = (lines[None, :] + nh * np.arange(p.o.n_levels)[:, None]).ravel()
    for name, a, b in (("q^{n+1}", gb, ob), ("filtered q^n", ga, oa)):
        assert_groups(a[:, idx], b[:, idx], TOL64, "full-size imex %s, sampled lines" % name)


def test_imex_zero_steps_leave_states_untouched(torch_cuda, oracle_mod):
    p = Pair_(terrain_box(3), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 9))
    a, b = p.dev(q0), p.dev(2.0 * q0)
    p.g.imex_step(a, b, 0.1, 0.05, 0)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(p.host(a), q0) and np.array_equal(p.host(b), 2.0 * q0)
