"""The split DSS of a fused stage (NUMA_STAGE_SPLIT) against the oracle.

The element kernel's workgroup holds a run of consecutive elements along x:
it adds the copies of the x faces shared inside the run and finishes the
nodes whose copies it then holds; the element faces in y and z and the x
faces that start a run are finished by a second kernel from contributions
written in rows along x.  The meshes cover runs that stay in one row of
elements, runs that wrap onto the next row or layer (nx not a multiple of,
or smaller than, the run length: 2 elements at N = 8, 4 at N = 7, 5 at
N = 6, 7 at N = 5, 10 at N = 4, 16 at N = 3, 28 at N = 2, 64 at N = 1),
walls and periodic z.  FP64 takes the split DSS up to N = 8, mixed precision
up to N = 4 (above, the gather, which these tests then check as well).  FP64 within 1e-12 and mixed
precision within 1e-5, relative max-norm per variable group, for the
right-hand side (numa_stage_rhs), for steps of both integrators (the
five-stage one writes a stage over its own input), for the filtered step and
the explicit stage of the IMEX step; resume and batching bitwise.
"""
import numpy as np
import pytest

from paper_1511_01561_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, Pair, assert_groups, group_err  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


# (N, elements, periodic z)
CASES = [
    (4, (20, 3, 2), False),   # two whole runs per row
    (4, (12, 3, 3), False),   # runs wrap onto the next row
    (4, (4, 3, 2), False),    # nx < run: a run spans rows and layers
    (4, (8, 4, 4), True),     # periodic z
    (3, (16, 2, 3), False),
    (3, (6, 5, 2), True),
    (2, (30, 2, 2), False),
    (2, (5, 3, 3), True),
    (1, (4, 4, 3), False),
    (1, (3, 2, 2), True),
    (5, (7, 3, 2), False),    # FP64 only (mixed precision takes the gather)
    (5, (3, 2, 3), True),
    (6, (5, 3, 2), False),
    (6, (4, 2, 2), True),
    (7, (5, 2, 2), False),
    (7, (3, 2, 2), True),
    (8, (4, 2, 2), False),
    (8, (2, 2, 2), True),
]


def _wl(N, ne, perz):
    nx, ny, nz = ne
    return inputs.box_workload(nx, ny, nz, N, nx * 3.0e3, ny * 2.5e3, nz * 1.5e3, terrain=350.0,
                               bubble_centre=(nx * 1.5e3, ny * 1.25e3, 1.5e3), bubble_radius=3.0e3,
                               periodic_z=perz)


def _pair(wl, oracle_mod, prec_mask=3):
    from paper_1511_01561_amd import numa
    p = Pair(wl, oracle_mod, prec_mask=prec_mask)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    p.g.set_stage(numa.STAGE_SPLIT)
    return p


@pytest.mark.parametrize("N,ne,perz", CASES)
def test_split_stage_rhs(torch_cuda, oracle_mod, N, ne, perz):
    from paper_1511_01561_amd import numa
    print("split rhs N=%d ne=%s perz=%d" % (N, ne, perz), flush=True)
    p = _pair(_wl(N, ne, perz), oracle_mod)
    q = inputs.random_state(p.nu, seed=200 + N)
    Ro = p.o.dss(p.o.rhs(q), 3)
    qd = p.dev(q)
    assert_groups(p.host(p.g.stage_rhs(qd, prec=numa.PREC_FP64)), Ro, TOL64, "split rhs N=%d ne=%s" % (N, ne))
    assert_groups(p.host(p.g.stage_rhs(qd, prec=numa.PREC_MIXED)), Ro, TOLMIX, "split mixed rhs N=%d ne=%s" % (N, ne))


@pytest.mark.parametrize("N,ne,perz", CASES)
def test_split_step(torch_cuda, oracle_mod, N, ne, perz):
    """Two SSP-RK3 steps (FP64 stages fold q_s into the contributions away
    from the walls, in the face rows and in the run-interior nodes alike);
    mixed precision within 1e-5 of the increment."""
    from paper_1511_01561_amd import numa
    print("split step N=%d ne=%s perz=%d" % (N, ne, perz), flush=True)
    p = _pair(_wl(N, ne, perz), oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, N))
    qo = p.o.step(q0, 0.05, 2)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    assert_groups(p.host(qg), qo, TOL64, "split step N=%d ne=%s" % (N, ne))
    qm = p.dev(q0)
    p.g.step(qm, 0.05, 2, prec=numa.PREC_MIXED)
    e = group_err(p.host(qm) - q0, qo - q0)
    print("split mixed 2-step increment", {k: "%.1e" % v for k, v in e.items()}, flush=True)
    assert max(e.values()) <= TOLMIX


@pytest.mark.parametrize("N,ne,perz", [(4, (12, 3, 3), False), (3, (6, 5, 2), True), (2, (5, 3, 3), False)])
def test_split_ssp53_step(torch_cuda, oracle_mod, N, ne, perz):
    """The five-stage integrator: its fourth stage writes the buffer it
    reads (the split stage finishes run-interior nodes while other
    workgroups gather, which only this workgroup reads)."""
    from paper_1511_01561_amd import numa
    print("split ssp53 N=%d ne=%s" % (N, ne), flush=True)
    p = _pair(_wl(N, ne, perz), oracle_mod)
    p.g.set_integrator(numa.RK_SSP53)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 30 + N))
    qo = p.o.step(q0, 0.05, 2, scheme="ssp53")
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    assert_groups(p.host(qg), qo, TOL64, "split ssp53 N=%d" % N)


def test_split_filtered_step(torch_cuda, oracle_mod):
    """A step that ends with the Boyd-Vandeven filter: the split stages, then
    the filter with its own DSS."""
    print("split filtered step", flush=True)
    p = _pair(_wl(4, (12, 3, 3), False), oracle_mod)
    p.g.set_filter(16.0, 1)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 3))
    qo = q0
    for _ in range(2):
        qo = p.o.filter(p.o.step(qo, 0.05, 1), 16.0, 1)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    p.g.set_filter(None)
    assert_groups(p.host(qg), qo, TOL64, "split filtered step")


def test_split_imex_step(torch_cuda, oracle_mod):
    """The IMEX step's explicit leap-frog stage (a = 1, b = 0: no q_s term)
    through the split stage."""
    from paper_1511_01561_amd import numa
    print("split imex step", flush=True)
    p = _pair(_wl(4, (12, 3, 3), False), oracle_mod, prec_mask=3 | numa.WS_IMEX)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 4))
    dt, ra = 0.2, 0.05
    qm = p.o.step(q0, -dt, 1)
    oa, ob = p.o.imex_step(qm, q0, dt, ra, 3)
    ga, gb = p.dev(qm), p.dev(q0)
    p.g.imex_step(ga, gb, dt, ra, 3)
    assert_groups(p.host(ga), oa, TOL64, "split imex previous level")
    assert_groups(p.host(gb), ob, TOL64, "split imex current level")


@pytest.mark.parametrize("prec", [0, 1])
def test_split_resume_and_batch_bitwise(torch_cuda, oracle_mod, prec):
    """step(4) == step(2) step(2) bit for bit, and a batch that mixes split
    meshes of different run layouts with a gather mesh gives every item its
    result alone."""
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    print("split resume/batch prec=%d" % prec, flush=True)
    meshes = []
    for k, ne in enumerate(((12, 3, 3), (4, 3, 2), (20, 3, 2), (12, 3, 3))):
        wl = _wl(4, ne, False)
        g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=3)
        g.set_metric(numa.METRIC_RECOMPUTE)
        g.set_stage(numa.STAGE_SPLIT if k < 3 else numa.STAGE_GATHER)
        q = g.init_state(wl["ic"], inputs.device_noise(g.n_unique, len(meshes)))
        meshes.append((g, q))
    g0, q0 = meshes[0]
    a, b = q0.clone(), q0.clone()
    g0.step(a, 0.05, 4, prec=prec)
    g0.step(b, 0.05, 2, prec=prec)
    g0.step(b, 0.05, 2, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    alone = []
    for g, q in meshes:
        a = q.clone()
        g.step(a, 0.05, 3, prec=prec)
        alone.append(a)
    items = [(g, q.clone(), numa.alloc_scratch(g, prec), 0.05) for g, q in meshes]
    numa.step_batch(items, 3, prec)
    torch.cuda.synchronize()
    for k, (it, a) in enumerate(zip(items, alone)):
        assert torch.equal(it[1], a), k


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7, 8])
def test_split_full_size(torch_cuda, oracle_mod, N):
    """The 64 x 64 x 16 box: the right-hand side at 1e-12 (FP64) and 1e-5
    (mixed), and one FP64 step against the oracle's."""
    from paper_1511_01561_amd import numa
    print("split full size N=%d" % N, flush=True)
    p = _pair(inputs.gpu_box(N), oracle_mod)
    q = inputs.random_state(p.nu, seed=7)
    Ro = p.o.dss(p.o.rhs(q), 3)
    qd = p.dev(q)
    assert_groups(p.host(p.g.stage_rhs(qd)), Ro, TOL64, "split full rhs N=%d" % N)
    assert_groups(p.host(p.g.stage_rhs(qd, prec=numa.PREC_MIXED)), Ro, TOLMIX, "split full mixed rhs N=%d" % N)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    qo = p.o.step(q0, 0.05, 1)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 1)
    assert_groups(p.host(qg), qo, TOL64, "split full step N=%d" % N)
