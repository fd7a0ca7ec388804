"""The fused block stage (NUMA_STAGE_BLOCK: a workgroup per block of element
columns: element right-hand side, DSS inside the block, M^-1, wall projection
and stage update in one kernel; the nodes shared between blocks summed by a
second kernel) and the colour passes (NUMA_STAGE_COLOUR: 8 colour launches
add J w R into a unique-node accumulator, a pointwise kernel finishes)
against the oracle.

The block stage runs for box meshes with no-flux walls, the recomputed metric, N = 2..4,
nx a multiple of 4 (N = 4) or 8 (N = 2, 3) and ny even.  The cases cover
blocks one layer tall (a z face between every layer), taller blocks (levels
carried from layer to layer, and z faces), a single block in x and y (the
western halo is the block's own last element column), and the full
64 x 64 x 16 box (one block per column, no z face).  The colour passes need
N <= 4 and nx, ny, nz even; cases a mode does not take run the gather stage.
FP64 within 1e-12 and mixed precision within 1e-5, relative max-norm per
variable group.
"""
import numpy as np
import pytest

from paper_1511_01561_amd import inputs
from test_gpu_parity import TOL64, TOLMIX, Pair, assert_groups, group_err, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu

# (N, elements): block layers chosen by the library from the mesh size
CASES = [
    (4, (8, 4, 3)),    # 2 x 2 blocks of one layer: z faces between all layers
    (4, (64, 32, 4)),  # 16 x 16 blocks of two layers: carried level and one z face
    (4, (4, 2, 2)),    # one block: halo and y faces wrap onto the block itself
    (3, (16, 4, 3)),
    (3, (8, 2, 2)),
    (2, (8, 4, 2)),
    (4, (8, 4, 4)),    # even nz: the colour passes (odd nz falls back to the gather stage)
    (3, (8, 6, 2)),
    (1, (4, 4, 2)),    # colour passes only (the block stage needs N >= 2)
]


def _wl(N, ne):
    nx, ny, nz = ne
    return inputs.box_workload(nx, ny, nz, N, nx * 3.0e3, ny * 2.5e3, nz * 1.5e3, terrain=350.0,
                               bubble_centre=(nx * 1.5e3, ny * 1.25e3, 1.5e3), bubble_radius=3.0e3)


def _pair(N, ne, oracle_mod, mode=1):
    from paper_1511_01561_amd import numa
    p = Pair(_wl(N, ne), oracle_mod)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    p.g.set_stage(mode)
    return p


MODES = [1, 2, 3]  # NUMA_STAGE_BLOCK, NUMA_STAGE_COLOUR, NUMA_STAGE_SPLIT


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("N,ne", CASES)
def test_pencil_stage_rhs(torch_cuda, oracle_mod, N, ne, mode):
    from paper_1511_01561_amd import numa
    p = _pair(N, ne, oracle_mod, mode)
    q = inputs.random_state(p.nu, seed=100 + N)
    Ro = p.o.dss(p.o.rhs(q), 3)
    qd = p.dev(q)
    assert_groups(p.host(p.g.stage_rhs(qd, prec=numa.PREC_FP64)), Ro, TOL64, "pencil rhs N=%d ne=%s" % (N, ne))
    assert_groups(p.host(p.g.stage_rhs(qd, prec=numa.PREC_MIXED)), Ro, TOLMIX, "pencil mixed rhs N=%d ne=%s" % (N, ne))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("N,ne", CASES)
def test_pencil_step(torch_cuda, oracle_mod, N, ne, mode):
    """Two SSP-RK3 steps (the FP64 stages fold q_s into the contributions
    away from the walls) from the bubble and noise; mixed precision within
    1e-5 of the increment."""
    from paper_1511_01561_amd import numa
    p = _pair(N, ne, oracle_mod, mode)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, N))
    qo = p.o.step(q0, 0.05, 2)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    assert_groups(p.host(qg), qo, TOL64, "pencil step N=%d ne=%s" % (N, ne))
    qm = p.dev(q0)
    p.g.step(qm, 0.05, 2, prec=numa.PREC_MIXED)
    e = group_err(p.host(qm) - q0, qo - q0)
    print("pencil mixed 2-step increment", {k: "%.1e" % v for k, v in e.items()}, flush=True)
    assert max(e.values()) <= TOLMIX


@pytest.mark.parametrize("mode", MODES)
def test_pencil_resume_is_bitwise(torch_cuda, oracle_mod, mode):
    torch = torch_cuda
    p = _pair(4, (8, 4, 4), oracle_mod, mode)
    q0 = p.dev(p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 1)))
    a, b = q0.clone(), q0.clone()
    p.g.step(a, 0.05, 4)
    p.g.step(b, 0.05, 2)
    p.g.step(b, 0.05, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec", [0, 1])
def test_pencil_batch_with_other_meshes_is_bitwise_alone(torch_cuda, oracle_mod, prec, mode):
    """A batch that mixes meshes the mode takes (8 x 4 x 4, 64 x 32 x 4) with
    ones it does not (ny odd, or gather mode: the two-kernel stage) gives
    every item the result of numa_step on it alone."""
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    meshes = []
    for k, ne in enumerate(((8, 4, 4), (4, 3, 2), (64, 32, 4), (8, 4, 4), (8, 4, 2))):
        wl = _wl(4, ne)
        g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=3)
        g.set_metric(numa.METRIC_RECOMPUTE)
        g.set_stage(mode if k < 4 else numa.STAGE_GATHER)
        q = g.init_state(wl["ic"], inputs.device_noise(g.n_unique, len(meshes)))
        meshes.append((g, q))
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


@pytest.mark.parametrize("mode", MODES)
def test_pencil_full_size_step(torch_cuda, oracle_mod, mode):
    """The benchmark's 64 x 64 x 16, N = 4 box: one FP64 step against the
    oracle's, and the right-hand side at 1e-12 (FP64) and 1e-5 (mixed)."""
    from paper_1511_01561_amd import numa
    p = Pair(inputs.gpu_box(4), oracle_mod)
    p.g.set_metric(numa.METRIC_RECOMPUTE)
    p.g.set_stage(mode)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    qo = p.o.step(q0, 0.05, 1)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 1)
    assert_groups(p.host(qg), qo, TOL64, "pencil full step")
    q = inputs.random_state(p.nu, seed=5)
    Ro = p.o.dss(p.o.rhs(q), 3)
    qd = p.dev(q)
    assert_groups(p.host(p.g.stage_rhs(qd)), Ro, TOL64, "pencil full rhs")
    assert_groups(p.host(p.g.stage_rhs(qd, prec=numa.PREC_MIXED)), Ro, TOLMIX, "pencil full mixed rhs")
