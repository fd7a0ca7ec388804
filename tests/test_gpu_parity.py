"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 results within 1e-12 relative max-norm per variable group
(rho'; u, v, w; theta'), err = max|a - b| / max|b|; the mixed-precision
right-hand side within 1e-5 of the FP64 oracle in the same norm.  Connectivity
is compared bit for bit in the host tests.
"""
import numpy as np
import pytest

from paper_1511_01561_amd import inputs

pytestmark = pytest.mark.gpu

GROUPS = {"rho": [0], "u": [1, 2, 3], "theta": [4]}
TOL64 = 1e-12
TOLMIX = 1e-5


def group_err(a, b):
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    out = {}
    for g, rows in GROUPS.items():
        den = np.max(np.abs(b[rows]))
        num = np.max(np.abs(a[rows] - b[rows]))
        out[g] = num / den if den > 0 else num
    return out


def assert_groups(a, b, tol, what=""):
    e = group_err(a, b)
    print(what, {k: "%.2e" % v for k, v in e.items()}, flush=True)
    for g, v in e.items():
        assert v <= tol, "%s group %s: %.3e > %.1e" % (what, g, v, tol)


def scale_err(a, b, scale):
    """max|a - b| per group over the group's term scale (the sum of the
    magnitudes of the individual terms, from the oracle): the norm for groups
    whose result is nearly cancelled."""
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    scale = np.asarray(scale).reshape(5, -1)
    return {g: np.max(np.abs(a[r] - b[r])) / np.max(scale[r]) for g, r in GROUPS.items()}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


class Pair:
    """The same workload built by the oracle and by the library."""

    def __init__(self, wl, oracle_mod, prec_mask=3):
        from paper_1511_01561_amd import numa
        mm = wl["mesh"]
        self.wl = wl
        self.o = oracle_mod.OracleMesh(mm["kind"], mm["N"], mm["ne"], mm["periodic"], mm["extent"], mm["h0"],
                                       wl["phys"])
        self.g = numa.Mesh(mm, wl["phys"], prec_mask=prec_mask)
        self.nu = self.o.n_unique
        self.nl = self.o.n_local

    def dev(self, a):
        import torch
        return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")

    @staticmethod
    def host(t):
        import torch
        torch.cuda.synchronize()
        return t.cpu().numpy()


def small_box_terrain(N):
    return inputs.box_workload(4, 3, 3, N, 12e3, 9e3, 6e3, terrain=400.0, bubble_centre=(6e3, 4.5e3, 2e3),
                               bubble_radius=2.5e3)


def small_shell(N=4):
    return inputs.shell_workload(ne=3, nz=2, N=N, seed=0)


@pytest.fixture(scope="module")
def box4(torch_cuda, oracle_mod):
    return Pair(inputs.small_box(), oracle_mod)


@pytest.fixture(scope="module")
def shell4(torch_cuda, oracle_mod):
    return Pair(small_shell(), oracle_mod)


# -------------------------------------------------------------------- geometry
@pytest.mark.parametrize("which", ["box", "terrain", "shell"])
def test_geometry_parity(torch_cuda, oracle_mod, which):
    from paper_1511_01561_amd import numa
    wl = {"box": inputs.small_box(), "terrain": small_box_terrain(3), "shell": small_shell(4)}[which]
    p = Pair(wl, oracle_mod)
    g, o = p.g, p.o
    M = p.host(g.export(numa.FIELD_MASS))
    np.testing.assert_allclose(M, o.get("mass"), rtol=1e-13)
    ref = p.host(g.export(numa.FIELD_REF))
    np.testing.assert_allclose(ref, o.get("ref"), rtol=1e-13)
    xu = p.host(g.export(numa.FIELD_COORDS))
    scale = np.abs(o.get("xu")).max()
    assert np.abs(xu - o.get("xu")).max() <= 1e-14 * scale
    xl = p.host(g.export(numa.FIELD_LOCAL_COORDS))
    assert np.abs(xl - o.get("xl")).max() <= 1e-14 * scale
    met = p.host(g.export(numa.FIELD_METRIC))
    om = o.get("metric")
    # inverse-metric entries share one scale (off-diagonal ones may be pure roundoff)
    sc = np.abs(om[:9]).max()
    err = [np.abs(met[c] - om[c]).max() / sc for c in range(9)]
    print(which, "metric rel err", ["%.1e" % e for e in err], flush=True)
    assert max(err) <= 1e-12
    assert np.abs(met[9] - om[9]).max() <= 1e-12 * np.abs(om[9]).max()
    grav = p.host(g.export(numa.FIELD_GRAVITY))
    np.testing.assert_allclose(grav, o.get("gravity"), rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- init state
@pytest.mark.parametrize("which", ["box", "shell"])
def test_init_state_parity(torch_cuda, oracle_mod, which, box4, shell4):
    p = box4 if which == "box" else shell4
    nz = inputs.noise(p.nu, 3) if which == "box" else None
    qo = p.o.init_state(p.wl["ic"], nz)
    qg = p.host(p.g.init_state(p.wl["ic"], p.dev(nz) if nz is not None else None))
    # per variable group (w of the tangential jet is pure roundoff on its own)
    assert_groups(qg, qo, 1e-13, "init state")


# ----------------------------------------------------------------------- rhs
def test_rest_state_rhs_exactly_zero(torch_cuda, box4, shell4):
    for p in (box4, shell4):
        C = p.host(p.g.rhs(p.dev(np.zeros((5, p.nu)))))
        assert np.all(C == 0.0)


@pytest.mark.parametrize("N", range(1, 9))
def test_rhs_parity_random_state_all_orders(torch_cuda, oracle_mod, N):
    p = Pair(small_box_terrain(N), oracle_mod)
    q = inputs.random_state(p.nu, seed=N)
    Co = p.o.rhs(q)
    Cg = p.host(p.g.rhs(p.dev(q)))
    assert_groups(Cg, Co, TOL64, "rhs N=%d" % N)


def test_rhs_parity_bubble_box(torch_cuda, box4):
    p = box4
    nz = inputs.noise(p.nu, 0)
    q = p.o.init_state(p.wl["ic"], nz)
    Co = p.o.rhs(q)
    Cg = p.host(p.g.rhs(p.dev(q)))
    assert_groups(Cg, Co, TOL64, "rhs bubble")


@pytest.mark.parametrize("N", [2, 4, 5])
def test_rhs_parity_shell(torch_cuda, oracle_mod, N):
    p = Pair(small_shell(N), oracle_mod)
    q = p.o.init_state(p.wl["ic"], None)
    q[1:4] += 0.5 * inputs.noise(p.nu, 7)        # arbitrary (non-tangential) wind
    Co = p.o.rhs(q)
    Cg = p.host(p.g.rhs(p.dev(q)))
    assert_groups(Cg, Co, TOL64, "rhs shell N=%d" % N)


@pytest.mark.parametrize("N", [3, 4, 5, 6, 8])
def test_rhs_mixed_precision_within_tolerance(torch_cuda, oracle_mod, N):
    from paper_1511_01561_amd import numa
    p = Pair(small_box_terrain(N), oracle_mod)
    q = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 1))
    Co = p.o.rhs(q)
    Cg = p.host(p.g.rhs(p.dev(q), prec=numa.PREC_MIXED))
    assert_groups(Cg, Co, TOLMIX, "mixed rhs N=%d" % N)


def test_rhs_mixed_precision_shell(torch_cuda, shell4):
    """The balanced jet makes R_rho' (a divergence-free wind) and R_theta'
    (wind normal to grad theta_bar) nearly cancel: the mixed tolerance is
    taken against the term scale; the u group is not cancelled."""
    from paper_1511_01561_amd import numa
    p = shell4
    q = p.o.init_state(p.wl["ic"], None)
    Co = p.o.rhs(q)
    Cg = p.host(p.g.rhs(p.dev(q), prec=numa.PREC_MIXED))
    e = scale_err(Cg, Co, p.o.rhs_scale(q))
    print("mixed rhs shell, term-scale norm", {k: "%.2e" % v for k, v in e.items()},
          "plain norm", {k: "%.2e" % v for k, v in group_err(Cg, Co).items()}, flush=True)
    assert max(e.values()) <= TOLMIX
    assert group_err(Cg, Co)["u"] <= TOLMIX


# ----------------------------------------------------------------------- dss
@pytest.mark.parametrize("flags", [0, 1, 3])
def test_dss_parity(torch_cuda, box4, shell4, flags):
    for p in (box4, shell4):
        rng = np.random.default_rng(flags)
        C = rng.standard_normal((5, p.nl))
        out_o = p.o.dss(C, flags)
        out_g = p.host(p.g.dss(p.dev(C), flags))
        sc = np.abs(out_o).max()
        assert np.abs(out_g - out_o).max() <= 1e-13 * sc
        if flags == 0:
            assert np.array_equal(out_g, out_o)     # same copies, same order, no weights


def test_dss_other_nvar(torch_cuda, box4):
    p = box4
    C = np.random.default_rng(5).standard_normal((7, p.nl))
    out_o = p.o.dss(C, 1)
    out_g = p.host(p.g.dss(p.dev(C), 1))
    assert np.abs(out_g - out_o).max() <= 1e-13 * np.abs(out_o).max()


# ------------------------------------------------------------------ rk stage
def test_rk_stage_parity(torch_cuda, box4):
    p = box4
    rng = np.random.default_rng(9)
    qn, qs, r = (rng.standard_normal((5, p.nu)) for _ in range(3))
    for s in range(3):
        o = p.o.rk_stage(s, 0.05, qn, qs, r)
        g = p.host(p.g.rk_stage(s, 0.05, p.dev(qn), p.dev(qs), p.dev(r)))
        assert np.abs(g - o).max() <= 4e-16 * np.abs(o).max()


# ---------------------------------------------------------------------- step
def test_step_parity_small_box_10_steps(torch_cuda, box4):
    p = box4
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    qo = p.o.step(q0, 0.05, 10)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 10)
    qh = p.host(qg)
    # the increment of theta' over 10 steps is ~1e-7 K on a 0.5 K state: its
    # difference is below the state's own rounding, so the state is compared
    print("increment", group_err(qh - q0, qo - q0))
    assert_groups(qh, qo, TOL64, "step state")


def test_step_equals_composition(torch_cuda, box4):
    from paper_1511_01561_amd import numa
    p = box4
    g = p.g
    q0 = p.dev(p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0)))
    # composition of the separate calls
    q = q0.clone()
    R = g.dss(g.rhs(q), numa.DSS_MASS | numa.DSS_NOFLUX)
    q1 = g.rk_stage(0, 0.05, q, q, R)
    R = g.dss(g.rhs(q1), numa.DSS_MASS | numa.DSS_NOFLUX)
    q2 = g.rk_stage(1, 0.05, q, q1, R)
    R = g.dss(g.rhs(q2), numa.DSS_MASS | numa.DSS_NOFLUX)
    q3 = g.rk_stage(2, 0.05, q, q2, R)
    qf = q0.clone()
    g.step(qf, 0.05, 1)
    a, b = p.host(qf), p.host(q3)
    # The fused FP64 step folds q_s into the element contributions away from
    # the walls (J w (q_s + cdt R), summed and multiplied by M^-1), so the two
    # agree to rounding of the state rather than of the increment: the states
    # within the FP64 bar, and within ~100 ulps of each group's largest value.
    assert_groups(a, b, TOL64, "fused vs composed")
    e = group_err(a, b)
    print("fused vs composed, state", {k: "%.1e" % v for k, v in e.items()}, flush=True)
    assert max(e.values()) <= 1e-14


def test_step_resume_and_determinism_bitwise(torch_cuda, box4):
    p = box4
    q0 = p.dev(p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0)))
    a = q0.clone(); p.g.step(a, 0.05, 10)
    b = q0.clone(); p.g.step(b, 0.05, 5); p.g.step(b, 0.05, 5)
    c = q0.clone(); p.g.step(c, 0.05, 10)
    A, B, C = p.host(a), p.host(b), p.host(c)
    assert np.array_equal(A, B)
    assert np.array_equal(A, C)


def test_step_mass_conservation_affine_gpu(torch_cuda, box4):
    from paper_1511_01561_amd import numa
    p = box4
    q0 = p.dev(p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0)))
    q = q0.clone()
    p.g.step(q, 0.05, 10)
    M = p.host(p.g.export(numa.FIELD_MASS))
    rb = p.host(p.g.export(numa.FIELD_REF))[0]
    d = abs((M * p.host(q)[0]).sum() - (M * p.host(q0)[0]).sum())
    assert d <= 1e-13 * (M * rb).sum()


def test_step_parity_shell(torch_cuda, shell4):
    p = shell4
    q0 = p.o.init_state(p.wl["ic"], None)
    qo = p.o.step(q0, 0.5, 5)
    qg = p.dev(q0)
    p.g.step(qg, 0.5, 5)
    qh = p.host(qg)
    print("shell increment", group_err(qh - q0, qo - q0))
    assert_groups(qh, qo, TOL64, "shell step state")


def test_step_mixed_precision_drift(torch_cuda, box4):
    from paper_1511_01561_amd import numa
    p = box4
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    qo = p.o.step(q0, 0.05, 10)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 10, prec=numa.PREC_MIXED)
    e = group_err(p.host(qg) - q0, qo - q0)
    print("mixed 10-step increment error", e)
    assert max(e.values()) <= TOLMIX


# ------------------------------------------------- full one-GPU workload size
@pytest.fixture(scope="module")
def full(torch_cuda, oracle_mod):
    """The 64x64x16, N = 4 terrain box in the launch configuration the
    benchmark times (the oracle runs it with OpenMP on the host)."""
    return Pair(inputs.gpu_box(), oracle_mod)


def test_full_size_rhs_and_dss_parity(full):
    from paper_1511_01561_amd import numa
    p = full
    q = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    qg = p.g.init_state(p.wl["ic"], p.dev(inputs.noise(p.nu, 0)))
    qh = p.host(qg)
    for v in range(5):
        assert np.abs(qh[v] - q[v]).max() <= 1e-13 * max(np.abs(q[v]).max(), 1e-300), v
    Co = p.o.rhs(q)
    Cg = p.g.rhs(p.dev(q))
    assert_groups(p.host(Cg), Co, TOL64, "full rhs")
    Ro = p.o.dss(Co, 3)
    Rg = p.host(p.g.dss(Cg, numa.DSS_MASS | numa.DSS_NOFLUX))
    assert_groups(Rg, Ro, TOL64, "full rhs+dss")
    Cm = p.host(p.g.rhs(p.dev(q), prec=numa.PREC_MIXED))
    assert_groups(Cm, Co, TOLMIX, "full mixed rhs")


def test_full_size_step_parity(full):
    p = full
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, 0))
    qo = p.o.step(q0, 0.05, 2)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    qh = p.host(qg)
    print("full increment", group_err(qh - q0, qo - q0))
    assert_groups(qh, qo, TOL64, "full 2-step state")


# ------------------------------------------- fused step across orders/meshes
@pytest.mark.parametrize("N,ne,perz", [(1, (8, 4, 3), 0), (2, (8, 4, 3), 0), (3, (8, 3, 2), 0), (4, (8, 4, 2), 1),
                                       (5, (4, 3, 2), 0), (6, (4, 2, 2), 0), (7, (4, 2, 2), 1), (8, (4, 2, 2), 0),
                                       (4, (6, 4, 3), 0), (3, (5, 2, 2), 1)])
def test_step_parity_orders_and_meshes(torch_cuda, oracle_mod, N, ne, perz):
    """Covers the box finish kernel for every order (including periodic z and
    the top-wall layer) and the generic finish when nx is not a multiple of
    the block's x-segment (nx = 6 at N = 4, nx = 5 at N = 3)."""
    wl = inputs.box_workload(*ne, N, 1.2e4, 9e3, 6e3, terrain=300.0, bubble_centre=(6e3, 4.5e3, 2.5e3),
                             bubble_radius=2.5e3, periodic_z=bool(perz))
    p = Pair(wl, oracle_mod)
    q0 = p.o.init_state(p.wl["ic"], inputs.noise(p.nu, N))
    qo = p.o.step(q0, 0.05, 2)
    qg = p.dev(q0)
    p.g.step(qg, 0.05, 2)
    qh = p.host(qg)
    assert_groups(qh, qo, TOL64, "step N=%d ne=%s perz=%d" % (N, ne, perz))
    # and the mixed path stays within the mixed tolerance of the FP64 result
    from paper_1511_01561_amd import numa
    qm = p.dev(q0)
    p.g.step(qm, 0.05, 2, prec=numa.PREC_MIXED)
    e = group_err(p.host(qm) - q0, qo - q0)
    print("mixed 2-step increment", {k: "%.1e" % v for k, v in e.items()})
    assert max(e.values()) <= TOLMIX


# ---------------------------------------------------------------- edge cases
@pytest.mark.parametrize("which", ["box4", "nx6", "shell"])
def test_zero_steps_leave_the_state_untouched(torch_cuda, oracle_mod, which):
    """nsteps = 0 through the batched box path, the generic path (nx = 6 at
    N = 4) and the shell path: the state is bitwise unchanged."""
    from paper_1511_01561_amd import numa
    torch = torch_cuda
    if which == "box4":
        wl = inputs.small_box()
    elif which == "nx6":
        wl = inputs.box_workload(6, 4, 2, 4, 1.2e4, 9e3, 6e3, terrain=300.0, bubble_centre=(6e3, 4.5e3, 2.5e3),
                                 bubble_radius=2.5e3)
    else:
        wl = small_shell(3)
    g = numa.Mesh(wl["mesh"], wl["phys"], prec_mask=3)
    noise = inputs.device_noise(g.n_unique, 3) if wl["ic"]["noise_amp"] else None
    q = g.init_state(wl["ic"], noise)
    q0 = q.clone()
    for prec in (0, 1):
        g.step(q, 0.05, 0, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(q, q0)
    if wl["mesh"]["kind"] == 0 and wl["mesh"]["ne"][0] % 4 == 0:
        numa.step_batch([(g, q, numa.alloc_scratch(g, 0), 0.05)], 0, 0)
        torch.cuda.synchronize()
        assert torch.equal(q, q0)
