"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a special case that reduces to a textbook result or a library
routine, or a brute-force evaluation of the paper's definitions.
"""
import math

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

from paper_1511_01561_amd import inputs

PHYS = dict(inputs.PHYS, T0=300.0)


# --------------------------------------------------------------------------
# GLL basis (Sec. "Spatial Discretization": Lobatto points, Lagrange basis)
# --------------------------------------------------------------------------
CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(oracle_mod, N):
    xi, w, _ = oracle_mod.gll(N)
    np.testing.assert_allclose(xi, CLOSED[N][0], rtol=0, atol=4e-16)
    np.testing.assert_allclose(w, CLOSED[N][1], rtol=4e-16, atol=0)


@pytest.mark.parametrize("N", range(1, 9))
def test_gll_nodes_are_roots_of_legendre_derivative(oracle_mod, N):
    xi, w, _ = oracle_mod.gll(N)
    roots = np.sort(npleg.Legendre.basis(N).deriv().roots().real) if N > 1 else np.array([])
    np.testing.assert_allclose(xi[1:-1], roots, atol=1e-14)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    assert np.all(xi[::-1] == -xi)          # exact symmetry
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("N", range(1, 9))
def test_gll_quadrature_exactness(oracle_mod, N):
    xi, w, _ = oracle_mod.gll(N)
    for k in range(0, 2 * N):                # exact for degree <= 2N-1
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14
    k = 2 * N                                # and not for degree 2N
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("N", range(1, 9))
def test_derivative_matrix_exact_on_polynomials(oracle_mod, N):
    xi, _, D = oracle_mod.gll(N)
    for k in range(0, N + 1):
        d = D @ xi ** k
        ref = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.max(np.abs(d - ref)) < 1e-12 * max(1, N * N)
    # one degree too many is not differentiated exactly
    k = N + 1
    assert np.max(np.abs(D @ xi ** k - k * xi ** (k - 1))) > 1e-3
    # centro-antisymmetry and zero row sums
    P = N + 1
    for i in range(P):
        for m in range(P):
            assert abs(D[P - 1 - i, P - 1 - m] + D[i, m]) < 1e-13
    assert np.max(np.abs(D.sum(axis=1))) < 1e-12


def test_derivative_matrix_corner_value(oracle_mod):
    _, _, D = oracle_mod.gll(4)
    assert D[0, 0] == -5.0 and D[4, 4] == 5.0


@pytest.mark.parametrize("N", range(1, 9))
def test_lagrange_brute_force(oracle_mod, N):
    """psi_m from the product formula of the paper; its derivative at the
    nodes by the exact product rule, against D."""
    xi, _, D = oracle_mod.gll(N)
    P = N + 1

    def psi(m, x):
        r = 1.0
        for n in range(P):
            if n != m:
                r *= (x - xi[n]) / (xi[m] - xi[n])
        return r

    def dpsi(m, x):
        s = 0.0
        for k in range(P):
            if k == m:
                continue
            t = 1.0 / (xi[m] - xi[k])
            for n in range(P):
                if n != m and n != k:
                    t *= (x - xi[n]) / (xi[m] - xi[n])
            s += t
        return s

    for i in range(P):
        for m in range(P):
            assert abs(psi(m, xi[i]) - (1.0 if i == m else 0.0)) < 1e-14
            assert abs(dpsi(m, xi[i]) - D[i, m]) < 2e-13 * N * N


# --------------------------------------------------------------------------
# Connectivity (CG storage: one copy per unique grid point)
# --------------------------------------------------------------------------
def _box(oracle_mod, nx=4, ny=4, nz=3, N=3, periodic_z=0, h0=0.0, ext=(1e4, 2e4, 5e3), phys=None):
    return oracle_mod.OracleMesh(0, N, (nx, ny, nz), (1, 1, periodic_z), ext, h0, phys or PHYS)


def test_box_unique_count_and_multiplicity(oracle_mod):
    nx, ny, nz, N = 4, 6, 3, 3
    m = _box(oracle_mod, nx, ny, nz, N)
    assert m.n_unique == (nx * N) * (ny * N) * (nz * N + 1)
    G = m.get("gather").ravel()
    mult = np.bincount(G, minlength=m.n_unique)
    assert set(np.unique(mult)) == {1, 2, 4, 8}
    # interior lattice counts: a node is shared by 2 per direction where it sits on an element face
    ni, nj, nk = nx * N, ny * N, nz * N + 1
    gi, gj, gk = np.meshgrid(np.arange(ni), np.arange(nj), np.arange(nk), indexing="ij")
    fx = np.where(gi % N == 0, 2, 1)
    fy = np.where(gj % N == 0, 2, 1)
    fz = np.where((gk % N == 0) & (gk > 0) & (gk < nk - 1), 2, 1)
    expect = (fx * fy * fz).transpose(2, 1, 0).ravel()   # id = gi + ni (gj + nj gk)
    np.testing.assert_array_equal(mult, expect)


def test_box_periodic_z_count(oracle_mod):
    m = _box(oracle_mod, 2, 2, 2, 2, periodic_z=1)
    assert m.n_unique == 4 * 4 * 4
    # fully periodic 2x2x2 elements of order 2: every element vertex is shared by 8
    mult = np.bincount(m.get("gather").ravel(), minlength=m.n_unique)
    assert mult.sum() == m.n_local and set(np.unique(mult)) == {1, 2, 4, 8}


def test_box_copies_share_coordinates(oracle_mod):
    m = _box(oracle_mod, h0=300.0)
    G = m.get("gather").ravel()
    xl, xu = m.get("xl"), m.get("xu")
    L = np.array([1e4, 2e4])
    for a in range(2):
        d = xl[a] - xu[a][G]
        shift = np.round(d / L[a])
        assert np.all(np.isin(shift, [0.0, 1.0]))
        np.testing.assert_allclose(d - shift * L[a], 0.0, atol=1e-9)
    # z: identical where no periodic shift happened
    unshifted = np.isclose(xl[0], xu[0][G]) & np.isclose(xl[1], xu[1][G])
    np.testing.assert_allclose(xl[2][unshifted], xu[2][G][unshifted], rtol=0, atol=1e-9)


def test_shell_unique_count_and_corner_columns(oracle_mod):
    ne, nz, N = 3, 2, 3
    m = oracle_mod.OracleMesh(1, N, (ne, ne, nz), (0, 0, 0), (6.371e6, 0.0, 3e4), 0.0, dict(inputs.PHYS, T0=250.0))
    L = ne * N
    assert m.n_unique == (6 * L * L + 2) * (nz * N + 1)
    assert m.n_elem == 6 * ne * ne * nz
    G = m.get("gather").ravel()
    mult = np.bincount(G, minlength=m.n_unique)
    assert mult.sum() == m.n_local
    assert set(np.unique(mult)) <= {1, 2, 3, 4, 6, 8}
    # horizontal multiplicity 3 only at the 8 cube corners, on every level
    bottom = mult[: m.n_horiz]
    assert np.sum(bottom == 3) == 8
    # copies share coordinates bitwise (built from one lattice)
    xl, xu = m.get("xl"), m.get("xu")
    for a in range(3):
        assert np.array_equal(xl[a], xu[a][G])
    # radius at each level is constant
    r = np.sqrt((xu ** 2).sum(0))
    r_lev = r.reshape(m.n_levels, m.n_horiz)
    assert np.max(np.abs(r_lev - r_lev[:, :1])) < 1e-8 * 6.4e6


# --------------------------------------------------------------------------
# Geometry: metric and mass (Eq. (derivatives), Eq. (discstrongform))
# --------------------------------------------------------------------------
def test_undeformed_metric_closed_form(oracle_mod):
    nx, ny, nz, N = 4, 6, 3, 3
    Lx, Ly, H = 1e4, 2e4, 5e3
    m = _box(oracle_mod, nx, ny, nz, N, ext=(Lx, Ly, H))
    met = m.get("metric")
    np.testing.assert_allclose(met[0], 2 * nx / Lx, rtol=1e-13)
    np.testing.assert_allclose(met[4], 2 * ny / Ly, rtol=1e-13)
    np.testing.assert_allclose(met[8], 2 * nz / H, rtol=1e-13)
    for c in (1, 2, 3, 5, 6, 7):
        assert np.max(np.abs(met[c])) < 1e-16
    xi, w, _ = oracle_mod.gll(N)
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    J = Lx * Ly * H / (8 * nx * ny * nz)
    np.testing.assert_allclose(met[9].reshape(-1, (N + 1) ** 3), np.tile(J * W, (m.n_elem, 1)), rtol=1e-13)
    assert abs(m.get("mass").sum() - Lx * Ly * H) < 1e-12 * Lx * Ly * H


def test_terrain_mass_is_volume(oracle_mod):
    Lx, Ly, H = 1e4, 2e4, 5e3
    m = _box(oracle_mod, ext=(Lx, Ly, H), h0=400.0)
    assert abs(m.get("mass").sum() - Lx * Ly * H) < 1e-12 * Lx * Ly * H
    met = m.get("metric")
    assert np.max(np.abs(met[6])) > 1e-6       # zeta_x is exercised by the terrain


def test_shell_mass_converges_to_volume(oracle_mod):
    a, H = 6.371e6, 3e4
    vol = 4.0 * math.pi / 3.0 * ((a + H) ** 3 - a ** 3)
    errs = []
    for N in (2, 4, 6):
        m = oracle_mod.OracleMesh(1, N, (2, 2, 1), (0, 0, 0), (a, 0.0, H), 0.0, dict(inputs.PHYS, T0=250.0))
        errs.append(abs(m.get("mass").sum() - vol) / vol)
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 1e-9


# --------------------------------------------------------------------------
# Terrain-following box geometry (Sec. "Spatial Discretization": isoparametric
# hexahedra; Eq. (derivatives): the metric terms).  Everything the pins below
# compare with is computed here from the map itself, with GLL nodes taken as
# numpy's roots of P'_N, never from the oracle's arrays.
# --------------------------------------------------------------------------
TERRAIN = dict(nx=4, ny=4, nz=3, N=4, Lx=4.0e4, Ly=3.0e4, H=6.0e3, h0=500.0)


def _numpy_gll_nodes(N):
    inner = np.sort(npleg.Legendre.basis(N).deriv().roots().real)
    return np.concatenate([[-1.0], inner, [1.0]])


def _terrain(x, y, t=TERRAIN):
    """h(x, y) of the map and its gradient"""
    kx, ky = 2 * math.pi / t["Lx"], 2 * math.pi / t["Ly"]
    h = t["h0"] * np.sin(kx * x) * np.sin(ky * y)
    return h, t["h0"] * kx * np.cos(kx * x) * np.sin(ky * y), t["h0"] * ky * np.sin(kx * x) * np.cos(ky * y)


def _terrain_unique_coords(t=TERRAIN):
    """unique-node coordinates of the terrain box in canonical order
    (x fastest; x, y periodic, so the lattice stops one point short of Lx, Ly):
    x = Lx (ex + (1 + xi_i)/2)/nx and likewise y, z; z' = z + h(x, y)(1 - z/H)"""
    N, nx, ny, nz = t["N"], t["nx"], t["ny"], t["nz"]
    xi = _numpy_gll_nodes(N)

    def axis(n, L, closed):
        c = np.arange(n * N + (1 if closed else 0))
        e = np.minimum(c // N, n - 1)
        return L * (e + (1 + xi[c - N * e]) / 2) / n

    ax, ay, az = axis(nx, t["Lx"], False), axis(ny, t["Ly"], False), axis(nz, t["H"], True)
    z, y, x = np.meshgrid(az, ay, ax, indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    h = _terrain(x, y, t)[0]
    return x, y, z + h * (1 - z / t["H"])


def _terrain_box(oracle_mod, phys=None, N=None):
    t = TERRAIN
    return oracle_mod.OracleMesh(0, N or t["N"], (t["nx"], t["ny"], t["nz"]), (1, 1, 0), (t["Lx"], t["Ly"], t["H"]),
                                 t["h0"], phys or PHYS)


def test_terrain_coordinates_follow_the_map(oracle_mod):
    m = _terrain_box(oracle_mod)
    x, y, z = _terrain_unique_coords()
    xu = m.get("xu")
    assert xu.shape[1] == x.size
    np.testing.assert_allclose(xu[0], x, rtol=0, atol=1e-9)
    np.testing.assert_allclose(xu[1], y, rtol=0, atol=1e-9)
    np.testing.assert_allclose(xu[2], z, rtol=0, atol=1e-9)
    # the terrain is really there: the bottom layer is not flat
    assert np.ptp(xu[2][:m.n_horiz]) > 1.9 * TERRAIN["h0"]


def _seam_free_mask(m, t=TERRAIN):
    """element-local mask of the elements that do not touch the periodic seam:
    there a field linear in the wrapped unique coordinates is not linear in the
    element's own coordinates"""
    e = np.arange(m.n_elem)
    ok = (e % t["nx"] < t["nx"] - 1) & ((e // t["nx"]) % t["ny"] < t["ny"] - 1)
    return np.repeat(ok, m.np)


def test_terrain_linear_theta_is_advected_exactly(oracle_mod):
    """theta' linear in the physical coordinates is in the isoparametric
    element's interpolation space, so the chain rule through the terrain
    metric (zeta_x, zeta_y from z_xi, z_eta) gives its exact gradient at every
    node: with constant u, g0 = 0 and rho' = -rho_bar theta'/(theta_bar + theta')
    (p' = 0), R_theta' = -u.grad(theta') = -(u b + v c + w d)."""
    t = TERRAIN
    m = _terrain_box(oracle_mod, phys=dict(PHYS, g0=0.0))
    x, y, z = _terrain_unique_coords()
    b, c, d = 0.3 / t["Lx"], -0.2 / t["Ly"], 0.4 / t["H"]
    tp = 0.1 + b * x + c * y + d * z
    u, v, w = 3.0, -2.0, 0.5
    rb, tb, _ = m.get("ref")
    q = np.stack([-rb * tp / (tb + tp), np.full_like(tp, u), np.full_like(tp, v), np.full_like(tp, w), tp])
    R = m.rhs(q) / m.get("metric")[9]
    mask = _seam_free_mask(m)
    exact = -(u * b + v * c + w * d)
    assert np.max(np.abs(R[4][mask] - exact)) < 1e-12 * abs(exact)
    # the same field differentiated along z only would be off by the terrain slope
    assert abs(exact + w * d) > 0.5 * abs(exact)


def test_terrain_linear_velocity_is_differentiated_exactly(oracle_mod):
    """u, v, w linear in the physical coordinates, rho' = theta' = 0, g0 = 0
    (constant rho_bar): R_u = -(u.grad)u and R_rho' = -rho_bar div(u) exactly,
    with every entry of the velocity gradient non-zero, so that each metric
    term (xi_x, eta_y, zeta_x, zeta_y, zeta_z) enters."""
    t = TERRAIN
    m = _terrain_box(oracle_mod, phys=dict(PHYS, g0=0.0))
    x, y, z = _terrain_unique_coords()
    G = np.array([[0.7 / t["Lx"], -0.4 / t["Ly"], 0.9 / t["H"]],
                  [0.3 / t["Lx"], 0.5 / t["Ly"], -0.6 / t["H"]],
                  [-0.2 / t["Lx"], 0.8 / t["Ly"], 0.35 / t["H"]]])  # G[a, c] = d u_a / d x_c
    u0 = np.array([2.0, -1.5, 0.4])
    X = np.stack([x, y, z])
    vel = u0[:, None] + G @ X
    q = np.zeros((5, m.n_unique))
    q[1:4] = vel
    R = m.rhs(q) / m.get("metric")[9]
    mask = _seam_free_mask(m)
    Gm = m.get("gather").ravel()[mask]
    rb = m.get("ref")[0][Gm]
    assert np.ptp(rb) == 0.0  # g0 = 0: constant reference density
    exact_u = -(G @ vel)  # -(u.grad) u_a = -sum_c u_c G[a, c]
    for a in range(3):
        ex = exact_u[a][Gm]
        assert np.max(np.abs(R[1 + a][mask] - ex)) < 1e-12 * np.max(np.abs(ex)), a
    ex0 = -rb * np.trace(G)
    assert np.max(np.abs(R[0][mask] - ex0)) < 1e-12 * np.max(np.abs(ex0))


def test_terrain_bottom_normal_is_the_analytic_terrain_normal(oracle_mod):
    """bottom wall: n = (-h_x, -h_y, 1)/|.| of the map's terrain; top: +z"""
    m = _terrain_box(oracle_mod)
    x, y, _ = _terrain_unique_coords()
    nrm, isb = m.get("normals"), m.get("isbnd").astype(bool)
    nh = m.n_horiz
    _, hx, hy = _terrain(x[:nh], y[:nh])
    s = np.sqrt(hx * hx + hy * hy + 1.0)
    np.testing.assert_allclose(nrm[:, :nh], np.stack([-hx / s, -hy / s, 1.0 / s]), rtol=0, atol=1e-13)
    np.testing.assert_allclose(nrm[:, -nh:], np.tile([[0.0], [0.0], [1.0]], (1, nh)), rtol=0, atol=0)
    assert isb[:nh].all() and isb[-nh:].all() and not isb[nh:-nh].any()
    assert np.max(np.abs(nrm[0, :nh])) > 0.05  # the slope is resolved, not negligible


def test_terrain_bottom_normal_matches_grad_zeta(oracle_mod):
    """The bottom surface of the isoparametric mesh has normal grad(zeta)/|.|
    (zeta = -1 there), taken from the oracle's metric; it converges
    spectrally in N to the wall normal the no-flux projection uses."""
    errs = []
    for N in (2, 4, 6, 8):
        m = _terrain_box(oracle_mod, N=N)
        met, G = m.get("metric"), m.get("gather").ravel()
        nrm = m.get("normals")
        P = N + 1
        k = (np.arange(m.n_local) % m.np) // (P * P)
        bottom = (k == 0) & (G < m.n_horiz)
        gz = met[6:9][:, bottom]
        gz = gz / np.sqrt((gz ** 2).sum(0))
        errs.append(np.max(np.abs(gz - nrm[:, G[bottom]])))
    assert errs[3] < errs[2] < errs[1] < errs[0]
    assert errs[3] < 1e-6


# --------------------------------------------------------------------------
# Reference state: hydrostatic balance and the equation of state
# --------------------------------------------------------------------------
def test_isentropic_reference_is_hydrostatic(oracle_mod):
    m = _box(oracle_mod, 2, 2, 4, 6, ext=(1e4, 1e4, 1e4))
    ref, xu = m.get("ref"), m.get("xu")
    z = xu[2]
    rb, tb, pb = ref
    assert np.all(tb == 300.0)
    # pressure from the equation of state equals the closed-form hydrostatic profile
    R, cp, g0, p0 = 287.0, 1004.5, 9.81, 1e5
    pi = 1 - g0 * z / (cp * 300.0)
    np.testing.assert_allclose(pb, p0 * pi ** (cp / R), rtol=1e-13)
    # dp/dz = -rho g along a column (by finite differences on the exact profile)
    h = 1e-2
    dp = (p0 * (1 - g0 * (z + h) / (cp * 300)) ** (cp / R) - p0 * (1 - g0 * (z - h) / (cp * 300)) ** (cp / R)) / (2 * h)
    np.testing.assert_allclose(dp, -rb * g0, rtol=1e-6)


def test_isothermal_shell_reference_is_hydrostatic(oracle_mod):
    a = 6.371e6
    m = oracle_mod.OracleMesh(1, 3, (2, 2, 2), (0, 0, 0), (a, 0.0, 3e4), 0.0, dict(inputs.PHYS, T0=250.0))
    ref, xu, g = m.get("ref"), m.get("xu"), m.get("gravity")
    r = np.sqrt((xu ** 2).sum(0))
    rb, tb, pb = ref
    R, cp, g0, p0 = 287.0, 1004.5, 9.81, 1e5
    np.testing.assert_allclose(pb, rb * R * 250.0, rtol=1e-12)               # isothermal ideal gas
    np.testing.assert_allclose(tb * (pb / p0) ** (R / cp), 250.0, rtol=1e-12)  # theta definition
    gr = np.sqrt((g ** 2).sum(0))
    np.testing.assert_allclose(gr, g0 * (a / r) ** 2, rtol=1e-13)
    np.testing.assert_allclose((g * xu).sum(0), -gr * r, rtol=1e-12)         # points inward
    # dp/dr = -rho g(r) from the closed form
    f = lambda rr: p0 * np.exp(-(g0 * a / (R * 250.0)) * (1 - a / rr))
    dp = (f(r + 1e-1) - f(r - 1e-1)) / 0.2
    np.testing.assert_allclose(dp, -rb * gr, rtol=1e-6)


# --------------------------------------------------------------------------
# Right-hand side (create_rhs, Eq. (discstrongform) and Eq. (derivatives))
# --------------------------------------------------------------------------
def _elem_view(m, a):
    return a.reshape(a.shape[0], m.n_elem, m.np)


def test_rest_state_rhs_is_exactly_zero_box(oracle_mod):
    m = _box(oracle_mod, h0=500.0)
    C = m.rhs(np.zeros((5, m.n_unique)))
    assert np.all(C == 0.0)


def test_rest_state_rhs_is_exactly_zero_shell(oracle_mod):
    m = oracle_mod.OracleMesh(1, 4, (2, 2, 2), (0, 0, 0), (6.371e6, 0.0, 3e4), 0.0, dict(inputs.PHYS, T0=250.0))
    C = m.rhs(np.zeros((5, m.n_unique)))
    assert np.all(C == 0.0)


def test_uniform_flow_triply_periodic_no_gravity(oracle_mod):
    phys = dict(PHYS, g0=0.0)
    m = _box(oracle_mod, 4, 4, 4, 4, periodic_z=1, phys=phys)
    q = np.zeros((5, m.n_unique))
    q[0] = -0.01; q[1] = 3.0; q[2] = -2.0; q[3] = 1.5; q[4] = 0.7
    C = m.rhs(q)
    Jw = m.get("metric")[9]
    R = C / Jw
    # every term is a derivative of a constant field: roundoff only
    assert np.max(np.abs(R)) < 1e-13 * 4.0 * 16 / 2500.0 * 1e3


def _affine_interior(m, nx, ny):
    """element-local mask of elements away from the periodic seam"""
    e = np.arange(m.n_elem)
    ex, ey = e % nx, (e // nx) % ny
    ok = (ex < nx - 1) & (ey < ny - 1)
    return np.repeat(ok, m.np)


def test_polynomial_advection_is_exact(oracle_mod):
    """Affine mesh, g = 0, constant background, polynomial u, v, w, theta' of
    degree <= N per direction, rho' chosen so that p' = 0: R_u = -(u.grad)u and
    R_theta' = -u.grad theta' exactly at the nodes."""
    nx, ny, nz, N = 4, 4, 3, 4
    Lx, Ly, H = 1e4, 1e4, 6e3
    phys = dict(PHYS, g0=0.0)
    m = _box(oracle_mod, nx, ny, nz, N, ext=(Lx, Ly, H), phys=phys)
    x, y, z = (m.get("xu")[a] / s for a, s in zip(range(3), (Lx, Ly, H)))
    u = 1.0 + 0.3 * x + 0.2 * y * y - 0.1 * x * z + 0.05 * z ** 3
    v = -0.5 + 0.4 * y * z + 0.1 * x ** 4
    w = 0.2 * x * y - 0.3 * z * z + 0.02 * y ** 3 * z
    tp = 0.5 * x * y * z + 0.1 * z ** 2 - 0.2 * x ** 3
    rb, tb, _ = m.get("ref")
    q = np.stack([-rb * tp / (tb + tp), u, v, w, tp])
    C = m.rhs(q)
    R = C / m.get("metric")[9]
    # analytic derivatives (d/dx = (1/Lx) d/dx' etc.)
    ux, uy, uz = (0.3 - 0.1 * z) / Lx, 0.4 * y / Ly, (-0.1 * x + 0.15 * z * z) / H
    vx, vy, vz = 0.4 * x ** 3 / Lx, 0.4 * z / Ly, 0.4 * y / H
    wx, wy, wz = 0.2 * y / Lx, (0.2 * x + 0.06 * y * y * z) / Ly, (-0.6 * z + 0.02 * y ** 3) / H
    tx, ty, tz = (0.5 * y * z - 0.6 * x * x) / Lx, 0.5 * x * z / Ly, (0.5 * x * y + 0.2 * z) / H
    exact = [-(u * ux + v * uy + w * uz), -(u * vx + v * vy + w * vz), -(u * wx + v * wy + w * wz),
             -(u * tx + v * ty + w * tz)]
    G = m.get("gather").ravel()
    mask = _affine_interior(m, nx, ny)
    for s, ex in zip((1, 2, 3, 4), exact):
        got = R[s][mask]
        ref = ex[G][mask]
        assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref)), s


def test_polynomial_divergence_is_exact(oracle_mod):
    """theta' = rho' = 0: R_rho' = -rho_bar div(u) exactly."""
    nx, ny, nz, N = 4, 4, 3, 3
    Lx, Ly, H = 1e4, 1e4, 6e3
    m = _box(oracle_mod, nx, ny, nz, N, ext=(Lx, Ly, H), phys=dict(PHYS, g0=0.0))
    x, y, z = (m.get("xu")[a] / s for a, s in zip(range(3), (Lx, Ly, H)))
    q = np.zeros((5, m.n_unique))
    q[1] = x * y + z ** 3
    q[2] = y ** 2 * x - z
    q[3] = x * z * y + x ** 3
    div = y / Lx + 2 * x * y / Ly + x * y / H
    rb = m.get("ref")[0]
    R = m.rhs(q) / m.get("metric")[9]
    G = m.get("gather").ravel()
    mask = _affine_interior(m, nx, ny)
    ref = (-rb * div)[G][mask]
    assert np.max(np.abs(R[0][mask] - ref)) < 1e-11 * np.max(np.abs(ref))


def test_pressure_gradient_term(oracle_mod):
    """u = 0, rho' = 0, theta' chosen so that p' is a given polynomial P:
    R_u = -grad(P)/rho_bar; R_rho' = R_theta' = 0."""
    nx, ny, nz, N = 4, 4, 3, 4
    Lx, Ly, H = 1e4, 1e4, 6e3
    m = _box(oracle_mod, nx, ny, nz, N, ext=(Lx, Ly, H), phys=dict(PHYS, g0=0.0))
    x, y, z = (m.get("xu")[a] / s for a, s in zip(range(3), (Lx, Ly, H)))
    rb, tb, pb = m.get("ref")
    gamma = 1004.5 / (1004.5 - 287.0)
    Pp = 20.0 * x * y - 15.0 * z ** 2 + 5.0 * x ** 3 * z
    q = np.zeros((5, m.n_unique))
    q[4] = tb * ((1 + Pp / pb) ** (1 / gamma) - 1)
    R = m.rhs(q) / m.get("metric")[9]
    G = m.get("gather").ravel()
    mask = _affine_interior(m, nx, ny)
    grad = [(20 * y + 15 * x * x * z) / Lx, 20 * x / Ly, (-30 * z + 5 * x ** 3) / H]
    for s in range(3):
        ref = (-grad[s] / rb)[G][mask]
        assert np.max(np.abs(R[1 + s][mask] - ref)) < 1e-9 * np.max(np.abs(ref)), s
    assert np.all(R[0] == 0.0) and np.all(R[4] == 0.0)


def test_buoyancy_term(oracle_mod):
    """u = 0, constant rho', theta' with Delta = 0 (p' = 0): R_w = -(rho'/rho) g0."""
    m = _box(oracle_mod, 4, 4, 3, 3, ext=(1e4, 1e4, 6e3), h0=300.0)
    rb, tb, _ = m.get("ref")
    rp = -0.01
    q = np.zeros((5, m.n_unique))
    q[0] = rp
    q[4] = -rp * tb / (rb + rp)
    R = m.rhs(q) / m.get("metric")[9]
    G = m.get("gather").ravel()
    ref = (-rp / (rb + rp) * 9.81)[G]
    np.testing.assert_allclose(R[3], ref, rtol=1e-9)
    assert np.max(np.abs(R[1])) < 1e-9 * np.max(np.abs(ref))
    assert np.max(np.abs(R[2])) < 1e-9 * np.max(np.abs(ref))
    assert np.all(R[0] == 0.0) and np.all(R[4] == 0.0)


def test_buoyancy_term_shell_is_radial(oracle_mod):
    a = 6.371e6
    m = oracle_mod.OracleMesh(1, 3, (2, 2, 2), (0, 0, 0), (a, 0.0, 3e4), 0.0, dict(inputs.PHYS, T0=250.0))
    rb, tb, _ = m.get("ref")
    rp = 0.003
    q = np.zeros((5, m.n_unique))
    q[0] = rp
    q[4] = -rp * tb / (rb + rp)
    R = m.rhs(q) / m.get("metric")[9]
    G = m.get("gather").ravel()
    xu = m.get("xu")
    r = np.sqrt((xu ** 2).sum(0))
    gmag = 9.81 * (a / r) ** 2
    for s in range(3):
        ref = (-(rp / (rb + rp)) * gmag * xu[s] / r)[G]
        np.testing.assert_allclose(R[1 + s], ref, rtol=1e-8, atol=1e-9 * np.max(np.abs(ref)))


def test_shell_background_theta_gradient_converges(oracle_mod):
    """Radial wind u0 r_hat over the isothermal background: R_theta' = -u0 dtheta_bar/dr,
    with spectral convergence in N."""
    a, H = 6.371e6, 3e4
    R_, cp = 287.0, 1004.5
    errs = []
    for N in (2, 4, 6):
        m = oracle_mod.OracleMesh(1, N, (2, 2, 2), (0, 0, 0), (a, 0.0, H), 0.0, dict(inputs.PHYS, T0=250.0))
        xu = m.get("xu")
        r = np.sqrt((xu ** 2).sum(0))
        q = np.zeros((5, m.n_unique))
        q[1:4] = 2.0 * xu / r
        Rr = m.rhs(q)[4] / m.get("metric")[9]
        rb, tb, pb = m.get("ref")
        # theta = T0 (p0/p)^(R/cp), dp/dr = -rho g  =>  dtheta/dr = -(R/cp) theta/p dp/dr
        dth = (R_ / cp) * tb / pb * rb * 9.81 * (a / r) ** 2
        G = m.get("gather").ravel()
        ref = (-2.0 * dth)[G]
        errs.append(np.max(np.abs(Rr - ref)) / np.max(np.abs(ref)))
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 1e-6


# --------------------------------------------------------------------------
# DSS (text after Eq. (derivatives)) and the mass matrix
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [0, 1])
def test_dss_of_continuous_field_is_identity(oracle_mod, kind):
    if kind == 0:
        m = _box(oracle_mod, h0=500.0)
    else:
        m = oracle_mod.OracleMesh(1, 3, (2, 2, 2), (0, 0, 0), (6.371e6, 0.0, 3e4), 0.0, dict(inputs.PHYS, T0=250.0))
    rng = np.random.default_rng(1)
    f = rng.standard_normal((2, m.n_unique))
    G = m.get("gather").ravel()
    Jw = m.get("metric")[9]
    out = m.dss(f[:, G] * Jw, flags=1)
    np.testing.assert_allclose(out, f, rtol=1e-13, atol=1e-13)
    # plain sum counts copies
    ones = m.dss(np.ones((1, m.n_local)), flags=0)[0]
    np.testing.assert_array_equal(ones, np.bincount(G, minlength=m.n_unique).astype(float))


def test_dss_conserves_weighted_sum(oracle_mod):
    m = _box(oracle_mod, h0=500.0)
    rng = np.random.default_rng(2)
    C = rng.standard_normal((3, m.n_local))
    out = m.dss(C, flags=1)
    M = m.get("mass")
    np.testing.assert_allclose((out * M).sum(1), C.sum(1), rtol=1e-12, atol=1e-10)


def test_noflux_projection_removes_normal_component(oracle_mod):
    m = _box(oracle_mod, h0=500.0)
    rng = np.random.default_rng(3)
    C = rng.standard_normal((5, m.n_local))
    out = m.dss(C, flags=3)
    nrm, isb = m.get("normals"), m.get("isbnd").astype(bool)
    dn = (out[1:4] * nrm).sum(0)
    assert np.max(np.abs(dn[isb])) < 1e-14 * np.max(np.abs(out))
    ref = m.dss(C, flags=1)
    np.testing.assert_array_equal(out[:, ~isb], ref[:, ~isb])
    np.testing.assert_array_equal(out[0], ref[0])
    np.testing.assert_array_equal(out[4], ref[4])
    assert isb.sum() == 2 * m.n_horiz


# --------------------------------------------------------------------------
# SSP-RK3 ("update q")
# --------------------------------------------------------------------------
def test_rk3_linear_amplification(oracle_mod):
    m = _box(oracle_mod, 2, 2, 1, 1)
    lam, dt = -0.7 + 0.0, 0.3
    rng = np.random.default_rng(4)
    q0 = rng.standard_normal((5, m.n_unique))
    q1 = m.rk_stage(0, dt, q0, q0, lam * q0)
    q2 = m.rk_stage(1, dt, q0, q1, lam * q1)
    q3 = m.rk_stage(2, dt, q0, q2, lam * q2)
    z = lam * dt
    np.testing.assert_allclose(q3, (1 + z + z * z / 2 + z ** 3 / 6) * q0, rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# Time stepping invariants on the small box workload
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small(oracle_mod):
    wl = inputs.small_box()
    mm = wl["mesh"]
    m = oracle_mod.OracleMesh(mm["kind"], mm["N"], mm["ne"], mm["periodic"], mm["extent"], mm["h0"], wl["phys"])
    return m, wl


def test_mass_conservation_affine(small):
    m, wl = small
    q0 = m.init_state(wl["ic"], inputs.noise(m.n_unique, 0))
    M = m.get("mass")
    rb = m.get("ref")[0]
    q = m.step(q0, 0.05, 10)
    assert abs((M * q[0]).sum() - (M * q0[0]).sum()) <= 1e-13 * (M * rb).sum()
    assert np.abs(q - q0).max() > 0


def test_mirror_symmetry_without_noise(small):
    m, wl = small
    q = m.step(m.init_state(wl["ic"], None), 0.05, 10)
    N = m.N
    ni = nj = 4 * N
    nk = 4 * N + 1
    Q = q.reshape(5, nk, nj, ni)
    scale = np.abs(Q).reshape(5, -1).max(1)
    mx = np.roll(Q[:, :, :, ::-1], 1, axis=3)           # gi -> (ni - gi) mod ni
    sx = np.array([1, -1, 1, 1, 1])[:, None, None, None]
    assert np.max(np.abs(mx * sx - Q).reshape(5, -1).max(1) / np.maximum(scale, 1e-300)) < 1e-10
    # x <-> y with u <-> v
    T = Q.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]]
    assert np.max(np.abs(T - Q).reshape(5, -1).max(1) / np.maximum(scale, 1e-300)) < 1e-10


def test_step_resume_is_bitwise(small):
    m, wl = small
    q0 = m.init_state(wl["ic"], inputs.noise(m.n_unique, 0))
    a = m.step(q0, 0.05, 4)
    b = m.step(m.step(q0, 0.05, 2), 0.05, 2)
    assert np.array_equal(a, b)


def test_initial_state_balanced_pressure(small):
    m, wl = small
    q = m.init_state(wl["ic"], None)
    rb, tb, _ = m.get("ref")
    delta = q[0] * tb + rb * q[4] + q[0] * q[4]
    assert np.max(np.abs(delta)) < 1e-13
    assert 0.45 < q[4].max() <= 0.5
    # the cosine bell at the nodes, from the node coordinates
    x, y, z = m.get("xu")
    r = np.sqrt((x - 5e3) ** 2 + (y - 5e3) ** 2 + (z - 2e3) ** 2)
    bell = np.where(r < 2e3, 0.25 * (1 + np.cos(np.pi * r / 2e3)), 0.0)
    np.testing.assert_allclose(q[4], bell, rtol=1e-14, atol=1e-16)


# --------------------------------------------------------------------------
# Boyd-Vandeven filter (Sec. "Filter"; Code example 1: filter, then DSS and
# inverse mass).  Order and cutoff are inputs (the paper gives neither).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,order,cutoff", [(4, 12.0, 1), (6, 8.0, 2), (8, 16.0, 4), (8, 4.0, 0), (7, 36.0, 3)])
def test_filter_sigma_shape(oracle_mod, N, order, cutoff):
    s = oracle_mod.filter_sigma(N, order, cutoff)
    np.testing.assert_array_equal(s[:cutoff + 1], 1.0)      # modes up to the cutoff untouched
    assert s[N] == 0.0                                       # top mode removed
    assert np.all(np.diff(s) <= 0) and np.all(s >= 0)        # monotone damping
    # the erfc-log form is odd about t = 1/2: sigma(t) + sigma(1 - t) = 1
    k = np.arange(cutoff, N + 1)
    np.testing.assert_allclose(s[k] + s[k[::-1]], 1.0, rtol=0, atol=1e-15)
    if (N - cutoff) % 2 == 0:
        assert abs(s[(N + cutoff) // 2] - 0.5) < 1e-16


def test_filter_sigma_sharpens_with_order(oracle_mod):
    # larger order -> closer to the sharp cut at t = 1/2
    lo = oracle_mod.filter_sigma(8, 2.0, 0)
    hi = oracle_mod.filter_sigma(8, 200.0, 0)
    assert np.all(hi[:4] >= lo[:4]) and np.all(hi[5:] <= lo[5:])
    assert hi[3] > 0.999 and hi[5] < 1e-3
    assert lo[3] < 0.9 and lo[5] > 0.1


@pytest.mark.parametrize("N,order,cutoff", [(2, 12.0, 0), (4, 12.0, 1), (8, 16.0, 4), (5, 6.0, 2)])
def test_filter_matrix_is_modal_damping(oracle_mod, N, order, cutoff):
    """F applied to P_k at the GLL nodes gives sigma_k P_k (numpy's Legendre series)."""
    xi, _, _ = oracle_mod.gll(N)
    F = oracle_mod.filter_matrix(N, order, cutoff)
    s = oracle_mod.filter_sigma(N, order, cutoff)
    for k in range(N + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        pk = npleg.legval(xi, c)
        np.testing.assert_allclose(F @ pk, s[k] * pk, rtol=0, atol=2e-14)


def test_filter_matrix_low_order_closed_forms(oracle_mod):
    # N = 1, cutoff 0: the constant mode only, i.e. the two-node mean
    np.testing.assert_allclose(oracle_mod.filter_matrix(1, 12.0, 0), np.full((2, 2), 0.5), rtol=0, atol=1e-16)
    # N = 2, cutoff 0: sigma = (1, 1/2, 0) on nodes (-1, 0, 1), P_2 = (3x^2 - 1)/2;
    # a = c0 + c1 x + c2 P2(x): c0 = (a0 + 4 a1 + a2)/6, c1 = (a2 - a0)/2, c2 = (a0 - 2 a1 + a2)/3
    C = np.array([[1 / 6, 4 / 6, 1 / 6], [-0.5, 0.0, 0.5], [1 / 3, -2 / 3, 1 / 3]])
    V = np.array([[1.0, -1.0, 1.0], [1.0, 0.0, -0.5], [1.0, 1.0, 1.0]])
    F2 = V @ np.diag([1.0, 0.5, 0.0]) @ C
    np.testing.assert_allclose(oracle_mod.filter_matrix(2, 12.0, 0), F2, rtol=0, atol=1e-15)
    # cutoff at N: the identity
    np.testing.assert_allclose(oracle_mod.filter_matrix(6, 12.0, 6), np.eye(7), rtol=0, atol=1e-14)


def _filter_box(oracle_mod, N=4, nz=2, h0=0.0):
    return _box(oracle_mod, 2, 2, nz, N, h0=h0, ext=(2e3, 3e3, 1e3))


def test_filter_single_vertical_mode(oracle_mod):
    """A state that is P_k(zeta) in every element of a one-layer box comes back
    as sigma_k P_k: the whole path (element matrix, J w, DSS / M) is exact."""
    N, order, cutoff = 6, 10.0, 2
    m = _filter_box(oracle_mod, N, nz=1)
    z = m.get("xu")[2]
    zeta = 2.0 * z / 1e3 - 1.0
    s = oracle_mod.filter_sigma(N, order, cutoff)
    for k in range(N + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        pk = npleg.legval(zeta, c)
        q = np.zeros((5, m.n_unique))
        q[0] = pk
        q[4] = 2.0 * pk
        out = m.filter(q, order, cutoff)
        np.testing.assert_allclose(out[0], s[k] * pk, rtol=0, atol=1e-13)
        np.testing.assert_allclose(out[4], 2.0 * s[k] * pk, rtol=0, atol=2e-13)
        assert np.all(out[1:4] == 0.0)


def test_filter_horizontal_brute_force(oracle_mod):
    """x- and y-dependent state, expected value by per-element Legendre fits
    (numpy) and the plain average of the two copies on element faces."""
    N, order, cutoff = 4, 12.0, 1
    Lx, Ly = 2e3, 3e3
    m = _filter_box(oracle_mod, N, nz=1)
    x, y, _ = m.get("xu")
    f = (x - Lx / 2) ** 4 / Lx ** 4 + 0.5 * (y - Ly / 2) ** 3 * (y - Ly / 2) / Ly ** 4   # periodic, continuous
    q = np.zeros((5, m.n_unique))
    q[0] = f
    out = m.filter(q, order, cutoff)
    s = oracle_mod.filter_sigma(N, order, cutoff)
    xi, _, _ = oracle_mod.gll(N)

    def damp1d(g, lo, L):        # filtered 1D profile of one element at its GLL nodes
        xs = lo + (xi + 1) * L / 4
        coef = npleg.legfit(xi, g(xs), N)
        return xs, npleg.legval(xi, coef * s)

    gx = lambda t: (t - Lx / 2) ** 4 / Lx ** 4
    gy = lambda t: 0.5 * (t - Ly / 2) ** 4 / Ly ** 4
    # f is a sum of an x- and a y-profile; sigma_0 = 1 keeps constants, so each
    # filtered element is the sum of the filtered profiles; on faces the two
    # element copies have equal J w and average.
    def nodal(g, L):
        vals = {}
        for e in range(2):
            xs, v = damp1d(g, e * L / 2, L)
            for a, b in zip(xs, v):
                key = round((a % L) / L * 4 * N) % (4 * N)
                vals.setdefault(key, []).append(b)
        return {k: np.mean(v) for k, v in vals.items()}
    ex, ey = nodal(gx, Lx), nodal(gy, Ly)
    kx = np.round((x % Lx) / Lx * 4 * N).astype(int) % (4 * N)
    ky = np.round((y % Ly) / Ly * 4 * N).astype(int) % (4 * N)
    want = np.array([ex[a] for a in kx]) + np.array([ey[b] for b in ky])
    np.testing.assert_allclose(out[0], want, rtol=0, atol=1e-14)
    assert np.abs(out[0] - f).max() > 1e-4          # the top modes were there and were damped


def test_filter_preserves_low_degree_and_is_identity_at_full_cutoff(oracle_mod):
    N = 5
    m = _filter_box(oracle_mod, N, nz=2, h0=0.0)
    x, y, z = m.get("xu")
    lowdeg = 1.0 + 1e-3 * z + 1e-7 * z * z     # degree 2 in z, constant in x, y
    q = np.zeros((5, m.n_unique))
    q[0] = lowdeg
    q[4] = 3.0 - 2e-3 * z
    out = m.filter(q, 10.0, 2)
    np.testing.assert_allclose(out, q, rtol=0, atol=1e-13)
    rng = np.random.default_rng(7)
    r = np.zeros((5, m.n_unique))
    r[0], r[4] = rng.standard_normal((2, m.n_unique))
    np.testing.assert_allclose(m.filter(r, 10.0, N), r, rtol=0, atol=1e-13)


def test_filter_conserves_mass_and_respects_walls(oracle_mod):
    """Affine elements: the GLL-weighted element integral keeps only the mean
    mode, which sigma_0 = 1 leaves, so sum M q is unchanged for rho' and theta';
    the velocity has no normal component at the walls afterwards."""
    m = _filter_box(oracle_mod, 4, nz=2)
    rng = np.random.default_rng(8)
    q = rng.standard_normal((5, m.n_unique))
    out = m.filter(q, 8.0, 1)
    M = m.get("mass")
    for v in (0, 4):
        assert abs((M * out[v]).sum() - (M * q[v]).sum()) < 1e-12 * (M * np.abs(q[v])).sum()
    assert np.abs(out - q).max() > 0.1
    nrm, isb = m.get("normals"), m.get("isbnd").astype(bool)
    assert np.abs((out[1:4] * nrm).sum(0)[isb]).max() < 1e-14


# --------------------------------------------------------------------------
# SSP-RK(5,3) (Sec. "Time Discretization": five stages, third order; the
# coefficients are those of Spiteri and Ruuth's optimal SSP(5,3) method)
# --------------------------------------------------------------------------
def _butcher(alpha, beta):
    """Shu-Osher (alpha, beta) -> Butcher A (rows: stages 1..5 in terms of L(u_0..u_4))."""
    A = np.zeros((6, 5))
    for i in range(1, 6):
        for k in range(i):
            A[i] += alpha[i, k] * A[k]
            A[i, k] += beta[i, k]
    return A[:5], A[5]


def test_rk53_order_conditions(oracle_mod):
    alpha, beta = oracle_mod.rk53_coeffs()
    np.testing.assert_allclose(alpha[1:].sum(1), 1.0, rtol=0, atol=2e-15)     # consistency
    assert np.all(alpha >= 0) and np.all(beta >= 0)                            # SSP form
    A, b = _butcher(alpha, beta)
    c = A.sum(1)
    assert abs(b.sum() - 1) < 2e-15
    assert abs(b @ c - 1 / 2) < 2e-15
    assert abs(b @ c ** 2 - 1 / 3) < 2e-15
    assert abs(b @ A @ c - 1 / 6) < 2e-15
    # third order exactly: the fourth-order conditions fail
    assert abs(b @ c ** 3 - 1 / 4) > 1e-3 or abs(b @ A @ A @ c - 1 / 24) > 1e-3
    # an optimal SSP method: every nonzero beta_ik has the same alpha_ik / beta_ik
    r = alpha[beta > 0] / beta[beta > 0]
    assert np.ptp(r) < 1e-12 * r[0] and 2.6 < r[0] < 2.7


def test_rk53_linear_amplification(oracle_mod):
    """L(u) = lam u through the stage combination: R(z) agrees with the
    Butcher form's polynomial, whose first four terms are those of exp(z)."""
    alpha, beta = oracle_mod.rk53_coeffs()
    A, b = _butcher(alpha, beta)
    coef = [1.0] + [b @ np.linalg.matrix_power(A, k) @ np.ones(5) for k in range(5)]
    np.testing.assert_allclose(coef[:4], [1, 1, 1 / 2, 1 / 6], rtol=0, atol=2e-15)
    for z in (-0.3, -1.2, -2.5):
        lam, dt = z, 1.0
        U, L = np.zeros((6, 1)), np.zeros((5, 1))
        U[0] = 1.0
        for i in range(1, 6):
            L[i - 1] = lam * U[i - 1]
            U[i] = oracle_mod.rk53_combine(i, dt, U, L)
        assert abs(U[5, 0] - sum(cf * z ** k for k, cf in enumerate(coef))) < 1e-14


def test_rk53_third_order_convergence(oracle_mod):
    """y' = -y^2, y(0) = 1 (y = 1/(1+t)) to t = 1: the error falls 8x per halving."""
    def run(dt):
        y = np.array([[1.0]])
        for _ in range(int(round(1.0 / dt))):
            U, L = np.zeros((6, 1)), np.zeros((5, 1))
            U[0] = y[0]
            for i in range(1, 6):
                L[i - 1] = -U[i - 1] ** 2
                U[i] = oracle_mod.rk53_combine(i, dt, U, L)
            y = U[5:6]
        return abs(y[0, 0] - 0.5)
    e = [run(dt) for dt in (0.2, 0.1, 0.05)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all((rates > 2.8) & (rates < 3.3)), rates


def test_rk53_mesh_invariants(small):
    m, wl = small
    q0 = m.init_state(wl["ic"], inputs.noise(m.n_unique, 0))
    M = m.get("mass")
    rb = m.get("ref")[0]
    q = m.step(q0, 0.05, 6, scheme="ssp53")
    assert abs((M * q[0]).sum() - (M * q0[0]).sum()) <= 1e-13 * (M * rb).sum()
    assert np.array_equal(q, m.step(m.step(q0, 0.05, 3, scheme="ssp53"), 0.05, 3, scheme="ssp53"))


def test_rk53_and_rk3_agree_to_third_order(small):
    """Both schemes are third order: their difference after a fixed time falls
    about 8x when dt halves."""
    m, wl = small
    q0 = m.init_state(wl["ic"], inputs.noise(m.n_unique, 0))
    d = []
    for dt, n in ((0.4, 4), (0.2, 8), (0.1, 16)):
        a = m.step(q0, dt, n, scheme="ssp53")
        b = m.step(q0, dt, n)
        d.append(np.abs(a[4] - b[4]).max())
    rates = np.log2(np.array(d[:-1]) / np.array(d[1:]))
    assert np.all((rates > 2.6) & (rates < 3.4)), (d, rates)


# --------------------------------------------------------------------------
# 1D-IMEX (Sec. "Time Discretization": implicit vertical corrections after an
# explicit leap-frog step; Code example 1: IMEX corrections per column)
# --------------------------------------------------------------------------
def _isentropic(z, ph):
    R, cp, g0, p0, T0 = ph["R"], ph["cp"], ph["g0"], ph["p0"], ph["T0"]
    cv = cp - R
    pi = 1 - g0 * z / (cp * T0)
    rb = p0 / (R * T0) * pi ** (cv / R)
    drb = rb * (cv / R) / pi * (-g0 / (cp * T0))
    return rb, drb, cp / cv


@pytest.mark.parametrize("N,tol", [(4, 1e-6), (6, 1e-9)])
def test_imex_operator_closed_forms(oracle_mod, N, tol):
    """V on states whose vertical terms have closed forms over the isentropic
    reference: w = 1 gives V_rho' = -d rho_bar/dz; rho' = d rho_bar gives
    V_w = (gamma - 1) g0 d (pressure gradient and buoyancy); momentum rows are
    zero at the walls and V_u = V_v = 0; V_theta' vanishes (theta_bar const)."""
    wl = inputs.small_box(N)
    mm, ph = wl["mesh"], wl["phys"]
    m = oracle_mod.OracleMesh(mm["kind"], N, mm["ne"], mm["periodic"], mm["extent"], mm["h0"], ph)
    rb, drb, gam = _isentropic(m.get("xu")[2], ph)
    q = np.zeros((5, m.n_unique))
    q[3] = 1.0
    V = m.imex_V(q)
    assert np.abs(V[0] + drb).max() <= tol * np.abs(drb).max()
    assert np.all(V[1:4] == 0.0) and np.abs(V[4]).max() < 1e-12
    d = 1e-3
    q = np.zeros((5, m.n_unique))
    q[0] = d * rb
    V = m.imex_V(q)
    isb = m.get("isbnd").astype(bool)
    want = (gam - 1) * ph["g0"] * d
    assert np.abs(V[3][~isb] - want).max() <= 10 * tol * want
    assert np.all(V[3][isb] == 0.0) and np.all(V[0] == 0.0) and np.all(V[[1, 2, 4]] == 0.0)


def test_imex_operator_acts_along_vertical_lines(oracle_mod):
    """A unit value at one node: V's response stays on the node's vertical
    lattice line (terrain-following map: d/dz acts along zeta), terrain included."""
    m = _box(oracle_mod, 3, 3, 3, 4, h0=400.0)
    nh = m.n_horiz
    for comp in (0, 3, 4):
        for I in (nh * 5 + 7, nh * 0 + 4, nh * (m.n_levels - 1) + 2):
            E = np.zeros((5, m.n_unique))
            E[comp, I] = 1.0
            V = m.imex_V(E)
            on = np.zeros(m.n_unique, bool)
            on[I % nh::nh] = True
            assert np.abs(V[:, ~on]).max() <= 1e-13 * max(np.abs(V[:, on]).max(), 1.0)


def test_imex_conserves_mass_flat_box(small):
    m, wl = small
    q0 = m.init_state(wl["ic"], inputs.noise(m.n_unique, 0))
    M, rb = m.get("mass"), m.get("ref")[0]
    a, b = m.imex_step(q0, q0, 0.1, 0.05, 6)
    for x in (a, b):
        assert abs((M * x[0]).sum() - (M * q0[0]).sum()) <= 1e-13 * (M * rb).sum()
    assert np.abs(b - q0).max() > 0


def test_imex_second_order(small):
    """Against a fine SSP-RK3 reference to t = 0.8 s, started from the exact
    previous level (one RK3 step back): the error falls 4x per halving of dt
    (leap-frog with a trapezoidal vertical part, no Robert-Asselin filter)."""
    m, wl = small
    q0 = m.init_state(wl["ic"], inputs.noise(m.n_unique, 0))
    ref = m.step(q0, 0.005, 160)
    err = []
    for dt in (0.2, 0.1, 0.05):
        _, b = m.imex_step(m.step(q0, -dt, 1), q0, dt, 0.0, int(round(0.8 / dt)))
        err.append([np.abs(b[v] - ref[v]).max() for v in (0, 3, 4)])
    rates = np.log2(np.array(err[:-1]) / np.array(err[1:]))
    assert np.all((rates > 1.8) & (rates < 2.3)), rates


def test_imex_stable_beyond_the_vertical_acoustic_limit(oracle_mod):
    """Vertical spacing 8x finer than horizontal: explicit SSP-RK3 blows up at
    dt = 0.5 s; the 1D-IMEX step stays bounded at dt = 2 s."""
    wl = inputs.box_workload(4, 4, 8, 4, 40e3, 40e3, 5e3, terrain=0.0, bubble_centre=(20e3, 20e3, 2e3),
                             bubble_radius=2e3)
    mm = wl["mesh"]
    m = oracle_mod.OracleMesh(mm["kind"], mm["N"], mm["ne"], mm["periodic"], mm["extent"], mm["h0"], wl["phys"])
    q0 = m.init_state(wl["ic"], inputs.noise(m.n_unique, 0))
    with np.errstate(all="ignore"):
        x = m.step(q0, 0.5, 80)
    assert not np.all(np.isfinite(x)) or np.abs(x[3]).max() > 1e3
    a, b = m.imex_step(q0, q0, 2.0, 0.05, 20)
    assert np.all(np.isfinite(b)) and np.abs(b[3]).max() < 2 * np.abs(m.step(q0, 0.1, 400)[3]).max()


def test_imex_refuses_periodic_z(oracle_mod):
    m = _box(oracle_mod, 2, 2, 2, 3, periodic_z=1)
    q = np.zeros((5, m.n_unique))
    with pytest.raises(ValueError):
        m.imex_step(q, q, 0.1, 0.0, 1)


def _shell(oracle_mod, ne, nz, N, H):
    wl = inputs.shell_workload(ne=ne, nz=nz, N=N, seed=0, H=H)
    mm = wl["mesh"]
    return oracle_mod.OracleMesh(mm["kind"], N, mm["ne"], mm["periodic"], mm["extent"], mm["h0"], wl["phys"]), wl


def test_imex_operator_closed_forms_shell(oracle_mod):
    """Shell, N = 8: w_r = 1 gives V_rho' = -(1/r^2) d(r^2 rho_bar)/dr (the
    2 rho_bar/r term is 2e-3 of the result), rho' = d rho_bar gives a radial
    V_u = (gamma - 1) g0 (a/r)^2 d over the isothermal reference; no
    tangential part, zero momentum rows at the walls."""
    m, wl = _shell(oracle_mod, 2, 4, 8, 30e3)
    ph, a = wl["phys"], wl["mesh"]["extent"][0]
    xu = m.get("xu")
    r = np.linalg.norm(xu, axis=0)
    n = xu / r
    rb = m.get("ref")[0]
    drb = rb * (-(ph["g0"] * a / (ph["R"] * ph["T0"])) * (a / r ** 2))
    q = np.zeros((5, m.n_unique))
    q[1:4] = n
    V = m.imex_V(q)
    want = -(2 * rb / r + drb)
    assert np.abs(V[0] - want).max() <= 1e-7 * np.abs(want).max()
    d = 1e-3
    q = np.zeros((5, m.n_unique))
    q[0] = d * rb
    V = m.imex_V(q)
    isb = m.get("isbnd").astype(bool)
    gam = ph["cp"] / (ph["cp"] - ph["R"])
    want = (gam - 1) * ph["g0"] * (a / r) ** 2 * d
    Vn = (V[1:4] * n).sum(0)
    assert np.abs(Vn[~isb] - want[~isb]).max() <= 1e-7 * want.max()
    assert np.abs(V[1:4] - Vn * n).max() <= 1e-14 * want.max()
    assert np.all(V[1:4][:, isb] == 0.0)


def test_imex_operator_acts_along_radial_lines(oracle_mod):
    m, _ = _shell(oracle_mod, 3, 4, 4, 30e3)
    nh = m.n_horiz
    for comp in (0, 1, 3, 4):
        I = nh * 5 + 7
        E = np.zeros((5, m.n_unique))
        E[comp, I] = 1.0
        V = m.imex_V(E)
        on = np.zeros(m.n_unique, bool)
        on[I % nh::nh] = True
        assert np.abs(V[:, ~on]).max() <= 1e-15 * np.abs(V[:, on]).max()


def test_imex_second_order_shell(oracle_mod):
    m, wl = _shell(oracle_mod, 3, 4, 4, 30e3)
    q0 = m.init_state(wl["ic"], None)
    ref = m.step(q0, 0.02, 400)
    err = []
    for dt in (2.0, 1.0, 0.5):
        _, b = m.imex_step(m.step(q0, -dt, 1), q0, dt, 0.0, int(round(8.0 / dt)))
        err.append([np.abs(b[v] - ref[v]).max() for v in (0, 1, 4)])
    rates = np.log2(np.array(err[:-1]) / np.array(err[1:]))
    assert np.all((rates > 1.8) & (rates < 2.3)), rates


def test_imex_stable_beyond_the_radial_acoustic_limit(oracle_mod):
    """1.25 km layers under ~840 km horizontal spacing: SSP-RK3 blows up at
    dt = 2 s; 1D-IMEX stays bounded at dt = 20 s for 200 s."""
    m, wl = _shell(oracle_mod, 3, 8, 4, 10e3)
    q0 = m.init_state(wl["ic"], None)
    with np.errstate(all="ignore"):
        x = m.step(q0, 2.0, 20)
    assert not np.all(np.isfinite(x)) or np.abs(x[1:4]).max() > 1e3
    _, b = m.imex_step(q0, q0, 20.0, 0.05, 10)
    assert np.all(np.isfinite(b)) and np.abs(b[1:4]).max() < 1.01 * np.abs(q0[1:4]).max()
