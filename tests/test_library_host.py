"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every declared symbol, and its host mesh numbering matches the oracle's
bit for bit."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_1511_01561_amd import inputs, numa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(numa.LIB_PATH):
        from paper_1511_01561_amd import build
        build.build()
    return numa.lib()


def test_every_declared_symbol_is_exported(L):
    hdr = open(os.path.join(ROOT, "include", "numa.h")).read()
    declared = set(re.findall(r"^\s*(?:const\s+char\s*\*|int32_t)\s*(numa_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(numa.EXPORTED)
    for name in declared:
        assert hasattr(L, name)


def _create(desc):
    d = numa.numa_mesh_desc()
    d.kind = desc["kind"]; d.order = desc["N"]
    for a in range(3):
        d.ne[a] = desc["ne"][a]; d.periodic[a] = desc["periodic"][a]; d.extent[a] = desc["extent"][a]
    d.terrain_amp = desc.get("h0", 0.0)
    h = ct.c_void_p()
    rc = numa.lib().numa_mesh_create(ct.byref(d), ct.byref(h))
    return rc, h


MESHES = [
    dict(kind=0, N=4, ne=(4, 4, 4), periodic=(1, 1, 0), extent=(1e4, 1e4, 1e4), h0=0.0),
    dict(kind=0, N=3, ne=(6, 4, 2), periodic=(1, 1, 1), extent=(1e4, 2e4, 3e3), h0=100.0),
    dict(kind=0, N=1, ne=(2, 2, 1), periodic=(1, 1, 0), extent=(1e3, 1e3, 1e3), h0=0.0),
    dict(kind=0, N=8, ne=(2, 3, 2), periodic=(1, 1, 0), extent=(1e4, 1e4, 1e4), h0=0.0),
    dict(kind=1, N=4, ne=(3, 3, 2), periodic=(0, 0, 0), extent=(6.371e6, 0.0, 3e4), h0=0.0),
    dict(kind=1, N=2, ne=(1, 1, 1), periodic=(0, 0, 0), extent=(6.371e6, 0.0, 3e4), h0=0.0),
    dict(kind=1, N=5, ne=(2, 2, 3), periodic=(0, 0, 0), extent=(6.371e6, 0.0, 3e4), h0=0.0),
]


@pytest.mark.parametrize("desc", MESHES)
def test_gather_map_bit_exact_vs_oracle(L, oracle_mod, desc):
    rc, h = _create(desc)
    assert rc == 0, L.numa_last_error()
    try:
        vals = [ct.c_int64() for _ in range(5)]
        assert L.numa_mesh_info(h, *[ct.byref(v) for v in vals]) == 0
        ne, nl, nu, nh, nk = (v.value for v in vals)
        om = oracle_mod.OracleMesh(desc["kind"], desc["N"], desc["ne"], desc["periodic"], desc["extent"],
                                   desc["h0"], dict(inputs.PHYS, T0=300.0 if desc["kind"] == 0 else 250.0))
        assert (ne, nl, nu, nh, nk) == (om.n_elem, om.n_local, om.n_unique, om.n_horiz, om.n_levels)
        G = np.zeros(nl, dtype=np.int32)
        assert L.numa_mesh_gather_map(h, G.ctypes.data) == 0
        assert np.array_equal(G, om.get("gather").ravel())
    finally:
        L.numa_mesh_destroy(h)


@pytest.mark.parametrize("N", range(1, 9))
def test_library_gll_matches_oracle(L, oracle_mod, N):
    xi, w, D = numa.numa_gll(N)
    oxi, ow, oD = oracle_mod.gll(N)
    np.testing.assert_allclose(xi, oxi, rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, ow, rtol=4e-15, atol=0)
    np.testing.assert_allclose(D, oD, rtol=0, atol=2e-13 * N * N)


@pytest.mark.parametrize("bad", [
    dict(kind=0, N=0, ne=(2, 2, 2), periodic=(1, 1, 0), extent=(1, 1, 1)),
    dict(kind=0, N=9, ne=(2, 2, 2), periodic=(1, 1, 0), extent=(1, 1, 1)),
    dict(kind=0, N=3, ne=(1, 2, 2), periodic=(1, 1, 0), extent=(1, 1, 1)),
    dict(kind=0, N=3, ne=(2, 2, 1), periodic=(1, 1, 1), extent=(1, 1, 1)),
    dict(kind=0, N=3, ne=(2, 2, 2), periodic=(0, 1, 0), extent=(1, 1, 1)),
    dict(kind=0, N=3, ne=(2, 2, 0), periodic=(1, 1, 0), extent=(1, 1, 1)),
    dict(kind=0, N=3, ne=(2, 2, 2), periodic=(1, 1, 0), extent=(1, -1, 1)),
    dict(kind=1, N=3, ne=(0, 0, 2), periodic=(0, 0, 0), extent=(1, 0, 1)),
    dict(kind=7, N=3, ne=(2, 2, 2), periodic=(1, 1, 0), extent=(1, 1, 1)),
])
def test_invalid_mesh_rejected(L, bad):
    rc, h = _create(dict(bad, h0=0.0))
    assert rc == numa.NUMA_OK - 1 and not h.value
    assert len(L.numa_last_error()) > 0


def test_calls_before_setup_are_rejected(L):
    rc, h = _create(MESHES[0])
    assert rc == 0
    try:
        # no workspace: device calls refuse with ENOMEM before touching the GPU
        assert L.numa_rhs(h, 0, ct.c_void_p(16), ct.c_void_p(16), None) == -2
        assert L.numa_step(h, 0, 0.1, 1, ct.c_void_p(16), None) == -2
        assert L.numa_geometry(h, None, None) == -1
        nb = ct.c_uint64()
        assert L.numa_mesh_workspace_bytes(h, 1, ct.byref(nb)) == 0 and nb.value > 0
        nb3 = ct.c_uint64()
        L.numa_mesh_workspace_bytes(h, 3, ct.byref(nb3))
        assert nb3.value > nb.value                    # the mixed path adds the FP32 metric
        assert L.numa_mesh_attach_workspace(h, ct.c_void_p(256), nb.value - 1, 1) == -2
        assert L.numa_mesh_attach_workspace(h, ct.c_void_p(257), nb.value, 1) == -1
    finally:
        L.numa_mesh_destroy(h)


def test_gll_rejects_bad_order(L):
    buf = np.zeros(100)
    assert L.numa_gll(0, buf.ctypes.data, buf.ctypes.data, buf.ctypes.data) == -1
    assert L.numa_gll(9, buf.ctypes.data, buf.ctypes.data, buf.ctypes.data) == -1


def test_mesh_beyond_32bit_indices_rejected(L):
    """n_local >= 2^31 (the index width of the gather map and the E-vector
    copies) is refused before anything is allocated."""
    rc, h = _create(dict(kind=0, N=1, ne=(1300, 1300, 1300), periodic=(1, 1, 0), extent=(1, 1, 1), h0=0.0))
    assert rc == -4 and not h.value
    assert b"32-bit" in L.numa_last_error()


@pytest.mark.parametrize("N,ne,nz", [(1, 2, 2), (3, 2, 3), (4, 3, 2)])
def test_shell_copies_factor_horizontal_times_radial(L, N, ne, nz):
    """The shell's fused finish builds the copies of unique node h + n_h gk as
    (the copies of horizontal node h in the bottom layer) x (the radial
    copies: local k = 0 of layer gk/N and k = N of the layer below on a layer
    boundary, else the one layer).  Check that against the gather map."""
    rc, h = _create(dict(kind=1, N=N, ne=(ne, ne, nz), periodic=(0, 0, 0), extent=(6.371e6, 0.0, 3e4)))
    assert rc == 0
    try:
        vals = [ct.c_int64() for _ in range(5)]
        assert L.numa_mesh_info(h, *[ct.byref(v) for v in vals]) == 0
        n_elem, n_local, n_unique, nh, nk = (v.value for v in vals)
        G = np.zeros(n_local, dtype=np.int32)
        assert L.numa_mesh_gather_map(h, G.ctypes.data) == 0
    finally:
        L.numa_mesh_destroy(h)
    P = N + 1
    np_, pp = P ** 3, P * P
    neh = 6 * ne * ne
    assert nh == 6 * (ne * N) ** 2 + 2 and nk == nz * N + 1
    # horizontal copy lists from the bottom layer, ascending e*np + l
    hcopies = [[] for _ in range(nh)]
    for eh in range(neh):
        for c in range(pp):
            hcopies[G[eh * np_ + c]].append(eh * np_ + c)
    expected = [[] for _ in range(n_unique)]
    for c, I in enumerate(G):
        expected[I].append(c)
    top = nz * N
    for I in range(n_unique):
        hh, gk = I % nh, I // nh
        if gk == top:
            rad = [(nz - 1, N)]
        else:
            ez, kz = gk // N, gk % N
            rad = [(ez, kz)] + ([(ez - 1, N)] if kz == 0 and ez > 0 else [])
        got = sorted(ez * neh * np_ + pp * kz + hc for ez, kz in rad for hc in hcopies[hh])
        assert got == sorted(expected[I]), I
        assert 1 <= len(hcopies[hh]) <= 4


def test_missing_library_fails_loudly():
    """Without the built HIP library the binding raises; nothing falls back
    to a CPU path."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1511_01561_amd import numa\n"
            "numa.LIB_PATH = '/nonexistent/libnuma.so'\n"
            "try:\n    numa.lib()\nexcept numa.NumaError as e:\n    print('raised', e)\n"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert "raised" in out.stdout and "no CPU fallback" in out.stdout, out.stdout + out.stderr


def test_empty_batch_rejected(L):
    """A batch without items is an argument error, refused before any device work."""
    assert L.numa_step_batch(None, 0, 0, 1, None) == -1
    assert b"no items" in L.numa_last_error()
    h = ct.c_void_p()
    assert L.numa_batch_capture(None, 0, 0, 1, None, ct.byref(h)) == -1


@pytest.mark.parametrize("N,order,cutoff", [(1, 12.0, 0), (2, 12.0, 0), (4, 12.0, 1), (5, 6.0, 2), (6, 36.0, 3),
                                            (7, 8.0, 0), (8, 16.0, 4), (8, 16.0, 8), (3, 2.0, 9)])
def test_library_filter_matrix_matches_oracle(L, oracle_mod, N, order, cutoff):
    """Host part of numa_filter: the library's nodal filter matrix (V^-1 from
    the discrete GLL orthogonality) against the oracle's (Gauss-Jordan)."""
    F = numa.numa_filter_matrix(N, order, cutoff)
    np.testing.assert_allclose(F, oracle_mod.filter_matrix(N, order, cutoff), rtol=0, atol=5e-15 * N)


def test_filter_rejects_bad_parameters(L):
    buf = np.zeros(100)
    for order, fo, cut in ((0, 12.0, 1), (9, 12.0, 1), (4, 0.0, 1), (4, -1.0, 1), (4, float("nan"), 1),
                           (4, float("inf"), 1), (4, 12.0, -1)):
        assert L.numa_filter_matrix(order, fo, cut, buf.ctypes.data) == -1, (order, fo, cut)
        assert len(L.numa_last_error()) > 0
    assert L.numa_filter_matrix(4, 12.0, 1, None) == -1
    rc, h = _create(MESHES[0])
    assert rc == 0
    try:   # no workspace: refused before touching the GPU
        assert L.numa_filter(h, 12.0, 1, ct.c_void_p(16), None) == -2
    finally:
        L.numa_mesh_destroy(h)


def test_set_filter_validates_on_the_host(L):
    rc, h = _create(MESHES[0])
    assert rc == 0
    try:
        assert L.numa_mesh_set_filter(h, 1, 12.0, 1) == 0
        assert L.numa_mesh_set_filter(h, 1, 0.0, 1) == -1
        assert L.numa_mesh_set_filter(h, 1, 12.0, -1) == -1
        assert L.numa_mesh_set_filter(h, 0, float("nan"), -5) == 0     # off: parameters ignored
        assert L.numa_mesh_set_filter(None, 0, 0.0, 0) == -1
    finally:
        L.numa_mesh_destroy(h)


def test_integrator_setting_and_scratch_size(L):
    rc, h = _create(MESHES[0])
    assert rc == 0
    try:
        a, b = ct.c_uint64(), ct.c_uint64()
        assert L.numa_step_scratch_bytes(h, 0, ct.byref(a)) == 0
        assert L.numa_mesh_set_integrator(h, numa.RK_SSP53) == 0
        assert L.numa_step_scratch_bytes(h, 0, ct.byref(b)) == 0
        nu, nl = ct.c_int64(), ct.c_int64()
        assert L.numa_mesh_info(h, None, ct.byref(nl), ct.byref(nu), None, None) == 0
        # both integrators keep two stage states (no stage writes its own input)
        # beside the contributions (FP64 element-local, or an FP64 unique-node sum)
        r = lambda x: (x + 255) // 256 * 256
        assert a.value == b.value == 2 * r(40 * nu.value) + r(max(40 * nl.value, 40 * nu.value))
        m = ct.c_uint64()
        assert L.numa_step_scratch_bytes(h, 1, ct.byref(m)) == 0
        assert m.value == 2 * r(40 * nu.value) + r(max(20 * nl.value, 40 * nu.value))
        assert L.numa_mesh_set_integrator(h, 2) == -1 and L.numa_mesh_set_integrator(h, -1) == -1
        assert L.numa_mesh_set_integrator(None, 0) == -1
        assert L.numa_mesh_set_integrator(h, numa.RK_SSP33) == 0
    finally:
        L.numa_mesh_destroy(h)


def test_imex_step_refused_before_setup(L):
    assert L.numa_imex_step(None, 0, 0.1, 0.0, 1, ct.c_void_p(16), ct.c_void_p(32), None) == -1
    rc, h = _create(MESHES[0])
    assert rc == 0
    try:   # no workspace: refused before touching the GPU
        assert L.numa_imex_step(h, 0, 0.1, 0.0, 1, ct.c_void_p(16), ct.c_void_p(32), None) == -2
        nb, nb4 = ct.c_uint64(), ct.c_uint64()
        assert L.numa_mesh_workspace_bytes(h, 1, ct.byref(nb)) == 0
        assert L.numa_mesh_workspace_bytes(h, 1 | numa.WS_IMEX, ct.byref(nb4)) == 0
        assert nb4.value > nb.value          # the line factors
    finally:
        L.numa_mesh_destroy(h)


def test_lean_workspace_holds_only_what_batched_steps_read(L):
    """NUMA_WS_LEAN: the inverse map, reference, M, M^-1, the recomputed
    mass, wall normals, coordinates, column factors and the GLL tables, each
    256-byte aligned; refused on meshes the batched steps do not take."""
    def a256(x):
        return (x + 255) // 256 * 256

    wl = inputs.box_workload(8, 4, 3, 4, 5e4, 2.5e4, 6e3, terrain=300.0)
    rc, h = _create(wl["mesh"])
    assert rc == 0
    try:
        ne, nl, nu, nh, nk = (ct.c_int64() for _ in range(5))
        assert L.numa_mesh_info(h, ct.byref(ne), ct.byref(nl), ct.byref(nu), ct.byref(nh), ct.byref(nk)) == 0
        nl, nu, nh, P, kp = nl.value, nu.value, nh.value, 5, 9
        want = (a256(4 * (nu + 1)) + a256(4 * nl) + a256(24 * nu) + 3 * a256(8 * nu) + a256(48 * nh)
                + a256(24 * nu) + a256(32 * 8 * 4 * P * P) + a256(8 * kp * kp) + a256(4 * kp * kp)
                + 2 * a256(8 * kp) + a256(4))
        lean, full = ct.c_uint64(), ct.c_uint64()
        assert L.numa_mesh_workspace_bytes(h, 3 | numa.WS_LEAN, ct.byref(lean)) == 0
        assert L.numa_mesh_workspace_bytes(h, 3, ct.byref(full)) == 0
        assert lean.value == want and full.value > 4 * lean.value
        # binding a lean workspace is host-only; the device calls then still need the geometry
        assert L.numa_mesh_attach_workspace(h, ct.c_void_p(256), lean.value, 3 | numa.WS_LEAN) == 0
    finally:
        L.numa_mesh_destroy(h)
    for mesh in (inputs.shell_workload(ne=3, nz=2, N=4, seed=0)["mesh"],             # shell
                 inputs.box_workload(6, 4, 3, 4, 5e4, 2.5e4, 6e3)["mesh"]):           # nx not a multiple of 4
        rc, h = _create(mesh)
        assert rc == 0
        try:
            nb = ct.c_uint64()
            assert L.numa_mesh_workspace_bytes(h, 1 | numa.WS_LEAN, ct.byref(nb)) == 0
            assert L.numa_mesh_attach_workspace(h, ct.c_void_p(256), nb.value, 1 | numa.WS_LEAN) == -4
        finally:
            L.numa_mesh_destroy(h)
