"""FP64 CPU oracle for the NUMA spectral-element hot path (test infrastructure).

This package is test infrastructure only: the test suite, the smoke check and
the CPU-baseline leg of the benchmark may load it; the product path never does.
It wraps ``numa_oracle.c`` (plain C, FP64, no FMA contraction) through ctypes.
The C source cites, routine by routine, the section or equation of the paper
(Mueller et al., IJHPCA 2016) that it follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "numa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _MeshDesc(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("N", ct.c_int32), ("ne", ct.c_int32 * 3),
                ("periodic", ct.c_int32 * 3), ("extent", ct.c_double * 3), ("h0", ct.c_double)]


class _Phys(ct.Structure):
    _fields_ = [("R", ct.c_double), ("cp", ct.c_double), ("g0", ct.c_double),
                ("p0", ct.c_double), ("T0", ct.c_double)]


class _IC(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("amp", ct.c_double), ("radius", ct.c_double),
                ("c", ct.c_double * 3), ("lz", ct.c_double), ("jet_u0", ct.c_double),
                ("noise_amp", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ct.CDLL(_LIB)
        P = ct.c_void_p
        L.or_create.restype = P
        L.or_create.argtypes = [ct.POINTER(_MeshDesc), ct.POINTER(_Phys)]
        L.or_destroy.argtypes = [P]
        L.or_info.argtypes = [P, P]
        L.or_get.argtypes = [P, ct.c_int, P]
        L.or_set.argtypes = [P, ct.c_int, P]
        L.or_gll.argtypes = [ct.c_int, P, P, P]
        L.or_counts.argtypes = [ct.POINTER(_MeshDesc), P, P, P]
        L.or_init_state.argtypes = [P, ct.POINTER(_IC), P, P]
        L.or_rhs.argtypes = [P, P, P]
        L.or_rhs_scale.argtypes = [P, P, P]
        L.or_dss.argtypes = [P, ct.c_int, P, ct.c_int, P]
        L.or_rk_stage.argtypes = [P, ct.c_int, ct.c_double, P, P, P, P]
        L.or_step.argtypes = [P, ct.c_double, ct.c_int, P]
        L.or_filter_sigma.argtypes = [ct.c_int, ct.c_double, ct.c_int, P]
        L.or_filter_matrix.argtypes = [ct.c_int, ct.c_double, ct.c_int, P]
        L.or_filter.argtypes = [P, ct.c_double, ct.c_int, P]
        L.or_rk53_coeffs.argtypes = [P, P]
        L.or_rk53_combine.argtypes = [ct.c_int64, ct.c_int, ct.c_double, P, P, P]
        L.or_step_rk53.argtypes = [P, ct.c_double, ct.c_int, P]
        L.or_imex_V.argtypes = [P, P, P]
        L.or_imex_step.argtypes = [P, ct.c_double, ct.c_double, ct.c_int, P, P, P, ct.c_int]
        L.or_set_threads.argtypes = [ct.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ct.c_void_p)


def gll(N: int):
    """(xi, w, D) of order N from the oracle; D[i, m] = dpsi_m/dxi at xi_i."""
    xi = np.zeros(N + 1); w = np.zeros(N + 1); D = np.zeros((N + 1, N + 1))
    if lib().or_gll(N, _p(xi), _p(w), _p(D)) != 0:
        raise ValueError("order out of range")
    return xi, w, D


def _desc(kind, N, ne, periodic, extent, h0):
    d = _MeshDesc()
    d.kind = kind; d.N = N
    for a in range(3):
        d.ne[a] = int(ne[a]); d.periodic[a] = int(periodic[a]); d.extent[a] = float(extent[a])
    d.h0 = float(h0)
    return d


def _phys(phys):
    p = _Phys()
    for k, v in phys.items():
        setattr(p, k, float(v))
    return p


def counts(kind, N, ne, periodic=(1, 1, 0), extent=(1.0, 1.0, 1.0), h0=0.0):
    d = _desc(kind, N, ne, periodic, extent, h0)
    a = np.zeros(3, dtype=np.int64)
    if lib().or_counts(ct.byref(d), _p(a[0:1]), _p(a[1:2]), _p(a[2:3])) != 0:
        raise ValueError("invalid mesh description")
    return int(a[0]), int(a[1]), int(a[2])


class OracleMesh:
    """Mesh, geometry and reference state built by the oracle, plus the RHS,
    DSS, RK-stage and step operators on it.  All arrays are numpy FP64."""

    def __init__(self, kind, N, ne, periodic=(1, 1, 0), extent=(1.0, 1.0, 1.0), h0=0.0,
                 phys=None):
        self.phys = dict(R=287.0, cp=1004.5, g0=9.81, p0=1.0e5, T0=300.0)
        if phys:
            self.phys.update(phys)
        self._d = _desc(kind, N, ne, periodic, extent, h0)
        self._ph = _phys(self.phys)
        self._h = lib().or_create(ct.byref(self._d), ct.byref(self._ph))
        if not self._h:
            raise ValueError("oracle: invalid mesh or non-positive Jacobian")
        info = np.zeros(5, dtype=np.int64)
        lib().or_info(self._h, _p(info))
        self.kind, self.N = kind, N
        self.P = N + 1
        self.np = self.P ** 3
        self.n_elem, self.n_local, self.n_unique, self.n_horiz, self.n_levels = (int(x) for x in info)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    def get(self, name: str) -> np.ndarray:
        nl, nu = self.n_local, self.n_unique
        spec = {"gather": (0, (self.n_elem, self.np), np.int32),
                "xl": (1, (3, nl), np.float64), "xu": (2, (3, nu), np.float64),
                "metric": (3, (10, nl), np.float64), "mass": (4, (nu,), np.float64),
                "ref": (5, (3, nu), np.float64), "gravity": (6, (3, nu), np.float64),
                "normals": (7, (3, nu), np.float64), "isbnd": (8, (nu,), np.int32)}
        if name == "gll":
            buf = np.zeros(2 * self.P + self.P * self.P)
            lib().or_get(self._h, 9, _p(buf))
            return buf[:self.P], buf[self.P:2 * self.P], buf[2 * self.P:].reshape(self.P, self.P)
        code, shape, dt = spec[name]
        out = np.zeros(shape, dtype=dt)
        lib().or_get(self._h, code, _p(out))
        return out

    def set_reference(self, ref: np.ndarray) -> None:
        ref = np.ascontiguousarray(ref, dtype=np.float64).reshape(3, self.n_unique)
        lib().or_set(self._h, 5, _p(ref))

    def set_gravity(self, g: np.ndarray) -> None:
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(3, self.n_unique)
        lib().or_set(self._h, 6, _p(g))

    def init_state(self, ic: dict, noise: np.ndarray | None = None) -> np.ndarray:
        d = _IC()
        d.kind = int(ic.get("kind", 0))
        d.amp = float(ic.get("amp", 0.0)); d.radius = float(ic.get("radius", 1.0))
        c = ic.get("centre", (0.0, 0.0, 0.0))
        for a in range(3):
            d.c[a] = float(c[a])
        d.lz = float(ic.get("lz", 1.0)); d.jet_u0 = float(ic.get("jet_u0", 0.0))
        d.noise_amp = float(ic.get("noise_amp", 0.0))
        q = np.zeros((5, self.n_unique))
        nz = None
        if noise is not None:
            nz = np.ascontiguousarray(noise, dtype=np.float64).reshape(3, self.n_unique)
        lib().or_init_state(self._h, ct.byref(d), _p(nz) if nz is not None else None, _p(q))
        return q

    def rhs(self, q: np.ndarray) -> np.ndarray:
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(5, self.n_unique)
        out = np.zeros((5, self.n_local))
        lib().or_rhs(self._h, _p(q), _p(out))
        return out

    def rhs_scale(self, q: np.ndarray) -> np.ndarray:
        """J w times the sum of |individual terms| of each R (conditioning scale)."""
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(5, self.n_unique)
        out = np.zeros((5, self.n_local))
        lib().or_rhs_scale(self._h, _p(q), _p(out))
        return out

    def dss(self, cin: np.ndarray, flags: int = 1) -> np.ndarray:
        cin = np.ascontiguousarray(cin, dtype=np.float64)
        nvar = cin.size // self.n_local
        cin = cin.reshape(nvar, self.n_local)
        out = np.zeros((nvar, self.n_unique))
        lib().or_dss(self._h, nvar, _p(cin), flags, _p(out))
        return out

    def rk_stage(self, stage, dt, qn, qs, r) -> np.ndarray:
        qn = np.ascontiguousarray(qn, dtype=np.float64).reshape(5, self.n_unique)
        qs = np.ascontiguousarray(qs, dtype=np.float64).reshape(5, self.n_unique)
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(5, self.n_unique)
        out = np.zeros((5, self.n_unique))
        lib().or_rk_stage(self._h, stage, dt, _p(qn), _p(qs), _p(r), _p(out))
        return out

    def filter(self, q: np.ndarray, order: float, cutoff: int) -> np.ndarray:
        """Filtered state: element filter, J w weighting, DSS / M, no-flux."""
        q = np.array(q, dtype=np.float64, copy=True).reshape(5, self.n_unique)
        rc = lib().or_filter(self._h, float(order), int(cutoff), _p(q))
        if rc != 0:
            raise ValueError("oracle filter (%d)" % rc)
        return q

    def imex_V(self, q: np.ndarray) -> np.ndarray:
        """The vertical linear operator of the 1D-IMEX correction."""
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(5, self.n_unique)
        out = np.zeros((5, self.n_unique))
        if lib().or_imex_V(self._h, _p(q), _p(out)) != 0:
            raise MemoryError("oracle imex_V")
        return out

    def imex_step(self, qprev, qcur, dt: float, ra: float, nsteps: int, lines=None):
        """nsteps 1D-IMEX leap-frog steps; returns the new (qprev, qcur)."""
        a = np.array(qprev, dtype=np.float64, copy=True).reshape(5, self.n_unique)
        b = np.array(qcur, dtype=np.float64, copy=True).reshape(5, self.n_unique)
        ln = None if lines is None else np.ascontiguousarray(lines, dtype=np.int32)
        rc = lib().or_imex_step(self._h, float(dt), float(ra), int(nsteps), _p(a), _p(b),
                                None if ln is None else _p(ln), 0 if ln is None else len(ln))
        if rc != 0:
            raise ValueError("oracle imex step (%d)" % rc)
        return a, b

    def step(self, q: np.ndarray, dt: float, nsteps: int, scheme: str = "ssp33") -> np.ndarray:
        """nsteps steps of SSP-RK3 (scheme "ssp33") or SSP-RK(5,3) ("ssp53")."""
        q = np.array(q, dtype=np.float64, copy=True).reshape(5, self.n_unique)
        fn = {"ssp33": lib().or_step, "ssp53": lib().or_step_rk53}[scheme]
        if fn(self._h, dt, nsteps, _p(q)) != 0:
            raise MemoryError("oracle step")
        return q


def filter_sigma(N: int, order: float, cutoff: int) -> np.ndarray:
    """Boyd-Vandeven modal factors sigma_0..sigma_N (erfc-log form)."""
    s = np.zeros(N + 1)
    if lib().or_filter_sigma(N, float(order), int(cutoff), _p(s)) != 0:
        raise ValueError("filter parameters")
    return s


def filter_matrix(N: int, order: float, cutoff: int) -> np.ndarray:
    """1D nodal filter matrix V diag(sigma) V^-1, F[i, m]."""
    F = np.zeros((N + 1, N + 1))
    if lib().or_filter_matrix(N, float(order), int(cutoff), _p(F)) != 0:
        raise ValueError("filter parameters")
    return F


def rk53_coeffs():
    """alpha, beta ([6][5]) of the oracle's SSP-RK(5,3) Shu-Osher form."""
    a, b = np.zeros((6, 5)), np.zeros((6, 5))
    lib().or_rk53_coeffs(_p(a), _p(b))
    return a, b


def rk53_combine(i: int, dt: float, U: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Stage i (1..5) from the stage values U [6][n] and L(u_k) [5][n]."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    n = U.shape[1]
    out = np.zeros(n)
    if lib().or_rk53_combine(n, i, float(dt), _p(U), _p(L), _p(out)) != 0:
        raise ValueError("stage index")
    return out


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (timing only)."""
    lib().or_set_threads(int(n))
