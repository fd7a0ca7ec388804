"""Thin ctypes binding of libnuma (include/numa.h), same names as the C ABI.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  torch supplies device memory (the workspace and the state tensors)
and the stream (torch.cuda.current_stream()).  If libnuma.so has not been
built, loading fails with an error; there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnuma.so")

NUMA_OK = 0
MESH_BOX, MESH_SHELL = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
DSS_MASS, DSS_NOFLUX = 1, 2
METRIC_STORED, METRIC_RECOMPUTE = 0, 1
RK_SSP33, RK_SSP53 = 0, 1
STAGE_GATHER, STAGE_BLOCK, STAGE_COLOUR, STAGE_SPLIT, STAGE_AUTO = 0, 1, 2, 3, 4
WS_IMEX = 4
WS_LEAN = 8
FIELD_MASS, FIELD_REF, FIELD_COORDS, FIELD_METRIC, FIELD_GRAVITY, FIELD_LOCAL_COORDS = range(6)

EXPORTED = ["numa_last_error", "numa_gll", "numa_mesh_create", "numa_mesh_destroy", "numa_mesh_info",
            "numa_mesh_gather_map", "numa_mesh_workspace_bytes", "numa_mesh_attach_workspace",
            "numa_geometry", "numa_export", "numa_init_state", "numa_rhs", "numa_dss",
            "numa_rk_stage", "numa_step", "numa_profile", "numa_profile_read", "numa_step_scratch_bytes",
            "numa_step_batch", "numa_batch_capture", "numa_graph_launch", "numa_graph_destroy",
            "numa_mesh_set_metric", "numa_filter", "numa_filter_matrix", "numa_mesh_set_filter",
            "numa_mesh_set_integrator", "numa_imex_step", "numa_stage_rhs", "numa_mesh_set_stage",
            "numa_step_batch_noalloc", "numa_mesh_set_step_graph"]


class numa_mesh_desc(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("order", ct.c_int32), ("ne", ct.c_int32 * 3),
                ("periodic", ct.c_int32 * 3), ("extent", ct.c_double * 3), ("terrain_amp", ct.c_double)]


class numa_phys(ct.Structure):
    _fields_ = [("R", ct.c_double), ("cp", ct.c_double), ("g0", ct.c_double), ("p0", ct.c_double),
                ("T0", ct.c_double)]


class numa_ic(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("amp", ct.c_double), ("radius", ct.c_double), ("c", ct.c_double * 3),
                ("lz", ct.c_double), ("jet_u0", ct.c_double), ("noise_amp", ct.c_double)]


class numa_batch_item(ct.Structure):
    _fields_ = [("mesh", ct.c_void_p), ("q", ct.c_void_p), ("scratch", ct.c_void_p), ("scratch_bytes", ct.c_uint64),
                ("dt", ct.c_double), ("nonfinite", ct.c_void_p)]


class NumaError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libnuma.so (built in-tree by paper_1511_01561_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NumaError("libnuma.so is not built (run python -m paper_1511_01561_amd.build); "
                        "there is no CPU fallback")
    L = ct.CDLL(LIB_PATH)
    P, I32, I64, D = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_double
    sig = {
        "numa_last_error": (ct.c_char_p, []),
        "numa_gll": (I32, [I32, P, P, P]),
        "numa_mesh_create": (I32, [ct.POINTER(numa_mesh_desc), ct.POINTER(P)]),
        "numa_mesh_destroy": (I32, [P]),
        "numa_mesh_info": (I32, [P, P, P, P, P, P]),
        "numa_mesh_gather_map": (I32, [P, P]),
        "numa_mesh_workspace_bytes": (I32, [P, I32, ct.POINTER(ct.c_uint64)]),
        "numa_mesh_attach_workspace": (I32, [P, P, ct.c_uint64, I32]),
        "numa_geometry": (I32, [P, ct.POINTER(numa_phys), P]),
        "numa_export": (I32, [P, I32, P, P]),
        "numa_init_state": (I32, [P, ct.POINTER(numa_ic), P, P, P]),
        "numa_rhs": (I32, [P, I32, P, P, P]),
        "numa_dss": (I32, [P, I32, P, P, I32, P]),
        "numa_rk_stage": (I32, [P, I32, D, P, P, P, P, P]),
        "numa_filter": (I32, [P, D, I32, P, P]),
        "numa_filter_matrix": (I32, [I32, D, I32, P]),
        "numa_mesh_set_filter": (I32, [P, I32, D, I32]),
        "numa_mesh_set_integrator": (I32, [P, I32]),
        "numa_imex_step": (I32, [P, I32, D, D, I32, P, P, P]),
        "numa_step": (I32, [P, I32, D, I32, P, P]),
        "numa_stage_rhs": (I32, [P, I32, P, P, P]),
        "numa_profile": (I32, [P, I32]),
        "numa_profile_read": (I32, [P, P]),
        "numa_step_scratch_bytes": (I32, [P, I32, ct.POINTER(ct.c_uint64)]),
        "numa_step_batch": (I32, [ct.POINTER(numa_batch_item), I32, I32, I32, P]),
        "numa_step_batch_noalloc": (I32, [ct.POINTER(numa_batch_item), I32, I32, I32, P]),
        "numa_mesh_set_step_graph": (I32, [P, I32]),
        "numa_batch_capture": (I32, [ct.POINTER(numa_batch_item), I32, I32, I32, P, ct.POINTER(P)]),
        "numa_graph_launch": (I32, [P, P]),
        "numa_graph_destroy": (I32, [P]),
        "numa_mesh_set_metric": (I32, [P, I32]),
        "numa_mesh_set_stage": (I32, [P, I32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != NUMA_OK:
        raise NumaError("libnuma error %d: %s" % (rc, lib().numa_last_error().decode()))


def numa_gll(order: int):
    import numpy as np
    xi = np.zeros(order + 1); w = np.zeros(order + 1); D = np.zeros((order + 1, order + 1))
    check(lib().numa_gll(order, xi.ctypes.data, w.ctypes.data, D.ctypes.data))
    return xi, w, D


def numa_filter_matrix(order: int, filter_order: float, cutoff: int):
    import numpy as np
    F = np.zeros((order + 1, order + 1))
    check(lib().numa_filter_matrix(order, float(filter_order), int(cutoff), F.ctypes.data))
    return F


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous() and t.dtype.is_floating_point, "device FP64 contiguous tensor expected"
    return ct.c_void_p(t.data_ptr())


def _desc(mesh: dict):
    d = numa_mesh_desc()
    d.kind = int(mesh["kind"]); d.order = int(mesh["N"])
    for a in range(3):
        d.ne[a] = int(mesh["ne"][a]); d.periodic[a] = int(mesh["periodic"][a])
        d.extent[a] = float(mesh["extent"][a])
    d.terrain_amp = float(mesh.get("h0", 0.0))
    return d


def mesh_sizes(mesh: dict, prec_mask: int, prec: int):
    """Host only: (device workspace bytes, unique nodes, batch scratch bytes of
    one item in precision prec) of a mesh description, without building it on
    the device."""
    d = _desc(mesh)
    h = ct.c_void_p()
    check(lib().numa_mesh_create(ct.byref(d), ct.byref(h)))
    try:
        nb, sb, nu = ct.c_uint64(), ct.c_uint64(), ct.c_int64()
        check(lib().numa_mesh_workspace_bytes(h, prec_mask, ct.byref(nb)))
        check(lib().numa_step_scratch_bytes(h, prec, ct.byref(sb)))
        check(lib().numa_mesh_info(h, None, None, ct.byref(nu), None, None))
        return nb.value, nu.value, sb.value
    finally:
        lib().numa_mesh_destroy(h)


class Mesh:
    """A mesh handle with its device workspace (a torch uint8 tensor)."""

    def __init__(self, mesh: dict, phys: dict, prec_mask: int = 3, device="cuda:0", stream=None):
        import torch
        self.device = torch.device(device)
        d = _desc(mesh)
        self._desc = d
        h = ct.c_void_p()
        check(lib().numa_mesh_create(ct.byref(d), ct.byref(h)))
        self._h = h
        vals = [ct.c_int64() for _ in range(5)]
        check(lib().numa_mesh_info(h, *[ct.byref(v) for v in vals]))
        self.n_elem, self.n_local, self.n_unique, self.n_horiz, self.n_levels = (v.value for v in vals)
        self.N = d.order
        self.np = (self.N + 1) ** 3
        nb = ct.c_uint64()
        check(lib().numa_mesh_workspace_bytes(h, prec_mask, ct.byref(nb)))
        self.workspace_bytes = nb.value
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        check(lib().numa_mesh_attach_workspace(h, ct.c_void_p(base + off), nb.value, prec_mask))
        ph = numa_phys()
        for k in ("R", "cp", "g0", "p0", "T0"):
            setattr(ph, k, float(phys[k]))
        self._phys = ph
        check(lib().numa_geometry(h, ct.byref(ph), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.numa_mesh_destroy(self._h)
            self._h = None

    __del__ = close

    # -- host -----------------------------------------------------------------
    def gather_map(self):
        import numpy as np
        out = np.zeros((self.n_elem, self.np), dtype=np.int32)
        check(lib().numa_mesh_gather_map(self._h, out.ctypes.data))
        return out

    # -- device ---------------------------------------------------------------
    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def export(self, what: int, stream=None):
        nu, nl = self.n_unique, self.n_local
        shape = {FIELD_MASS: (nu,), FIELD_REF: (3, nu), FIELD_COORDS: (3, nu), FIELD_METRIC: (10, nl),
                 FIELD_GRAVITY: (3, nu), FIELD_LOCAL_COORDS: (3, nl)}[what]
        out = self._empty(*shape)
        check(lib().numa_export(self._h, what, _ptr(out), _stream(stream)))
        return out

    def init_state(self, ic: dict, noise=None, stream=None):
        d = numa_ic()
        d.kind = int(ic.get("kind", 0)); d.amp = float(ic.get("amp", 0.0)); d.radius = float(ic.get("radius", 1.0))
        c = ic.get("centre", (0.0, 0.0, 0.0))
        for a in range(3):
            d.c[a] = float(c[a])
        d.lz = float(ic.get("lz", 1.0)); d.jet_u0 = float(ic.get("jet_u0", 0.0))
        d.noise_amp = float(ic.get("noise_amp", 0.0))
        q = self._empty(5, self.n_unique)
        check(lib().numa_init_state(self._h, ct.byref(d), _ptr(noise), _ptr(q), _stream(stream)))
        return q

    def rhs(self, q, prec=PREC_FP64, out=None, stream=None):
        if out is None:
            out = self._empty(5, self.n_local)
        check(lib().numa_rhs(self._h, prec, _ptr(q), _ptr(out), _stream(stream)))
        return out

    def stage_rhs(self, q, prec=PREC_FP64, out=None, stream=None):
        """M^-1 DSS(J w R) with the wall projection, by numa_step's stage kernels."""
        if out is None:
            out = self._empty(5, self.n_unique)
        check(lib().numa_stage_rhs(self._h, prec, _ptr(q), _ptr(out), _stream(stream)))
        return out

    def dss(self, c_elem, flags=DSS_MASS, out=None, stream=None):
        nvar = c_elem.numel() // self.n_local
        if out is None:
            out = self._empty(nvar, self.n_unique)
        check(lib().numa_dss(self._h, nvar, _ptr(c_elem), _ptr(out), flags, _stream(stream)))
        return out

    def filter(self, q, filter_order, cutoff, stream=None):
        """Boyd-Vandeven filter of the state q [5][n_unique] in place."""
        check(lib().numa_filter(self._h, float(filter_order), int(cutoff), _ptr(q), _stream(stream)))
        return q

    def imex_step(self, qprev, qcur, dt, ra, nsteps, prec=PREC_FP64, stream=None):
        """nsteps 1D-IMEX leap-frog steps on the pair (q^{n-1}, q^n), in place."""
        check(lib().numa_imex_step(self._h, prec, float(dt), float(ra), int(nsteps), _ptr(qprev), _ptr(qcur),
                                   _stream(stream)))
        return qprev, qcur

    def set_integrator(self, integrator: int):
        """RK_SSP33 (default) or RK_SSP53 for step() and the batched steps."""
        check(lib().numa_mesh_set_integrator(self._h, int(integrator)))

    def set_filter(self, filter_order=None, cutoff=0):
        """Filter after every step of step() and the batched steps (None: off)."""
        on = filter_order is not None
        check(lib().numa_mesh_set_filter(self._h, 1 if on else 0, float(filter_order or 0.0), int(cutoff)))

    def rk_stage(self, stage, dt, qn, qs, r, out=None, stream=None):
        if out is None:
            out = self._empty(5, self.n_unique)
        check(lib().numa_rk_stage(self._h, stage, float(dt), _ptr(qn), _ptr(qs), _ptr(r), _ptr(out),
                                  _stream(stream)))
        return out

    def set_metric(self, mode: int):
        """METRIC_STORED or METRIC_RECOMPUTE (box meshes)."""
        check(lib().numa_mesh_set_metric(self._h, mode))

    def set_step_graph(self, enable: bool):
        """numa_step replays a captured step (default) or launches directly"""
        check(lib().numa_mesh_set_step_graph(self._h, int(bool(enable))))

    def set_stage(self, mode: int):
        """STAGE_AUTO (default), STAGE_GATHER, STAGE_BLOCK, STAGE_COLOUR or STAGE_SPLIT: how a fused stage sums the copies."""
        check(lib().numa_mesh_set_stage(self._h, mode))

    def profile(self, enable: bool):
        check(lib().numa_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(element-kernel ms total, launches, finish ms total, launches)"""
        out = (ct.c_double * 4)()
        check(lib().numa_profile_read(self._h, out))
        return tuple(out)

    def step(self, q, dt, nsteps, prec=PREC_FP64, stream=None):
        """nsteps steps of the mesh's integrator in place on q (device [5][n_unique] FP64)."""
        check(lib().numa_step(self._h, prec, float(dt), int(nsteps), _ptr(q), _stream(stream)))
        return q


def step_scratch_bytes(mesh: Mesh, prec: int) -> int:
    nb = ct.c_uint64()
    check(lib().numa_step_scratch_bytes(mesh._h, prec, ct.byref(nb)))
    return nb.value


def alloc_scratch(mesh: Mesh, prec: int):
    """Device scratch for one batch item (a torch uint8 tensor, 256-byte aligned view)."""
    import torch
    nb = step_scratch_bytes(mesh, prec)
    buf = torch.empty(nb + 256, dtype=torch.uint8, device=mesh.device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nb]


def _items(items):
    """items: sequence of (mesh, q, scratch, dt) or (mesh, q, scratch, dt, flag),
    scratch None for the library's own, flag a device int32 tensor element (a
    view of one element) or None"""
    arr = (numa_batch_item * len(items))()
    for k, it in enumerate(items):
        m, q, scr, dt = it[:4]
        flag = it[4] if len(it) > 4 else None
        arr[k].mesh = m._h.value if isinstance(m._h, ct.c_void_p) else m._h
        arr[k].q = q.data_ptr()
        arr[k].scratch = scr.data_ptr() if scr is not None else None
        arr[k].scratch_bytes = scr.numel() * scr.element_size() if scr is not None else 0
        arr[k].dt = float(dt)
        arr[k].nonfinite = flag.data_ptr() if flag is not None else None
    return arr


def step_batch(items, nsteps: int, prec: int = PREC_FP64, stream=None):
    """Advance every (mesh, q, scratch, dt[, flag]) item by nsteps steps in
    batched launches (same order, metric mode and integrator, box meshes)."""
    arr = _items(items)
    check(lib().numa_step_batch(arr, len(items), prec, int(nsteps), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 128 << 20
NOALLOC_MAX_ITEMS = 64


def step_batch_noalloc(items, nsteps: int, prec: int = PREC_FP64, stream=None):
    """step_batch over (mesh, q, dt[, flag]) items whose scratch the library
    takes from its static device array (numa_step_batch_noalloc); nsteps = 0
    with no items only looks up the array on the current device."""
    arr = _items([(it[0], it[1], None) + tuple(it[2:]) for it in items])
    check(lib().numa_step_batch_noalloc(arr, len(items), prec, int(nsteps), _stream(stream)))


class Graph:
    """A captured batch step (numa_batch_capture); replay with launch()."""

    def __init__(self, items, nsteps: int, prec: int, stream):
        arr = _items(items)
        h = ct.c_void_p()
        check(lib().numa_batch_capture(arr, len(items), prec, int(nsteps), _stream(stream), ct.byref(h)))
        self._h = h

    def launch(self, stream=None):
        check(lib().numa_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.numa_graph_destroy(self._h)
            self._h = None

    __del__ = close
