"""Benchmark of the NUMA hot path on one MI355X.

A step is one SSP-RK3 step (three stages of right-hand side + DSS + stage
update) over the 64 x 64 x 16 element, N = 4 terrain-following box
(400 x 400 x 20 km, 4,259,840 unique grid points), inputs resident in HBM.
The metric counts grid-point RHS updates: unique nodes x 3 stages per step.

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# the stage kernels' sources: a traffic record holds only while they are unchanged
_STAGE_SOURCES = [os.path.join(ROOT, "paper_1511_01561_amd", "csrc", f) for f in ("kernels.h", "batch.hip")]
_FILTER_SOURCES = _STAGE_SOURCES + [os.path.join(ROOT, "paper_1511_01561_amd", "csrc", "filter.hip")]
KERNEL_SOURCES = {"element": _STAGE_SOURCES, "finish": _STAGE_SOURCES, "filter": _FILTER_SOURCES,
                  "filter_finish": _FILTER_SOURCES}


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def element_bytes(nu, nl, prec, metric):
    """Algorithmic HBM bytes of one launch of the element kernel of a fused
    stage on the box: the unique state (5 x 8 B) and reference read once
    (rho_bar, theta_bar, p_bar: 3 x 8 B; the recomputed-metric kernels take the
    isentropic theta_bar = theta0 as a constant: 2 x 8 B); per element-local
    node the contribution written once (5 x 8 B, or 5 x 4 B mixed) and, with
    the stored metric, the 9 inverse-metric entries and J w (10 x 8 B, or
    10 x 4 B mixed).  Unique ids follow from the lattice and a recomputed
    metric costs no traffic."""
    contrib = 20 if prec == "mixed" else 40
    met = 0 if metric == "recompute" else (40 if prec == "mixed" else 80)
    ref = 16 if metric == "recompute" else 24
    return nu * (40 + ref) + nl * (met + contrib)


def finish_bytes(nu, nl, n_wall, prec):
    """Algorithmic bytes of one finish launch on the box (averaged over the 3
    stages): per unique node M^-1 (8 B), q^n (2 of 3 stages) and the new state
    (5 x 8 B each); the stage state (5 x 8 B) at the wall nodes in FP64 (the
    FP64 element kernels fold it into the contributions elsewhere) and at
    every node in mixed precision; per element-local node its contribution
    (5 x 8 B, or 5 x 4 B mixed); the wall normals.  Copies follow from the
    lattice position."""
    contrib = 20 if prec == "mixed" else 40
    qs_nodes = nu if prec == "mixed" else n_wall
    return nu * (8 + 40 * 2.0 / 3.0 + 40) + qs_nodes * 40 + nl * contrib + n_wall * 24


def split_layout(ne3, N):
    """Node and contribution counts of the split DSS (NUMA_STAGE_SPLIT) on a
    box of ne3 = (nx, ny, nz) elements: workgroups of EB consecutive elements
    (EB = 256 // (N+1)^2); a run's first element (e % EB == 0 or ex == 0)
    and an element whose east neighbour is in another run (e % EB == EB - 1 or
    ex == nx - 1) write extra copies; the element kernel finishes the interior
    rows of the other elements.  Returns (nodes finished by the element
    kernel, face-row contribution values, run-boundary contribution values)."""
    nx, ny, nz = ne3
    ne = nx * ny * nz
    EB = 256 // (N + 1) ** 2
    e = np.arange(ne)
    ex = e % nx
    first = (e % EB == 0) | (ex == 0)
    last = (e % EB == EB - 1) | (ex == nx - 1)
    nip = (N - 1) ** 2
    n_int = int((~first).sum()) * nip * N
    fa = ne * 4 * N * N * 5
    fb = (int(last.sum()) * (4 * N + nip) + int(first.sum()) * nip * N) * 5
    return n_int, fa, fb


def split_kernel_bytes(nu, n_wall, ne3, N, prec):
    """Bytes of one launch of each split-DSS kernel (averaged over the 3
    stages): the element kernel reads the state (5 x 8 B) and rho_bar, p_bar
    (2 x 8 B) per unique node, writes the face-row and run-boundary
    contributions, and finishes its nodes (M^-1, q^n in 2 of 3 stages, the new
    state; the stage state too in mixed precision); the face kernel reads the
    contributions back and finishes the rest (plus the stage state and normals
    at the walls, the stage state everywhere in mixed precision)."""
    n_int, fa, fb = split_layout(ne3, N)
    w = 4 if prec == "mixed" else 8
    upd = 8 + 40 * 2.0 / 3.0 + 40 + (40 if prec == "mixed" else 0)
    el = nu * 56 + n_int * upd + (fa + fb) * w
    n_face = nu - n_int
    fin = n_face * upd + (0 if prec == "mixed" else n_wall * 40) + n_wall * 24 + (fa + fb) * w
    return el, fin, 2 * (fa + fb) * w


def stage_bytes(nu, ncol_nodes, prec):
    """Algorithmic HBM bytes of one fused stage (right-hand side, DSS, M^-1,
    update) with the metric recomputed every stage: per unique node the state
    read (5 x 8 B), q^n read in two of the three stages (5 x 8 x 2/3 B), the new
    state written (5 x 8 B), the reference rho_bar, theta_bar, p_bar (3 x 8 B)
    and M^-1 (8 B, or 4 B in mixed precision); plus the column factors of the
    metric (4 x 8 B per element column node (i, j)), read once.  Element-local
    intermediates (the contributions' round trip) are not algorithmic."""
    minv = 4 if prec == "mixed" else 8
    return nu * (40 + 40 * 2.0 / 3.0 + 40 + 24 + minv) + 32 * ncol_nodes


def load_traffic(kernel, workload):
    """HBM bytes per launch measured by rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, calibrated on a copy kernel), if taken on the current source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("source_sha") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, steps=100, budget_s=45.0):
    """Time the FP64 oracle (OpenMP over elements / unique nodes) on this host:
    up to `steps` SSP-RK3 steps of the same workload with all threads (stopping
    early after budget_s), then one step on one thread.  Returns the record and
    the oracle states after the first and after the last step (accuracy of the
    GPU results)."""
    import numpy as np
    import oracle
    from paper_1511_01561_amd import inputs
    mm = wl["mesh"]
    t0 = time.perf_counter()
    om = oracle.OracleMesh(mm["kind"], mm["N"], mm["ne"], mm["periodic"], mm["extent"], mm["h0"], wl["phys"])
    q0 = om.init_state(wl["ic"], inputs.noise(om.n_unique, 0))
    _log("oracle setup %.1f s" % (time.perf_counter() - t0))
    nthreads = oracle.num_threads()
    q, q1, per = q0, None, []
    while len(per) < steps and sum(per) < budget_s:
        t = time.perf_counter()
        q = om.step(q, 0.05, 1)
        per.append(time.perf_counter() - t)
        if q1 is None:
            q1 = q.copy()
        if len(per) % 10 == 0:
            _log("oracle step %d: %.2f s" % (len(per), sum(per)))
    assert np.isfinite(q).all()
    oracle.set_threads(1)
    t = time.perf_counter()
    om.step(q0, 0.05, 1)
    one = time.perf_counter() - t
    oracle.set_threads(nthreads)
    _log("oracle: %d steps on %d threads, median %.3f s/step; 1 thread %.2f s/step" % (len(per), nthreads,
                                                                                    float(np.median(per)), one))
    el = sum(per)
    rec = dict(value=om.n_unique * 3 * len(per) / el, unit="grid-point RHS updates/s", cores=nthreads, kind="oracle",
               sample="%d SSP-RK3 steps of the full 64x64x16 N=4 box (the timed workload), FP64, %d OpenMP threads, "
                      "%.1f s" % (len(per), nthreads, el),
               steps=len(per), median_s_per_step=float(np.median(per)),
               one_thread_s_per_step=one, one_thread_value=om.n_unique * 3 / one, cpu_model=cpu_model())
    return rec, q0, q1, q, len(per)


def serving(n_req, budget_gb, precs, loads=(0.5, 0.8), seed=0):
    """Ensemble serving: requests of box meshes {8^3, 16^3, 32x32x8, 64x64x16}
    with N in {3, 4, 5, 6} and K = 50 SSP-RK3 steps.  First back-to-back (all
    requests available at once) to measure the capacity C in requests/s, then
    Poisson arrivals at rate load*C for p50/p99 latency (arrival to completion)."""
    import torch
    from paper_1511_01561_amd import inputs
    from paper_1511_01561_amd.serve import GpuExecutor, Request, Server

    def make(rate, s):
        return [Request(id=r["id"], arrival=r["arrival"], workload=r["workload"], noise_seed=r["noise_seed"],
                        steps=r["steps"]) for r in inputs.serving_requests(n_req, s, rate)]

    out = {"requests": n_req, "budget_gb": budget_gb, "steps_per_request": 50,
           "budget_covers": "request states, scratch and flags, and every geometry workspace (LRU eviction of idle ones)",
           "mix": "box {8^3, 16^3, 32x32x8, 64x64x16} x N {3,4,5,6}, uniform"}
    for prec, name in precs:
        ex = GpuExecutor(prec=prec)
        srv = Server(ex, budget_bytes=int(budget_gb * 2 ** 30))
        b2b = make(1.0, seed)
        srv.prewarm(b2b, fraction=0.7)
        rec0 = {"geometry_gb_prewarmed": srv.geom_bytes / 2 ** 30}
        st = srv.run(b2b, realtime=False)
        cap = n_req / st.wall
        rec = dict(rec0, capacity_req_per_s=cap, throughput_updates_per_s=st.updates / st.wall,
                   back_to_back_wall_s=st.wall, max_active=st.max_active, peak_gb=st.peak_bytes / 2 ** 30,
                   failed=st.failed)
        _log("serving %s: capacity %.2f req/s, %.3e updates/s, max %d active" % (name, cap, st.updates / st.wall,
                                                                                st.max_active))
        for load in loads:
            reqs = make(load * cap, seed + 1)
            srv.prewarm(reqs, fraction=0.7)
            st = srv.run(reqs, realtime=True)
            rec["load_%.1f" % load] = {"rate_req_per_s": load * cap, "p50_s": st.percentile(50),
                                       "p99_s": st.percentile(99), "throughput_updates_per_s": st.updates / st.wall,
                                       "max_active": st.max_active, "peak_gb": st.peak_bytes / 2 ** 30,
                                       "failed": st.failed}
            _log("serving %s at %.1f C: p50 %.3f s, p99 %.3f s" % (name, load, st.percentile(50), st.percentile(99)))
        ex.drop_graphs()
        out[name] = rec
        del ex, srv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def group_err(a, b):
    """max|a - b| / max|b| per variable group (rho'; u, v, w; theta')."""
    import numpy as np
    out = {}
    for g, rows in (("rho", [0]), ("u", [1, 2, 3]), ("theta", [4])):
        den = float(np.abs(b[rows]).max())
        out[g] = float(np.abs(a[rows] - b[rows]).max()) / den if den > 0 else 0.0
    return out


def sweep(orders, shell_steps, long_steps, oracle_check=True):
    """Order sweep on the 64x64x16 terrain box and the 6x32x32x10 shell:
    FP64 and mixed step time, and the mixed result against FP64 after 1 and
    `long_steps` steps (FP64 GPU result after 1 step also against the oracle)."""
    import numpy as np
    import torch
    from paper_1511_01561_amd import inputs, numa
    res = {"box": {}, "shell": None}

    def timed(g, q0, prec, dt, steps=5):
        q = q0.clone()
        g.step(q, dt, 1, prec=prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.step(q, dt, steps, prec=prec)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    def run(wl, dt, nlong, name, long_oracle=False):
        mm = wl["mesh"]
        g = numa.Mesh(mm, wl["phys"], prec_mask=3 | numa.WS_IMEX)
        nz = torch.as_tensor(inputs.noise(g.n_unique, 0), device="cuda:0") if wl["ic"]["noise_amp"] else None
        q0 = g.init_state(wl["ic"], nz)
        t64, tmx = timed(g, q0, numa.PREC_FP64, dt), timed(g, q0, numa.PREC_MIXED, dt)
        rec = {"unique_nodes": g.n_unique, "local_nodes": g.n_local,
               "fp64_ms_per_step": 1e3 * t64, "mixed_ms_per_step": 1e3 * tmx, "speedup": t64 / tmx,
               "fp64_updates_per_s": 3 * g.n_unique / t64, "mixed_updates_per_s": 3 * g.n_unique / tmx}
        # the same steps with the metric recomputed per stage
        g.set_metric(numa.METRIC_RECOMPUTE)
        r64, rmx = timed(g, q0, numa.PREC_FP64, dt), timed(g, q0, numa.PREC_MIXED, dt)
        a, b = q0.clone(), q0.clone()
        g.step(a, dt, 1, prec=numa.PREC_FP64)
        g.set_metric(numa.METRIC_STORED)
        g.step(b, dt, 1, prec=numa.PREC_FP64)
        rec["recompute"] = {"fp64_ms_per_step": 1e3 * r64, "mixed_ms_per_step": 1e3 * rmx,
                            "speedup": r64 / rmx, "fp64_updates_per_s": 3 * g.n_unique / r64,
                            "mixed_updates_per_s": 3 * g.n_unique / rmx,
                            "vs_stored_state_1": group_err(a.cpu().numpy(), b.cpu().numpy())}
        h0 = q0.cpu().numpy()
        for n in (1, nlong):
            a, b = q0.clone(), q0.clone()
            g.step(a, dt, n, prec=numa.PREC_FP64)
            g.step(b, dt, n, prec=numa.PREC_MIXED)
            A, B = a.cpu().numpy(), b.cpu().numpy()
            rec["mixed_vs_fp64_state_%d" % n] = group_err(B, A)
            rec["mixed_vs_fp64_increment_%d" % n] = group_err(B - h0, A - h0)
            if n == nlong and oracle_check and long_oracle:
                # the whole run on the oracle (the 64x64x16 N = 4 box and the shell only)
                import oracle
                om = oracle.OracleMesh(mm["kind"], mm["N"], mm["ne"], mm["periodic"], mm["extent"], mm["h0"],
                                       wl["phys"])
                t0 = time.perf_counter()
                qo = om.step(h0, dt, n)
                _log("%s: oracle %d steps %.1f s" % (name, n, time.perf_counter() - t0))
                rec["fp64_vs_oracle_state_%d" % n] = group_err(A, qo)
                del om
            if n == 1 and oracle_check:
                import oracle
                om = oracle.OracleMesh(mm["kind"], mm["N"], mm["ne"], mm["periodic"], mm["extent"], mm["h0"],
                                       wl["phys"])
                qo = om.step(h0, dt, 1)
                rec["fp64_vs_oracle_state_1"] = group_err(A, qo)
                rec["mixed_vs_oracle_increment_1"] = group_err(B - h0, qo - h0)
                del om
        _log("%s: fp64 %.3f ms, mixed %.3f ms (x%.2f); mixed-fp64 after %d steps %s"
             % (name, rec["fp64_ms_per_step"], rec["mixed_ms_per_step"], rec["speedup"], nlong,
                {k: "%.1e" % v for k, v in rec["mixed_vs_fp64_state_%d" % nlong].items()}))
        if "recompute" in rec:
            _log("%s, recomputed metric: fp64 %.3f ms, mixed %.3f ms (x%.2f)"
                 % (name, rec["recompute"]["fp64_ms_per_step"], rec["recompute"]["mixed_ms_per_step"],
                    rec["recompute"]["speedup"]))
        del g
        torch.cuda.empty_cache()
        return rec

    for N in orders:
        res["box"]["N%d" % N] = run(inputs.gpu_box(N), 0.05, long_steps, "box64x64x16 N=%d" % N, long_oracle=N == 4)
    if shell_steps:
        res["shell"] = run(inputs.shell_workload(32, 10, 4, seed=0), 0.5, shell_steps, "shell6x32x32x10 N=4",
                           long_oracle=True)
    return res


FILTER_ORDER, FILTER_CUTOFF = 16.0, 1


def filter_leg(g, q0, dt, steps, stream, workload):
    """The Boyd-Vandeven filter on the bench state: the element filter and
    its DSS (two launches), timed with events on the launch stream, against
    the state read once and written once (80 B per unique node); and the FP64
    step with the filter at its end."""
    import torch
    from paper_1511_01561_amd import numa
    q = q0.clone()
    for _ in range(2):
        g.filter(q, FILTER_ORDER, FILTER_CUTOFF)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        g.filter(q, FILTER_ORDER, FILTER_CUTOFF)
    e1.record(stream)
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / steps
    algo = 80 * g.n_unique
    g.set_filter(FILTER_ORDER, FILTER_CUTOFF)
    q = q0.clone()
    g.step(q, dt, 1)
    torch.cuda.synchronize()
    e0.record(stream)
    g.step(q, dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    g.set_filter(None)
    assert torch.isfinite(q).all().item()
    tf, tn = load_traffic("filter", workload), load_traffic("filter_finish", workload)
    return {"order": FILTER_ORDER, "cutoff": FILTER_CUTOFF, "avg_us": s * 1e6, "algorithmic_bytes": algo,
            "achieved_GBs": algo / s / 1e9, "frac": algo / s / 1e9 / HBM_PEAK_GBS,
            "traffic": tf + tn if tf is not None and tn is not None else None,
            "step_with_filter_ms": e0.elapsed_time(e1) / steps}


def rk53_leg(g, q0, dt, steps, stream):
    """The same FP64 step with the five-stage SSP-RK(5,3) integrator: five
    RHS evaluations per step."""
    import torch
    from paper_1511_01561_amd import numa
    g.set_integrator(numa.RK_SSP53)
    q = q0.clone()
    g.step(q, dt, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    g.step(q, dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    g.set_integrator(numa.RK_SSP33)
    assert torch.isfinite(q).all().item()
    ms = e0.elapsed_time(e1) / steps
    return {"ms_per_step": ms, "value": 5 * g.n_unique / (ms * 1e-3), "stages": 5}


IMEX_RA = 0.05


def imex_leg(g, q0, dt, steps, stream):
    """The 1D-IMEX leap-frog step (explicit stage, vertical line solves,
    Robert-Asselin filter) at the same dt, FP64, after the factorisation of
    the line matrices (first call)."""
    import torch
    a, b = q0.clone(), q0.clone()
    g.imex_step(a, b, dt, IMEX_RA, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    g.imex_step(a, b, dt, IMEX_RA, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    assert torch.isfinite(b).all().item()
    return {"ms_per_step": e0.elapsed_time(e1) / steps, "ra": IMEX_RA, "lines": g.n_horiz,
            "levels": g.n_levels}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--small", action="store_true", help="4x4x4 box instead of the one-GPU workload")
    ap.add_argument("--sweep", action="store_true", help="order sweep and shell instead of the bench line")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests per serving run (0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=28.0,
                    help="device memory for geometry and requests (admission binds below it)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_01561_amd import inputs, numa

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    numa.lib()
    if args.sweep:
        print(json.dumps(sweep((3, 4, 5, 6, 8), shell_steps=200, long_steps=100)), flush=True)
        return
    wl = inputs.small_box() if args.small else inputs.gpu_box()
    mm = wl["mesh"]
    workload = "box%dx%dx%d_N%d_terrain%g" % (*mm["ne"], mm["N"], mm["h0"])
    _log("workload %s" % workload)
    stream = torch.cuda.current_stream()
    g = numa.Mesh(mm, wl["phys"], prec_mask=3 | numa.WS_IMEX)
    nz = torch.as_tensor(inputs.noise(g.n_unique, 0), device="cuda:0")
    q0 = g.init_state(wl["ic"], nz)
    torch.cuda.synchronize()
    _log("mesh: %d elements, %d local, %d unique nodes; workspace %.2f GB"
         % (g.n_elem, g.n_local, g.n_unique, g.workspace_bytes / 1e9))

    dt = 0.05

    def timed_steps(prec):
        q = q0.clone()
        g.step(q, dt, args.warmup, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        g.step(q, dt, args.steps, prec=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert torch.isfinite(q).all().item()
        return e0.elapsed_time(e1) / 1e3, wall

    n_wall = 0 if mm["periodic"][2] else 2 * g.n_horiz

    def measure(metric):
        g.set_metric(numa.METRIC_RECOMPUTE if metric == "recompute" else numa.METRIC_STORED)
        rec = {}
        for prec, name in ((numa.PREC_FP64, "fp64"), (numa.PREC_MIXED, "mixed")):
            if name == "mixed" and args.no_mixed:
                continue
            gpu_s, wall_s = timed_steps(prec)
            r = {"value": g.n_unique * 3 * args.steps / wall_s, "ms_per_step": 1e3 * wall_s / args.steps}
            # per-launch durations of the two stage kernels, from HIP events the
            # library records on the stream it launches them on
            q = q0.clone()
            g.step(q, dt, 1, prec=prec)
            torch.cuda.synchronize()
            g.profile(True)
            g.step(q, dt, args.steps, prec=prec)
            el_ms, el_n, fin_ms, fin_n = g.profile_read()
            g.profile(False)
            el_s, fin_s = el_ms / el_n * 1e-3, fin_ms / fin_n * 1e-3
            if metric == "recompute" and name == "fp64":  # NUMA_STAGE_AUTO: the split DSS in FP64
                ea, fa, _ = split_kernel_bytes(g.n_unique, n_wall, mm["ne"], mm["N"], name)
            else:
                ea = element_bytes(g.n_unique, g.n_local, name, metric)
                fa = finish_bytes(g.n_unique, g.n_local, n_wall, name)
            r["element_kernel"] = {"avg_launch_us": el_s * 1e6, "algorithmic_bytes": ea, "achieved_GBs": ea / el_s / 1e9}
            r["finish_kernel"] = {"avg_launch_us": fin_s * 1e6, "algorithmic_bytes": fa, "achieved_GBs": fa / fin_s / 1e9}
            _log("%s metric, %s: %.3f ms/step, %.3e updates/s; element %.1f us (%.0f GB/s), finish %.1f us (%.0f GB/s)"
                 % (metric, name, r["ms_per_step"], r["value"], el_s * 1e6, ea / el_s / 1e9, fin_s * 1e6,
                    fa / fin_s / 1e9))
            rec[name] = r
        if "mixed" in rec:
            rec["mixed"]["speedup_vs_fp64"] = rec["fp64"]["ms_per_step"] / rec["mixed"]["ms_per_step"]
        return rec

    stored = measure("stored")
    recomp = measure("recompute")
    head = recomp["fp64"]
    value, ms_step = head["value"], head["ms_per_step"]
    mixed = recomp.get("mixed")
    if mixed is not None:
        mixed["dtype"] = "f32 contractions / f64 state"

    # achievable rate: a plain device copy (1 GiB each way), timed with events
    src = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_GBs = 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    _log("device copy: %.0f GB/s" % copy_GBs)

    # roofline of the whole fused stage (element kernel + finish kernel): the
    # algorithmic bytes of a stage over the two kernels' average durations
    ncol = mm["ne"][0] * mm["ne"][1] * (mm["N"] + 1) ** 2

    def stage_roofline(r, prec):
        el, fin = r["element_kernel"], r["finish_kernel"]
        st_us = el["avg_launch_us"] + fin["avg_launch_us"]
        algo = stage_bytes(g.n_unique, ncol, prec)
        ach = algo / (st_us * 1e-6) / 1e9
        N = mm["N"]
        if prec == "fp64":  # NUMA_STAGE_AUTO: the split DSS
            kernel = ("fused SSP-RK3 stage: k_elem_col2<%d,double> + k_fin_split<%d,double,false> (recomputed metric, "
                      "split DSS)" % (N, N))
            trip = split_kernel_bytes(g.n_unique, n_wall, mm["ne"], N, prec)[2]
        else:
            kernel = ("fused SSP-RK3 stage: k_elem_col<%d,float> + k_fin_batch<%d,%d,float> (recomputed metric, "
                      "gather DSS)" % (N, N, 4))
            trip = 2 * 20 * g.n_local
        return dict(kernel=kernel, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    algorithmic_bytes=algo, stage_us=st_us, copy_GBs=copy_GBs, copy_frac=ach / copy_GBs,
                    contribution_round_trip_bytes=trip, element_kernel=el, finish_kernel=fin)

    roofline = stage_roofline(head, "fp64")
    te, tf = load_traffic("element", workload), load_traffic("finish", workload)
    roofline["traffic"] = te + tf if te is not None and tf is not None else None
    roofline["traffic_by_kernel"] = {"element": te, "finish": tf}
    if mixed is not None:
        mixed["roofline"] = stage_roofline(mixed, "mixed")
    _log("stage: %.1f us, %.0f GB/s algorithmic = %.3f of 8 TB/s, %.3f of the copy rate"
         % (roofline["stage_us"], roofline["achieved"], roofline["frac"], roofline["copy_frac"]))

    # the DSS schedules of a stage on the same mesh (numa_mesh_set_stage; the
    # default NUMA_STAGE_AUTO is the split one in FP64, the gather in mixed)
    g.set_metric(numa.METRIC_RECOMPUTE)
    modes = {}
    for mode, mname in ((numa.STAGE_GATHER, "gather"), (numa.STAGE_SPLIT, "split"), (numa.STAGE_BLOCK, "block"),
                        (numa.STAGE_COLOUR, "colour")):
        g.set_stage(mode)
        modes[mname] = {}
        for prec, name in ((numa.PREC_FP64, "fp64"), (numa.PREC_MIXED, "mixed")):
            if name == "mixed" and args.no_mixed:
                continue
            gpu_s, wall_s = timed_steps(prec)
            modes[mname][name] = {"ms_per_step": 1e3 * wall_s / args.steps}
        _log("stage mode %s: %s" % (mname, {k: "%.3f ms" % v["ms_per_step"] for k, v in modes[mname].items()}))
    g.set_stage(numa.STAGE_AUTO)

    # accuracy: FP64 and mixed states after 1 and after the oracle's steps
    # (100 unless the CPU budget stopped it earlier)
    def states(n):
        out = {}
        for prec, name in ((numa.PREC_FP64, "fp64"), (numa.PREC_MIXED, "mixed")):
            if name == "mixed" and args.no_mixed:
                continue
            q = q0.clone()
            g.step(q, dt, n, prec=prec)
            out[name] = q.cpu().numpy()
        return out

    acc_states = {1: states(1), 100: states(100)}
    q0h = q0.cpu().numpy()
    g.set_metric(numa.METRIC_RECOMPUTE)
    filt = filter_leg(g, q0, dt, args.steps, stream, workload)
    rk53 = rk53_leg(g, q0, dt, args.steps, stream)
    _log("SSP-RK(5,3): %.3f ms/step, %.3e updates/s" % (rk53["ms_per_step"], rk53["value"]))
    imex = imex_leg(g, q0, dt, args.steps, stream)
    _log("1D-IMEX leap-frog: %.3f ms/step (explicit stage and line solves)" % imex["ms_per_step"])
    _log("filter (p=%g, cutoff %d): %.1f us per launch pair, %.0f GB/s algorithmic; step with filter %.3f ms"
         % (filt["order"], filt["cutoff"], filt["avg_us"], filt["achieved_GBs"], filt["step_with_filter_ms"]))

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log("copy probe: 3 x %d MiB device copies" % args.copy_probe)
        del src, dst

    n_elem, n_unique, n_local = g.n_elem, g.n_unique, g.n_local
    serve = None
    if args.serve_requests > 0:
        del q0, g
        torch.cuda.empty_cache()
        precs = [(numa.PREC_FP64, "fp64")] + ([] if args.no_mixed else [(numa.PREC_MIXED, "mixed")])
        serve = serving(args.serve_requests, args.serve_budget_gb, precs)

    cpu = None
    accuracy = {}
    for n, st in acc_states.items():
        if "mixed" in st:
            accuracy["mixed_vs_fp64_state_%d" % n] = group_err(st["mixed"], st["fp64"])
            accuracy["mixed_vs_fp64_increment_%d" % n] = group_err(st["mixed"] - q0h, st["fp64"] - q0h)
    if not args.no_cpu:
        cpu, _, o1, on, nsteps = cpu_baseline(wl)
        _log("cpu oracle: %.3e updates/s" % cpu["value"])
        accuracy["fp64_vs_oracle_state_1"] = group_err(acc_states[1]["fp64"], o1)
        accuracy["fp64_vs_oracle_increment_1"] = group_err(acc_states[1]["fp64"] - q0h, o1 - q0h)
        if "mixed" in acc_states[1]:
            accuracy["mixed_vs_oracle_increment_1"] = group_err(acc_states[1]["mixed"] - q0h, o1 - q0h)
        if nsteps == 100:
            accuracy["fp64_vs_oracle_state_100"] = group_err(acc_states[100]["fp64"], on)
            if "mixed" in acc_states[100]:
                accuracy["mixed_vs_oracle_state_100"] = group_err(acc_states[100]["mixed"], on)
    accuracy["norm"] = "max|a - b| / max|b| per variable group (rho'; u, v, w; theta')"
    _log("accuracy: %s" % {k: ({g: "%.1e" % e for g, e in v.items()} if isinstance(v, dict) else v)
                           for k, v in accuracy.items()})

    out = {
        "metric": "grid-point RHS updates/s",
        "value": value,
        "unit": "grid-point RHS updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "elements": n_elem, "order": mm["N"], "unique_nodes": n_unique,
                   "local_nodes": n_local, "dt": dt, "integrator": "SSP-RK3", "metric": "recomputed each stage",
                   "parallelism": "single GPU"},
        "mixed": mixed,
        "stored_metric": stored,
        "roofline": roofline,
        "accuracy": accuracy,
        "stage_modes": modes,
        "filter": filt,
        "ssp53": rk53,
        "imex": imex,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
