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

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {
    "stage": os.path.join(ROOT, "paper_1511_01561_amd", "csrc", "rhs.hip"),
}


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def element_bytes(nu, nl, prec):
    """Algorithmic HBM bytes of one launch of the element kernel of a fused
    stage: the unique state (5 x 8 B) and reference (3 x 8 B) read once; per
    element-local node the gather map (4 B), the metric terms with J w
    (10 x 8 B, or 10 x 4 B mixed) and the contribution written once
    (5 x 8 B, or 5 x 4 B mixed)."""
    met, contrib = (40, 20) if prec == "mixed" else (80, 40)
    return nu * (40 + 24) + nl * (4 + met + contrib)


def finish_bytes(nu, nl, n_wall, prec):
    """Algorithmic bytes of one finish launch (averaged over the 3 stages):
    the node order (4 B) and copy offsets (8 B) per unique node, the copy list
    (4 B) and contribution (5 x 8 B or 5 x 4 B) per element-local node, M^-1
    (8 B), the stage state, q^n (2 of 3 stages) and the new state (5 x 8 B
    each) per unique node, and the wall normals."""
    contrib = 20 if prec == "mixed" else 40
    return nu * (4 + 8 + 8 + 40 + 40 * 2.0 / 3.0 + 40) + nl * (4 + contrib) + n_wall * 24


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


def cpu_baseline(wl, budget_s=15.0):
    """Time the FP64 oracle (OpenMP over elements / unique nodes) on this host
    for whole SSP-RK3 steps of the same workload until ~budget_s has elapsed."""
    import numpy as np
    import oracle
    from paper_1511_01561_amd import inputs
    mm = wl["mesh"]
    t0 = time.perf_counter()
    om = oracle.OracleMesh(mm["kind"], mm["N"], mm["ne"], mm["periodic"], mm["extent"], mm["h0"], wl["phys"])
    q = om.init_state(wl["ic"], inputs.noise(om.n_unique, 0))
    _log("oracle setup %.1f s" % (time.perf_counter() - t0))
    steps, el = 0, 0.0
    while el < budget_s and steps < 100:
        t = time.perf_counter()
        q = om.step(q, 0.05, 1)
        el += time.perf_counter() - t
        steps += 1
        _log("oracle step %d: %.2f s" % (steps, el))
    assert np.isfinite(q).all()
    return dict(value=om.n_unique * 3 * steps / el, unit="grid-point RHS updates/s",
                cores=oracle.num_threads(), kind="oracle",
                sample="%d SSP-RK3 step(s) of the full 64x64x16 N=4 box, FP64, %d OpenMP threads, %.1f s"
                       % (steps, oracle.num_threads(), el))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--small", action="store_true", help="4x4x4 box instead of the one-GPU workload")
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
    wl = inputs.small_box() if args.small else inputs.gpu_box()
    mm = wl["mesh"]
    workload = "box%dx%dx%d_N%d_terrain%g" % (*mm["ne"], mm["N"], mm["h0"])
    _log("workload %s" % workload)
    stream = torch.cuda.current_stream()
    g = numa.Mesh(mm, wl["phys"], prec_mask=3)
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

    gpu_s, wall_s = timed_steps(numa.PREC_FP64)
    ms_step = 1e3 * wall_s / args.steps
    value = g.n_unique * 3 * args.steps / wall_s
    _log("fp64: %.3f ms/step (events %.3f), %.3e updates/s" % (ms_step, 1e3 * gpu_s / args.steps, value))

    mixed = None
    if not args.no_mixed:
        mg, mw = timed_steps(numa.PREC_MIXED)
        mixed = dict(value=g.n_unique * 3 * args.steps / mw, ms_per_step=1e3 * mw / args.steps,
                     speedup_vs_fp64=wall_s / mw, dtype="f32 contractions / f64 state")
        _log("mixed: %.3f ms/step, speedup %.2f" % (mixed["ms_per_step"], mixed["speedup_vs_fp64"]))

    # the dominant kernel: per-launch durations of the two stage kernels from
    # HIP events the library records on the stream it launches them on
    n_wall = 0 if mm["periodic"][2] else 2 * g.n_horiz
    prof = {}
    for prec, name in ((numa.PREC_FP64, "fp64"), (numa.PREC_MIXED, "mixed")):
        if name == "mixed" and args.no_mixed:
            continue
        q = q0.clone()
        g.step(q, dt, 1, prec=prec)
        torch.cuda.synchronize()
        g.profile(True)
        g.step(q, dt, args.steps, prec=prec)
        el_ms, el_n, fin_ms, fin_n = g.profile_read()
        g.profile(False)
        prof[name] = (el_ms / el_n * 1e-3, fin_ms / fin_n * 1e-3)
        _log("%s stage kernels: element %.1f us, finish %.1f us per launch"
             % (name, prof[name][0] * 1e6, prof[name][1] * 1e6))
    el_s, fin_s = prof["fp64"]
    alg = element_bytes(g.n_unique, g.n_local, "fp64")
    achieved = alg / el_s / 1e9
    fin_alg = finish_bytes(g.n_unique, g.n_local, n_wall, "fp64")
    _log("element kernel %.0f GB/s algorithmic; finish kernel %.0f GB/s" % (achieved, fin_alg / fin_s / 1e9))
    traffic = load_traffic("stage", workload)
    roofline = dict(kernel="k_rhs<4,double> (element kernel of the fused stage)", bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=traffic, algorithmic_bytes=alg,
                    avg_launch_us=el_s * 1e6,
                    finish_kernel=dict(avg_launch_us=fin_s * 1e6, algorithmic_bytes=fin_alg,
                                       achieved=fin_alg / fin_s / 1e9))
    if "mixed" in prof and mixed is not None:
        malg = element_bytes(g.n_unique, g.n_local, "mixed")
        mixed["element_kernel"] = dict(avg_launch_us=prof["mixed"][0] * 1e6, algorithmic_bytes=malg,
                                       achieved=malg / prof["mixed"][0] / 1e9)

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log("copy probe: 3 x %d MiB device copies" % args.copy_probe)
        del src, dst

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl)
        _log("cpu oracle: %.3e updates/s" % cpu["value"])

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
        "config": {"workload": workload, "elements": g.n_elem, "order": mm["N"], "unique_nodes": g.n_unique,
                   "local_nodes": g.n_local, "dt": dt, "integrator": "SSP-RK3", "parallelism": "single GPU"},
        "mixed": mixed,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
