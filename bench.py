#!/usr/bin/env python3
"""Benchmark of near-circulant splitting (NCS) on one MI355X.

Workload: one 256 x 256 parallel-beam CT slice (360 angles over [0, pi), 367
unit detector bins), anisotropic-TV least squares with lambda = 0.005, on a
seeded random-ellipse phantom (seed 0) with b = E x_true + 1% Gaussian noise
(synthetic stand-in for the patient data of the paper's experiments).

A step is one NCS iteration: backprojection + divergence, circulant solve
(2D DFT, multiplier, inverse DFT) with the primal update, TV dual update,
forward projection + data prox, and the objective in double precision.

Printed: one JSON line with iterations/s over exactly --steps timed
iterations (after --warmup), the per-kernel times from HIP events, the
roofline of the dominant kernel, the time to a 1e-4 relative objective gap
(f* from a long double-precision run of the same library), and the CPU
oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NCS iters/s and time to 1e-4 rel. obj gap per 256² slice, plain vs warm-start"
N_SIDE, N_ANGLES, N_BINS, LAMBDA, SEED = 256, 360, 367, 0.005, 0
ALPHA, BETA_RATIO, GAMMA_FRAC = 3e-4, 3.0, 0.3     # beta = 3 alpha, gamma = 0.3 alpha C_R
GAP = 1e-4
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
COPY_MIB = 256          # plain device copy used to calibrate the HBM byte counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1810_13100_amd", "csrc", "ncs_kernels.hip")


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def params(ncs):
    c_r = N_ANGLES * N_SIDE / math.pi
    return ncs.Params(ALPHA, BETA_RATIO * ALPHA, GAMMA_FRAC * ALPHA * c_r, LAMBDA)


def make_data(ncs, torch, dev):
    """b = E x_true + sigma eps on the device (E from the library's own projector)."""
    import ncs_inputs
    geom = ncs.Geometry(N_SIDE, N_ANGLES, N_BINS)
    op = ncs.Solver(geom, params(ncs))
    x_true = torch.tensor(ncs_inputs.phantom(N_SIDE, SEED).ravel(), dtype=torch.float32, device=dev)
    clean = op.forward(x_true)
    sigma = 0.01 * float(clean.max())
    eps = torch.tensor(ncs_inputs.gaussian_noise(SEED, geom.m), dtype=torch.float32, device=dev)
    b = clean + sigma * eps
    torch.cuda.synchronize()
    op.close()
    return geom, b


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(KERNEL_SOURCE, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != digest:
        return None
    entry = rec.get("kernels", {}).get(kernel)
    return None if entry is None else entry.get("bytes_per_launch")


def calibration_copy(torch, dev) -> None:
    """One plain device-to-device copy of COPY_MIB MiB (its FETCH_SIZE and
    WRITE_SIZE calibrate the byte counters of the other kernels)."""
    n = COPY_MIB * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cpu_baseline(iters: int) -> dict:
    """The FP64 oracle on the same workload, timed on the host (assembly excluded)."""
    from oracle import problems, solvers
    progress("cpu baseline: assembling the oracle's sparse E")
    prob = problems.ct_problem(N_SIDE, N_ANGLES, N_BINS, SEED, LAMBDA)
    c_r = N_ANGLES * N_SIDE / math.pi
    par = problems.Params(ALPHA, BETA_RATIO * ALPHA, GAMMA_FRAC * ALPHA * c_r)
    progress(f"cpu baseline: {iters} oracle iterations")
    t0 = time.perf_counter()
    solvers.ncs(prob, par, iters)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": iters / dt, "unit": "iterations/s", "cores": 1, "kind": "oracle",
        "sample": f"{iters} FP64 oracle NCS iterations on the same 256^2 workload (SciPy CSR E and E^T, "
                  f"numpy FFT, objective every iteration; E assembly excluded); single-threaded "
                  f"({os.cpu_count()} host CPUs visible: {cpu})",
        "seconds": dt,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=60, help="oracle iterations of the CPU baseline (0: skip)")
    ap.add_argument("--no-gap", action="store_true", help="skip the time-to-gap measurement")
    ap.add_argument("--fstar-iters", type=int, default=20000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(slices shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        return 2
    import torch
    from paper_1810_13100_amd import ncs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    progress(f"device {torch.cuda.get_device_name(dev)}")
    geom, b = make_data(ncs, torch, dev)
    s = ncs.Solver(geom, params(ncs), b=b, dtype=torch.float32)
    info = s.info()
    s.set_init()

    progress(f"warmup {args.warmup} iterations")
    s.iterate(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    progress(f"timing {args.steps} iterations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.iterate(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    its = 1000.0 / ms_per_step

    progress("per-kernel timing (HIP events)")
    phases = s.time_phases(50)
    calibration_copy(torch, dev)
    dominant = max(phases, key=phases.get)
    flops = 2.0 * info["nnz"]          # one multiply-add per nonzero of E
    dom_ms = phases[dominant]
    if dominant in ("project_dataprox_tv", "backproject"):
        achieved = flops / (dom_ms * 1e-3) / 1e12
        roof = {"kernel": dominant, "bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic(dominant),
                "work_per_launch": f"2 x nnz(E) = {flops:.4g} flop", "ms_per_launch": dom_ms}
    else:
        roof = {"kernel": dominant, "bound": "hbm", "achieved": None, "peak": 8000.0, "unit": "GB/s",
                "frac": None, "traffic": None, "ms_per_launch": dom_ms}

    gap = None
    if not args.no_gap:
        progress(f"f*: {args.fstar_iters} double-precision iterations")
        s64 = ncs.Solver(geom, params(ncs), b=b.double(), dtype=torch.float64)
        s64.set_init()
        chunk = 5000
        done = 0
        fmin = math.inf
        while done < args.fstar_iters:
            k = min(chunk, args.fstar_iters - done)
            obj = s64.iterate(k, record=True)
            fmin = min(fmin, float(obj.min()))
            done += k
            progress(f"  f* run: {done} iterations, f = {obj[-1]:.10g}")
        tail_change = float(abs(obj[-1] - obj[-1000]) / abs(obj[-1])) if len(obj) >= 1000 else None
        s64.close()
        target = fmin * (1.0 + GAP)
        progress("time to gap (plain, x0 = 0)")
        s.set_init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, iters, f = s.solve(50000, target)
        t_gap = time.perf_counter() - t0
        gap = {"plain": {"seconds": t_gap, "iterations": iters, "reached": st == ncs.NCS_OK, "f": f},
               "warm": None, "f_star": fmin, "f_star_rel_change_last_1000": tail_change,
               "rel_gap": GAP, "f_star_source": f"min f over {args.fstar_iters} FP64 iterations"}

    cpu = cpu_baseline(args.cpu_iters) if args.cpu_iters > 0 else None
    s.close()
    out = {
        "metric": METRIC, "value": its, "unit": "iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "256^2 parallel-beam CT, anisotropic TV (lambda 0.005), 360 angles x 367 bins, "
                               "random-ellipse phantom seed 0, 1% Gaussian noise",
                   "n_side": N_SIDE, "n_angles": N_ANGLES, "n_bins": N_BINS, "alpha": ALPHA,
                   "beta": BETA_RATIO * ALPHA, "gamma": GAMMA_FRAC * ALPHA * N_ANGLES * N_SIDE / math.pi,
                   "nnz_E": info["nnz"]},
        "wall_s_timed": wall, "phases_ms": phases, "roofline": roof, "time_to_gap": gap,
        "cpu_baseline": cpu, "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
