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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NCS iters/s and time to 1e-4 rel. obj gap per 256² slice, plain vs warm-start"
N_SIDE, N_ANGLES, N_BINS, LAMBDA, SEED = 256, 360, 367, 0.005, 0
# beta = 3 alpha, gamma = 0.3 alpha C_R; alpha the fastest of a scan of the
# iterations of 8 slices to the 1e-4 gap (gamma = 0.25 alpha C_R diverges)
ALPHA, BETA_RATIO, GAMMA_FRAC = 2.4e-3, 3.0, 0.3
# f* runs: the smaller alpha, whose FP64 run gets closer to the minimum in a
# fixed number of iterations (f* is a property of the problem, not of alpha)
FSTAR_ALPHA = 3e-4
PDHG_ALPHA = 3e-4
GAP = 1e-4
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
COPY_MIB = 256          # plain device copy used to calibrate the HBM byte counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1810_13100_amd", "csrc", "ncs_kernels.hip")
CONE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cone_traffic.json")
CONE_SOURCE = os.path.join(ROOT, "paper_1810_13100_amd", "csrc", "cone.hip")


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def params(ncs, alpha: float = ALPHA):
    c_r = N_ANGLES * N_SIDE / math.pi
    return ncs.Params(alpha, BETA_RATIO * alpha, GAMMA_FRAC * alpha * c_r, LAMBDA)


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


def measured_traffic(kernel: str, traffic_file: str = TRAFFIC_FILE, source: str = KERNEL_SOURCE,
                     variants: dict | None = None):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel source changed since the counters were taken or the
    counters were taken with other kernel variants than `variants`."""
    import hashlib
    try:
        with open(traffic_file) as f:
            rec = json.load(f)
        with open(source, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != digest:
        return None
    if variants and any(rec.get(k) != v for k, v in variants.items()):
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


WEIGHTS = os.path.join(ROOT, "paper_1810_13100_amd", "weights", "warmstart_ct256.npy")


def time_to_gap(ncs, torch, dev, geom, args) -> dict:
    """Plain NCS from zero and the learned warm start, each run on its own
    evaluation slice (seeds 0..n-1) to f <= f* (1 + 1e-4), f* the smallest
    objective of a long double-precision run of the same slice.  Wall time
    from "b on the device, setup done" to the stopping iteration."""
    from paper_1810_13100_amd import warmstart
    seeds = list(range(args.gap_seeds))
    op = ncs.Solver(geom, params(ncs))
    bs = [warmstart.ct_sinogram(op, s) for s in seeds]
    op.close()
    progress(f"f*: {args.fstar_iters} double-precision iterations on {len(seeds)} slices")
    ref = ncs.Batch([geom] * len(seeds), [params(ncs, FSTAR_ALPHA)] * len(seeds), [b.double() for b in bs],
                    dtype=torch.float64)
    ref.set_init()
    fstar = np.full(len(seeds), np.inf)
    done = 0
    while done < args.fstar_iters:
        k = min(2000, args.fstar_iters - done)
        _, _, f = ref.solve(k)
        fstar = np.minimum(fstar, f)
        done += k
    tail = [float(abs(ref.slice(i).objectives(done - 1, 1)[0] - ref.slice(i).objectives(done - 1000, 1)[0])
                  / abs(fstar[i])) for i in range(len(seeds))]
    ref.close()
    net, meta = None, None
    if os.path.exists(WEIGHTS):
        from paper_1810_13100_amd import cnn
        net = cnn.WarmStartNet(1, N_SIDE, N_SIDE)
        net.set_params(warmstart.load_params(WEIGHTS))
        meta_path = os.path.splitext(WEIGHTS)[0] + ".json"
        if os.path.exists(meta_path):
            with open(meta_path) as f:
                meta = json.load(f)
    k0 = int(meta["k0"]) if meta else 300
    if net is not None:   # the network's kernels run once before any timing
        net.forward(torch.zeros((1, N_SIDE, N_SIDE), dtype=torch.float32, device=dev))
    plain_t, plain_it, warm_t, warm_it = [], [], [], []
    for i, b in enumerate(bs):
        target = fstar[i] * (1.0 + GAP)
        s = ncs.Solver(geom, params(ncs), b=b)
        s.set_init()
        s.iterate(64)   # warm-up: the replayed graphs are captured and every kernel has run once
        torch.cuda.synchronize()

        def plain():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.set_init()
            st, it, _ = s.solve(50000, target)
            torch.cuda.synchronize()
            plain_t.append(time.perf_counter() - t0)
            plain_it.append(it if st == ncs.NCS_OK else None)

        def warm():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, _ = warmstart.warm_solve(s, net, k0, 50000, target)
            torch.cuda.synchronize()
            warm_t.append(time.perf_counter() - t0)
            warm_it.append(it if st == ncs.NCS_OK else None)

        # the two legs alternate in order from slice to slice
        legs = [plain] if net is None else ([plain, warm] if i % 2 == 0 else [warm, plain])
        for leg in legs:
            leg()
        s.close()
        progress(f"  slice {i}: plain {plain_it[-1]} it {plain_t[-1]:.3f} s" +
                 (f", warm {warm_it[-1]} it {warm_t[-1]:.3f} s" if net is not None else ""))
    # PDHG (eq. PDHG) on the same kernels and the first slice: M = gamma_P I with
    # gamma_P = 1.05 alpha lambda_max(A^T A); lambda_max(E^T E) by power iteration,
    # plus (beta/alpha)^2 * 8 for D^T D (its largest eigenvalue is below 8)
    progress("PDHG: power iteration for lambda_max(E^T E)")
    op = ncs.Solver(geom, params(ncs))
    g = torch.Generator(device="cpu").manual_seed(3)
    v = torch.randn(geom.n, generator=g, dtype=torch.float32).to(dev)
    lam_e = 0.0
    for _ in range(60):
        w = op.adjoint(op.forward(v / torch.linalg.norm(v)))
        lam_e = float(torch.linalg.norm(w))
        v = w
    op.close()
    # PDHG at its own alpha: 3e-4 took 9,741 iterations on this slice, 2.4e-3 14,268
    gamma_p = 1.05 * PDHG_ALPHA * (lam_e + (BETA_RATIO ** 2) * 8.0)
    pp = ncs.Params(PDHG_ALPHA, BETA_RATIO * PDHG_ALPHA, gamma_p, LAMBDA, method=ncs.METHOD_PDHG)
    s = ncs.Solver(geom, pp, b=bs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_init()
    st, it_p, f_p = s.solve(args.pdhg_iters, fstar[0] * (1.0 + GAP))
    torch.cuda.synchronize()
    pdhg = {"slice": 0, "alpha": PDHG_ALPHA, "gamma_p": gamma_p, "lambda_max_EtE": lam_e, "seconds": time.perf_counter() - t0,
            "iterations": it_p, "reached": st == ncs.NCS_OK, "rel_gap_at_end": (f_p - fstar[0]) / abs(fstar[0]),
            "ncs_iterations_same_slice": plain_it[0]}
    s.close()
    progress(f"PDHG: {it_p} iterations, reached {st == ncs.NCS_OK} (NCS: {plain_it[0]})")
    # ADMM with 10 preconditioned CG steps per linear solve on the same slice
    pa = ncs.Params(ALPHA, BETA_RATIO * ALPHA, GAMMA_FRAC * ALPHA * N_ANGLES * N_SIDE / math.pi, LAMBDA,
                    method=ncs.METHOD_ADMM_CG, cg_iters=10, cg_precondition=1)
    s = ncs.Solver(geom, pa, b=bs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_init()
    st, it_a, f_a = s.solve(args.admm_iters, fstar[0] * (1.0 + GAP))
    torch.cuda.synchronize()
    admm = {"slice": 0, "cg_iters": 10, "preconditioner": "alpha M^+ (the NCS circulant)",
            "seconds": time.perf_counter() - t0, "iterations": it_a, "reached": st == ncs.NCS_OK,
            "rel_gap_at_end": (f_a - fstar[0]) / abs(fstar[0])}
    s.close()
    progress(f"ADMM-CG: {it_a} iterations, reached {st == ncs.NCS_OK}")
    ok = lambda v: bool(v) and all(x is not None for x in v)
    med = lambda v: float(np.median(v)) if ok(v) else None
    iqr = lambda v: [float(np.percentile(v, 25)), float(np.percentile(v, 75))] if ok(v) else None
    out = {"seeds": seeds, "rel_gap": GAP, "f_star": fstar.tolist(),
           "f_star_source": f"min f over {args.fstar_iters} FP64 NCS iterations of each slice at alpha "
                            f"{FSTAR_ALPHA:g}",
           "f_star_rel_change_last_1000": tail,
           "protocol": "per slice: one handle, 64 warm-up iterations (graph capture), then the two legs "
                       "in alternating order, each from set_init; wall time from the leg's start to the "
                       "iteration that first reaches f* (1 + 1e-4)",
           "plain": {"seconds_median": med(plain_t), "seconds_iqr": iqr(plain_t), "iterations_median": med(plain_it),
                     "iterations_iqr": iqr(plain_it), "seconds": plain_t, "iterations": plain_it},
           "pdhg": pdhg, "admm_cg": admm}
    if net is not None:
        out["warm"] = {"seconds_median": med(warm_t), "seconds_iqr": iqr(warm_t), "iterations_median": med(warm_it),
                       "iterations_iqr": iqr(warm_it), "seconds": warm_t, "iterations": warm_it, "k0": k0,
                       "weights": os.path.relpath(WEIGHTS, ROOT), "training": meta,
                       "description": f"{k0} plain iterations, x <- x + N(x) by the network, NCS continued "
                                      f"with its own duals"}
        if ok(plain_t) and ok(warm_t):
            rt = np.array(warm_t) / np.array(plain_t)
            ri = np.array(warm_it, dtype=float) / np.array(plain_it, dtype=float)
            out["warm_vs_plain"] = {"time_ratio_median": float(np.median(rt)),
                                    "time_ratio_iqr": [float(np.percentile(rt, 25)), float(np.percentile(rt, 75))],
                                    "iteration_ratio_median": float(np.median(ri)),
                                    "slices_faster": int((rt < 1.0).sum()), "slices": len(rt)}
        net.close()
    else:
        out["warm"] = None
    return out


# PET: the fastest of a scan of alpha in {0.01, ..., 1} and gamma/(alpha C_R)
# in {0.1, ..., 1} by the iterations to the gap (38,263 at alpha 1, gamma =
# alpha C_R; 3,957 here; smaller alpha or gamma stalls); f* from a long FP64
# run at alpha 0.2, whose objective settles to 2e-9 per 1,000 iterations.
# With x >= 0 the fastest of alpha in {0.05, ..., 2} is 0.3 (5,184 iterations
# to the projected gap; 35,328 at alpha 1, gamma = alpha C_R; 29,120 at 0.05).
PET_ALPHA, PET_GAMMA_FRAC, PET_FSTAR_ALPHA, PET_POS_ALPHA = 0.05, 0.3, 0.2, 0.3


def _pet_fstar(ncs, geom, p, b64, bg64, iters: int, label: str):
    """A long double-precision run: the smallest finite objective, the
    relative change over its last 1,000 iterations, min x and the last
    objective."""
    s64 = ncs.Solver(geom, p, b=b64, bg=bg64, dtype=b64.dtype)
    s64.set_init()
    best, done, obj = np.inf, 0, None
    while done < iters:
        k = min(20000, iters - done)
        obj = s64.iterate(k, record=True)
        best = min(best, float(obj[np.isfinite(obj)].min()))
        done += k
        progress(f"{label} f*: {done}/{iters} double-precision iterations")
    xmin = float(s64.x().min())
    s64.close()
    return best, float(abs(obj[-1] - obj[-1001]) / abs(obj[-1])), xmin, float(obj[-1])


def pet_data(ncs, torch, dev):
    """The PET workload's data: 128^2 activity phantom (seed 0) scaled to 1e6
    expected counts over 180 angles x 185 bins with a uniform 5% background,
    Poisson counts (FP64 tensors on the device)."""
    import ncs_inputs
    n, na, nb = 128, 180, 185
    geom = ncs.Geometry(n, na, nb)
    op = ncs.Solver(geom, pet_params(ncs, na * n / math.pi, PET_ALPHA, PET_GAMMA_FRAC))
    base = torch.tensor(ncs_inputs.phantom(n, 0).ravel(), dtype=torch.float32, device=dev)
    proj = op.forward(base).double()
    scale = 1e6 / (1.05 * float(proj.sum()))
    clean = (proj * scale).cpu().numpy()
    bg = np.full(clean.size, 0.05 * clean.sum() / clean.size)
    counts = ncs_inputs.poisson_counts(0, clean + bg)
    op.close()
    return (geom, na * n / math.pi, torch.tensor(counts, dtype=torch.float64, device=dev),
            torch.tensor(bg, dtype=torch.float64, device=dev))


def pet_params(ncs, c_r: float, alpha: float, gamma_frac: float, positivity: int = 0):
    return ncs.Params(alpha, 3.0 * alpha, gamma_frac * alpha * c_r, 0.02, data_term=ncs.DATA_POISSON,
                      tv_term=ncs.TV_ISO, positivity=positivity)


def solve_projected(s, f_target: float, max_iters: int, chunk: int = 64):
    """Iterations until the projection max(x^k, 0) has f <= f_target, tested
    every `chunk` iterations (and after the last of max_iters).  With x >= 0 the objective the library reports
    for x^k leaves out the indicator, so an infeasible iterate can lie below
    the constrained minimum; the projection is feasible, and its objective is
    the constrained one."""
    done = 0
    while done < max_iters:
        k = min(chunk, max_iters - done)
        s.iterate(k)
        done += k
        f = s.objective(s.x().clamp_(min=0))
        if f <= f_target:
            return done, f
    return None, None


def pet_time_to_gap(ncs, torch, dev, fstar_iters: int) -> dict:
    """The PET workload (isotropic TV, lambda = 0.02).  Plain NCS from zero to
    f <= f* (1 + 1e-4), f* the smallest objective of a long double-precision run."""
    geom, c_r, b64, bg64 = pet_data(ncs, torch, dev)

    def pp(a, positivity=0, gf=PET_GAMMA_FRAC):
        return pet_params(ncs, c_r, a, gf, positivity)
    p = pp(PET_ALPHA)
    fstar, tail, _, _ = _pet_fstar(ncs, geom, pp(PET_FSTAR_ALPHA), b64, bg64, fstar_iters, "PET")
    s = ncs.Solver(geom, p, b=b64.float(), bg=bg64.float())
    s.set_init()
    s.iterate(64)   # warm-up: graphs captured
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_init()
    st, it, f = s.solve(50000, fstar * (1.0 + GAP))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    xmin_free = float(s.x().min())
    s.close()
    # the same workload with the constraint x >= 0 (remark in Section 4.2): its
    # f* is the last objective of a long double-precision constrained run (its
    # smallest objective falls in the early, infeasible iterations)
    _, tail_pos, xmin_ref, fstar_pos = _pet_fstar(ncs, geom, pp(PET_FSTAR_ALPHA, 1), b64, bg64, fstar_iters,
                                                  "PET with x >= 0")
    s = ncs.Solver(geom, pp(PET_POS_ALPHA, 1), b=b64.float(), bg=bg64.float())
    s.set_init()
    s.iterate(64)
    s.objective(s.x().clamp_(min=0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_init()
    it_p, f_p = solve_projected(s, fstar_pos * (1.0 + GAP), 50000)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    xmax = float(s.x().max())
    xmin_pos = float(s.x().min())
    s.close()
    progress(f"PET: plain {it} iterations, with x >= 0 {it_p} iterations")
    return {"workload": "128^2 PET, 180 x 185, 1e6 counts, 5% background, isotropic TV lambda 0.02, seed 0",
            "params": f"alpha {PET_ALPHA:g}, beta 3 alpha, gamma = {PET_GAMMA_FRAC:g} alpha C_R", "f_star": fstar,
            "f_star_source": f"min finite f over {fstar_iters} FP64 iterations at alpha {PET_FSTAR_ALPHA:g} "
                             f"(objective includes sum log Gamma(b+1))",
            "f_star_rel_change_last_1000": tail,
            "seconds": dt, "iterations": it if st == ncs.NCS_OK else None, "reached": st == ncs.NCS_OK,
            "min_x_at_gap": xmin_free,
            "positivity": {"params": f"alpha {PET_POS_ALPHA:g}, beta 3 alpha, gamma = {PET_GAMMA_FRAC:g} alpha C_R",
                           "f_star": fstar_pos,
                           "f_star_source": f"last f of {fstar_iters} FP64 constrained iterations at alpha "
                                            f"{PET_FSTAR_ALPHA:g}",
                           "f_star_rel_change_last_1000": tail_pos, "min_x_f_star_run": xmin_ref,
                           "stop": "f(max(x^k, 0)) <= f* (1 + 1e-4), tested every 64 iterations (in the time)",
                           "seconds": dt_p, "iterations": it_p, "reached": it_p is not None,
                           "f_projected_at_stop": f_p, "min_x_at_gap": xmin_pos, "max_x_at_gap": xmax,
                           "note": "x >= 0 as a third block of A"}}


def fan_time_to_gap(ncs, torch, dev, fstar_iters: int) -> dict:
    """The fan-beam workload: 256^2, 90 source positions over a full turn x 368
    equi-angular bins, source at 512 pixels from the centre, random-ellipse
    phantom (seed 0), 1% Gaussian noise, anisotropic TV lambda 0.005.  E^T E's
    multiplier is the 16-probe estimate of eq. H-fan.  NCS and PDHG from zero
    to f <= f* (1 + 1e-4), f* the smallest objective of a long double-precision
    NCS run."""
    import ncs_inputs
    n, nv, nb, rs, lam, alpha = 256, 90, 368, 512.0, 0.005, 1e-3
    geom = ncs.Geometry(n, nv, nb, beam=ncs.BEAM_FAN, source_radius=rs)
    gamma = alpha * nv * n / (2.0 * math.pi)     # 0.3 of this diverged with the probe estimate
    p = ncs.Params(alpha, BETA_RATIO * alpha, gamma, lam)
    op = ncs.Solver(geom, p)
    x = torch.tensor(ncs_inputs.phantom(n, 0).ravel(), dtype=torch.float32, device=dev)
    clean = op.forward(x)
    eps = torch.tensor(ncs_inputs.gaussian_noise(0, geom.m), dtype=torch.float32, device=dev)
    b = (clean + 0.01 * float(clean.max()) * eps).contiguous()
    v = torch.randn(geom.n, generator=torch.Generator(device="cpu").manual_seed(3)).to(dev)
    lam_e = 0.0
    for _ in range(60):
        w = op.adjoint(op.forward(v / torch.linalg.norm(v)))
        lam_e = float(torch.linalg.norm(w))
        v = w
    op.close()
    progress(f"fan beam f*: {fstar_iters} double-precision iterations")
    s64 = ncs.Solver(geom, p, b=b.double(), dtype=torch.float64)
    s64.set_init()
    fstar = np.inf
    done = 0
    while done < fstar_iters:
        k = min(5000, fstar_iters - done)
        obj = s64.iterate(k, record=True)
        fstar = min(fstar, float(obj.min()))
        done += k
    s64.close()
    out = {"workload": "256^2 fan beam, 90 views x 368 bins, source radius 512, anisotropic TV lambda 0.005, seed 0",
           "params": f"alpha {alpha}, beta 3 alpha, gamma = alpha N_v N / (2 pi) = {gamma:.4g}, 16 probes (eq. H-fan)",
           "f_star": fstar, "f_star_source": f"min f over {fstar_iters} FP64 NCS iterations",
           "f_star_rel_change_last_1000": float(abs(obj[-1] - obj[-1001]) / abs(obj[-1]))}
    gamma_p = 1.05 * alpha * (lam_e + (BETA_RATIO ** 2) * 8.0)
    for name, pp, budget in (("ncs", p, 60000),
                             ("pdhg", ncs.Params(alpha, BETA_RATIO * alpha, gamma_p, lam, method=ncs.METHOD_PDHG),
                              200000)):
        s = ncs.Solver(geom, pp, b=b)
        s.set_init()
        s.iterate(1)
        s.set_init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, f = s.solve(budget, fstar * (1.0 + GAP))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        out[name] = {"seconds": dt, "iterations": it, "reached": st == ncs.NCS_OK, "it_per_s": it / dt}
        progress(f"fan beam {name}: {it} iterations, {dt:.3f} s, reached {st == ncs.NCS_OK}")
    out["pdhg"]["gamma_p"] = gamma_p
    return out


def cone_data(cone, ncs, torch, dev, geom, seed: int = 0):
    """b = E x_true + 1% Gaussian noise for the random-ellipsoid volume of `seed`."""
    import ncs_inputs
    op = cone.ConeSolver(geom, cone.ConeParams(1e-3, 3e-3, 1.0, 0.0, method=ncs.METHOD_PDHG))
    x = torch.tensor(ncs_inputs.phantom3d(geom.n_side, geom.n_slices, seed).ravel(), dtype=torch.float32,
                     device=dev)
    clean = op.forward(x)
    eps = torch.tensor(ncs_inputs.gaussian_noise(seed, geom.m), dtype=torch.float32, device=dev)
    b = (clean + 0.01 * float(clean.max()) * eps).contiguous()
    # lambda_max(E^T E) by power iteration (the PDHG step)
    v = torch.randn(geom.n, generator=torch.Generator(device="cpu").manual_seed(3)).to(dev)
    lam_e = 0.0
    for _ in range(60):
        w = op.adjoint(op.forward(v / torch.linalg.norm(v)))
        lam_e = float(torch.linalg.norm(w))
        v = w
    torch.cuda.synchronize()
    op.close()
    return b, lam_e


def cone_legs(ncs, torch, dev, steps: int, fstar_iters: int) -> dict:
    """Cone-beam CT on volumes (ncs_cone.h).

    Throughput: 256^2 x 64 voxels, 72 source positions over a full turn, a
    cylindrical detector of 64 rows x 368 equi-angular columns, source at 512
    voxels; `steps` timed FP32 NCS iterations and the per-phase times.

    Time to gap: 128^2 x 32 voxels, 48 views x 32 rows x 184 columns, source at
    256; NCS and PDHG (FP32) from zero to f <= f* (1 + 1e-4), f* the smallest
    objective of long FP64 NCS and PDHG runs of the same library.  The solvers
    are checked every 10 iterations (the time includes at most 9 iterations
    past the target).  Both use alpha = 3e-3, beta = 3 alpha, lambda = 0.005;
    NCS gamma = 3.2 alpha N_v N / (2 pi) (smaller factors break M >= alpha A^T A
    with the probe-estimated multiplier), PDHG gamma_P = 1.05 alpha
    (lambda_max(E^T E) + 9 x 12)."""
    from paper_1810_13100_amd import cone
    lam, alpha = 0.005, 3e-3
    out = {}
    geom = cone.ConeGeometry(256, 64, 72, 368, 64, 512.0)
    gamma = 3.2 * cone.default_gamma(geom, alpha)
    progress("cone beam 256^2 x 64: data and setup")
    b, _ = cone_data(cone, ncs, torch, dev, geom)
    t0 = time.perf_counter()
    s = cone.ConeSolver(geom, cone.ConeParams(alpha, 3 * alpha, gamma, lam), b=b)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    s.set_init()
    s.iterate(5)
    torch.cuda.synchronize()
    progress(f"cone beam: timing {steps} iterations")
    t0 = time.perf_counter()
    s.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = s.info()
    phases = s.time_phases(10)
    s.close()
    dom = max(phases, key=phases.get)
    flops = 2.0 * info["nnz"]
    roof = {"kernel": dom, "ms_per_launch": phases[dom]}
    if dom in ("backproject", "project_dataprox"):
        ach = flops / (phases[dom] * 1e-3) / 1e12
        roof.update({"bound": "alu", "achieved": ach, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(dom, CONE_TRAFFIC_FILE, CONE_SOURCE),
                     "work_per_launch": f"2 x nnz(E) = {flops:.4g} flop"})
    out["throughput"] = {
        "workload": "256^2 x 64 cone beam, 72 views x 64 rows x 368 columns, source radius 512, "
                    "anisotropic 3D TV lambda 0.005, random-ellipsoid volume seed 0, 1% Gaussian noise",
        "dtype": "f32", "iterations": steps, "seconds": dt, "it_per_s": steps / dt, "ms_per_iteration": 1e3 * dt / steps,
        "setup_s": setup_s, "nnz_E": info["nnz"], "phases_ms": phases, "roofline": roof,
        "bin_window": info["bin_window"]}
    progress(f"cone beam: {steps / dt:.1f} it/s, phases {phases}")
    if fstar_iters <= 0:
        return out

    geom = cone.ConeGeometry(128, 32, 48, 184, 32, 256.0)
    gamma = 3.2 * cone.default_gamma(geom, alpha)
    b, lam_e = cone_data(cone, ncs, torch, dev, geom)
    gamma_p = 1.05 * alpha * (lam_e + 9.0 * 12.0)
    p_ncs = cone.ConeParams(alpha, 3 * alpha, gamma, lam)
    p_pdhg = cone.ConeParams(alpha, 3 * alpha, gamma_p, lam, method=ncs.METHOD_PDHG)
    progress(f"cone beam f*: {fstar_iters} FP64 NCS and PDHG iterations at 128^2 x 32")
    fstar = np.inf
    tails = []
    for pp in (p_ncs, p_pdhg):
        s64 = cone.ConeSolver(geom, pp, b=b.double(), dtype=torch.float64)
        s64.set_init()
        done = 0
        while done < fstar_iters:
            k = min(2000, fstar_iters - done)
            obj = s64.iterate(k, record=True)
            fstar = min(fstar, float(np.nanmin(obj)))
            done += k
        tails.append(float(abs(obj[-1] - obj[-1001]) / abs(obj[-1])))
        s64.close()
    gap = {"workload": "128^2 x 32 cone beam, 48 views x 32 rows x 184 columns, source radius 256, "
                       "anisotropic 3D TV lambda 0.005, seed 0, 1% noise",
           "params": f"alpha {alpha}, beta 3 alpha, NCS gamma 3.2 alpha N_v N / (2 pi) = {gamma:.4g}, "
                     f"PDHG gamma_P = {gamma_p:.4g}, 16 probes (eq. H-fan, 3D DFT)",
           "f_star": fstar, "f_star_source": f"min f over {fstar_iters} FP64 NCS and {fstar_iters} FP64 PDHG iterations",
           "f_star_rel_change_last_1000": {"ncs": tails[0], "pdhg": tails[1]}}
    target = fstar * (1.0 + GAP)
    for name, pp, budget in (("ncs", p_ncs, 40000), ("pdhg", p_pdhg, 80000)):
        s = cone.ConeSolver(geom, pp, b=b)
        s.set_init()
        s.iterate(2)
        s.set_init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, hit = 0, None
        while done < budget and hit is None:
            obj = s.iterate(10, record=True)
            below = np.nonzero(obj <= target)[0]
            if below.size:
                hit = done + int(below[0]) + 1
            done += 10
        dt = time.perf_counter() - t0
        s.close()
        gap[name] = {"seconds": dt, "iterations": hit if hit is not None else done, "reached": hit is not None,
                     "it_per_s": done / dt}
        progress(f"cone beam {name}: {gap[name]['iterations']} iterations, {dt:.3f} s, reached {hit is not None}")
    gap["pdhg"]["gamma_p"] = gamma_p
    out["time_to_gap"] = gap
    return out


# alpha per image side of the uneven batch: the fastest of a scan over
# alpha in {1/4, ..., 8} x 3e-4 (256/N)^2 and beta/alpha in {1, 3, 10}
# (iterations of one slice to the 1e-4 gap); beta = 3 alpha, gamma = 0.3 alpha C_R
BATCH_ALPHA = {128: 2.4e-3, 256: 6e-4, 512: 3e-4}


def batch_slices(ncs, torch, dev):
    """The uneven batch: 205 slices of 128^2, 205 of 256^2 and 102 of 512^2
    (angles round(1.4 side), bins side + side/64), shuffled; every slice has its
    own seeded phantom and 1% Gaussian noise."""
    import ncs_inputs
    sides = ncs_inputs.batch_sides()
    ops, geoms, pars, bs = {}, [], [], []
    progress(f"batch: preparing {len(sides)} slices")
    for i, side in enumerate(sides):
        n, na, nb = ncs_inputs.batch_geometry(int(side))
        g = ncs.Geometry(n, na, nb)
        alpha = BATCH_ALPHA[n]
        p = ncs.Params(alpha, BETA_RATIO * alpha, GAMMA_FRAC * alpha * na * n / math.pi, LAMBDA)
        if n not in ops:
            ops[n] = ncs.Solver(g, p)
        seed = 10_000 + i
        x = torch.tensor(ncs_inputs.phantom(n, seed).ravel(), dtype=torch.float32, device=dev)
        clean = ops[n].forward(x)
        eps = torch.tensor(ncs_inputs.gaussian_noise(seed, g.m), dtype=torch.float32, device=dev)
        bs.append((clean + 0.01 * float(clean.max()) * eps).contiguous())
        geoms.append(g)
        pars.append(p)
    for o in ops.values():
        o.close()
    torch.cuda.synchronize()
    return sides, geoms, pars, bs


def batch_legs(ncs, torch, dev, iters: int, gap_ref_iters: int) -> dict:
    """Timed: `iters` batch iterations of all 512 slices in shared launches
    (replayed graphs, objective every iteration).  With gap_ref_iters > 0 also
    the wall time until every slice has stopped at its own target
    f* (1 + 1e-4), f* the smallest objective of the slice over gap_ref_iters
    FP32 iterations of the same batch (each slice stops on the device; stopped
    slices leave the shared launches)."""
    sides, geoms, pars, bs = batch_slices(ncs, torch, dev)
    t0 = time.perf_counter()
    bat = ncs.Batch(geoms, pars, bs)
    setup_s = time.perf_counter() - t0
    bat.set_init()
    bat.solve(50)   # graphs captured, every kernel run once
    torch.cuda.synchronize()
    progress(f"batch: timing {iters} iterations of {len(sides)} slices")
    t0 = time.perf_counter()
    _, it, _ = bat.solve(iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    taps = sum(1.8 * g.n_side * (g.n_side + 1) * g.n_angles for g in geoms)   # nnz(E) estimate per slice
    out = {"slices": len(sides), "mix": {"128": int((sides == 128).sum()), "256": int((sides == 256).sum()),
                                         "512": int((sides == 512).sum())},
           "iterations": iters, "seconds": dt, "slice_iterations_per_s": len(sides) * iters / dt,
           "ms_per_batch_iteration": dt / iters * 1e3, "est_taps_per_s": 2 * taps * iters / dt,
           "setup_s": setup_s,
           "alpha": {str(k): v for k, v in BATCH_ALPHA.items()}, "beta": "3 alpha", "gamma": "0.3 alpha C_R",
           "time_to_all_stop": None}
    if gap_ref_iters > 0:
        n = len(sides)
        fstar = np.full(n, np.inf)
        bat.set_init()
        done, t0 = 0, time.perf_counter()
        last = np.zeros(n)
        while done < gap_ref_iters:
            k = min(4000, gap_ref_iters - done)
            bat.solve(k)
            for i in range(n):
                h = bat.slice(i).objectives(done, k)
                fstar[i] = min(fstar[i], float(h.min()))
                if done + k == gap_ref_iters:
                    last[i] = abs(h[-1] - h[-1001]) / abs(fstar[i]) if k > 1000 else np.nan
            done += k
            progress(f"batch f*: {done}/{gap_ref_iters} iterations ({time.perf_counter() - t0:.0f} s)")
        ref_s = time.perf_counter() - t0
        bat.set_init()
        torch.cuda.synchronize()
        progress("batch: timing the per-slice stop at the 1e-4 gap")
        # calls of at most 2000 iterations; a slice that has stopped sits out
        # the later calls (target -inf)
        target = fstar * (1.0 + GAP)
        its, f = np.zeros(n, dtype=np.int64), np.full(n, np.inf)
        done_mask = np.zeros(n, dtype=bool)
        t0 = time.perf_counter()
        run = 0
        while run < gap_ref_iters and not done_mask.all():
            k = min(2000, gap_ref_iters - run)
            _, it_c, f_c = bat.solve(k, np.where(done_mask, -np.inf, target))
            its += np.asarray(it_c)
            f = np.where(done_mask, f, f_c)
            done_mask |= f_c <= target
            run += k
            progress(f"batch: {int(done_mask.sum())}/{n} slices stopped after {run} iterations "
                     f"({time.perf_counter() - t0:.0f} s)")
        torch.cuda.synchronize()
        m4 = time.perf_counter() - t0
        per = {}
        for side in (128, 256, 512):
            sel = its[sides == side]
            per[str(side)] = {"median": float(np.median(sel)), "min": int(sel.min()), "max": int(sel.max())}
        out["time_to_all_stop"] = {
            "seconds": m4, "reached": int(np.sum(f <= fstar * (1.0 + GAP))), "slices": n,
            "iterations_by_side": per, "slice_iterations": int(its.sum()),
            "f_star_source": f"min f of each slice over {gap_ref_iters} FP32 iterations of the same batch "
                             f"({ref_s:.0f} s)",
            "f_star_rel_change_last_1000_max": float(np.nanmax(last)),
            "check_every": 50, "rel_gap": GAP}
        progress(f"batch: all {n} slices stopped after {m4:.1f} s (max {int(its.max())} iterations)")
    bat.close()
    return out


def paper_context(ncs, torch, dev, iters: int = 500) -> dict:
    """The paper's parallel-beam experiment shape, 512^2 with 60 angles x 729
    bins and lambda = 1 (its data are not available: a seeded random-ellipse
    phantom with 1% noise stands in), timed like the headline: iterations/s of
    replayed graphs with the objective every iteration.  Context beside the
    paper's Table 1 (1000 iterations at 512^2 in 5.32 s on its GPU, angles not
    stated there)."""
    import ncs_inputs
    n, na, nb = 512, 60, 729
    g = ncs.Geometry(n, na, nb)
    alpha = 1e-4
    p = ncs.Params(alpha, BETA_RATIO * alpha, GAMMA_FRAC * alpha * na * n / math.pi, 1.0)
    op = ncs.Solver(g, p)
    x = torch.tensor(ncs_inputs.phantom(n, 0).ravel(), dtype=torch.float32, device=dev)
    clean = op.forward(x)
    eps = torch.tensor(ncs_inputs.gaussian_noise(0, g.m), dtype=torch.float32, device=dev)
    b = (clean + 0.01 * float(clean.max()) * eps).contiguous()
    op.close()
    s = ncs.Solver(g, p, b=b)
    s.set_init()
    s.iterate(100)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.iterate(iters)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    info = s.info()
    s.close()
    return {"workload": "512^2 parallel-beam CT, 60 angles x 729 bins, lambda 1, random-ellipse phantom seed 0, "
                        "1% Gaussian noise", "iterations": iters, "it_per_s": 1000.0 / ms, "ms_per_iteration": ms,
            "kernels": {"projector": info["projector"], "backprojector": info["backprojector"]},
            "paper_table1_512": {"it_per_s": 1000 / 5.32, "hardware": "NVIDIA TITAN Xp, MATLAB; angles not stated"}}


class _BlockRows:
    """y = A @ x for a CSR matrix split into row blocks, one block per pool
    thread (SciPy's CSR product releases the GIL, so the blocks run in parallel)."""

    def __init__(self, a, pool, parts):
        self.shape = a.shape
        self.cuts = np.linspace(0, a.shape[0], parts + 1).astype(int)
        self.blocks = [a[self.cuts[i]:self.cuts[i + 1]] for i in range(parts)]
        self.pool = pool

    def __matmul__(self, x):
        out = np.empty(self.shape[0])

        def part(i):
            out[self.cuts[i]:self.cuts[i + 1]] = self.blocks[i] @ x
        list(self.pool.map(part, range(len(self.blocks))))
        return out


def cpu_baseline(iters: int) -> dict:
    """The FP64 oracle on the same workload, timed on the host (assembly
    excluded): as it stands (SciPy CSR products and numpy FFTs, one core), and
    a threaded variant of the same iterations (E and E^T as row blocks on a
    thread pool, scipy.fft with that many workers)."""
    import copy
    from concurrent.futures import ThreadPoolExecutor
    from unittest import mock

    import scipy.fft

    from oracle import operators, problems, solvers
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
    # threads: the CPUs this process may run on, capped at 16
    threads = min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count())
    with ThreadPoolExecutor(threads) as pool:
        tp = copy.copy(prob)
        for name in ("E", "Et"):   # D and D^T (2 nonzeros a row) gain nothing from threads
            setattr(tp, name, _BlockRows(getattr(prob, name), pool, threads))

        def circulant(h, img):
            return np.real(scipy.fft.ifft2(h * scipy.fft.fft2(img, workers=threads), workers=threads))
        progress(f"cpu baseline: {iters} oracle iterations on {threads} threads")
        with mock.patch.object(operators, "apply_circulant", circulant):
            t0 = time.perf_counter()
            solvers.ncs(tp, par, iters)
            dt_t = time.perf_counter() - t0
    return {
        "value": iters / dt, "unit": "iterations/s", "cores": 1, "kind": "oracle",
        "sample": f"{iters} FP64 oracle NCS iterations on the same 256^2 workload (SciPy CSR E and E^T, "
                  f"numpy FFT, objective every iteration; E assembly excluded); single-threaded "
                  f"({os.cpu_count()} host CPUs visible: {cpu})",
        "seconds": dt,
        "threaded": {"value": iters / dt_t, "unit": "iterations/s", "cores": threads, "seconds": dt_t,
                     "sample": f"the same {iters} iterations with E and E^T split into {threads} row blocks "
                               f"on a pool of {threads} threads and scipy.fft with workers={threads}"},
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=200, help="oracle iterations of the CPU baseline (0: skip)")
    ap.add_argument("--no-gap", action="store_true", help="skip the time-to-gap measurement")
    ap.add_argument("--fstar-iters", type=int, default=24000)
    ap.add_argument("--gap-seeds", type=int, default=32, help="evaluation slices of the time-to-gap measurement")
    ap.add_argument("--pdhg-iters", type=int, default=100000, help="iteration budget of the PDHG comparison")
    ap.add_argument("--admm-iters", type=int, default=5000, help="iteration budget of the ADMM-CG comparison")
    ap.add_argument("--batch-iters", type=int, default=40, help="iterations of the uneven 512-slice batch (0: skip)")
    ap.add_argument("--batch-gap-iters", type=int, default=0,
                    help="FP32 iterations of the batch's f* run before timing the per-slice stop at the 1e-4 gap "
                         "(0: skip; the 512^2 slices need about 16000 iterations, the leg takes about 15 minutes)")
    ap.add_argument("--projector", type=int, default=0,
                    help="forward-projector kernel of the headline solver (0: the setup timing picks it)")
    ap.add_argument("--backprojector", type=int, default=0,
                    help="backprojector kernel of the headline solver (0: the setup timing picks it)")
    ap.add_argument("--cone-steps", type=int, default=50, help="timed cone-beam iterations (0: skip the cone legs)")
    ap.add_argument("--steady-runs", type=int, default=5, help="more runs of 2,000 iterations after the timed steps")
    ap.add_argument("--cone-fstar-iters", type=int, default=20000)
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
    p_head = params(ncs)
    p_head.projector, p_head.backprojector = args.projector, args.backprojector
    s = ncs.Solver(geom, p_head, b=b, dtype=torch.float32)
    info = s.info()
    # the other measurements first: the headline steps are then timed on a GPU
    # that has been busy for a while, as it is in service (a cold GPU runs a
    # 20-step sample about 4% slower)
    gap = None
    if not args.no_gap:
        gap = time_to_gap(ncs, torch, dev, geom, args)

    pet = None if args.no_gap else pet_time_to_gap(ncs, torch, dev, 100000)
    fan = None if args.no_gap else fan_time_to_gap(ncs, torch, dev, 60000)
    batch = batch_legs(ncs, torch, dev, args.batch_iters, args.batch_gap_iters) if args.batch_iters > 0 else None
    cone_out = None
    if args.cone_steps > 0:
        cone_out = cone_legs(ncs, torch, dev, args.cone_steps, 0 if args.no_gap else args.cone_fstar_iters)
    context = None if args.no_gap else paper_context(ncs, torch, dev)

    # per-kernel timing: HIP events around 50 back-to-back launches of each
    # phase on the solver's stream; it moves the state, so the timed run
    # starts again from x = 0 (set_init)
    progress("per-kernel timing (HIP events)")
    phases = s.time_phases(50)
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

    # steady state as a distribution: 5 more runs of 2,000 replayed iterations
    # (HIP events on the solver's stream), reported beside the timed steps
    m1 = []
    for _ in range(args.steady_runs):
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        s.iterate(2000)
        f1.record(stream)
        torch.cuda.synchronize()
        m1.append(2000 * 1000.0 / f0.elapsed_time(f1))
    m1_out = {"iterations": 2000, "it_per_s": m1, "median": float(np.median(m1))} if m1 else None

    calibration_copy(torch, dev)
    dominant = max(phases, key=phases.get)
    flops = 2.0 * info["nnz"]          # one multiply-add per nonzero of E
    dom_ms = phases[dominant]
    if dominant in ("project_dataprox_tv", "backproject"):
        achieved = flops / (dom_ms * 1e-3) / 1e12
        roof = {"kernel": dominant, "bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic(dominant, variants={"projector": info["projector"],
                                                                "backprojector": info["backprojector"]}),
                "work_per_launch": f"2 x nnz(E) = {flops:.4g} flop", "ms_per_launch": dom_ms}
    else:
        roof = {"kernel": dominant, "bound": "hbm", "achieved": None, "peak": 8000.0, "unit": "GB/s",
                "frac": None, "traffic": None, "ms_per_launch": dom_ms}

    # every kernel of the iteration against its own bound: the projector pair
    # against the FP32 vector peak (2 flops per nonzero of E), the DFT passes
    # against HBM with their algorithmic bytes (the arrays they must read and
    # write once; FP32 values, complex half spectrum of (N/2 + 1) N entries)
    n2 = N_SIDE * N_SIDE
    half = (N_SIDE // 2 + 1) * N_SIDE
    fft_bytes = {"fft_rows": 4 * n2 + 8 * half, "fft_cols_multiplier": 16 * half + 4 * half,
                 "fft_rows_inv_update": 8 * half + 4 * n2 + 3 * 4 * n2}
    per_kernel = {}
    for k, ms in phases.items():
        if k in ("project_dataprox_tv", "backproject"):
            a = flops / (ms * 1e-3) / 1e12
            per_kernel[k] = {"bound": "alu", "achieved": a, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": a / FP32_VECTOR_PEAK_TFLOPS, "ms_per_launch": ms}
        elif k in fft_bytes:
            a = fft_bytes[k] / (ms * 1e-3) / 1e9
            per_kernel[k] = {"bound": "hbm", "achieved": a, "peak": 8000.0, "unit": "GB/s", "frac": a / 8000.0,
                             "algorithmic_bytes": fft_bytes[k], "ms_per_launch": ms}
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
        "kernels": {"projector": info["projector"], "backprojector": info["backprojector"],
                    "chosen_by": "setup timing" if args.projector == 0 and args.backprojector == 0 else "flags"},
        "wall_s_timed": wall, "steady_state_5x2000": m1_out, "phases_ms": phases, "roofline": roof, "roofline_per_kernel": per_kernel, "time_to_gap": gap, "pet_time_to_gap": pet, "fan_time_to_gap": fan,
        "batch": batch, "cone": cone_out, "paper_context_512": context,
        "cpu_baseline": cpu, "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
