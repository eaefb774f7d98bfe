"""Shared helpers of the GPU parity tests: seeded oracle problems (cached) and
the conversion between the oracle's numpy arrays and device tensors."""
from __future__ import annotations

import functools
import sys

import numpy as np

from oracle import operators, problems, projector, solvers

# (n_side, n_angles, n_bins) of the workloads and of the edge cases
GEOMS = {
    "tiny": (16, 7, 23),        # ragged: 23 bins = one partial ray block, odd angle count
    "c1": (64, 90, 92),         # 64^2 CT, 90 x 92
    "c3": (128, 180, 185),      # 128^2 PET, 180 x 185
    "c4s": (128, 179, 130),     # smallest slice of the uneven batch (narrow detector)
    "c4m": (256, 358, 260),
    "c2": (256, 360, 367),      # 256^2 CT, 360 x 367
}
LAMBDA = {"c1": 0.01, "c2": 0.005, "c3": 0.02}


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def joseph(n_side: int, n_angles: int, n_bins: int):
    return projector.joseph_matrix(n_side, n_angles, n_bins)


def ct_params(n_side: int, n_angles: int, alpha: float = 0.01, ratio: float = 3.0, g: float = 0.3):
    """CT parameters: beta = ratio alpha, gamma = g alpha C_R."""
    return problems.Params(alpha, ratio * alpha, g * alpha * operators.default_c_r(n_side, n_angles))


@functools.lru_cache(maxsize=None)
def ct_problem(key: str, seed: int = 0, lam: float | None = None, tv: str = "aniso"):
    n, na, ns = GEOMS[key]
    lam = LAMBDA.get(key, 0.01) if lam is None else lam
    return problems.ct_problem(n, na, ns, seed, lam, tv=tv, E=joseph(n, na, ns))


@functools.lru_cache(maxsize=None)
def pet_problem(key: str, seed: int = 0, lam: float | None = None):
    n, na, ns = GEOMS[key]
    lam = LAMBDA.get(key, 0.02) if lam is None else lam
    return problems.pet_problem(n, na, ns, seed, lam, tv="iso", E=joseph(n, na, ns))


_traj_cache = {}


def oracle_ncs(prob, par, iters):
    key = (id(prob), par.alpha, par.beta, par.gamma, par.c_r, par.mu_dc, iters)
    if key not in _traj_cache:
        _traj_cache[key] = solvers.ncs(prob, par, iters)
    return _traj_cache[key]


def assert_converging(obj) -> None:
    """A trajectory compared for parity must come from a convergent run: its
    objective ends finite, below the first value and within 5% of its minimum
    (relative errors between two diverging runs say nothing)."""
    obj = np.asarray(obj, dtype=np.float64)
    fin = obj[np.isfinite(obj)]
    assert fin.size and np.isfinite(obj[-1]), "objective not finite at the end"
    assert obj[-1] < fin[0] and obj[-1] <= fin.min() + 0.05 * abs(fin.min()), (fin[0], fin.min(), obj[-1])


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
