"""Write the long FP64 oracle trajectories that the long-run GPU parity tests read.

Only ``oracle/`` (and the seeded input generator ``ncs_inputs`` through it) is
called here; nothing comes from the HIP library.  Each case is one seeded
problem run by the oracle's NCS (the CT form of Section 4.1 or the PET form of
Section 4.2) from x = u = v = 0:

* ``ct256_s<seed>``: 256 x 256 parallel-beam CT, 360 angles x 367 bins,
  anisotropic TV lambda = 0.005, alpha = 2.4e-3, beta = 3 alpha,
  gamma = 0.3 alpha C_R.  The image and duals are stored after ``k_state``
  iterations (the iteration at which the single-precision run of that slice
  first reaches the 1e-4 relative objective gap) and the objective f(x^k) for
  every k up to ``k_total``, whose minimum is the reference value f* of the
  relative gap.
* ``pet128_s<seed>``: 128 x 128 PET, 180 x 185, 1e6 expected counts with a 5%
  uniform background, isotropic TV lambda = 0.02, alpha = 0.05, beta = 3 alpha,
  gamma = 0.3 alpha C_R, to the same kind of ``k_state``.

Output: ``<case>.npz`` next to this script with arrays ``x``, ``u``, ``v`` (at
``k_state``), ``obj`` (f(x^1) ... f(x^k_total)) and scalars ``k_state``,
``k_total``, ``seed``, ``alpha``, ``beta``, ``gamma``, ``lam``.

Usage: ``python tests/golden/make_long.py [case ...]`` (default: every case).
The CT cases take about half an hour each on one core.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import operators, problems, projector, solvers  # noqa: E402

# case -> (kind, seed, k_state, k_total)
CASES = {
    "ct256_s0": ("ct", 0, 2258, 12000),
    "ct256_s1": ("ct", 1, 2492, 12000),
    "pet128_s0": ("pet", 0, 3957, 3957),
}


def case_problem(kind: str, seed: int):
    if kind == "ct":
        n, na, ns, lam, alpha = 256, 360, 367, 0.005, 2.4e-3
        gamma = 0.3 * alpha * operators.default_c_r(n, na)
        prob = problems.ct_problem(n, na, ns, seed, lam, E=projector.joseph_matrix(n, na, ns))
    else:
        n, na, ns, lam, alpha = 128, 180, 185, 0.02, 0.05
        gamma = 0.3 * alpha * operators.default_c_r(n, na)
        prob = problems.pet_problem(n, na, ns, seed, lam, tv="iso", E=projector.joseph_matrix(n, na, ns))
    return prob, problems.Params(alpha, 3.0 * alpha, gamma)


def run(case: str) -> str:
    kind, seed, k_state, k_total = CASES[case]
    prob, par = case_problem(kind, seed)
    t0 = time.perf_counter()
    first = solvers.ncs(prob, par, k_state)
    obj = [first.obj]
    print(f"{case}: {k_state} iterations in {time.perf_counter() - t0:.0f} s", flush=True)
    if k_total > k_state:
        rest = solvers.ncs(prob, par, k_total - k_state, x0=first.x, u0=first.u, v0=first.v)
        obj.append(rest.obj)
        print(f"{case}: {k_total} iterations in {time.perf_counter() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, case + ".npz")
    np.savez_compressed(out, x=first.x, u=first.u, v=first.v, obj=np.concatenate(obj),
                        k_state=k_state, k_total=k_total, seed=seed, alpha=par.alpha,
                        beta=par.beta, gamma=par.gamma, lam=prob.lam)
    return out


if __name__ == "__main__":
    for c in sys.argv[1:] or list(CASES):
        print(run(c), flush=True)
