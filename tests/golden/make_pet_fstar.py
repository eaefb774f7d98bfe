"""Write the oracle's long double-precision PET runs that pin the reference
value f* of the PET time-to-gap measurements.

Only ``oracle/`` (and the seeded input generator ``ncs_inputs`` through it) is
called here; nothing comes from the HIP library.  The problem is the 128 x 128
PET slice of ``make_long.py`` (Section 4.2: 180 x 185, 1e6 expected counts, a
5% uniform background, isotropic TV lambda = 0.02, seed 0), run by the oracle's
NCS from x = u = v = 0 at alpha = 0.2, beta = 3 alpha, gamma = 0.3 alpha C_R
for 100,000 iterations:

* ``pet128_s0_fstar``: without constraints; f* is the smallest finite
  objective;
* ``pet128_s0_pos_fstar``: with x >= 0 as a third block of A (remark in
  Section 4.2); f* is the last objective (the smallest one falls in the
  early, infeasible iterations, where the objective without the indicator
  lies below the constrained minimum).

Output: ``<case>.npz`` with ``obj_every_1000`` (f(x^1000), f(x^2000), ...),
``obj_last_1000`` (the last 1,000 objectives), ``f_min`` (smallest finite
objective) and its 1-based iteration ``k_min``, ``x`` (x^100000), and the
scalars ``iters``, ``positivity``, ``alpha``, ``beta``, ``gamma``, ``lam``.

Usage: ``python tests/golden/make_pet_fstar.py [case ...]``; each case takes
about 45 min on one core.
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

ITERS = 100000
CASES = {"pet128_s0_fstar": False, "pet128_s0_pos_fstar": True}


def run(case: str) -> str:
    positivity = CASES[case]
    n, na, ns, lam, alpha = 128, 180, 185, 0.02, 0.2
    prob = problems.pet_problem(n, na, ns, 0, lam, tv="iso", E=projector.joseph_matrix(n, na, ns))
    par = problems.Params(alpha, 3.0 * alpha, 0.3 * alpha * operators.default_c_r(n, na))
    t0 = time.perf_counter()
    x = u = v = t = None
    objs = []
    chunk = 10000
    for done in range(0, ITERS, chunk):
        tr = solvers.ncs(prob, par, chunk, x0=x, u0=u, v0=v, positivity=positivity, t0=t)
        x, u, v, t = tr.x, tr.u, tr.v, getattr(tr, "t", None)
        objs.append(tr.obj)
        print(f"{case}: {done + chunk} iterations in {time.perf_counter() - t0:.0f} s", flush=True)
    obj = np.concatenate(objs)
    fin = np.isfinite(obj)
    k_min = int(np.argmin(np.where(fin, obj, np.inf))) + 1
    out = os.path.join(HERE, case + ".npz")
    np.savez_compressed(out, obj_every_1000=obj[999::1000], obj_last_1000=obj[-1000:], f_min=obj[k_min - 1],
                        k_min=k_min, x=x, iters=ITERS, positivity=int(positivity), alpha=par.alpha,
                        beta=par.beta, gamma=par.gamma, lam=prob.lam)
    return out


if __name__ == "__main__":
    for c in sys.argv[1:] or list(CASES):
        print(run(c), flush=True)
