"""The stored long oracle runs (tests/golden/make_long.py and
make_pet_fstar.py) against facts that do not depend on the oracle's code:

* a convergent NCS run (Theorem 1) has settled at its end: the objective's
  relative change over its last 1,000 iterations is well below the 1e-4 gap;
* the reference value f* of a relative gap lies at or below every objective of
  the run it is taken from (without constraints every iterate with a finite
  objective is feasible, so f* <= f(x^k) for all k);
* with x >= 0 (remark in Section 4.2) the limit is feasible, and the
  constrained minimum is at least the unconstrained one of the same problem;
* the state stored for the single-precision parity runs sits where the oracle's
  own relative gap at that iteration is small (the library's FP32 run reaches
  1e-4 there, the oracle's trajectory is within a few times that)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(case):
    d = np.load(os.path.join(GOLDEN, case + ".npz"))
    return {k: d[k] for k in d.files}


@pytest.mark.parametrize("case", ["ct256_s0", "ct256_s1"])
def test_ct256_runs_settle_and_gap_at_the_state(case):
    fx = _load(case)
    obj, k = fx["obj"], int(fx["k_state"])
    assert np.all(np.isfinite(obj))
    fstar = obj.min()
    assert abs(obj[-1] - obj[-1001]) <= 1e-5 * abs(fstar)   # 1.1e-6 and 1.2e-6 at alpha 2.4e-3
    gap = (obj[k - 1] - fstar) / abs(fstar)
    assert 0.0 < gap <= 3e-4, gap


def test_pet_run_to_the_state_is_in_the_domain():
    fx = _load("pet128_s0")
    obj = fx["obj"]
    assert np.isfinite(obj[-1]) and obj[-1] < obj[np.isfinite(obj)][0]


def test_pet_f_star_runs():
    free, pos = _load("pet128_s0_fstar"), _load("pet128_s0_pos_fstar")
    for fx in (free, pos):
        assert int(fx["iters"]) == 100000
        tail = fx["obj_last_1000"]
        assert np.all(np.isfinite(tail))
        assert abs(tail[-1] - tail[0]) <= 1e-7 * abs(tail[-1])
    # without constraints: the smallest objective is the run's f*, at or below every stored value
    fmin = float(free["f_min"])
    assert fmin <= np.nanmin(free["obj_every_1000"]) and fmin <= free["obj_last_1000"].min()
    # with x >= 0: the limit is feasible, and its objective is the constrained
    # minimum, at least the unconstrained one
    x = pos["x"]
    assert x.min() >= -1e-8 * x.max()
    assert pos["obj_last_1000"][-1] >= fmin
    # the unconstrained limit uses negative values (so the constraint is active)
    assert free["x"].min() < -1e-3 * free["x"].max()
    # both runs share the problem and parameters
    for k in ("alpha", "beta", "gamma", "lam"):
        assert float(free[k]) == float(pos[k])
    # the same PET slice as the stored FP32-length run, at the same lambda
    assert float(free["lam"]) == float(_load("pet128_s0")["lam"])
