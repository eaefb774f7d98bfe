"""Host-side helpers of bench.py, on the CPU: the counted-traffic lookup is
reported only for the kernel source and variants it was taken with, and the
threaded row-block product of the CPU baseline equals the plain CSR product,
and the constrained time-to-gap stops on the objective of the projected iterate."""
import hashlib
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _record(tmp_path, source_text, variants):
    src = tmp_path / "kernels.hip"
    src.write_text(source_text)
    rec = {"kernel_source_sha256": hashlib.sha256(source_text.encode()).hexdigest(),
           "kernels": {"project_dataprox_tv": {"bytes_per_launch": 123.0}}, **variants}
    tf = tmp_path / "traffic.json"
    tf.write_text(json.dumps(rec))
    return str(tf), str(src)


def test_traffic_needs_the_same_source_and_variants(tmp_path):
    tf, src = _record(tmp_path, "kernel text", {"projector": 1, "backprojector": 1})
    v = {"projector": 1, "backprojector": 1}
    assert bench.measured_traffic("project_dataprox_tv", tf, src, v) == 123.0
    assert bench.measured_traffic("backproject", tf, src, v) is None               # kernel not counted
    assert bench.measured_traffic("project_dataprox_tv", tf, src, {"projector": 2, "backprojector": 1}) is None
    with open(src, "w") as f:
        f.write("kernel text changed")
    assert bench.measured_traffic("project_dataprox_tv", tf, src, v) is None      # source changed
    assert bench.measured_traffic("project_dataprox_tv", str(tmp_path / "missing.json"), src, v) is None


def test_threaded_row_blocks_equal_the_csr_product():
    rng = np.random.default_rng(0)
    a = sp.random(1000, 700, density=0.02, random_state=1, format="csr")
    x = rng.standard_normal(700)
    with ThreadPoolExecutor(4) as pool:
        for parts in (1, 3, 4, 7):
            b = bench._BlockRows(a, pool, parts)
            np.testing.assert_array_equal(b @ x, a @ x)


class _FakeSolver:
    """A stand-in for a constrained solve: x^k approaches the constrained
    minimiser (1, 0) from the infeasible side, x^k = (1, -0.5^k), and the
    objective is f(x) = (x0 - 1)^2 + x1 (without the indicator of x >= 0), so
    f(x^k) lies below the constrained minimum f* = 0 at every k."""
    def __init__(self):
        self.k = 0

    def iterate(self, k, record=False):
        self.k += k

    def x(self):
        import torch
        return torch.tensor([1.0, -0.5 ** self.k], dtype=torch.float64)

    def objective(self, x):
        return float((x[0] - 1.0) ** 2 + x[1])


def test_projected_stop_ignores_infeasible_iterates_below_f_star():
    s = _FakeSolver()
    assert s.objective(s.x()) < 0.0          # the raw objective is below f* already
    it, f = bench.solve_projected(s, 0.0, 1000, chunk=4)
    assert it == 4 and f == 0.0              # the projection (1, 0) attains f* = 0

    class _Shifted(_FakeSolver):             # x^k = (1 + 2^-k, -0.5^k): projected f = 4^-k
        def x(self):
            import torch
            return torch.tensor([1.0 + 0.5 ** self.k, -0.5 ** self.k], dtype=torch.float64)
    s = _Shifted()
    it, f = bench.solve_projected(s, 1e-4, 1000, chunk=2)
    assert it == 8 and abs(f - 0.5 ** 16) < 1e-18    # first chunk end with 4^-k <= 1e-4
    assert bench.solve_projected(_Shifted(), 1e-4, 6, chunk=2) == (None, None)
    s = _Shifted()
    assert bench.solve_projected(s, 1e-4, 6, chunk=4) == (None, None) and s.k == 6   # no overshoot
    it, f = bench.solve_projected(_Shifted(), 1e-4, 7, chunk=4)
    assert it == 7 and f == 0.25 ** 7                  # tested after the last iteration (4^-7 <= 1e-4)
