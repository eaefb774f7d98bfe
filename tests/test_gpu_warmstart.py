"""What the learned warm start gains over plain NCS, at the 64^2 geometry
(90 angles x 92 bins, lambda = 0.01).

A network is trained on the GPU by the library's own kernels on pairs
(x^k0, x_ref) from seeded training phantoms, then evaluated on disjoint
seeds: plain NCS from x = 0 and the warm start (k0 plain iterations, the
network's correction of the iterate, NCS continued with its own duals) run to
the same target f* (1 + 1e-4), f* the smallest objective of a long
double-precision run.  Both runs are decided by NCS.  The test checks that
the network moves the iterate towards the reference on held-out slices, that
the warm start reaches the same target, and reports the iterations it saves
(at this lambda the solution is dominated by amplified noise, which a local
network cannot predict, so the saving is small; it must not be a loss).
"""
import math

import numpy as np
import pytest
import torch

import ncs_inputs
from gpu_common import log
from paper_1810_13100_amd import cnn, ncs, warmstart

pytestmark = pytest.mark.gpu

N, NA, NS, LAM, ALPHA = 64, 90, 92, 0.01, 0.01
K0, REF = 100, 3000


def params():
    c_r = NA * N / math.pi
    return ncs.Params(ALPHA, 3 * ALPHA, 0.3 * ALPHA * c_r, LAM)


def test_warm_start_gain():
    geom = ncs.Geometry(N, NA, NS)
    par = params()
    XK, XR = warmstart.make_pairs(geom, par, [1_000_000 + i for i in range(512)], K0, REF)
    VK, VR = warmstart.make_pairs(geom, par, [2_000_000 + i for i in range(64)], K0, REF)
    net = cnn.WarmStartNet(16, N, N)
    net.set_params(ncs_inputs.cnn_init(5))
    warmstart.train(net, XK, XR, steps=1500, batch=16, lr=1e-3)
    e_in, e_out = warmstart.rel_error(net, VK, VR)
    log(f"held-out |x - x_ref| / |x_ref|: iterate {e_in:.4f}, corrected {e_out:.4f}")
    assert e_out < e_in

    test_seeds = list(range(8))
    op = ncs.Solver(geom, par)
    bs = [warmstart.ct_sinogram(op, s) for s in test_seeds]
    op.close()
    ref = ncs.Batch([geom] * len(bs), [par] * len(bs), [b.double() for b in bs], dtype=torch.float64)
    ref.set_init()
    _, _, fref = ref.solve(20000)
    ref.close()
    plain, warm = [], []
    for b, fs in zip(bs, fref):
        s = ncs.Solver(geom, par, b=b)
        s.set_init()
        st, it, _ = s.solve(20000, fs * (1 + 1e-4))
        assert st == ncs.NCS_OK
        plain.append(it)
        st, it, f = warmstart.warm_solve(s, net, K0, 20000, fs * (1 + 1e-4))
        assert st == ncs.NCS_OK and f <= fs * (1 + 1e-4)
        warm.append(it)
        s.close()
    log(f"iterations to the 1e-4 gap: plain {plain}, warm {warm}; "
        f"median plain {np.median(plain):.0f}, warm {np.median(warm):.0f} "
        f"({100 * (1 - np.sum(warm) / np.sum(plain)):.1f}% fewer in total)")
    assert np.sum(warm) <= np.sum(plain)
    net.close()
