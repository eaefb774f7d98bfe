"""What the learned warm start gains over plain NCS.

* At the 64^2 geometry (90 angles x 92 bins, lambda = 0.01) a network is
  trained on the GPU by the library's own kernels on pairs (x^k0, x_ref) from
  seeded training phantoms, then evaluated on disjoint seeds: plain NCS from
  x = 0 and the warm start (k0 plain iterations, the network's correction of
  the iterate, NCS continued with its own duals) run to the same target
  f* (1 + 1e-4), f* the smallest objective of a long double-precision run.
  Both runs are decided by NCS.  The test checks that the network moves the
  iterate towards the reference on held-out slices and that the warm start
  reaches the same target in no more iterations in total (at this lambda the
  solution is dominated by amplified noise, which a local network cannot
  predict, so the saving is small).
* The committed network for the 256^2 workload (360 x 367, lambda 0.005;
  trained on seeds 1000000 + i) on 16 held-out slices (seeds 100..115): every
  warm start reaches the target, the total iteration count falls by at least
  the stated fraction and most slices are faster.
"""
import json
import math
import os

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


W_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1810_13100_amd",
                      "weights", "warmstart_ct256")
MIN_SAVING = 0.01      # at least 1% fewer iterations in total over the held-out slices


def test_committed_weights_on_held_out_ct256_slices():
    with open(W_PATH + ".json") as f:
        meta = json.load(f)
    n, na, ns = meta["geometry"]
    geom = ncs.Geometry(n, na, ns)
    par = ncs.Params(meta["alpha"], meta["beta"], meta["gamma"], meta["lambda"])
    k0 = int(meta["k0"])
    net = cnn.WarmStartNet(1, n, n)
    net.set_params(warmstart.load_params(W_PATH + ".npy"))
    seeds = list(range(100, 116))
    op = ncs.Solver(geom, par)
    bs = [warmstart.ct_sinogram(op, s) for s in seeds]
    op.close()
    log(f"f*: 12000 FP64 iterations on {len(seeds)} held-out slices")
    ref = ncs.Batch([geom] * len(bs), [par] * len(bs), [b.double() for b in bs], dtype=torch.float64)
    ref.set_init()
    fstar = np.full(len(bs), np.inf)
    for _ in range(6):
        _, _, f = ref.solve(2000)
        fstar = np.minimum(fstar, f)
    ref.close()
    plain, warm = [], []
    for i, (b, fs) in enumerate(zip(bs, fstar)):
        s = ncs.Solver(geom, par, b=b)
        target = fs * (1 + 1e-4)
        s.set_init()
        st, it, _ = s.solve(50000, target)
        assert st == ncs.NCS_OK
        plain.append(it)
        st, it, f = warmstart.warm_solve(s, net, k0, 50000, target)
        assert st == ncs.NCS_OK and f <= target
        warm.append(it)
        s.close()
        log(f"  seed {seeds[i]}: plain {plain[-1]}, warm {warm[-1]}")
    net.close()
    saving = 1 - np.sum(warm) / np.sum(plain)
    faster = int(np.sum(np.array(warm) < np.array(plain)))
    log(f"held-out 256^2: median plain {np.median(plain):.0f}, warm {np.median(warm):.0f}; "
        f"{100 * saving:.2f}% fewer iterations in total, {faster}/{len(seeds)} slices faster")
    assert saving >= MIN_SAVING
    assert faster > len(seeds) // 2
