"""Learned warm start of NCS.

The initial point is x0 = z + N(z), where z = alpha M^+ E^T b is the
backprojection filtered by the method's own circulant inverse (eq. circ_R,
Section 4.1.1) and N is the residual network of ``include/ncs_cnn.h``.  NCS
starts from x0 with duals from the fixed-point relations (Section 3.2) and
runs to the same objective target as a cold start, so plain NCS still decides
the result; the network only moves the starting point.

Training pairs (z, x_NCS) come from the batched solver on seeded synthetic
slices (random-ellipse phantoms, Gaussian noise of 1% of max(E x_true); the
paper's patient data are not available).  Everything that computes runs in
the HIP library: this module only sequences calls and moves tensors.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

import ncs_inputs

from . import cnn, ncs


def ct_sinogram(op: ncs.Solver, seed: int, noise: float = 0.01) -> torch.Tensor:
    """b = E x_true + noise * max(E x_true) * eps for the phantom of `seed`, on the device."""
    g = op.geom
    x = torch.tensor(ncs_inputs.phantom(g.n_side, seed).ravel(), dtype=torch.float32, device=op.device)
    clean = op.forward(x)
    eps = torch.tensor(ncs_inputs.gaussian_noise(seed, g.m), dtype=torch.float32, device=op.device)
    return (clean + noise * float(clean.max()) * eps).contiguous()


def make_pairs(geom: ncs.Geometry, params: ncs.Params, seeds, iters: int, chunk: int = 128,
               progress=None) -> tuple[torch.Tensor, torch.Tensor]:
    """(Z, X): pre-filtered backprojections and NCS iterates after `iters`
    iterations from zero, float32 [len(seeds), N, N] on the device."""
    seeds = list(seeds)
    N = geom.n_side
    dev = torch.device("cuda", torch.cuda.current_device())
    Z = torch.empty((len(seeds), N, N), dtype=torch.float32, device=dev)
    X = torch.empty((len(seeds), N, N), dtype=torch.float32, device=dev)
    op = ncs.Solver(geom, params)
    t0 = time.perf_counter()
    for c0 in range(0, len(seeds), chunk):
        part = seeds[c0:c0 + chunk]
        bs = [ct_sinogram(op, s) for s in part]
        bat = ncs.Batch([geom] * len(part), [params] * len(part), bs)
        bat.set_init()
        bat.solve(iters)
        for i in range(len(part)):
            v = bat.slice(i)
            X[c0 + i] = v.x().view(N, N)
            Z[c0 + i] = v.prefilter(bs[i]).view(N, N)
        bat.close()
        if progress:
            progress(f"pairs {c0 + len(part)}/{len(seeds)} ({time.perf_counter() - t0:.1f} s)")
    op.close()
    torch.cuda.synchronize()
    return Z, X


def train(net: cnn.WarmStartNet, Z: torch.Tensor, X: torch.Tensor, steps: int, batch: int, lr: float,
          lr_final: float | None = None, seed: int = 0, log_every: int = 0, progress=None) -> list:
    """Adam on the mean squared error with a cosine learning-rate decay from lr
    to lr_final over `steps` minibatches drawn with replacement."""
    lr_final = lr * 0.05 if lr_final is None else lr_final
    rng = np.random.default_rng(seed)
    n = Z.shape[0]
    losses = []
    for k in range(steps):
        idx = torch.tensor(rng.integers(0, n, batch), device=Z.device)
        zb = Z.index_select(0, idx).contiguous()
        xb = X.index_select(0, idx).contiguous()
        rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / max(steps - 1, 1)))
        want = log_every > 0 and (k % log_every == 0 or k == steps - 1)
        loss = net.train_step(zb, xb.view(-1), rate, want_loss=want)
        if want:
            losses.append((k, loss))
            if progress:
                progress(f"train step {k}: loss {loss:.4e} (lr {rate:.2e})")
    return losses


def initial_point(solver: ncs.Solver, b: torch.Tensor, net: cnn.WarmStartNet) -> torch.Tensor:
    """x0 = z + N(z) with z = alpha M^+ E^T b."""
    N = solver.geom.n_side
    z = solver.prefilter(b).view(1, N, N)
    return net.forward(z).view(-1)


def warm_start(solver: ncs.Solver, b: torch.Tensor, net: cnn.WarmStartNet) -> torch.Tensor:
    """Initial point from the network and duals from the fixed-point relations."""
    x0 = initial_point(solver, b, net)
    solver.set_init(x0, dual_from_x0=True)
    return x0


def save_params(path: str, theta: np.ndarray) -> None:
    np.save(path, np.asarray(theta, dtype=np.float32), allow_pickle=False)


def load_params(path: str) -> np.ndarray:
    a = np.load(path, allow_pickle=False)
    if a.dtype != np.float32 or a.size != cnn.N_PARAMS:
        raise ValueError(f"{path}: expected {cnn.N_PARAMS} float32 parameters")
    return a
