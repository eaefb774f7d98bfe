"""Learned warm start of NCS.

NCS runs k0 plain iterations from zero, the residual network of
``include/ncs_cnn.h`` corrects the iterate, x <- x^k0 + N(x^k0), and NCS
continues from the corrected iterate with its own duals (``Solver.set_x``)
to the same objective target as a plain run.  Plain NCS therefore still
decides the result; the network only moves the iterate.

The network is trained on pairs (x^k0, x_ref) made by the batched solver on
seeded synthetic slices (random-ellipse phantoms, Gaussian noise of 1% of
max(E x_true); the paper's patient data are not available), with x_ref the
iterate after `iters_ref` iterations.  Everything that computes runs in the
HIP library: this module only sequences calls and moves tensors.

Restarting with duals rebuilt from x0 (``set_init(x0, dual_from_x0=True)``)
is also available; at the benchmark's lambda it costs more iterations than
it saves unless x0 is within about 1% of the solution, so the corrected
iterate keeps the duals that NCS has already built.
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


def make_pairs(geom: ncs.Geometry, params: ncs.Params, seeds, k0: int, iters_ref: int, chunk: int = 128,
               progress=None) -> tuple[torch.Tensor, torch.Tensor]:
    """(XK, XR): NCS iterates after k0 and after iters_ref iterations from
    zero, float32 [len(seeds), N, N] on the device."""
    seeds = list(seeds)
    N = geom.n_side
    dev = torch.device("cuda", torch.cuda.current_device())
    XK = torch.empty((len(seeds), N, N), dtype=torch.float32, device=dev)
    XR = torch.empty((len(seeds), N, N), dtype=torch.float32, device=dev)
    op = ncs.Solver(geom, params)
    t0 = time.perf_counter()
    for c0 in range(0, len(seeds), chunk):
        part = seeds[c0:c0 + chunk]
        bs = [ct_sinogram(op, s) for s in part]
        bat = ncs.Batch([geom] * len(part), [params] * len(part), bs)
        bat.set_init()
        bat.solve(k0)
        for i in range(len(part)):
            XK[c0 + i] = bat.slice(i).x().view(N, N)
        bat.solve(iters_ref - k0)
        for i in range(len(part)):
            XR[c0 + i] = bat.slice(i).x().view(N, N)
        bat.close()
        if progress:
            progress(f"pairs {c0 + len(part)}/{len(seeds)} ({time.perf_counter() - t0:.1f} s)")
    op.close()
    torch.cuda.synchronize()
    return XK, XR


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


def rel_error(net: cnn.WarmStartNet, Z: torch.Tensor, X: torch.Tensor, batch: int = 16) -> tuple[float, float]:
    """Median over the images of |x - x_ref| / |x_ref| for x = Z (the input) and
    for x = Z + N(Z) (the corrected iterate)."""
    outs = torch.cat([net.forward(Z[i:i + batch].contiguous()) for i in range(0, Z.shape[0], batch)])
    n = Z.shape[0]
    ref = X.reshape(n, -1)
    den = torch.linalg.norm(ref, dim=1)
    e_in = torch.linalg.norm(Z.reshape(n, -1) - ref, dim=1) / den
    e_out = torch.linalg.norm(outs.reshape(n, -1) - ref, dim=1) / den
    return float(torch.median(e_in)), float(torch.median(e_out))


def warm_solve(solver: ncs.Solver, net: cnn.WarmStartNet, k0: int, max_iters: int,
               f_target: float = math.nan) -> tuple[int, int, float]:
    """NCS from zero for k0 iterations (stopping early if the target is met),
    then x <- x + N(x) with the duals kept, then NCS to the target.  Returns
    (status, total iterations, last objective) like Solver.solve."""
    N = solver.geom.n_side
    solver.set_init()
    st, it0, f = solver.solve(min(k0, max_iters), f_target)
    if st == ncs.NCS_OK or it0 >= max_iters:
        return st, it0, f
    x1 = net.forward(solver.x().view(1, N, N)).view(-1)
    solver.set_x(x1)
    st, it1, f = solver.solve(max_iters - it0, f_target)
    return st, it0 + it1, f


def save_params(path: str, theta: np.ndarray) -> None:
    np.save(path, np.asarray(theta, dtype=np.float32), allow_pickle=False)


def load_params(path: str) -> np.ndarray:
    a = np.load(path, allow_pickle=False)
    if a.dtype != np.float32 or a.size != cnn.N_PARAMS:
        raise ValueError(f"{path}: expected {cnn.N_PARAMS} float32 parameters")
    return a
