"""Train the warm-start network on the GPU and write its parameters.

Usage (from the repository root, one GPU):

    python -m paper_1810_13100_amd.train_warmstart --out paper_1810_13100_amd/weights/warmstart_ct256.npy

Training pairs (x^k0, x_ref) come from the batched solver on seeded
random-ellipse slices at the 256^2 CT geometry (360 angles, 367 bins,
lambda = 0.005, 1% Gaussian noise): training seeds 1,000,000 + i, validation
seeds 2,000,000 + i.  The network starts as the identity map (zero last
layer) and is trained by the library's own forward and backward kernels
with Adam.  A JSON file next to the parameters records the recipe and the
validation errors.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import torch

import ncs_inputs

from . import cnn, ncs, warmstart


def progress(msg: str) -> None:
    print(f"[train] {msg}", file=sys.stderr, flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n-side", type=int, default=256)
    ap.add_argument("--angles", type=int, default=360)
    ap.add_argument("--bins", type=int, default=367)
    ap.add_argument("--lam", type=float, default=0.005)
    ap.add_argument("--alpha", type=float, default=2.4e-3)
    ap.add_argument("--pairs", type=int, default=2048)
    ap.add_argument("--val", type=int, default=64)
    ap.add_argument("--k0", type=int, default=300)
    ap.add_argument("--iters-ref", type=int, default=6000)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("training needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    N = args.n_side
    geom = ncs.Geometry(N, args.angles, args.bins)
    c_r = args.angles * N / math.pi
    par = ncs.Params(args.alpha, 3 * args.alpha, 0.3 * args.alpha * c_r, args.lam)
    t0 = time.perf_counter()
    XK, XR = warmstart.make_pairs(geom, par, [1_000_000 + i for i in range(args.pairs)], args.k0, args.iters_ref,
                                  progress=progress)
    VK, VR = warmstart.make_pairs(geom, par, [2_000_000 + i for i in range(args.val)], args.k0, args.iters_ref)
    t_data = time.perf_counter() - t0
    net = cnn.WarmStartNet(max(args.batch, 16), N, N)
    net.set_params(ncs_inputs.cnn_init(args.seed))
    t0 = time.perf_counter()
    warmstart.train(net, XK, XR, args.steps, args.batch, args.lr, log_every=max(args.steps // 10, 1),
                    progress=progress)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    e_in, e_out = warmstart.rel_error(net, VK, VR)
    progress(f"validation: |x^k0 - x_ref| / |x_ref| = {e_in:.4f}, after the network {e_out:.4f}")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    warmstart.save_params(args.out, net.params())
    meta = {"geometry": [N, args.angles, args.bins], "lambda": args.lam, "alpha": args.alpha,
            "beta": 3 * args.alpha, "gamma": 0.3 * args.alpha * c_r, "k0": args.k0, "iters_ref": args.iters_ref,
            "pairs": args.pairs, "val": args.val, "steps": args.steps, "batch": args.batch, "lr": args.lr,
            "init_seed": args.seed, "val_rel_err_input": e_in, "val_rel_err_output": e_out,
            "data_seconds": t_data, "train_seconds": t_train,
            "train_seeds": "1000000 + i", "val_seeds": "2000000 + i"}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)
    net.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
