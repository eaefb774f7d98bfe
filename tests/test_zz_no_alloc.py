"""ncs_forward_noalloc (no handle, no allocation; workspace in a fixed device
array) against ncs_forward of a handle with the same kernel, through the C ABI:
two calls in a row, the second on a smaller geometry (whose padded rows reuse
memory the first call left behind), then a geometry whose workspace exceeds
the fixed array."""
import numpy as np
import pytest
import torch

import ncs_inputs
from gpu_common import log, rel_l2
from paper_1810_13100_amd import ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _reference(geom, x):
    s = ncs.Solver(geom, ncs.Params(0.01, 0.03, 1.0, 0.01, projector=2))
    y = s.forward(x)
    torch.cuda.synchronize()
    s.close()
    return y


def test_forward_noalloc_matches_forward():
    cases = [(ncs.Geometry(256, 360, 367), 0), (ncs.Geometry(64, 90, 92), 1)]
    for geom, seed in cases:
        img = ncs_inputs.phantom(geom.n_side, seed).ravel()
        x = torch.tensor(img, dtype=torch.float32, device=DEV)
        y = torch.full((geom.m,), float("nan"), dtype=torch.float32, device=DEV)
        ncs.forward_noalloc(geom, x, y)
        torch.cuda.synchronize()
        ref = _reference(geom, x)
        err = rel_l2(y.double().cpu().numpy(), ref.double().cpu().numpy())
        log(f"forward_noalloc {geom.n_side}^2, {geom.n_angles} x {geom.n_bins}: rel-L2 vs ncs_forward {err:.2e}")
        assert torch.isfinite(y).all()
        assert err <= 1e-6
    big = ncs.Geometry(1024, 1434, 1040)
    x = torch.zeros(big.n, dtype=torch.float32, device=DEV)
    y = torch.zeros(big.m, dtype=torch.float32, device=DEV)
    with pytest.raises(ncs.NcsError) as e:
        ncs.forward_noalloc(big, x, y)
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    assert "fixed array" in str(e.value)
