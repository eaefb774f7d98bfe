"""GPU parity of the warm-start network against the FP64 oracle, through the C ABI.

Gates:
* float -> bfloat16 rounding: bit-exact.
* one convolution layer with bfloat16-exact inputs and weights and a float
  output: max |gpu - oracle| <= 1e-5 max |oracle| (FP32 accumulation of at
  most 288 exact products).  With a bfloat16 output every value is within one
  bfloat16 step (2^-8 relative) of the rounded oracle value, and at least
  99.9% of them equal it (the two sides round different accumulations).
* weight gradients of one layer: max error <= 1e-5 max |oracle| (FP32 sums
  over every pixel).
* the whole network and its gradient, with the oracle emulating the bfloat16
  storage points: x0 rel-L2 <= 1e-4, loss <= 1e-4 relative, each layer's
  gradient rel-L2 <= 5e-3 (a few activations round to the neighbouring
  bfloat16 value on one side only).
* one and two Adam steps: within 1e-2 lr of the oracle's update per parameter.
"""
import numpy as np
import pytest
import torch

import ncs_inputs
from gpu_common import ct_params, ct_problem, log, rel_l2
from oracle import cnn as ocnn
from oracle import problems
from paper_1810_13100_amd import cnn, ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def bf16_dev(a: np.ndarray) -> torch.Tensor:
    t = torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)
    b = t.to(torch.bfloat16)
    assert torch.equal(b.float(), t), "test input is not bfloat16-exact"
    return b.contiguous()


def test_to_bf16_is_round_to_nearest_even():
    rng = np.random.default_rng(11)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        1.0 + (2 * np.arange(256) + 1) * 2.0 ** -8, -(1.0 + (2 * np.arange(256) + 1) * 2.0 ** -8),
                        [0.0, -0.0, 1e-40, -1e-40, 3.3e38]]).astype(np.float32)
    out = cnn.to_bf16(torch.tensor(a, device=DEV)).float().cpu().numpy().astype(np.float64)
    assert np.array_equal(out, ocnn.bf16_round(a))


SHAPES = [(1, 32), (32, 32), (32, 1)]


def layer_inputs(cin, cout, B=2, H=37, W=50, seed=0):
    x = ncs_inputs.bf16_exact(seed, (B, H, W, cin))
    w = ncs_inputs.bf16_exact(seed + 1, (9, cout, cin), exponent=11)
    bias = np.random.default_rng([seed, 9]).standard_normal(cout).astype(np.float32).astype(np.float64)
    return x, w, bias


@pytest.mark.parametrize("cin,cout", SHAPES)
def test_conv_layer_float_output(cin, cout):
    x, w, bias = layer_inputs(cin, cout)
    ref = ocnn.conv3x3(x, w, bias)
    out = cnn.conv3x3_bf16(bf16_dev(x), bf16_dev(w), torch.tensor(bias, dtype=torch.float32, device=DEV),
                           cnn.CONV_F32).double().cpu().numpy()
    err = np.max(np.abs(out.reshape(ref.shape) - ref)) / np.max(np.abs(ref))
    log(f"conv {cin}->{cout} float output: max rel err {err:.2e}")
    assert err <= 1e-5


def check_bf16_close(out, ref_exact, what):
    q = ocnn.bf16_round(ref_exact)
    step = np.maximum(np.abs(q), 1e-30) * 2.0 ** -8
    assert np.all(np.abs(out - q) <= step * 1.0001), what
    frac = np.mean(out == q)
    log(f"{what}: {frac * 100:.3f}% equal to the rounded oracle value")
    assert frac >= 0.999


@pytest.mark.parametrize("cin", [1, 32])
def test_conv_relu_and_mask_epilogues(cin):
    x, w, bias = layer_inputs(cin, 32, seed=3)
    exact = ocnn.conv3x3(x, w, bias)
    out = cnn.conv3x3_bf16(bf16_dev(x), bf16_dev(w), torch.tensor(bias, dtype=torch.float32, device=DEV),
                           cnn.CONV_RELU_BF16).double().cpu().numpy()
    check_bf16_close(out, np.maximum(exact, 0.0), f"conv {cin}->32 relu")
    mask = ncs_inputs.bf16_exact(5, exact.shape)          # about half positive
    nob = ocnn.conv3x3(x, w)
    out = cnn.conv3x3_bf16(bf16_dev(x), bf16_dev(w), None, cnn.CONV_MASK_BF16, mask=bf16_dev(mask)).double()
    check_bf16_close(out.cpu().numpy(), np.where(mask > 0, nob, 0.0), f"conv {cin}->32 mask")


def test_conv_residual_output():
    x, w, bias = layer_inputs(32, 1, seed=4)
    z = np.random.default_rng(6).standard_normal(x.shape[:3]).astype(np.float32)
    ref = z + ocnn.conv3x3(x, w, bias)[..., 0]
    out = cnn.conv3x3_bf16(bf16_dev(x), bf16_dev(w), torch.tensor(bias, dtype=torch.float32, device=DEV),
                           cnn.CONV_RESID_F32, resid=torch.tensor(z, device=DEV)).double().cpu().numpy()
    assert np.max(np.abs(out - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("cin,cout", SHAPES)
@pytest.mark.parametrize("shape", [(2, 37, 50), (1, 16, 16), (3, 5, 70)])
def test_weight_gradient(cin, cout, shape):
    B, H, W = shape
    x = ncs_inputs.bf16_exact(7, (B, H, W, cin))
    dz = ncs_inputs.bf16_exact(8, (B, H, W, cout))
    dw, db = ocnn.conv3x3_weight_grad(x, dz)
    ref = np.concatenate([dw.ravel(), db])
    out = cnn.conv3x3_wgrad_bf16(bf16_dev(x), bf16_dev(dz)).double().cpu().numpy()
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    log(f"wgrad {cin}->{cout} {shape}: max rel err {err:.2e}")
    assert err <= 1e-5


def test_network_forward_and_gradient():
    theta = ncs_inputs.cnn_init(21, scale_last=1.0)
    B, H, W = 2, 24, 40
    rng = np.random.default_rng(22)
    z = rng.uniform(0.0, 1.0, (B, H, W)).astype(np.float32)
    t = (z + 0.1 * rng.standard_normal((B, H, W))).astype(np.float32)
    loss_ref, x0_ref, g_ref = ocnn.loss_and_grad(theta, z.astype(np.float64), t.astype(np.float64), quant=True)
    net = cnn.WarmStartNet(B, H, W)
    net.set_params(theta)
    assert np.array_equal(net.params().astype(np.float64), theta)
    zt, tt = torch.tensor(z, device=DEV), torch.tensor(t, device=DEV)
    x0 = net.forward(zt).double().cpu().numpy()
    ex = rel_l2(x0 - z, x0_ref - z)
    loss, g = net.gradient(zt, tt)
    el = abs(loss - loss_ref) / loss_ref
    log(f"network: x0 residual rel-L2 {ex:.2e}, loss rel {el:.2e}")
    assert ex <= 1e-4 and el <= 1e-4
    k = 0
    for l, (ci, co) in enumerate(ocnn.LAYERS):
        n = 9 * co * ci + co
        e = rel_l2(g[k:k + n].astype(np.float64), g_ref[k:k + n])
        log(f"  layer {l} ({ci}->{co}) gradient rel-L2 {e:.2e}")
        assert e <= 5e-3, (l, e)
        k += n
    net.close()


def test_adam_steps_match_oracle():
    theta = ncs_inputs.cnn_init(31, scale_last=1.0)
    B, H, W = 1, 32, 32
    rng = np.random.default_rng(32)
    z = rng.uniform(0.0, 1.0, (B, H, W)).astype(np.float32)
    t = (z + 0.1 * rng.standard_normal((B, H, W))).astype(np.float32)
    net = cnn.WarmStartNet(B, H, W)
    net.set_params(theta)
    zt, tt = torch.tensor(z, device=DEV), torch.tensor(t, device=DEV)
    lr = 1e-3
    th, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for step in (1, 2):
        _, g_ref = ocnn.loss_and_grad(th, z.astype(np.float64), t.astype(np.float64), quant=True)[0::2]
        th, m, v = ocnn.adam(th, g_ref, m, v, step, lr)
        net.gradient(zt, tt)
        net.adam_step(lr)
        d = np.abs(net.params().astype(np.float64) - th)
        log(f"Adam step {step}: max |gpu - oracle| = {d.max():.2e} (lr {lr})")
        # a few parameters with a gradient near zero may step differently
        assert np.mean(d <= 1e-2 * lr) >= 0.999
        assert d.max() <= 2 * lr * step
    net.close()


def test_training_reduces_the_loss():
    B, H, W = 4, 32, 32
    z = np.stack([ncs_inputs.phantom(32, s) for s in range(B)]).astype(np.float32)
    t = np.stack([np.clip(ncs_inputs.phantom(32, s), 0, 0.8) for s in range(B)]).astype(np.float32)
    net = cnn.WarmStartNet(B, H, W)
    net.set_params(ncs_inputs.cnn_init(41))
    zt, tt = torch.tensor(z, device=DEV), torch.tensor(t, device=DEV)
    first = net.train_step(zt, tt, 1e-3, want_loss=True)
    for _ in range(300):
        net.train_step(zt, tt, 1e-3)
    last = net.last_loss()
    log(f"training: loss {first:.3e} -> {last:.3e}")
    assert last < 0.2 * first
    net.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_prefilter_matches_oracle(prec):
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    h = problems.multiplier(prob, par)
    ref = ocnn.prefilter(prob.E, h, par.alpha, prob.b).ravel()
    dt = torch.float64 if prec == "f64" else torch.float32
    p = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, c_r=par.c_r or 0.0, mu_dc=par.mu_dc or 0.0)
    s = ncs.Solver(ncs.Geometry(64, 90, 92), p, dtype=dt)
    out = s.prefilter(torch.tensor(prob.b, dtype=dt, device=DEV)).double().cpu().numpy()
    e = rel_l2(out, ref)
    log(f"prefilter {prec}: rel-L2 {e:.2e}")
    assert e <= (1e-11 if prec == "f64" else 1e-5)
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("key", ["c1", "tiny"])
def test_fbp_matches_oracle(prec, key):
    from gpu_common import GEOMS, joseph
    n, na, ns = GEOMS[key]
    E = joseph(n, na, ns)
    y = np.random.default_rng(12).standard_normal(na * ns) + E @ ncs_inputs.phantom(n, 3).ravel()
    ref = ocnn.fbp(E, na, ns, y)
    dt = torch.float64 if prec == "f64" else torch.float32
    s = ncs.Solver(ncs.Geometry(n, na, ns), ncs.Params(0.01, 0.03, 1.0, 0.01), dtype=dt)
    out = s.fbp(torch.tensor(y, dtype=dt, device=DEV)).double().cpu().numpy()
    e = rel_l2(out, ref)
    log(f"fbp {key} {prec}: rel-L2 {e:.2e}")
    assert e <= (1e-11 if prec == "f64" else 2e-5)
    s.close()
