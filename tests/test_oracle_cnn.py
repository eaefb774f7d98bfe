"""Pins of the oracle's warm-start network, loss gradient, Adam and pre-filter.

Each is checked against something other than itself: a library convolution
(SciPy), the adjoint identities of a linear map, central finite differences of
the loss, the closed form of Adam's first step, bfloat16 rounding by PyTorch,
and an identity that links the pre-filter to the NCS iteration.
"""
import numpy as np
import pytest
import scipy.signal
import torch

import ncs_inputs
from oracle import cnn, problems, solvers
from oracle.problems import Params


def rand(rng, *shape):
    return rng.standard_normal(shape)


def test_layer_table_and_parameter_count():
    assert cnn.n_params() == 9 * 32 + 32 + 4 * (9 * 32 * 32 + 32) + 9 * 32 + 1 == 37601
    theta = np.arange(cnn.n_params(), dtype=np.float64)
    assert np.array_equal(cnn.pack(cnn.unpack(theta)), theta)


def test_conv_matches_scipy_correlation():
    rng = np.random.default_rng(1)
    B, H, W, Ci, Co = 2, 7, 9, 3, 4
    x, w, b = rand(rng, B, H, W, Ci), rand(rng, 9, Co, Ci), rand(rng, Co)
    y = cnn.conv3x3(x, w, b)
    for bi in range(B):
        for o in range(Co):
            ref = np.full((H, W), b[o])
            for i in range(Ci):
                k = w[:, o, i].reshape(3, 3)        # k[dy + 1, dx + 1]
                ref += scipy.signal.correlate2d(x[bi, :, :, i], k, mode="same", boundary="fill")
            np.testing.assert_allclose(y[bi, :, :, o], ref, rtol=1e-12, atol=1e-12)


def test_conv_grads_are_adjoints():
    rng = np.random.default_rng(2)
    B, H, W, Ci, Co = 2, 6, 5, 3, 4
    x, w, g = rand(rng, B, H, W, Ci), rand(rng, 9, Co, Ci), rand(rng, B, H, W, Co)
    lhs = np.sum(cnn.conv3x3(x, w) * g)
    assert np.isclose(lhs, np.sum(x * cnn.conv3x3_input_grad(g, w)), rtol=1e-12)
    dw, db = cnn.conv3x3_weight_grad(x, g)
    assert np.isclose(lhs, np.sum(w * dw), rtol=1e-12)
    # bias gradient: <conv(x, 0, b), g> = <b, db>
    bb = rand(rng, Co)
    assert np.isclose(np.sum(cnn.conv3x3(np.zeros_like(x), w, bb) * g), bb @ db, rtol=1e-12)


def test_loss_gradient_by_finite_differences():
    rng = np.random.default_rng(3)
    theta = ncs_inputs.cnn_init(7, scale_last=1.0)
    z = rand(rng, 1, 6, 5)
    t = rand(rng, 1, 6, 5)
    loss, _, grad = cnn.loss_and_grad(theta, z, t)
    idx = rng.choice(theta.size, 60, replace=False)
    # always include biases and the first and last layers
    idx = np.unique(np.concatenate([idx, [0, 300, 320, 9567, 37600, 37311]]))
    eps = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (cnn.loss_and_grad(tp, z, t)[0] - cnn.loss_and_grad(tm, z, t)[0]) / (2 * eps)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(grad[k])) + 1e-9, (k, fd, grad[k])


def test_zero_last_layer_is_identity():
    theta = ncs_inputs.cnn_init(3)          # last layer starts at zero
    z = np.random.default_rng(4).standard_normal((2, 8, 8))
    x0, _ = cnn.forward(theta, z)
    assert np.array_equal(x0, z)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        # exact ties: 1 + (2k+1) 2^-8 sits halfway between two bfloat16 values
                        1.0 + (2 * np.arange(64) + 1) * 2.0 ** -8, -(1.0 + (2 * np.arange(64) + 1) * 2.0 ** -8),
                        [0.0, -0.0, 1e-40, 3.4e38]])
    ref = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(a), ref)


def test_quantised_forward_is_close_to_exact():
    theta = ncs_inputs.cnn_init(9, scale_last=1.0)
    z = np.random.default_rng(6).uniform(0, 1, (1, 16, 16))
    exact, _ = cnn.forward(theta, z)
    quant, acts = cnn.forward(theta, z, quant=True)
    for a in acts:
        assert np.array_equal(cnn.bf16_round(a), a)      # stored values are bfloat16
    rel = np.linalg.norm(quant - exact) / np.linalg.norm(exact - z)
    assert rel < 0.05, rel


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so the step is lr g / (|g| + eps)
    rng = np.random.default_rng(8)
    theta, g = rng.standard_normal(100), rng.standard_normal(100)
    new, m, v = cnn.adam(theta, g, np.zeros(100), np.zeros(100), 1, lr=0.01)
    np.testing.assert_allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(9)
    c = rng.standard_normal(20)
    th, m, v = np.zeros(20), np.zeros(20), np.zeros(20)
    for k in range(1, 3001):
        th, m, v = cnn.adam(th, 2 * (th - c), m, v, k, lr=0.01)
    assert np.max(np.abs(th - c)) < 1e-3


def test_prefilter_is_scaled_second_ncs_iterate():
    # From x = u = v = 0 the first CT iteration gives x1 = 0, u1 = -alpha b/(1+alpha),
    # v1 = 0, so the second gives x2 = alpha/(1+alpha) M^+ E^T b: the pre-filtered
    # backprojection is (1 + alpha) x2.
    prob = problems.ct_problem(16, 12, 23, 0, 0.01)
    par = Params(0.05, 0.15, 0.3 * 0.05 * 12 * 16 / np.pi)
    h = problems.multiplier(prob, par)
    z = cnn.prefilter(prob.E, h, par.alpha, prob.b)
    x2 = solvers.ncs(prob, par, 2, record=False).x
    np.testing.assert_allclose(z.ravel(), (1 + par.alpha) * x2, rtol=1e-12, atol=1e-14)


def test_shepp_logan_frequency_response():
    # sum_n h(n) e^{-i w n} = |sin(w / 2)| / pi: the ramp |w| / (2 pi) times sinc(w / (2 pi))
    h = cnn.shepp_logan(100001)
    n = np.arange(-100000, 100001)
    for w in (0.05, 0.3, 1.0, 2.0, 2.9, np.pi):
        assert abs(np.sum(h * np.cos(w * n)) - abs(np.sin(w / 2)) / np.pi) < 1e-9


def test_fbp_reconstructs_a_smooth_image():
    # FBP inverts the projector on a smooth image up to discretisation error
    from oracle import projector
    N, NA, NS = 64, 180, 92
    E = projector.joseph_matrix(N, NA, NS)
    c = np.arange(N) - (N - 1) / 2
    yy, xx = np.meshgrid(c, c, indexing="ij")
    img = np.exp(-((xx - 5) ** 2 + (yy + 3) ** 2) / (2 * 8.0 ** 2)) + 0.5 * np.exp(-((xx + 10) ** 2 + yy ** 2) / (2 * 4.0 ** 2))
    rec = cnn.fbp(E, NA, NS, E @ img.ravel())
    err = np.linalg.norm(rec - img.ravel()) / np.linalg.norm(img)
    assert err < 0.05, err
