"""Warm-start network of the learned initialisation, in FP64 (TEST
INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's
CPU baseline, never by the product path).

The network is not in the paper. It maps the circulant-filtered
backprojection z of a sinogram to an initial image, x0 = z + N(z). N is six
3x3 "same" convolutions with zero padding: 1 -> 32, four times 32 -> 32 and
32 -> 1, with ReLU after the first five.

Activations are NHWC arrays [B, H, W, C]. The weights of one layer are
[9, C_out, C_in]. Tap t = 3 (dy + 1) + (dx + 1) reads the input pixel
(row + dy, col + dx), so that

    y[b, r, c, o] = bias[o] + sum_t sum_i x[b, r + dy_t, c + dx_t, i] w[t, o, i].

The flat parameter vector stores, for each layer in order, w (row-major) and
then the bias.

With ``quant=True`` the storage points of the device implementation are
emulated: weights, the input, every stored activation and every stored
activation gradient are rounded to bfloat16 (round to nearest, ties to even,
after rounding to float32), while sums stay exact. With ``quant=False`` the
whole network is exact FP64; the finite-difference pins use that form.

Parity unpinned: the architecture, its initialisation and the training recipe
are not in the paper. They are fixed by the project. The arithmetic is pinned
(by a library convolution, adjoint identities, finite differences and a
closed-form Adam step), the choice of network is not.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]
TAPS = [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def n_params() -> int:
    return sum(9 * co * ci + co for ci, co in LAYERS)


def unpack(theta: np.ndarray) -> list[tuple[np.ndarray, np.ndarray]]:
    """Split the flat vector into [(w [9, C_out, C_in], bias [C_out]), ...]."""
    out, k = [], 0
    for ci, co in LAYERS:
        w = np.asarray(theta[k:k + 9 * co * ci], dtype=np.float64).reshape(9, co, ci)
        k += 9 * co * ci
        b = np.asarray(theta[k:k + co], dtype=np.float64)
        k += co
        out.append((w, b))
    assert k == theta.size
    return out


def pack(layers: list[tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), via float32; returned in float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def _pad(x: np.ndarray) -> np.ndarray:
    B, H, W, C = x.shape
    p = np.zeros((B, H + 2, W + 2, C))
    p[:, 1:H + 1, 1:W + 1, :] = x
    return p


def conv3x3(x: np.ndarray, w: np.ndarray, bias: np.ndarray | None = None) -> np.ndarray:
    """y = bias + sum over the nine taps of the shifted input times w[t]^T."""
    B, H, W, C = x.shape
    xp = _pad(x)
    y = np.zeros((B, H, W, w.shape[1]))
    for t, (dy, dx) in enumerate(TAPS):
        y += xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] @ w[t].T
    if bias is not None:
        y += bias
    return y


def conv3x3_input_grad(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 in its input: dx[q, i] = sum_t sum_o g[q - o_t, o] w[t, o, i]."""
    B, H, W, _ = g.shape
    gp = _pad(g)
    dx = np.zeros((B, H, W, w.shape[2]))
    for t, (dy, dxx) in enumerate(TAPS):
        dx += gp[:, 1 - dy:1 - dy + H, 1 - dxx:1 - dxx + W, :] @ w[t]
    return dx


def conv3x3_weight_grad(x: np.ndarray, g: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Adjoint of conv3x3 in its weights and bias:
    dw[t, o, i] = sum_p g[p, o] x[p + o_t, i],  dbias[o] = sum_p g[p, o]."""
    B, H, W, C = x.shape
    xp = _pad(x)
    gf = g.reshape(-1, g.shape[-1])
    dw = np.zeros((9, g.shape[-1], C))
    for t, (dy, dx) in enumerate(TAPS):
        dw[t] = gf.T @ xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :].reshape(-1, C)
    return dw, gf.sum(axis=0)


def forward(theta: np.ndarray, z: np.ndarray, quant: bool = False):
    """x0 = z + N(z) for z of shape [B, H, W]; also returns the stored activations
    (acts[0] is the input, acts[l + 1] the ReLU output of layer l < 5)."""
    q = bf16_round if quant else (lambda a: a)
    layers = unpack(theta)
    acts = [q(np.asarray(z, dtype=np.float64)[..., None])]
    for l in range(5):
        w, b = layers[l]
        acts.append(q(np.maximum(conv3x3(acts[-1], q(w), b), 0.0)))
    w, b = layers[5]
    out = conv3x3(acts[-1], q(w), b)[..., 0]
    return np.asarray(z, dtype=np.float64) + out, acts


def loss_and_grad(theta: np.ndarray, z: np.ndarray, target: np.ndarray, quant: bool = False):
    """Mean squared error L = mean((x0 - target)^2) over every pixel of the
    batch, and dL/dtheta by the chain rule through the layers in reverse."""
    q = bf16_round if quant else (lambda a: a)
    layers = unpack(theta)
    x0, acts = forward(theta, z, quant)
    r = x0 - target
    loss = float(np.mean(r * r))
    g = q((2.0 / r.size) * r)[..., None]         # dL/d(output of layer 5)
    grads = [None] * 6
    for l in range(5, -1, -1):
        w, _ = layers[l]
        dw, db = conv3x3_weight_grad(acts[l], g)
        grads[l] = (dw, db)
        if l > 0:
            g = q(conv3x3_input_grad(g, q(w)) * (acts[l] > 0))
    return loss, x0, pack(grads)


def adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) with bias correction at
    step number `step` >= 1.  Returns the new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def prefilter(E, h: np.ndarray, alpha: float, y: np.ndarray) -> np.ndarray:
    """z = alpha M^+ E^T y, the circulant-filtered backprojection that feeds the
    network (M^+ = F^-1 diag(h) F, h = 1/mu of Section 4.1)."""
    from .operators import apply_circulant
    n = h.shape[0]
    return alpha * apply_circulant(h, (E.T @ y).reshape(n, n))


def shepp_logan(n_bins: int) -> np.ndarray:
    """Shepp-Logan filter taps h(n) = -2 / (pi^2 (4 n^2 - 1)) for unit spacing,
    n = -(n_bins - 1) .. n_bins - 1 (Shepp and Logan, 1974)."""
    n = np.arange(-(n_bins - 1), n_bins, dtype=np.float64)
    return -2.0 / (np.pi ** 2 * (4.0 * n * n - 1.0))


def fbp(E, n_angles: int, n_bins: int, y: np.ndarray) -> np.ndarray:
    """Filtered backprojection (pi / N_theta) E^T q with q[a] the linear
    convolution of projection a with the Shepp-Logan filter, kept on the
    detector's n_bins samples (zero outside the detector)."""
    h = shepp_logan(n_bins)
    ys = np.asarray(y, dtype=np.float64).reshape(n_angles, n_bins)
    q = np.stack([np.convolve(row, h, mode="full")[n_bins - 1:2 * n_bins - 1] for row in ys])
    return (np.pi / n_angles) * (E.T @ q.ravel())
