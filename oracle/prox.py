"""Proximal maps used by the iterations (oracle, FP64).

Conventions follow Section 2: prox_{a g}(z) = argmin_x a g(x) + 1/2 |x - z|^2,
and the Moreau identity (eq. Moreau) prox_{a g*}(x) = x - a prox_{g/a}(x/a).

Maps on the dual side (what the iterations call):

* ``conj_quadratic``: g = 1/2 |.|^2, prox_{a g*}(w) = w / (1 + a)  (Section 4.1).
* ``box``: g = s' |.|_1 with its conjugate the indicator of [-s', s'];
  prox_{a g*} = projection onto [-s, s] componentwise, s = s' (Section 4.1,
  the map Pi_{[-s,s]}); with the scaled TV block s = lambda alpha / beta.
* ``l2_ball``: isotropic TV, g = s' sum_p |z_p|_2 over pixel pairs
  z_p = (horizontal, vertical); its conjugate is the indicator of the product
  of l2 balls of radius s'; prox = per-pixel projection (not in the paper,
  which uses anisotropic TV; required by the PET workload).
* ``poisson_s``: S(u; c) = 1 + (u - 1 - sqrt((u-1)^2 + 4c))/2 of Section 4.2,
  which is prox_{a l*}(u) for l(y) = y - b log y with c = a b.
* ``nonpositive``: g = indicator of the nonnegative orthant (the positivity
  block of the remark in Section 4.2); its conjugate is the indicator of the
  nonpositive orthant, so prox_{a g*} = min(., 0) for every a > 0.

Maps on the primal side (used only by the classic-ADMM cross-check of the
appendix): ``prox_quadratic``, ``soft_threshold``, ``prox_poisson``.

Parity: pinned against brute-force one-dimensional minimisation, the Moreau
identity with the primal maps, and closed special cases (S(u; 0) = min(u, 1)).
"""
from __future__ import annotations

import numpy as np


def conj_quadratic(w: np.ndarray, a: float) -> np.ndarray:
    return w / (1.0 + a)


def box(w: np.ndarray, s: float) -> np.ndarray:
    return np.clip(w, -s, s)


def l2_ball(wh: np.ndarray, wv: np.ndarray, s: float) -> tuple[np.ndarray, np.ndarray]:
    """Project each pixel pair (wh, wv) onto the disk of radius s."""
    norm = np.sqrt(wh * wh + wv * wv)
    scale = 1.0 / np.maximum(1.0, norm / s)
    return wh * scale, wv * scale


def poisson_s(u: np.ndarray, c: np.ndarray) -> np.ndarray:
    """S(u; c) exactly as printed in Section 4.2."""
    return 1.0 + (u - 1.0 - np.sqrt((u - 1.0) ** 2 + 4.0 * c)) / 2.0


def nonpositive(w: np.ndarray) -> np.ndarray:
    return np.minimum(w, 0.0)


def prox_quadratic(z: np.ndarray, t: float) -> np.ndarray:
    """prox_{t g} for g = 1/2 |.|^2."""
    return z / (1.0 + t)


def soft_threshold(z: np.ndarray, t: float) -> np.ndarray:
    """prox_{t |.|_1}."""
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def prox_poisson(z: np.ndarray, b: np.ndarray, t: float) -> np.ndarray:
    """prox_{t l} for l(y) = y - b log y (y > 0): positive root of y^2 - (z-t) y - t b = 0."""
    zt = z - t
    return (zt + np.sqrt(zt * zt + 4.0 * t * b)) / 2.0


def moreau_conj(prox_g_scaled, x: np.ndarray, a: float) -> np.ndarray:
    """prox_{a g*}(x) = x - a prox_{g/a}(x/a), with prox_g_scaled(z, t) = prox_{t g}(z)."""
    return x - a * prox_g_scaled(x / a, 1.0 / a)
