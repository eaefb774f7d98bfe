"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module draws random numbers and rasterises ellipses; it holds none of the
reconstruction method's arithmetic (no projector, no difference operator, no
Fourier multiplier, no proximal map).  The paper measures on patient CT data and
on PET data that are not available here, so seeded random-ellipse phantoms with
the paper's image sizes and sinogram shapes stand in for them.

Recipe (same for every consumer):

* phantom on [-1, 1]^2 sampled at pixel centres (2c+1)/N - 1 (columns) and
  (2r+1)/N - 1 (rows); K ~ U{5..10} ellipses; semi-axes a, b ~ U[0.05, 0.45];
  centre at radius rho ~ U[0, 1 - max(a, b)] and angle psi ~ U[0, 2 pi);
  rotation phi ~ U[0, pi); intensity ~ U[0, 1]; overlaps add.
* volume phantom on [-1, 1]^3 sampled at voxel centres (2c+1)/N - 1,
  (2r+1)/N - 1, (2z+1)/N_z - 1; K ~ U{5..10} ellipsoids; in-plane semi-axes
  a, b ~ U[0.05, 0.45], axial semi-axis c ~ U[0.1, 0.6]; centre at radius
  rho ~ U[0, 1 - max(a, b)], angle psi ~ U[0, 2 pi), height z0 ~ U[-0.5, 0.5];
  rotation phi ~ U[0, pi) about the z axis; intensity ~ U[0, 1]; overlaps
  add; RNG ``default_rng([seed, 5])``.
* phantom RNG ``numpy.random.default_rng(seed)``; Gaussian noise RNG
  ``default_rng([seed, 1])``; Poisson count RNG ``default_rng([seed, 2])``.
* the uneven 512-slice batch: 205 slices of 128^2, 205 of 256^2, 102 of 512^2,
  shuffled with ``default_rng(4242)``; angles = round(1.4 * side), bins =
  side + side // 64.
* warm-start network: initial parameters from ``default_rng([seed, 3])``,
  He-normal weights (std sqrt(2 / (9 C_in))) rounded to float32, zero biases,
  the last layer scaled by ``scale_last`` (0: the network starts as the
  identity map of its input); training slices use seeds 1,000,000 + i,
  validation 2,000,000 + i, evaluation 0..31.
* bfloat16-exact test tensors: k 2^-e with integer |k| <= 255, so every value
  is exactly representable in bfloat16 and float32.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "ellipse_params",
    "phantom",
    "ellipsoid_params",
    "phantom3d",
    "gaussian_noise",
    "poisson_counts",
    "batch_sides",
    "batch_geometry",
    "cnn_init",
    "bf16_exact",
    "CNN_LAYERS",
]

# (C_in, C_out) of the six 3x3 layers of the warm-start network
CNN_LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]


def ellipse_params(seed: int) -> np.ndarray:
    """Return a (K, 6) array of ellipses: a, b, x0, y0, phi, intensity."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(5, 11))
    a = rng.uniform(0.05, 0.45, k)
    b = rng.uniform(0.05, 0.45, k)
    rho = rng.uniform(0.0, 1.0, k) * (1.0 - np.maximum(a, b))
    psi = rng.uniform(0.0, 2.0 * np.pi, k)
    phi = rng.uniform(0.0, np.pi, k)
    inten = rng.uniform(0.0, 1.0, k)
    x0 = rho * np.cos(psi)
    y0 = rho * np.sin(psi)
    return np.stack([a, b, x0, y0, phi, inten], axis=1)


def phantom(n_side: int, seed: int) -> np.ndarray:
    """Random-ellipse phantom, float64 array of shape (n_side, n_side), row-major.

    Row index r runs along y, column index c along x.
    """
    t = (2.0 * np.arange(n_side) + 1.0) / n_side - 1.0
    yy, xx = np.meshgrid(t, t, indexing="ij")
    img = np.zeros((n_side, n_side))
    for a, b, x0, y0, phi, inten in ellipse_params(seed):
        dx = xx - x0
        dy = yy - y0
        cp, sp = np.cos(phi), np.sin(phi)
        u = (dx * cp + dy * sp) / a
        v = (-dx * sp + dy * cp) / b
        img += inten * (u * u + v * v <= 1.0)
    return img


def ellipsoid_params(seed: int) -> np.ndarray:
    """Return a (K, 8) array of ellipsoids: a, b, c, x0, y0, z0, phi, intensity."""
    rng = np.random.default_rng([seed, 5])
    k = int(rng.integers(5, 11))
    a = rng.uniform(0.05, 0.45, k)
    b = rng.uniform(0.05, 0.45, k)
    c = rng.uniform(0.1, 0.6, k)
    rho = rng.uniform(0.0, 1.0, k) * (1.0 - np.maximum(a, b))
    psi = rng.uniform(0.0, 2.0 * np.pi, k)
    z0 = rng.uniform(-0.5, 0.5, k)
    phi = rng.uniform(0.0, np.pi, k)
    inten = rng.uniform(0.0, 1.0, k)
    return np.stack([a, b, c, rho * np.cos(psi), rho * np.sin(psi), z0, phi, inten], axis=1)


def phantom3d(n_side: int, n_slices: int, seed: int) -> np.ndarray:
    """Random-ellipsoid volume phantom, float64 array of shape
    (n_slices, n_side, n_side): index [z, r, c], r along y, c along x."""
    t = (2.0 * np.arange(n_side) + 1.0) / n_side - 1.0
    tz = (2.0 * np.arange(n_slices) + 1.0) / n_slices - 1.0
    zz, yy, xx = np.meshgrid(tz, t, t, indexing="ij")
    vol = np.zeros((n_slices, n_side, n_side))
    for a, b, c, x0, y0, z0, phi, inten in ellipsoid_params(seed):
        dx, dy, dz = xx - x0, yy - y0, zz - z0
        cp, sp = np.cos(phi), np.sin(phi)
        u = (dx * cp + dy * sp) / a
        v = (-dx * sp + dy * cp) / b
        w = dz / c
        vol += inten * (u * u + v * v + w * w <= 1.0)
    return vol


def gaussian_noise(seed: int, m: int) -> np.ndarray:
    """Standard normal draws for the CT noise of slice ``seed``."""
    return np.random.default_rng([seed, 1]).standard_normal(m)


def poisson_counts(seed: int, mean: np.ndarray) -> np.ndarray:
    """Poisson draws with the given mean vector (PET counts), as float64."""
    return np.random.default_rng([seed, 2]).poisson(mean).astype(np.float64)


def batch_sides(n_small: int = 205, n_mid: int = 205, n_large: int = 102) -> np.ndarray:
    """Image sides of the uneven batch, in their shuffled order."""
    sides = np.array([128] * n_small + [256] * n_mid + [512] * n_large, dtype=np.int64)
    np.random.default_rng(4242).shuffle(sides)
    return sides


def batch_geometry(side: int) -> tuple[int, int, int]:
    """(n_side, n_angles, n_bins) of one slice of the uneven batch."""
    return int(side), int(round(1.4 * side)), int(side + side // 64)


def cnn_init(seed: int, scale_last: float = 0.0) -> np.ndarray:
    """Initial flat parameter vector of the warm-start network (float64 holding
    float32 values): per layer the weights [9, C_out, C_in], then the biases."""
    rng = np.random.default_rng([seed, 3])
    parts = []
    for l, (ci, co) in enumerate(CNN_LAYERS):
        w = rng.standard_normal(9 * co * ci) * np.sqrt(2.0 / (9 * ci))
        if l == len(CNN_LAYERS) - 1:
            w = w * scale_last
        parts += [w, np.zeros(co)]
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def bf16_exact(seed: int, shape, exponent: int = 8, positive: bool = False) -> np.ndarray:
    """Random values k * 2^-exponent with integer |k| <= 255 (k >= 0 if positive)."""
    rng = np.random.default_rng([seed, 4])
    k = rng.integers(0 if positive else -255, 256, size=shape)
    return k.astype(np.float64) * 2.0 ** -exponent
