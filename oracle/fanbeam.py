"""Fan-beam projector and the probe-estimated multiplier of eq. (H-fan) (oracle, FP64).

Section 4.1.1 (fan beam and cone beam geometry) takes E to be a discretisation
of the divergent-beam transform and replaces the analytic multiplier of
eq. (circ_R) by an estimate of the circulant closest to E^T E: for a
circulant C = F^-1 diag(h) F one has h_i = (F C v)_i / (F v)_i for every v,
and the paper averages (F E^T E v)_i / (F v)_i over many v.

The paper fixes neither the fan geometry nor the discretisation; this module
and the HIP library both use the following reading.

* Image: as in ``projector`` (unit pixels, centres (c - (N-1)/2, r - (N-1)/2)).
* Views a of N_v over a full turn: the source sits at
  S_a = R_s (cos beta_a, sin beta_a), beta_a = 2 pi a / N_v, and the central
  ray points at the origin, theta_c = beta_a + pi.
* Bins d of N_s on an equi-angular detector: ray (a, d) leaves S_a in the
  direction theta = theta_c + gamma_d, gamma_d = (d - (N_s-1)/2) dgamma, with
  dgamma = 2 asin(R_fov / R_s) / (N_s - 1) so that the fan just covers the
  circle of radius R_fov = N / sqrt(2) around the image.  Storage index
  a*N_s + d.
* Joseph's method per ray: with u = (cos theta, sin theta), the ray steps
  through image rows when |u_y| >= |u_x| - 1e-12 and through columns
  otherwise.  Stepping through row r it crosses y = y_r at column coordinate
  xi = S_x + (y_r - S_y) u_x / u_y + (N-1)/2; with c0 = floor(xi),
  f = xi - c0 it puts weight (1-f)/|u_y| on pixel (r, c0) and f/|u_y| on
  (r, c0+1), dropping pixels outside the image.  Columns swap x and y.

The estimate of eq. (H-fan) is taken as the least-squares average over the
probes, h_i = sum_v conj(F v)_i (F E^T E v)_i / sum_v |(F v)_i|^2 (real part):
the average of the ratios weighted by |(F v)_i|^2, which equals the paper's
ratio for one probe and does not blow up where a probe's spectrum is small.
The probes are Rademacher images (+-1) drawn bit by bit from SplitMix64
(Steele, Lea and Flood, 2014), seeded by the probe index, which the HIP
library implements from the same published definition.

Parity: ``fan_matrix`` is pinned by the analytic line integrals of a Gaussian
blob, the chord lengths of the unit image and its exact equivariance under a
quarter turn; ``probe_multiplier`` by exact recovery of a circulant operator,
and ``splitmix64`` by the published first outputs of the generator.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

MASK64 = (1 << 64) - 1
TIE = 1e-12


@dataclass(frozen=True)
class FanGeometry:
    n_side: int
    n_views: int
    n_bins: int
    source_radius: float

    @property
    def r_fov(self) -> float:
        return self.n_side / np.sqrt(2.0)

    @property
    def dgamma(self) -> float:
        return 2.0 * np.arcsin(self.r_fov / self.source_radius) / (self.n_bins - 1)


def rays(g: FanGeometry):
    """Per ray (a*N_s + d): source (sx, sy), direction (ux, uy), rows-stepping flag."""
    a = np.arange(g.n_views)
    beta = 2.0 * np.pi * a / g.n_views
    sx, sy = g.source_radius * np.cos(beta), g.source_radius * np.sin(beta)
    gam = (np.arange(g.n_bins) - (g.n_bins - 1) / 2.0) * g.dgamma
    theta = (beta + np.pi)[:, None] + gam[None, :]
    ux, uy = np.cos(theta).ravel(), np.sin(theta).ravel()
    sx = np.repeat(sx, g.n_bins)
    sy = np.repeat(sy, g.n_bins)
    rows = np.abs(uy) >= np.abs(ux) - TIE
    return sx, sy, ux, uy, rows


def fan_matrix(g: FanGeometry) -> sp.csr_matrix:
    """The (N_v N_s) x N^2 Joseph fan-beam matrix E, CSR, float64."""
    n = g.n_side
    half = (n - 1) / 2.0
    sx, sy, ux, uy, rows = rays(g)
    m = sx.size
    coord = np.arange(n) - half
    step = np.arange(n)
    ri, ci, vi = [], [], []
    for stepping_rows in (True, False):
        sel = np.nonzero(rows == stepping_rows)[0]
        if sel.size == 0:
            continue
        if stepping_rows:
            # column coordinate of each selected ray on each row
            xi = sx[sel, None] + (coord[None, :] - sy[sel, None]) * (ux[sel] / uy[sel])[:, None] + half
            w = 1.0 / np.abs(uy[sel])
        else:
            # row coordinate of each selected ray on each column
            xi = sy[sel, None] + (coord[None, :] - sx[sel, None]) * (uy[sel] / ux[sel])[:, None] + half
            w = 1.0 / np.abs(ux[sel])
        c0 = np.floor(xi)
        f = xi - c0
        c0 = c0.astype(np.int64)
        ray = np.broadcast_to(sel[:, None], xi.shape)
        stp = np.broadcast_to(step[None, :], xi.shape)
        for off, wt in ((0, 1.0 - f), (1, f)):
            tap = c0 + off
            ok = (tap >= 0) & (tap < n) & (wt != 0.0)
            pix = np.where(stepping_rows, stp * n + tap, tap * n + stp)
            ri.append(ray[ok])
            ci.append(pix[ok])
            vi.append((wt * w[:, None])[ok])
    return sp.csr_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))), shape=(m, n * n))


def splitmix64(seed: int, count: int) -> np.ndarray:
    """The first `count` outputs of SplitMix64 started from state `seed` (uint64)."""
    out = np.empty(count, dtype=np.uint64)
    x = seed & MASK64
    for i in range(count):
        x = (x + 0x9E3779B97F4A7C15) & MASK64
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out[i] = z ^ (z >> 31)
    return out


def rademacher_probe(index: int, n: int) -> np.ndarray:
    """Probe `index`: n values +-1, bit j of SplitMix64 output k (seeded by the
    index) giving entry 64 k + j (bit set: +1)."""
    words = splitmix64(index, (n + 63) // 64)
    bits = ((words[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)).ravel()[:n]
    return np.where(bits == 1, 1.0, -1.0)


def probe_multiplier(apply_ata, n_side: int, n_probes: int) -> np.ndarray:
    """Real part of sum_v conj(F v) F(A v) / sum_v |F v|^2 over the probes
    v = rademacher_probe(0..n_probes-1) (an N x N array)."""
    num = np.zeros((n_side, n_side), dtype=np.complex128)
    den = np.zeros((n_side, n_side))
    for k in range(n_probes):
        v = rademacher_probe(k, n_side * n_side)
        fv = np.fft.fft2(v.reshape(n_side, n_side))
        fz = np.fft.fft2(np.asarray(apply_ata(v), dtype=np.float64).reshape(n_side, n_side))
        num += np.conj(fv) * fz
        den += np.abs(fv) ** 2
    return np.real(num / den)
