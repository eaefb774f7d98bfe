"""Cone-beam CT on volumes: projector, 3D finite differences, the 3D
multiplier and the NCS iteration (oracle, FP64).

Section 4.1.1 (fan beam and cone beam geometry) takes E to be a
discretisation of the cone-beam transform for a source orbit in 3D and, as
for the fan beam, replaces the analytic multiplier of E^T E by the estimate
of eq. (H-fan), now with the 3D DFT.  The paper fixes neither the orbit nor
the detector nor the discretisation; this module and the HIP library both use
the following reading.

* Volume: N x N x N_z unit voxels with centres (c - (N-1)/2, r - (N-1)/2,
  z - (N_z-1)/2), stored (z N + r) N + c.
* Orbit: the source circles in the plane z = 0 at radius R_s; view a of N_v
  puts it at S_a = R_s (cos beta_a, sin beta_a, 0), beta_a = 2 pi a / N_v.
* Detector: cylindrical and centred on the source.  Its columns are the bins
  of the fan beam (``fanbeam``: equi-angular, fan step dgamma, central ray
  towards the axis); its rows are equally spaced in slope, z_rho =
  (rho - (N_r-1)/2) dz with dz = 2 z_max / (N_r - 1) and
  z_max = (N_z / 2) / (R_s - N / sqrt 2), so that the cone just covers the
  volume's height where the cylinder around the volume is nearest the
  source.  Ray (a, rho, d) is the half line S_a + s (cos theta, sin theta,
  z_rho), s >= 0 the in-plane distance, theta the fan ray's angle; it is
  stored at (a N_r + rho) N_s + d.
* Joseph's method: the ray steps through the planes of the in-plane axis the
  fan ray steps through (rows when |u_y| >= |u_x| - 1e-12).  At each plane
  its point has an in-plane coordinate xi (column or row) and a slice
  coordinate zeta = s z_rho + (N_z-1)/2; the four voxels around (xi, zeta)
  get the bilinear weights, times sqrt(1 + z_rho^2) / |u_y| (or |u_x|), the
  ray's length per plane.  Voxels outside the volume are dropped.
* D stacks the forward differences of Section 2 along x, y and z (each with
  a zero last row), so D^T D is the sum of the three Neumann Laplacians and
  its circulant approximation has the eigenvalues
  4 (sin^2(pi j/N) + sin^2(pi k/N) + sin^2(pi l/N_z)) (eq. circ_D in 3D).
* The multiplier: mu = gamma + alpha h_E + (beta^2/alpha) H_D3 with h_E the
  probe estimate of eq. (H-fan) taken with the 3D DFT (the least-squares
  average over Rademacher probes, as ``fanbeam.probe_multiplier``); the DC
  eigenvalue is gamma + alpha |E 1|^2 / n as for the other geometries.

Parity: ``cone_matrix`` is pinned by the analytic line integrals of a
Gaussian blob (rays of every slope), by the fan-beam matrix on the mid-plane
rows of a volume constant along z, by the chord lengths of the unit volume
and by its exact symmetries (a quarter turn about the axis shifts the views,
a flip along z mirrors the rows); ``diff_3d`` and ``multiplier_diff_3d`` by
the Kronecker form of D^T D and the periodic 7-point stencil;
``probe_multiplier_3d`` by exact recovery of a circulant operator; ``ncs3d``
by PDHG in its stacked form (a constant multiplier) and by the common limit
of NCS and PDHG; its positivity form by the stacked form of eq. (NCS) on
A' = [E; (beta/alpha) D; I] with the conjugate prox of the indicator from the
Moreau identity, and by a constrained limit that is nonnegative and lower
than every nonnegative point of the unconstrained run.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

import ncs_inputs

from . import fanbeam, operators, prox


@dataclass(frozen=True)
class ConeGeometry:
    n_side: int
    n_slices: int
    n_views: int
    n_bins: int
    n_rows: int
    source_radius: float

    @property
    def fan(self) -> fanbeam.FanGeometry:
        return fanbeam.FanGeometry(self.n_side, self.n_views, self.n_bins, self.source_radius)

    @property
    def dzeta(self) -> float:
        z_max = 0.5 * self.n_slices / (self.source_radius - self.n_side / np.sqrt(2.0))
        return 2.0 * z_max / (self.n_rows - 1)

    @property
    def slopes(self) -> np.ndarray:
        return (np.arange(self.n_rows) - (self.n_rows - 1) / 2.0) * self.dzeta

    @property
    def shape(self) -> tuple[int, int, int]:
        return (self.n_slices, self.n_side, self.n_side)

    @property
    def n(self) -> int:
        return self.n_slices * self.n_side * self.n_side

    @property
    def m(self) -> int:
        return self.n_views * self.n_rows * self.n_bins


def cone_matrix(g: ConeGeometry, views=None) -> sp.csr_matrix:
    """The (N_v N_r N_s) x (N_z N^2) Joseph cone-beam matrix E, CSR, float64.
    With ``views`` (a list of view indices) only the rows of those views are
    built, in the given order: the block of E for those views."""
    n, nz = g.n_side, g.n_slices
    half, half_z = (n - 1) / 2.0, (nz - 1) / 2.0
    sx, sy, ux, uy, rows = fanbeam.rays(g.fan)
    coord = np.arange(n) - half
    step = np.arange(n)
    keep = np.ones(rows.size, dtype=bool)
    slot = np.arange(g.n_views)
    if views is not None:
        views = np.asarray(views, dtype=np.int64)
        keep = np.isin(np.arange(rows.size) // g.n_bins, views)
        slot = np.full(g.n_views, -1)
        slot[views] = np.arange(views.size)
    ri, ci, vi = [], [], []
    for stepping_rows in (True, False):
        sel = np.nonzero((rows == stepping_rows) & keep)[0]       # fan rays a N_s + d
        if sel.size == 0:
            continue
        if stepping_rows:
            s = (coord[None, :] - sy[sel, None]) / uy[sel, None]      # in-plane distance at each row
            xi = sx[sel, None] + s * ux[sel, None] + half
            k_xy = 1.0 / np.abs(uy[sel])
        else:
            s = (coord[None, :] - sx[sel, None]) / ux[sel, None]
            xi = sy[sel, None] + s * uy[sel, None] + half
            k_xy = 1.0 / np.abs(ux[sel])
        c0 = np.floor(xi)
        f = xi - c0
        c0 = c0.astype(np.int64)
        a_idx, d_idx = slot[sel // g.n_bins], sel % g.n_bins
        stp = np.broadcast_to(step[None, :], xi.shape)
        for rho, zr in enumerate(g.slopes):
            zeta = s * zr + half_z
            z0 = np.floor(zeta)
            gz = zeta - z0
            z0 = z0.astype(np.int64)
            ray = np.broadcast_to(((a_idx * g.n_rows + rho) * g.n_bins + d_idx)[:, None], xi.shape)
            scale = (k_xy * np.sqrt(1.0 + zr * zr))[:, None]
            for dz_, wz in ((0, 1.0 - gz), (1, gz)):
                zt = z0 + dz_
                for dc_, wc in ((0, 1.0 - f), (1, f)):
                    tap = c0 + dc_
                    wt = wc * wz
                    ok = (tap >= 0) & (tap < n) & (zt >= 0) & (zt < nz) & (wt != 0.0)
                    inplane = np.where(stepping_rows, stp * n + tap, tap * n + stp)
                    ri.append(ray[ok])
                    ci.append((zt * n * n + inplane)[ok])
                    vi.append((wt * scale)[ok])
    n_rays = g.m if views is None else views.size * g.n_rows * g.n_bins
    return sp.csr_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))),
                         shape=(n_rays, g.n))


def diff_3d(n: int, nz: int) -> sp.csr_matrix:
    """3 N_z N^2 x N_z N^2: [D_x; D_y; D_z] with D_n of Section 2 along each axis."""
    dn, dz = operators.diff_1d(n), operators.diff_1d(nz)
    i_n, i_z = sp.identity(n, format="csr"), sp.identity(nz, format="csr")
    dx = sp.kron(i_z, sp.kron(i_n, dn))
    dy = sp.kron(i_z, sp.kron(dn, i_n))
    dzz = sp.kron(dz, sp.kron(i_n, i_n))
    return sp.vstack([dx, dy, dzz]).tocsr()


def multiplier_diff_3d(n: int, nz: int) -> np.ndarray:
    """Eigenvalues of the periodic 3D Laplacian, shape (N_z, N, N) in numpy FFT order."""
    s2 = np.sin(np.arange(n) * np.pi / n) ** 2
    s2z = np.sin(np.arange(nz) * np.pi / nz) ** 2
    return 4.0 * (s2z[:, None, None] + s2[None, :, None] + s2[None, None, :])


def probe_multiplier_3d(apply_ata, shape, n_probes: int) -> np.ndarray:
    """Real part of sum_v conj(F v) F(A v) / sum_v |F v|^2 with the 3D DFT, over
    the probes v = fanbeam.rademacher_probe(0..n_probes-1) laid out in `shape`."""
    n = int(np.prod(shape))
    num = np.zeros(shape, dtype=np.complex128)
    den = np.zeros(shape)
    for k in range(n_probes):
        v = fanbeam.rademacher_probe(k, n)
        fv = np.fft.fftn(v.reshape(shape))
        fz = np.fft.fftn(np.asarray(apply_ata(v), dtype=np.float64).reshape(shape))
        num += np.conj(fv) * fz
        den += np.abs(fv) ** 2
    return np.real(num / den)


@dataclass
class ConeProblem:
    """minimize 1/2 |E x - b|^2 + lambda |D x|_1 on a volume (Section 4.1 in 3D)."""
    geom: ConeGeometry
    lam: float
    E: sp.csr_matrix
    D: sp.csr_matrix
    b: np.ndarray
    x_true: np.ndarray
    Et: sp.csr_matrix = field(init=False)
    Dt: sp.csr_matrix = field(init=False)

    def __post_init__(self):
        self.Et = self.E.T.tocsr()
        self.Dt = self.D.T.tocsr()

    @property
    def n(self) -> int:
        return self.geom.n

    @property
    def m(self) -> int:
        return self.geom.m


def cone_problem(g: ConeGeometry, seed: int, lam: float, noise_frac: float = 0.01, E=None) -> ConeProblem:
    """b = E x_true + sigma eps with x_true = ncs_inputs.phantom3d, sigma = noise_frac max(E x_true)."""
    if E is None:
        E = cone_matrix(g)
    x_true = ncs_inputs.phantom3d(g.n_side, g.n_slices, seed).ravel()
    clean = E @ x_true
    sigma = noise_frac * float(np.max(clean))
    b = clean + sigma * ncs_inputs.gaussian_noise(seed, clean.size)
    return ConeProblem(g, lam, E, diff_3d(g.n_side, g.n_slices), b, x_true)


def objective3d(prob: ConeProblem, x: np.ndarray) -> float:
    r = prob.E @ x - prob.b
    return 0.5 * float(r @ r) + prob.lam * float(np.abs(prob.D @ x).sum())


def eigenvalues3d(prob: ConeProblem, alpha: float, beta: float, gamma: float, h_e: np.ndarray,
                  mu_dc: float | None = None, positivity: bool = False) -> np.ndarray:
    """mu = gamma + alpha h_E + (beta^2/alpha) H_D3, DC entry gamma + alpha |E 1|^2 / n;
    with ``positivity`` (the rows I of x >= 0 in A, remark in Section 4.2) every
    eigenvalue is raised by alpha."""
    g = prob.geom
    mu = gamma + alpha * h_e + (beta * beta / alpha) * multiplier_diff_3d(g.n_side, g.n_slices)
    if mu_dc is None:
        e1 = prob.E @ np.ones(prob.n)
        mu_dc = gamma + alpha * float(e1 @ e1) / prob.n
    mu[0, 0, 0] = mu_dc
    return mu + alpha if positivity else mu


def ncs3d(prob: ConeProblem, alpha: float, beta: float, h: np.ndarray, iters: int, x0=None,
          record: bool = True, positivity: bool = False, with_t: bool = False):
    """The CT form of eq. (NCS) on a volume (Section 4.1):

        x+ = x - (1/alpha) F^-1 diag(h) F (alpha E^T u + beta D^T v)
        u+ = (u + alpha E(2x+ - x) - alpha b) / (1 + alpha)
        v+ = Pi_[-s,s](v + beta D(2x+ - x)),  s = lambda alpha / beta

    with F the 3D DFT and h = 1/mu (a constant h = 1/gamma_P gives eq. PDHG).
    With ``positivity`` the constraint x >= 0 is a third block of A (rows I,
    the remark in Section 4.2) with its own dual t: alpha t joins the
    backprojection and t+ = min(t + alpha (2x+ - x), 0) (h must then invert
    the eigenvalues raised by alpha, ``eigenvalues3d(..., positivity=True)``).
    Returns x, u, v and the objective after each iteration (and t with
    ``with_t``)."""
    shape = prob.geom.shape
    s = prob.lam * alpha / beta
    x = np.zeros(prob.n) if x0 is None else np.array(x0, dtype=np.float64)
    u = np.zeros(prob.m)
    v = np.zeros(3 * prob.n)
    t = np.zeros(prob.n)
    obj = np.full(iters, np.nan)
    for k in range(iters):
        w = alpha * (prob.Et @ u) + beta * (prob.Dt @ v)
        if positivity:
            w = w + alpha * t
        x_new = x - np.real(np.fft.ifftn(h * np.fft.fftn(w.reshape(shape)))).ravel() / alpha
        xbar = 2.0 * x_new - x
        u = prox.conj_quadratic(u + alpha * (prob.E @ xbar) - alpha * prob.b, alpha)
        v = prox.box(v + beta * (prob.D @ xbar), s)
        if positivity:
            t = prox.nonpositive(t + alpha * xbar)
        x = x_new
        if record:
            obj[k] = objective3d(prob, x)
    return (x, u, v, obj, t) if with_t else (x, u, v, obj)
