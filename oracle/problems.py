"""Seeded synthetic CT and PET problems and NCS parameters (oracle, FP64).

The problem is eq. (RCP), minimize g(Ax - b), in the two instances of
Section 4:

* CT (Section 4.1): minimize 1/2 |E x - b|^2 + lambda TV(x), written as
  g(y, z) = 1/2 |y|^2 + (lambda alpha/beta) |z|_1 with
  A = [E; (beta/alpha) D] and offset [b; 0].
* PET (Section 4.2): minimize sum_i l((E x)_i + r_i; b_i) + lambda TV(x) with
  l(y; b) = y - b log y (b > 0), y + indicator(y >= 0) (b = 0); r is a known
  uniform background (not in the paper's l; see ``pet_problem``).

TV is anisotropic |Dx|_1 (the paper's choice) or isotropic
sum_p |(Dx)_p|_2 (the PET workload's choice).

Definitional choices that the paper does not fix and that are therefore
"parity unpinned" (both sides take them as inputs): the phantom recipe and
noise model (``ncs_inputs``), the default C_R (``operators.default_c_r``), the
default DC eigenvalue mu_DC = gamma + alpha |E 1|^2 / n (the Rayleigh quotient of
alpha A^T A on the constant image, since D 1 = 0; the paper tunes this entry by
hand, Section 4.1.1), and the values of alpha, beta, gamma.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

import ncs_inputs

from . import fanbeam, operators, projector


@dataclass
class Problem:
    kind: str                 # "ct" or "pet"
    tv: str                   # "aniso" or "iso"
    n_side: int
    n_angles: int
    n_bins: int
    lam: float
    E: sp.csr_matrix
    D: sp.csr_matrix
    b: np.ndarray
    bg: np.ndarray            # PET background r (zeros for CT)
    x_true: np.ndarray
    Et: sp.csr_matrix = field(init=False)
    Dt: sp.csr_matrix = field(init=False)

    def __post_init__(self):
        self.Et = self.E.T.tocsr()
        self.Dt = self.D.T.tocsr()

    @property
    def n(self) -> int:
        return self.n_side * self.n_side

    @property
    def m(self) -> int:
        return self.n_angles * self.n_bins


@dataclass
class Params:
    alpha: float
    beta: float
    gamma: float
    c_r: float | None = None      # None: N_theta N / pi
    mu_dc: float | None = None    # None: gamma + alpha |E 1|^2 / n
    h_e: np.ndarray | None = None  # N x N estimate of E^T E's multiplier (eq. H-fan); None: C_R / |omega|


def resolved_c_r(prob: Problem, par: Params) -> float:
    return operators.default_c_r(prob.n_side, prob.n_angles) if par.c_r is None else par.c_r


def resolved_mu_dc(prob: Problem, par: Params) -> float:
    if par.mu_dc is not None:
        return par.mu_dc
    e1 = prob.E @ np.ones(prob.n)
    return par.gamma + par.alpha * float(e1 @ e1) / prob.n


def multiplier(prob: Problem, par: Params, positivity: bool = False) -> np.ndarray:
    """h (N x N) for this problem and parameters (see ``eigenvalues``)."""
    return operators.pseudo_inverse_diag(eigenvalues(prob, par, positivity))


def eigenvalues(prob: Problem, par: Params, positivity: bool = False) -> np.ndarray:
    """mu = eig(M) (N x N).

    With the positivity block of the remark in Section 4.2, A gains the rows
    I (the block (delta/alpha) I with delta = alpha, scaled like the data
    block), so alpha A^T A gains alpha I and so does M: every eigenvalue,
    mu_DC included, is raised by alpha.
    """
    if par.h_e is None:
        mu = operators.ncs_eigenvalues(prob.n_side, par.alpha, par.beta, par.gamma,
                                       resolved_c_r(prob, par), resolved_mu_dc(prob, par))
    else:   # eq. (H-fan) for E^T E, eq. (circ_D) for D^T D, the DC entry as above
        mu = par.gamma + par.alpha * par.h_e + (par.beta ** 2 / par.alpha) * operators.multiplier_diff(prob.n_side)
        mu[0, 0] = resolved_mu_dc(prob, par)
    return mu + par.alpha if positivity else mu


def ct_problem(n_side: int, n_angles: int, n_bins: int, seed: int, lam: float,
               noise_frac: float = 0.01, tv: str = "aniso", E=None) -> Problem:
    """b = E x_true + sigma eps, sigma = noise_frac * max(E x_true), eps ~ N(0, I)."""
    if E is None:
        E = projector.joseph_matrix(n_side, n_angles, n_bins)
    x_true = ncs_inputs.phantom(n_side, seed).ravel()
    clean = E @ x_true
    sigma = noise_frac * float(np.max(clean))
    b = clean + sigma * ncs_inputs.gaussian_noise(seed, clean.size)
    return Problem("ct", tv, n_side, n_angles, n_bins, lam, E,
                   operators.diff_2d(n_side), b, np.zeros_like(b), x_true)


def fan_problem(n_side: int, n_views: int, n_bins: int, source_radius: float, seed: int, lam: float,
                noise_frac: float = 0.01, tv: str = "aniso", E=None) -> Problem:
    """The CT problem of ``ct_problem`` with the fan-beam E of ``fanbeam.fan_matrix``
    (n_angles holds the number of views)."""
    if E is None:
        E = fanbeam.fan_matrix(fanbeam.FanGeometry(n_side, n_views, n_bins, source_radius))
    x_true = ncs_inputs.phantom(n_side, seed).ravel()
    clean = E @ x_true
    sigma = noise_frac * float(np.max(clean))
    b = clean + sigma * ncs_inputs.gaussian_noise(seed, clean.size)
    return Problem("ct", tv, n_side, n_views, n_bins, lam, E,
                   operators.diff_2d(n_side), b, np.zeros_like(b), x_true)


def pet_problem(n_side: int, n_angles: int, n_bins: int, seed: int, lam: float,
                total_counts: float = 1e6, bg_frac: float = 0.05, tv: str = "iso",
                E=None) -> Problem:
    """Poisson counts b ~ Poisson(E x_true + r).

    x_true is the phantom scaled so that sum(E x_true + r) = total_counts with
    the uniform background r_i = bg_frac * sum(E x_true) / m.
    """
    if E is None:
        E = projector.joseph_matrix(n_side, n_angles, n_bins)
    base = ncs_inputs.phantom(n_side, seed).ravel()
    proj = E @ base
    m = proj.size
    scale = total_counts / ((1.0 + bg_frac) * float(proj.sum()))
    x_true = base * scale
    clean = E @ x_true
    bg = np.full(m, bg_frac * float(clean.sum()) / m)
    b = ncs_inputs.poisson_counts(seed, clean + bg)
    return Problem("pet", tv, n_side, n_angles, n_bins, lam, E,
                   operators.diff_2d(n_side), b, bg, x_true)
