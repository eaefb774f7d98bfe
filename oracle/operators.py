"""Finite differences and circulant multipliers (oracle, FP64).

* ``diff_1d`` is the paper's D_n of Section 2 (rows [1, -1]), padded with a zero
  last row so that it is n x n; ``diff_2d`` stacks the horizontal block
  I (x) D_n and the vertical block D_n (x) I, so that D^T D = I (x) L_n + L_n (x) I
  with L_n = D_n^T D_n (Section 2).  An image gradient is stored as two N x N
  planes (horizontal, vertical); the padded rows stay zero.
* ``laplacian_1d`` is L_n of Section 2 (Neumann) and ``periodic_laplacian_1d``
  is the circulant L~_n of Section 2.
* ``multiplier_radon`` is the mask H_R of eq. (circ_R) and
  ``multiplier_diff`` the mask H_D of eq. (circ_D), both indexed (j, k) with
  j, k = 0..N-1 in numpy FFT order.
* ``ncs_multiplier`` is h = diag(F M^+ F^-1) for M = gamma I + alpha C with
  C = H_R + (beta/alpha)^2 H_D the circulant approximation of A^T A for
  A = [E; (beta/alpha) D] (Sections 1.2 and 4.1); its DC entry is set
  separately (Section 4.1.1, Remark on the DC component).
* ``apply_circulant`` evaluates F^-1 diag(h) F x with numpy's FFT pair.

Parity: diff_2d and the masks are pinned by closed forms (D^T D identity,
DFT eigenvalues d_i = 4 sin^2(i pi / n) of L~_n), apply_circulant by the
periodic 5-point stencil it must reproduce.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def diff_1d(n: int) -> sp.csr_matrix:
    """n x n: row i (i < n-1) has +1 at i and -1 at i+1; last row zero."""
    i = np.arange(n - 1)
    rows = np.concatenate([i, i])
    cols = np.concatenate([i, i + 1])
    vals = np.concatenate([np.ones(n - 1), -np.ones(n - 1)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def diff_2d(n: int) -> sp.csr_matrix:
    """2n^2 x n^2: [I (x) D_n ; D_n (x) I] on row-major images."""
    d = diff_1d(n)
    eye = sp.identity(n, format="csr")
    return sp.vstack([sp.kron(eye, d), sp.kron(d, eye)]).tocsr()


def laplacian_1d(n: int) -> np.ndarray:
    """Dense L_n of Section 2: tridiagonal (-1, 2, -1) with corners 1."""
    lap = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    lap[0, 0] = 1.0
    lap[-1, -1] = 1.0
    return lap


def periodic_laplacian_1d(n: int) -> np.ndarray:
    """Dense circulant L~_n of Section 2: (-1, 2, -1) with wrap-around -1."""
    lap = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    lap[0, -1] = -1.0
    lap[-1, 0] = -1.0
    return lap


def _freq_index(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.minimum(j, n - j).astype(np.float64)


def multiplier_radon(n: int, c_r: float) -> np.ndarray:
    """H_R of eq. (circ_R): C_R (min(j,N-j)^2 + min(k,N-k)^2)^(-1/2); 0 at DC."""
    jj = _freq_index(n)
    rad2 = jj[:, None] ** 2 + jj[None, :] ** 2
    out = np.zeros((n, n))
    nz = rad2 > 0
    out[nz] = c_r / np.sqrt(rad2[nz])
    return out


def multiplier_diff(n: int) -> np.ndarray:
    """H_D of eq. (circ_D): 4 (sin^2(j pi/N) + sin^2(k pi/N))."""
    s2 = np.sin(np.arange(n) * np.pi / n) ** 2
    return 4.0 * (s2[:, None] + s2[None, :])


def default_c_r(n_side: int, n_angles: int) -> float:
    """C_R = N_theta N / pi.

    Reading of "C_R accounts for the scaling factor" (Section 4.1.1): the
    discrete E sums N_theta angles with unit bins, i.e. E^T E ~ (N_theta/pi)
    R*R; R*R convolves with 1/|r| (Section 2, eq. radon-formula) whose 2D
    Fourier transform is 1/|omega|, and DFT index j is frequency j/N.
    """
    return n_angles * n_side / np.pi


def ncs_eigenvalues(n: int, alpha: float, beta: float, gamma: float,
                    c_r: float, mu_dc: float) -> np.ndarray:
    """mu = eig(M) for M = gamma I + alpha H_R + (beta^2/alpha) H_D, mu[0,0] = mu_dc."""
    mu = gamma + alpha * multiplier_radon(n, c_r) + (beta * beta / alpha) * multiplier_diff(n)
    mu[0, 0] = mu_dc
    return mu


def pseudo_inverse_diag(mu: np.ndarray) -> np.ndarray:
    """diag(mu)^+ of Section 2: 1/mu_i where mu_i != 0, else 0."""
    out = np.zeros_like(mu)
    nz = mu != 0
    out[nz] = 1.0 / mu[nz]
    return out


def ncs_multiplier(n: int, alpha: float, beta: float, gamma: float,
                   c_r: float, mu_dc: float) -> np.ndarray:
    """h with diag(h) = F M^+ F^-1 (Section 4.1)."""
    return pseudo_inverse_diag(ncs_eigenvalues(n, alpha, beta, gamma, c_r, mu_dc))


def apply_circulant(h: np.ndarray, img: np.ndarray) -> np.ndarray:
    """Real part of F^-1 diag(h) F img for an N x N image (numpy fft2/ifft2 pair)."""
    return np.real(np.fft.ifft2(h * np.fft.fft2(img)))
