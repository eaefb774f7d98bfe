"""Explicit FP64 sparse matrix of the discrete Radon transform (oracle).

Section 4.1.1 of the paper takes E = R, "the discretization of the Radon
transform" of eq. (radon-def), R f(s, theta) = integral of f along the line
x cos(theta) + y sin(theta) = s, theta in [0, pi).  The paper does not fix the
discretisation (its experiments called a library routine), so both sides use
the Joseph ray-driven reading:

* pixel (r, c) of an N x N image has unit size and centre
  (x_c, y_r) = (c - (N-1)/2, r - (N-1)/2); storage index r*N + c;
* angle a of N_theta: theta_a = pi * a / N_theta;
* bin d of N_s: s_d = d - (N_s-1)/2; ray (a, d) is the line above; storage
  index a*N_s + d;
* a ray steps through rows when 4a <= N_theta or 4a >= 3 N_theta (an integer
  test, so the 45-degree ties do not depend on rounding) and through columns
  otherwise;
* stepping through row r, the ray crosses y = y_r at column coordinate
  xi = (s_d - y_r sin(theta)) / cos(theta) + (N-1)/2; with c0 = floor(xi),
  f = xi - c0 it puts weight (1-f)/|cos(theta)| on pixel (r, c0) and
  f/|cos(theta)| on pixel (r, c0+1) (pixels outside the image are dropped);
  1/|cos(theta)| is the length of the ray inside one pixel row;
* stepping through columns swaps the roles of x and y and of cos and sin.

Parity: pinned by tests against closed forms (theta = 0 and theta = pi/2 give
column and row sums), the analytic Radon transform of a Gaussian
(Section 2, eq. radon-def), chord lengths of the unit image, and the 1/|omega|
multiplier of R*R (Section 2, eq. radon-formula).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def row_stepping(n_angles: int) -> np.ndarray:
    """Boolean per angle: True when the ray marches through image rows."""
    a = np.arange(n_angles)
    return (4 * a <= n_angles) | (4 * a >= 3 * n_angles)


def joseph_matrix(n_side: int, n_angles: int, n_bins: int, angles=None) -> sp.csr_matrix:
    """The m x n matrix E (m = n_angles*n_bins, n = n_side**2), CSR, float64.

    With ``angles`` (a list of angle indices) only those rows are filled; the
    other rows are empty (used to check large geometries angle by angle).
    """
    n = n_side
    half_img = (n - 1) / 2.0
    s = np.arange(n_bins) - (n_bins - 1) / 2.0          # bin offsets s_d
    coord = np.arange(n) - half_img                      # pixel centre coordinates
    rows_all, cols_all, vals_all = [], [], []
    stepping_rows = row_stepping(n_angles)
    for a in (range(n_angles) if angles is None else angles):
        theta = np.pi * a / n_angles
        ct, st = np.cos(theta), np.sin(theta)
        ray = a * n_bins + np.arange(n_bins)             # (n_bins,)
        if stepping_rows[a]:
            # xi[d, r]: column coordinate of ray d on row r
            xi = (s[:, None] - coord[None, :] * st) / ct + half_img
            step = 1.0 / abs(ct)
        else:
            # eta[d, c]: row coordinate of ray d on column c
            xi = (s[:, None] - coord[None, :] * ct) / st + half_img
            step = 1.0 / abs(st)
        lo = np.floor(xi)
        f = xi - lo
        lo = lo.astype(np.int64)
        stepper = np.broadcast_to(np.arange(n)[None, :], xi.shape)
        rays = np.broadcast_to(ray[:, None], xi.shape)
        for off, w in ((0, (1.0 - f) * step), (1, f * step)):
            idx = lo + off
            keep = (idx >= 0) & (idx < n) & (w != 0.0)
            if stepping_rows[a]:
                pix = stepper[keep] * n + idx[keep]      # (r, c) with r stepped
            else:
                pix = idx[keep] * n + stepper[keep]      # (r, c) with c stepped
            rows_all.append(rays[keep])
            cols_all.append(pix)
            vals_all.append(w[keep])
    rows = np.concatenate(rows_all)
    cols = np.concatenate(cols_all)
    vals = np.concatenate(vals_all)
    m = n_angles * n_bins
    mat = sp.coo_matrix((vals, (rows, cols)), shape=(m, n * n)).tocsr()
    mat.sum_duplicates()
    return mat
