"""Pins of the oracle's discrete Radon transform (Definition of the Joseph model).

Each check is fixed by something other than the oracle itself: closed forms of
the projector at theta = 0 and pi/2, the analytic Radon transform of a Gaussian
(Section 2, eq. radon-def), chord lengths of the unit image, and the 1/|omega|
Fourier multiplier of R*R (Section 2, eq. radon-formula) that the circulant
mask eq. (circ_R) of Section 4.1.1 is built on.
"""
import numpy as np
import pytest

from oracle import operators, projector


@pytest.mark.parametrize("n_side,n_bins", [(16, 20), (32, 40)])
def test_theta0_even_offset_is_column_sums(n_side, n_bins):
    # theta = 0: ray d is the vertical line x = s_d; with N_s - N even every
    # ray passes through pixel centres, so E x = column sums (weight 1/|cos| = 1).
    E = projector.joseph_matrix(n_side, 6, n_bins)
    x = np.random.default_rng(1).standard_normal((n_side, n_side))
    y0 = (E @ x.ravel())[:n_bins]
    off = (n_bins - n_side) // 2
    expect = np.zeros(n_bins)
    expect[off:off + n_side] = x.sum(axis=0)
    np.testing.assert_allclose(y0, expect, rtol=0, atol=1e-12)


def test_theta0_odd_offset_is_mean_of_adjacent_columns():
    n_side, n_bins = 16, 21
    E = projector.joseph_matrix(n_side, 4, n_bins)
    x = np.random.default_rng(2).standard_normal((n_side, n_side))
    y0 = (E @ x.ravel())[:n_bins]
    cols = np.zeros(n_side + 2)
    cols[1:-1] = x.sum(axis=0)
    # s_d sits half-way between two columns: bin d sees columns d - 3 and d - 2
    full = 0.5 * (cols[:-1] + cols[1:])            # length n_side + 1
    expect = np.zeros(n_bins)
    off = (n_bins - (n_side + 1)) // 2
    expect[off:off + n_side + 1] = full
    np.testing.assert_allclose(y0, expect, rtol=0, atol=1e-12)


def test_theta_half_pi_is_row_sums():
    n_side, n_angles, n_bins = 16, 8, 20
    E = projector.joseph_matrix(n_side, n_angles, n_bins)
    x = np.random.default_rng(3).standard_normal((n_side, n_side))
    a = n_angles // 2                              # theta = pi/2: line y = s_d
    y = (E @ x.ravel())[a * n_bins:(a + 1) * n_bins]
    off = (n_bins - n_side) // 2
    expect = np.zeros(n_bins)
    expect[off:off + n_side] = x.sum(axis=1)
    np.testing.assert_allclose(y, expect, rtol=0, atol=1e-10)


def test_gaussian_matches_analytic_radon_transform():
    # f(x, y) = exp(-|(x,y) - c|^2 / (2 s^2)) has R f(s, theta) =
    # sqrt(2 pi) s exp(-(s - c.(cos, sin))^2 / (2 s^2)).  An off-centre blob
    # fixes the orientation of theta, s, rows (y) and columns (x).
    n_side, n_angles, n_bins = 64, 30, 92
    sig = 7.0
    cx, cy = 9.0, -13.0
    coord = np.arange(n_side) - (n_side - 1) / 2.0
    yy, xx = np.meshgrid(coord, coord, indexing="ij")
    img = np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * sig * sig))
    E = projector.joseph_matrix(n_side, n_angles, n_bins)
    y = (E @ img.ravel()).reshape(n_angles, n_bins)
    theta = np.pi * np.arange(n_angles) / n_angles
    s = np.arange(n_bins) - (n_bins - 1) / 2.0
    shift = cx * np.cos(theta) + cy * np.sin(theta)
    ref = np.sqrt(2 * np.pi) * sig * np.exp(-(s[None, :] - shift[:, None]) ** 2 / (2 * sig * sig))
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert rel < 5e-3, rel
    # a mistake in the orientation (theta -> -theta) is far off
    wrong = np.sqrt(2 * np.pi) * sig * np.exp(
        -(s[None, :] - (cx * np.cos(theta) - cy * np.sin(theta))[:, None]) ** 2 / (2 * sig * sig))
    assert np.linalg.norm(y - wrong) / np.linalg.norm(ref) > 0.3


def _chord(n_side, theta, s):
    # length of {x cos + y sin = s} inside the square [-N/2, N/2]^2
    h = n_side / 2.0
    c, si = np.cos(theta), np.sin(theta)
    pts = []
    for xb in (-h, h):
        if abs(si) > 1e-12:
            yv = (s - xb * c) / si
            if -h - 1e-9 <= yv <= h + 1e-9:
                pts.append((xb, yv))
    for yb in (-h, h):
        if abs(c) > 1e-12:
            xv = (s - yb * si) / c
            if -h - 1e-9 <= xv <= h + 1e-9:
                pts.append((xv, yb))
    if len(pts) < 2:
        return 0.0
    pts = np.array(pts)
    return float(max(np.linalg.norm(p - q) for p in pts for q in pts))


def test_ones_image_gives_chord_lengths():
    n_side, n_angles, n_bins = 32, 12, 48
    E = projector.joseph_matrix(n_side, n_angles, n_bins)
    e1 = (E @ np.ones(n_side * n_side)).reshape(n_angles, n_bins)
    s = np.arange(n_bins) - (n_bins - 1) / 2.0
    for a in range(n_angles):
        th = np.pi * a / n_angles
        kappa = 1.0 / max(abs(np.cos(th)), abs(np.sin(th)))
        for d in range(n_bins):
            ch = _chord(n_side, th, s[d])
            # interior: exact up to the half-pixel ends of the ray
            assert abs(e1[a, d] - ch) <= 2.0 * kappa + 1e-9, (a, d, e1[a, d], ch)


def test_adjoint_is_transpose_and_rows_nonnegative():
    E = projector.joseph_matrix(16, 10, 23)
    assert E.min() >= 0.0
    rng = np.random.default_rng(4)
    x = rng.standard_normal(E.shape[1])
    y = rng.standard_normal(E.shape[0])
    assert abs((E @ x) @ y - x @ (E.T @ y)) < 1e-10 * np.linalg.norm(E @ x) * np.linalg.norm(y)


def test_normal_operator_multiplier_is_c_r_over_frequency():
    # eq. (H-fan) probe: h_i = average over v of (F E^T E v)_i / (F v)_i.
    # At low frequencies it must follow C_R / |omega| with C_R = N_theta N / pi
    # (the reading of "C_R accounts for the scaling factor"); Joseph
    # interpolation only damps the highest frequencies.
    n_side, n_angles, n_bins = 64, 90, 92
    E = projector.joseph_matrix(n_side, n_angles, n_bins)
    Et = E.T.tocsr()
    rng = np.random.default_rng(0)
    acc = np.zeros((n_side, n_side))
    k = 24
    for _ in range(k):
        v = rng.standard_normal((n_side, n_side))
        cv = (Et @ (E @ v.ravel())).reshape(n_side, n_side)
        acc += (np.fft.fft2(cv) / np.fft.fft2(v)).real
    probe = acc / k
    c_r = operators.default_c_r(n_side, n_angles)
    hr = operators.multiplier_radon(n_side, c_r)
    j = np.minimum(np.arange(n_side), n_side - np.arange(n_side))
    rad = np.sqrt(j[:, None] ** 2 + j[None, :] ** 2)
    for r in (1, 2, 4, 8):
        ring = (rad >= r - 0.5) & (rad < r + 0.5)
        ratio = probe[ring].mean() / hr[ring].mean()
        assert 0.85 < ratio < 1.15, (r, ratio)
