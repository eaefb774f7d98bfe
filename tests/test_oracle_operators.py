"""Pins of the oracle's finite differences, circulant masks and proximal maps.

Closed forms from Section 2 (D_n, L_n, L~_n and the DFT eigenvalues
d_{i+1} = 4 sin^2(i pi / n) of eq. f-diff), the circulant pseudo-inverse of
Section 2, and brute-force one-dimensional minimisation for the proximal maps
of Section 4.1 (quadratic, box) and Section 4.2 (the Poisson map S).
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import operators, prox


def test_dtd_is_kron_of_neumann_laplacians():
    n = 8
    D = operators.diff_2d(n).toarray()
    # L_n as printed in Section 2: diagonal (1, 2, ..., 2, 1), off-diagonals -1
    L = np.diag([1.0] + [2.0] * (n - 2) + [1.0]) - np.eye(n, k=1) - np.eye(n, k=-1)
    I = np.eye(n)
    np.testing.assert_array_equal(D.T @ D, np.kron(I, L) + np.kron(L, I))
    Dn = operators.diff_1d(n).toarray()[: n - 1]
    # D_n of Section 2: rows [1, -1]
    np.testing.assert_array_equal(Dn[0, :2], [1.0, -1.0])
    np.testing.assert_array_equal(Dn.T @ Dn, L)


def test_gradient_layout_on_a_ramp():
    n = 6
    img = np.arange(n)[None, :] * 2.0 + np.arange(n)[:, None] * 5.0   # x[r, c] = 5 r + 2 c
    g = operators.diff_2d(n) @ img.ravel()
    gh, gv = g[: n * n].reshape(n, n), g[n * n:].reshape(n, n)
    assert np.all(gh[:, : n - 1] == -2.0) and np.all(gh[:, n - 1] == 0.0)
    assert np.all(gv[: n - 1, :] == -5.0) and np.all(gv[n - 1, :] == 0.0)


def test_periodic_laplacian_eigenvalues():
    # eq. (f-diff): L~_n = F^-1 diag(d) F, d_{i+1} = 4 sin^2(i pi / n)
    for n in (5, 8, 13):
        col = operators.periodic_laplacian_1d(n)[:, 0]
        d = np.fft.fft(col).real
        np.testing.assert_allclose(d, 4 * np.sin(np.arange(n) * np.pi / n) ** 2, atol=1e-12)


def test_h_d_mask_is_periodic_five_point_laplacian():
    n = 16
    x = np.random.default_rng(0).standard_normal((n, n))
    lap = 4 * x - np.roll(x, 1, 0) - np.roll(x, -1, 0) - np.roll(x, 1, 1) - np.roll(x, -1, 1)
    np.testing.assert_allclose(operators.apply_circulant(operators.multiplier_diff(n), x), lap, atol=1e-12)


def test_h_r_mask_closed_form():
    n = 8
    hr = operators.multiplier_radon(n, 3.0)
    assert hr[0, 0] == 0.0
    assert hr[1, 0] == pytest.approx(3.0)
    assert hr[7, 1] == pytest.approx(3.0 / np.sqrt(2.0))
    assert hr[4, 3] == pytest.approx(3.0 / 5.0)
    np.testing.assert_array_equal(hr, hr.T)


def test_ncs_multiplier_layout_and_dc():
    # index layout only (numpy FFT order, the DC slot, h = 1/mu); the weights of
    # the terms are pinned against the operators themselves in
    # test_mu_matches_the_probe_estimate_of_alpha_AtA
    n, a, b, g, cr, dc = 8, 0.3, 0.7, 2.0, 5.0, 11.0
    mu = operators.ncs_eigenvalues(n, a, b, g, cr, dc)
    assert mu[0, 0] == dc
    j, k = 3, 1
    expect = g + a * cr / np.sqrt(j * j + k * k) + (b * b / a) * 4 * (np.sin(j * np.pi / n) ** 2 + np.sin(k * np.pi / n) ** 2)
    assert mu[j, k] == pytest.approx(expect)
    h = operators.ncs_multiplier(n, a, b, g, cr, dc)
    np.testing.assert_allclose(h * mu, 1.0)


def _ring_ratios(est, mu_minus_gamma, n):
    """Sum of est over sum of mu - gamma on each ring round(|omega|) = 1, 2, ..."""
    jj = np.minimum(np.arange(n), n - np.arange(n))
    ring = np.rint(np.sqrt(jj[:, None] ** 2 + jj[None, :] ** 2)).astype(int)
    return np.array([est[ring == r].sum() / mu_minus_gamma[ring == r].sum() for r in range(1, ring.max() + 1)])


def test_mu_matches_the_probe_estimate_of_alpha_AtA():
    # M - gamma I = alpha C must approximate alpha A^T A = alpha E^T E + (beta^2/alpha) D^T D
    # (Sections 1.2 and 4.1.1: eq. circ_R for E^T E, eq. circ_D for D^T D).  The
    # multiplier of the actual operator alpha A^T A is estimated from 32 probes
    # (eq. H-fan) and compared with the oracle's mu - gamma ring by ring at 64^2.
    # Joseph interpolation damps E^T E at high frequencies (ratios fall to about
    # 0.64 there) but the low rings, where alpha C_R / |omega| dominates, agree
    # within 10%; with beta/alpha = 30 the difference term dominates every ring
    # and all agree within 10%.  A dropped alpha on H_R, a D weight of beta,
    # beta^2/alpha^2 or beta^2, or an M scaled by 2 breaks one of the bands.
    from oracle import fanbeam, problems, projector
    n, na, ns = 64, 90, 92
    E = projector.joseph_matrix(n, na, ns)
    Et = E.T.tocsr()
    D = operators.diff_2d(n)
    Dt = D.T.tocsr()
    z = np.zeros(E.shape[0])
    prob = problems.Problem("ct", "aniso", n, na, ns, 0.01, E, D, z, z, np.zeros(n * n))
    for a, b, lo_band, all_band in ((0.01, 0.03, (0.9, 1.05), (0.6, 1.05)),
                                   (0.01, 0.3, (0.9, 1.05), (0.9, 1.05))):
        g = 0.3 * a * operators.default_c_r(n, na)
        mu = problems.eigenvalues(prob, problems.Params(a, b, g))
        r2 = (b / a) ** 2
        est = a * fanbeam.probe_multiplier(lambda v: Et @ (E @ v) + r2 * (Dt @ (D @ v)), n, 32)
        rat = _ring_ratios(est, mu - g, n)
        assert lo_band[0] <= rat[:8].min() and rat[:8].max() <= lo_band[1], rat[:8]
        assert all_band[0] <= rat.min() and rat.max() <= all_band[1], rat


def test_circulant_pseudo_inverse():
    # Section 2: C^+ = F^-1 diag(h)^+ F with zero entries kept at zero.
    n = 8
    rng = np.random.default_rng(1)
    mu = np.abs(rng.standard_normal((n, n))) + 0.5
    mu = 0.5 * (mu + mu[(-np.arange(n)) % n][:, (-np.arange(n)) % n])   # real, even -> real operator
    mu[0, 0] = 0.0
    C = lambda z: operators.apply_circulant(mu, z)
    Cp = lambda z: operators.apply_circulant(operators.pseudo_inverse_diag(mu), z)
    x = rng.standard_normal((n, n))
    np.testing.assert_allclose(C(Cp(C(x))), C(x), atol=1e-12)           # C C^+ C = C
    np.testing.assert_allclose(Cp(np.ones((n, n))), 0.0, atol=1e-12)      # null space of the DC


# -- proximal maps -----------------------------------------------------------

def _brute_prox_conj_poisson(w, a, b):
    # argmin_u a l*(u) + (u - w)^2 / 2 with l*(u) = -b log(1 - u) + const (u < 1)
    # for b > 0 and l* = indicator(u <= 1) for b = 0.
    if b == 0:
        return min(w, 1.0)
    f = lambda u: -a * b * np.log(1.0 - u) + 0.5 * (u - w) ** 2
    lo = min(w, 0.0) - 10.0 - abs(w)
    res = minimize_scalar(f, bounds=(lo, 1.0 - 1e-14), method="bounded",
                          options={"xatol": 1e-13, "maxiter": 2000})
    return res.x


@pytest.mark.parametrize("w", [-3.0, -0.2, 0.5, 0.99, 1.5, 4.0])
@pytest.mark.parametrize("a,b", [(0.1, 3.0), (1.0, 0.5), (0.01, 30.0), (2.0, 0.0)])
def test_poisson_s_is_prox_of_conjugate(w, a, b):
    s = prox.poisson_s(np.array([w]), np.array([a * b]))[0]
    assert s == pytest.approx(_brute_prox_conj_poisson(w, a, b), abs=1e-6)
    assert s <= 1.0


def test_poisson_s_zero_counts_is_min_with_one():
    w = np.linspace(-3, 3, 13)
    np.testing.assert_allclose(prox.poisson_s(w, np.zeros_like(w)), np.minimum(w, 1.0))


def test_moreau_identity_poisson():
    rng = np.random.default_rng(2)
    w = rng.uniform(-3, 3, 50)
    b = rng.integers(0, 20, 50).astype(float)
    a = 0.3
    lhs = prox.poisson_s(w, a * b)
    rhs = prox.moreau_conj(lambda z, t: prox.prox_poisson(z, b, t), w, a)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_prox_poisson_brute_force():
    for z, b, t in [(0.3, 2.0, 0.5), (5.0, 1.0, 2.0), (-1.0, 3.0, 0.1)]:
        f = lambda y: t * (y - b * np.log(y)) + 0.5 * (y - z) ** 2
        res = minimize_scalar(f, bounds=(1e-12, 100.0), method="bounded", options={"xatol": 1e-12})
        assert prox.prox_poisson(np.array([z]), np.array([b]), t)[0] == pytest.approx(res.x, abs=1e-6)


def test_quadratic_and_box_via_moreau():
    w = np.linspace(-4, 4, 17)
    a = 0.7
    np.testing.assert_allclose(prox.conj_quadratic(w, a), prox.moreau_conj(prox.prox_quadratic, w, a))
    s = 0.9
    # g = s |.|_1 : prox_{a g*} = projection onto [-s, s] (Section 4.1)
    np.testing.assert_allclose(prox.box(w, s),
                               prox.moreau_conj(lambda z, t: prox.soft_threshold(z, t * s), w, a), atol=1e-12)
    # brute force of the quadratic conjugate prox: argmin a u^2/2 + (u - w)^2/2
    for wi in (-2.0, 0.3, 5.0):
        res = minimize_scalar(lambda u: a * u * u / 2 + (u - wi) ** 2 / 2)
        assert prox.conj_quadratic(wi, a) == pytest.approx(res.x, abs=1e-7)


def test_l2_ball_projection():
    rng = np.random.default_rng(3)
    wh, wv = rng.standard_normal(200) * 2, rng.standard_normal(200) * 2
    s = 1.3
    ph, pv = prox.l2_ball(wh, wv, s)
    nrm = np.sqrt(ph ** 2 + pv ** 2)
    assert np.all(nrm <= s + 1e-12)
    inside = np.sqrt(wh ** 2 + wv ** 2) <= s
    np.testing.assert_allclose(ph[inside], wh[inside])
    # outside: the projection is on the circle and on the ray through w
    out = ~inside
    np.testing.assert_allclose(nrm[out], s)
    np.testing.assert_allclose(ph[out] * wv[out] - pv[out] * wh[out], 0.0, atol=1e-12)
    assert np.all(ph[out] * wh[out] + pv[out] * wv[out] > 0)
