"""Pins of the oracle's fan-beam projector and of the probe estimate of
eq. (H-fan): analytic line integrals, chord lengths, a quarter-turn symmetry,
the published outputs of SplitMix64, exact recovery of a circulant operator,
and the common limit of NCS and PDHG on a fan-beam problem."""
import numpy as np
import pytest

from oracle import fanbeam, objective, operators, problems, solvers

G64 = fanbeam.FanGeometry(64, 60, 128, 120.0)


@pytest.fixture(scope="module")
def E64():
    return fanbeam.fan_matrix(G64)


def _grid(n):
    c = np.arange(n) - (n - 1) / 2.0
    return np.meshgrid(c, c)   # X[r, c] = x_c, Y[r, c] = y_r


def test_splitmix64_published_outputs():
    # the first three outputs from state 0 of the reference generator
    assert [int(v) for v in fanbeam.splitmix64(0, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                          0x06C45D188009454F]


def test_rademacher_probe_is_balanced_and_deterministic():
    v = fanbeam.rademacher_probe(3, 4096)
    assert set(np.unique(v)) == {-1.0, 1.0}
    assert abs(v.mean()) < 0.1
    assert np.array_equal(v, fanbeam.rademacher_probe(3, 4096))
    assert not np.array_equal(v, fanbeam.rademacher_probe(4, 4096))


@pytest.mark.parametrize("x0,y0", [(5.3, -7.1), (-11.0, 9.5)])
def test_gaussian_line_integrals(E64, x0, y0):
    # the divergent-beam transform of exp(-|p - p0|^2 / 2 s^2) along a line at
    # distance q from p0 is sqrt(2 pi) s exp(-q^2 / 2 s^2)
    sig = 4.0
    X, Y = _grid(64)
    img = np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * sig ** 2)).ravel()
    sx, sy, ux, uy, _ = fanbeam.rays(G64)
    q = np.abs((x0 - sx) * uy - (y0 - sy) * ux)
    ana = np.sqrt(2 * np.pi) * sig * np.exp(-q ** 2 / (2 * sig ** 2))
    assert np.max(np.abs(E64 @ img - ana)) <= 1.5e-2 * ana.max()


def test_chord_lengths_of_the_unit_image(E64):
    # E 1 is the length of each ray inside the image square, up to the two
    # partial pixels where it enters and leaves (at most 2 kappa)
    sx, sy, ux, uy, rows = fanbeam.rays(G64)
    half = 32.0
    tmin, tmax = np.full(sx.shape, -np.inf), np.full(sx.shape, np.inf)
    for s, u in ((sx, ux), (sy, uy)):
        with np.errstate(divide="ignore"):
            t1, t2 = (-half - s) / u, (half - s) / u
        tmin, tmax = np.maximum(tmin, np.minimum(t1, t2)), np.minimum(tmax, np.maximum(t1, t2))
    chord = np.maximum(tmax - tmin, 0.0)
    kappa = np.where(rows, 1 / np.abs(uy), 1 / np.abs(ux))
    assert np.all(np.abs(E64 @ np.ones(64 * 64) - chord) <= 2.0 * kappa)
    assert np.mean(chord > 0) > 0.8


def test_quarter_turn_shifts_the_views(E64):
    # turning the object by +90 degrees about the centre is turning the source
    # the other way: view a of the turned image is view a - N_v/4 of the original
    img = np.random.default_rng(0).standard_normal((64, 64))
    y = (E64 @ img.ravel()).reshape(60, 128)
    y_turned = (E64 @ np.rot90(img, -1).ravel()).reshape(60, 128)
    np.testing.assert_allclose(np.roll(y, 15, axis=0), y_turned, rtol=0, atol=1e-9 * np.abs(y).max())


def test_probe_estimate_recovers_a_circulant():
    # h_i = (F C v)_i / (F v)_i for every v when C is circulant (Section 4.1.1)
    n = 16
    h = 1.0 + operators.multiplier_diff(n) + 0.5 * np.cos(2 * np.pi * np.arange(n) / n)[None, :]
    h = 0.5 * (h + np.roll(np.flip(h), 1, axis=(0, 1)))   # h(-k) = h(k): C is real and symmetric
    est = fanbeam.probe_multiplier(lambda v: operators.apply_circulant(h, v.reshape(n, n)).ravel(), n, 3)
    np.testing.assert_allclose(est, h, rtol=1e-12, atol=1e-12)


def test_probe_estimate_of_the_fan_normal_operator_is_the_rayleigh_quotient():
    # the DC entry of the estimate is sum_v (1^T v)(1^T E^T E v) / sum_v (1^T v)^2,
    # and every entry is the least-squares fit of the probes' spectra
    g = fanbeam.FanGeometry(16, 24, 32, 30.0)
    E = fanbeam.fan_matrix(g)
    n = 16
    est = fanbeam.probe_multiplier(lambda v: E.T @ (E @ v), n, 4)
    num = den = 0.0
    for k in range(4):
        v = fanbeam.rademacher_probe(k, n * n)
        num += v.sum() * (E.T @ (E @ v)).sum()
        den += v.sum() ** 2
    assert est[0, 0] == pytest.approx(num / den, rel=1e-10)
    assert np.all(np.isfinite(est))


def test_fan_ncs_reaches_the_common_limit():
    # NCS with the estimated multiplier and a gamma meeting M >= alpha A^T A
    # converges to the minimiser PDHG reaches (Theorem 1)
    g = fanbeam.FanGeometry(16, 24, 32, 30.0)
    prob = problems.fan_problem(16, 24, 32, 30.0, 1, 0.05)
    h_e = fanbeam.probe_multiplier(lambda v: prob.Et @ (prob.E @ v), 16, 8)
    base = problems.Params(0.05, 0.1, 0.0, h_e=h_e)
    mu0 = problems.eigenvalues(prob, base)
    n = prob.n
    eye = np.eye(n).reshape(n, 16, 16)
    m0 = np.real(np.fft.ifft2(mu0[None] * np.fft.fft2(eye), axes=(1, 2))).reshape(n, n).T
    gam = float(np.linalg.eigvalsh(0.05 * solvers.normal_matrix(prob, base) - m0)[-1]) * 1.01 + 1e-9
    par = problems.Params(0.05, 0.1, max(gam, 0.0), h_e=h_e)
    tr = solvers.ncs(prob, par, 6000, record=False)
    gp = 1.05 * par.alpha * np.linalg.eigvalsh(solvers.normal_matrix(prob, par))[-1]
    x_p, _, _ = solvers.pdhg(prob, par, gp, 30000, record=False)
    assert np.linalg.norm(tr.x - x_p) <= 1e-5 * np.linalg.norm(x_p)
    assert objective.objective(prob, tr.x) <= objective.objective(prob, x_p) * (1 + 1e-9)
    assert g.n_bins == prob.n_bins
