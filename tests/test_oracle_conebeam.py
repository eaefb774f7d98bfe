"""Pins of the oracle's cone-beam path: analytic line integrals, the fan-beam
matrix on the mid-plane, chord lengths, exact symmetries of the orbit and the
detector, the Kronecker form of D^T D in 3D, the periodic 7-point stencil,
exact recovery of a 3D circulant, PDHG in its stacked form, and the common
limit of NCS and PDHG on a volume."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import conebeam, fanbeam, operators, prox

G = conebeam.ConeGeometry(32, 16, 24, 48, 11, 60.0)


@pytest.fixture(scope="module")
def E32():
    return conebeam.cone_matrix(G)


def _rays3d(g):
    """Source and unit direction of every ray (a, rho, d), in storage order."""
    sx, sy, ux, uy, _ = fanbeam.rays(g.fan)
    nv, ns, nr = g.n_views, g.n_bins, g.n_rows
    z = g.slopes
    shp = (nv, nr, ns)
    sx3 = np.broadcast_to(sx.reshape(nv, 1, ns), shp).ravel()
    sy3 = np.broadcast_to(sy.reshape(nv, 1, ns), shp).ravel()
    dx = np.broadcast_to(ux.reshape(nv, 1, ns), shp).ravel()
    dy = np.broadcast_to(uy.reshape(nv, 1, ns), shp).ravel()
    dz = np.broadcast_to(z.reshape(1, nr, 1), shp).ravel()
    nrm = np.sqrt(dx * dx + dy * dy + dz * dz)
    return sx3, sy3, dx / nrm, dy / nrm, dz / nrm


def _grid3d(g):
    c = np.arange(g.n_side) - (g.n_side - 1) / 2.0
    cz = np.arange(g.n_slices) - (g.n_slices - 1) / 2.0
    return np.meshgrid(cz, c, c, indexing="ij")   # Z, Y, X with [z, r, c]


@pytest.mark.parametrize("nz,rs,p0", [(32, 60.0, (3.3, -4.1, 1.7)), (32, 60.0, (-3.0, 2.5, -3.2)),
                                      (64, 40.0, (-3.0, 2.5, 20.0))])
def test_gaussian_line_integrals(nz, rs, p0):
    # the transform of exp(-|p - p0|^2 / 2 s^2) along a line at distance q from
    # p0 is sqrt(2 pi) s exp(-q^2 / 2 s^2), for every slope of the line; the
    # blob sits at least 3 s inside the volume, so truncation costs < 1%.
    # The tall volume with the source at R_s = 40 gives a wide cone (slopes up
    # to 1.8), and the blob high above the mid-plane is crossed only by rays of
    # slope 0.37 and 0.74, whose length per plane exceeds the in-plane one by
    # 7% and 25%.
    g = conebeam.ConeGeometry(32, nz, 24, 48, 11, rs)
    E = conebeam.cone_matrix(g)
    sig = 4.0
    Z, Y, X = _grid3d(g)
    vol = np.exp(-((X - p0[0]) ** 2 + (Y - p0[1]) ** 2 + (Z - p0[2]) ** 2) / (2 * sig ** 2)).ravel()
    sx, sy, dx, dy, dz = _rays3d(g)
    rx, ry, rz = p0[0] - sx, p0[1] - sy, p0[2]
    cx, cy, cz = ry * dz - rz * dy, rz * dx - rx * dz, rx * dy - ry * dx
    q = np.sqrt(cx * cx + cy * cy + cz * cz)
    ana = np.sqrt(2 * np.pi) * sig * np.exp(-q ** 2 / (2 * sig ** 2))
    got = E @ vol
    assert np.max(np.abs(got - ana)) <= 1.5e-2 * ana.max()
    # every ray through the blob, tilted ones included, within 5% of its value
    hit = ana >= 0.2 * ana.max()
    assert np.all(np.abs(got[hit] / ana[hit] - 1.0) <= 0.05)
    slope = np.abs(g.slopes[(np.arange(g.m) // g.n_bins) % g.n_rows])
    if nz == 64:
        assert np.count_nonzero(hit & (slope >= 0.5)) >= 20


def test_mid_plane_rows_of_an_axially_constant_volume_are_the_fan_beam(E32):
    # N_r odd: the middle row has slope 0; with N_z even it runs half way
    # between two slices, and a volume constant along z reproduces the fan beam
    img = np.random.default_rng(1).standard_normal((32, 32))
    vol = np.broadcast_to(img, (16, 32, 32)).ravel()
    y = (E32 @ vol).reshape(24, 11, 48)
    fan = (fanbeam.fan_matrix(G.fan) @ img.ravel()).reshape(24, 48)
    np.testing.assert_allclose(y[:, 5, :], fan, rtol=0, atol=1e-12 * np.abs(fan).max())


def test_chord_lengths_of_the_unit_volume(E32):
    # E 1 is the length of each ray inside the box, up to the partial voxels
    # where it enters and leaves (the interpolation ramps over one voxel on
    # each side of a face, centred on the face).  A ray that runs within one
    # voxel of a side for its whole length (in-plane slope under 1/50 against
    # the stepping axis) sees the ramp all along and is left out.
    sx, sy, dx, dy, dz = _rays3d(G)
    lo = np.array([-16.0, -16.0, -8.0])
    tmin, tmax = np.full(sx.shape, -np.inf), np.full(sx.shape, np.inf)
    for s0, u, l in ((sx, dx, lo[0]), (sy, dy, lo[1]), (np.zeros_like(sx), dz, lo[2])):
        with np.errstate(divide="ignore", invalid="ignore"):
            t1, t2 = (l - s0) / u, (-l - s0) / u
        t1 = np.where(u == 0, np.where(np.abs(s0) <= -l, -np.inf, np.inf), t1)
        t2 = np.where(u == 0, np.where(np.abs(s0) <= -l, np.inf, -np.inf), t2)
        tmin, tmax = np.maximum(tmin, np.minimum(t1, t2)), np.minimum(tmax, np.maximum(t1, t2))
    chord = np.maximum(tmax - tmin, 0.0)
    kappa = 1.0 / np.maximum(np.abs(dx), np.abs(dy))   # length per plane
    minor = np.minimum(np.abs(dx), np.abs(dy)) / np.maximum(np.abs(dx), np.abs(dy))
    transversal = minor >= 0.02
    err = np.abs(E32 @ np.ones(G.n) - chord)
    assert np.mean(transversal) > 0.95 and np.mean(chord > 0) > 0.6
    assert np.all(err[transversal] <= kappa[transversal])
    # rays that stay one voxel inside the slab meet only the side ramps
    z_end = np.maximum(np.abs(dz * tmin), np.abs(dz * tmax))
    inside = transversal & (chord > 0) & (z_end <= 7.0)
    assert inside.sum() > 3000 and np.all(err[inside] <= 0.5 * kappa[inside])


def test_view_subset_is_the_block_of_those_views(E32):
    sub = conebeam.cone_matrix(G, views=[17, 3])
    blk = G.n_rows * G.n_bins
    want = sp.vstack([E32[17 * blk:18 * blk], E32[3 * blk:4 * blk]]).tocsr()
    assert sub.shape == want.shape and abs(sub - want).max() == 0.0


def test_quarter_turn_shifts_the_views(E32):
    vol = np.random.default_rng(2).standard_normal((16, 32, 32))
    y = (E32 @ vol.ravel()).reshape(24, 11, 48)
    y_turned = (E32 @ np.rot90(vol, -1, axes=(1, 2)).ravel()).reshape(24, 11, 48)
    np.testing.assert_allclose(np.roll(y, 6, axis=0), y_turned, rtol=0, atol=1e-9 * np.abs(y).max())


def test_axial_flip_mirrors_the_detector_rows(E32):
    vol = np.random.default_rng(3).standard_normal((16, 32, 32))
    y = (E32 @ vol.ravel()).reshape(24, 11, 48)
    y_flip = (E32 @ vol[::-1].ravel()).reshape(24, 11, 48)
    np.testing.assert_allclose(y[:, ::-1, :], y_flip, rtol=0, atol=1e-9 * np.abs(y).max())


def test_diff_3d_normal_operator_is_the_sum_of_neumann_laplacians():
    n, nz = 5, 3
    D = conebeam.diff_3d(n, nz)
    ln, lz = operators.laplacian_1d(n), operators.laplacian_1d(nz)
    i_n, i_z = np.eye(n), np.eye(nz)
    want = np.kron(i_z, np.kron(i_n, ln)) + np.kron(i_z, np.kron(ln, i_n)) + np.kron(lz, np.kron(i_n, i_n))
    np.testing.assert_array_equal((D.T @ D).toarray(), want)
    assert D.shape == (3 * n * n * nz, n * n * nz)
    # the last difference along each axis is the padded zero row
    x = np.random.default_rng(0).standard_normal(n * n * nz)
    g = (D @ x).reshape(3, nz, n, n)
    assert np.all(g[0, :, :, -1] == 0) and np.all(g[1, :, -1, :] == 0) and np.all(g[2, -1] == 0)


def test_multiplier_diff_3d_is_the_periodic_seven_point_stencil():
    n, nz = 8, 4
    x = np.random.default_rng(4).standard_normal((nz, n, n))
    lap = 6 * x - sum(np.roll(x, s, axis=ax) for ax in range(3) for s in (1, -1))
    got = np.real(np.fft.ifftn(conebeam.multiplier_diff_3d(n, nz) * np.fft.fftn(x)))
    np.testing.assert_allclose(got, lap, rtol=0, atol=1e-12)


def test_probe_estimate_recovers_a_3d_circulant():
    n, nz = 8, 4
    h = 1.0 + conebeam.multiplier_diff_3d(n, nz) + 0.5 * np.cos(2 * np.pi * np.arange(nz) / nz)[:, None, None]
    h = 0.5 * (h + np.roll(np.flip(h), 1, axis=(0, 1, 2)))   # h(-k) = h(k)
    est = conebeam.probe_multiplier_3d(
        lambda v: np.real(np.fft.ifftn(h * np.fft.fftn(v.reshape(nz, n, n)))).ravel(), (nz, n, n), 3)
    np.testing.assert_allclose(est, h, rtol=1e-12, atol=1e-12)


def _tiny():
    g = conebeam.ConeGeometry(8, 4, 12, 16, 5, 20.0)
    return conebeam.cone_problem(g, 1, 0.05)


def test_constant_multiplier_is_pdhg_in_stacked_form():
    # eq. (PDHG) on y = [u; v], A = [E; (beta/alpha) D], b~ = [b; 0], with
    # prox_{alpha g*} from the Moreau identity and the primal proxes of g
    prob = _tiny()
    a, be, gp = 0.05, 0.15, 40.0
    s_tv = prob.lam * a / be
    x_n, u_n, v_n, _ = conebeam.ncs3d(prob, a, be, np.full(prob.geom.shape, 1.0 / gp), 25, record=False)
    m, n = prob.m, prob.n
    ratio = be / a
    x, y = np.zeros(n), np.zeros(m + 3 * n)
    for _ in range(25):
        aty = prob.Et @ y[:m] + ratio * (prob.Dt @ y[m:])
        x_new = x - aty / gp
        xb = 2 * x_new - x
        w = y + a * (np.concatenate([prob.E @ xb, ratio * (prob.D @ xb)]) - np.concatenate([prob.b, np.zeros(3 * n)]))
        y = np.concatenate([prox.moreau_conj(prox.prox_quadratic, w[:m], a),
                            prox.moreau_conj(lambda z, t: prox.soft_threshold(z, t * s_tv), w[m:], a)])
        x = x_new
    np.testing.assert_allclose(x_n, x, rtol=0, atol=1e-12 * np.abs(x).max())
    np.testing.assert_allclose(np.concatenate([u_n, v_n]), y, rtol=0, atol=1e-12 * np.abs(y).max())


def test_ncs_and_pdhg_reach_the_common_limit():
    # NCS with the probe-estimated multiplier and gamma meeting M >= alpha A^T A
    # converges to the minimiser PDHG reaches (Theorem 1)
    prob = _tiny()
    g = prob.geom
    a, be = 0.05, 0.1
    h_e = conebeam.probe_multiplier_3d(lambda v: prob.Et @ (prob.E @ v), g.shape, 8)
    ata = (prob.Et @ prob.E).toarray() + (be / a) ** 2 * (prob.Dt @ prob.D).toarray()
    mu0 = conebeam.eigenvalues3d(prob, a, be, 0.0, h_e)
    n = prob.n
    eye = np.eye(n).reshape(n, *g.shape)
    m0 = np.real(np.fft.ifftn(mu0[None] * np.fft.fftn(eye, axes=(1, 2, 3)), axes=(1, 2, 3))).reshape(n, n).T
    gam = max(float(np.linalg.eigvalsh(a * ata - m0)[-1]) * 1.01, 0.0) + 1e-9
    mu = conebeam.eigenvalues3d(prob, a, be, gam, h_e)
    x_n, _, _, _ = conebeam.ncs3d(prob, a, be, 1.0 / mu, 16000, record=False)
    gp = 1.05 * a * np.linalg.eigvalsh(ata)[-1]
    x_p, _, _, _ = conebeam.ncs3d(prob, a, be, np.full(g.shape, 1.0 / gp), 20000, record=False)
    assert np.linalg.norm(x_n - x_p) <= 1e-5 * np.linalg.norm(x_p)
    f_n, f_p = conebeam.objective3d(prob, x_n), conebeam.objective3d(prob, x_p)
    assert f_n <= f_p * (1 + 1e-9)
    # the sparse matrix has the expected shape and touches every voxel
    assert prob.E.shape == (g.m, g.n) and np.all(np.asarray(abs(prob.E).sum(axis=0)).ravel() > 0)
    assert isinstance(prob.E, sp.csr_matrix)


def test_positivity_form_is_the_stacked_iteration_with_the_identity_block():
    # eq. (NCS) on A' = [E; (beta/alpha) D; I] with M^+ = F^-1 diag(h') F, the
    # prox of alpha g* from the Moreau identity (primal proxes: quadratic,
    # soft threshold, max(., 0) for the indicator of x >= 0)
    prob = _tiny()
    g = prob.geom
    a, be = 0.05, 0.15
    s_tv = prob.lam * a / be
    h_e = conebeam.probe_multiplier_3d(lambda v: prob.Et @ (prob.E @ v), g.shape, 4)
    mu = conebeam.eigenvalues3d(prob, a, be, 2.0, h_e, positivity=True)
    h = 1.0 / mu
    x_n, u_n, v_n, _, t_n = conebeam.ncs3d(prob, a, be, h, 20, record=False, positivity=True, with_t=True)
    m, n = prob.m, prob.n
    ratio = be / a
    x, y = np.zeros(n), np.zeros(m + 4 * n)
    for _ in range(20):
        aty = prob.Et @ y[:m] + ratio * (prob.Dt @ y[m:m + 3 * n]) + y[m + 3 * n:]
        x_new = x - np.real(np.fft.ifftn(h * np.fft.fftn(aty.reshape(g.shape)))).ravel()
        xb = 2 * x_new - x
        w = y + a * (np.concatenate([prob.E @ xb - prob.b, ratio * (prob.D @ xb), xb]))
        y = np.concatenate([prox.moreau_conj(prox.prox_quadratic, w[:m], a),
                            prox.moreau_conj(lambda z, t: prox.soft_threshold(z, t * s_tv), w[m:m + 3 * n], a),
                            prox.moreau_conj(lambda z, t: np.maximum(z, 0.0), w[m + 3 * n:], a)])
        x = x_new
    np.testing.assert_allclose(x_n, x, rtol=0, atol=1e-12 * np.abs(x).max())
    np.testing.assert_allclose(np.concatenate([u_n, v_n, t_n]), y, rtol=0, atol=1e-12 * np.abs(y).max())
    assert np.all(t_n <= 0)


def test_positivity_limit_is_nonnegative_and_optimal():
    # with x >= 0 the iteration converges to a nonnegative point whose objective
    # is no higher than that of the clipped unconstrained minimiser
    prob = _tiny()
    g = prob.geom
    a, be = 0.05, 0.1
    h_e = conebeam.probe_multiplier_3d(lambda v: prob.Et @ (prob.E @ v), g.shape, 8)
    ata = (prob.Et @ prob.E).toarray() + (be / a) ** 2 * (prob.Dt @ prob.D).toarray() + np.eye(prob.n)
    gp = 1.05 * a * np.linalg.eigvalsh(ata)[-1]
    x_c, _, _, _, t_c = conebeam.ncs3d(prob, a, be, np.full(g.shape, 1.0 / gp), 20000, record=False,
                                       positivity=True, with_t=True)
    x_f, _, _, _ = conebeam.ncs3d(prob, a, be, np.full(g.shape, 1.0 / (1.05 * a * np.linalg.eigvalsh(ata - np.eye(prob.n))[-1])),
                                  20000, record=False)
    assert x_f.min() < -1e-3 * x_f.max()                 # the constraint matters
    assert x_c.min() >= -1e-7 * x_c.max()
    f_c = conebeam.objective3d(prob, x_c)
    assert f_c <= conebeam.objective3d(prob, np.maximum(x_f, 0.0)) + 1e-9 * abs(f_c)
    assert np.abs(t_c * x_c).max() <= 1e-6 * np.abs(t_c).max() * x_c.max()   # complementarity
