"""Pins of the oracle's iterations: special cases, the appendix change of
variables, the common limit of NCS / PDHG / ADMM (Theorem 1) with KKT
residuals, and the monotone / summable lemmas of Section 3.2 under A3.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import objective, operators, problems, solvers

N, NA, NS = 16, 24, 24


def _ct(tv="aniso", lam=0.05, seed=3):
    return problems.ct_problem(N, NA, NS, seed, lam, tv=tv)


def _pet(tv="iso", lam=0.5, seed=4):
    return problems.pet_problem(N, NA, NS, seed, lam, total_counts=2e4, tv=tv)


def _dense_circulant(mu):
    n = mu.shape[0]
    eye = np.eye(n * n).reshape(n * n, n, n)
    cols = np.real(np.fft.ifft2(mu[None] * np.fft.fft2(eye), axes=(1, 2)))
    return cols.reshape(n * n, n * n).T


def _gamma_a3(prob, par):
    """Smallest gamma with gamma I + M0 >= alpha A^T A (assumption A3)."""
    base = problems.Params(par.alpha, par.beta, 0.0, par.c_r,
                           problems.resolved_mu_dc(prob, problems.Params(par.alpha, par.beta, 0.0)))
    m0 = _dense_circulant(problems.eigenvalues(prob, base))
    ata = solvers.normal_matrix(prob, par)
    return float(np.linalg.eigvalsh(par.alpha * ata - m0)[-1])


def _a3_params(prob, alpha=0.05, beta=0.1):
    par = problems.Params(alpha, beta, 0.0)
    g = _gamma_a3(prob, par) * 1.01 + 1e-9
    return problems.Params(alpha, beta, g)


@pytest.mark.parametrize("kind", ["ct_aniso", "ct_iso", "pet_iso"])
def test_constant_multiplier_ncs_is_pdhg(kind):
    prob = {"ct_aniso": lambda: _ct("aniso"), "ct_iso": lambda: _ct("iso"), "pet_iso": _pet}[kind]()
    par = problems.Params(0.02, 0.05, 0.0)
    gp = 1.05 * par.alpha * np.linalg.eigvalsh(solvers.normal_matrix(prob, par))[-1]
    h = np.full((N, N), 1.0 / gp)
    tr = solvers.ncs(prob, par, 60, h=h)
    x, y, _ = solvers.pdhg(prob, par, gp, 60)
    np.testing.assert_allclose(tr.x, x, rtol=0, atol=1e-10 * np.abs(x).max())
    np.testing.assert_allclose(tr.u, y[: prob.m], rtol=0, atol=1e-10 * np.abs(y[: prob.m]).max())
    np.testing.assert_allclose(tr.v, y[prob.m:], rtol=0, atol=1e-10 * max(1.0, np.abs(y[prob.m:]).max()))


@pytest.mark.parametrize("kind", ["ct_aniso", "pet_iso"])
def test_application_form_is_general_ncs(kind):
    # The CT/PET forms of Section 4 with the mask equal eq. (NCS) with
    # M^+ = F^-1 diag(h) F on A = [E; (beta/alpha) D].
    prob = _ct() if kind == "ct_aniso" else _pet()
    par = problems.Params(0.03, 0.09, 20.0)
    h = problems.multiplier(prob, par)
    tr = solvers.ncs(prob, par, 40)
    x, y, _ = solvers.ncs_generic(prob, par, lambda z: operators.apply_circulant(h, z.reshape(N, N)).ravel(), 40)
    np.testing.assert_allclose(tr.x, x, rtol=0, atol=1e-10 * np.abs(x).max())
    np.testing.assert_allclose(tr.u, y[: prob.m], rtol=0, atol=1e-10 * np.abs(y[: prob.m]).max())


@pytest.mark.parametrize("kind", ["ct_aniso", "ct_iso", "pet_iso"])
def test_classic_admm_is_reduced_admm(kind):
    # Section 7.1: ADMM in the (z, x, multiplier) form equals eq. (ADMM) after the
    # change of variables y^{k+1} = prox_{alpha g*}(alpha(A x^k - b~ - l^k)).
    prob = {"ct_aniso": lambda: _ct("aniso"), "ct_iso": lambda: _ct("iso"), "pet_iso": _pet}[kind]()
    par = problems.Params(0.5, 0.2, 0.0)
    ata = solvers.normal_matrix(prob, par)
    cho = sla.cho_factor(ata)
    K = 25
    xs, y1 = solvers.admm_classic(prob, par, K, np.zeros(prob.n),
                                  np.zeros(prob.m + 2 * prob.n), lambda z: sla.cho_solve(cho, z))
    x, _, _ = solvers.admm(prob, par, K, x0=np.zeros(prob.n), y0=y1, record=False)
    np.testing.assert_allclose(x, xs[-1], rtol=0, atol=1e-8 * np.abs(xs[-1]).max())


def test_common_limit_and_kkt():
    # Theorem 1: NCS (A3 holds), PDHG and ADMM reach the same primal solution and
    # data dual (x* unique: E is injective here); KKT residuals vanish.
    prob = _ct("aniso")
    par = _a3_params(prob)
    assert np.linalg.svd(prob.E.toarray(), compute_uv=False)[-1] > 1e-6
    tr = solvers.ncs(prob, par, 6000, record=False)
    gp = 1.01 * par.alpha * np.linalg.eigvalsh(solvers.normal_matrix(prob, par))[-1]
    xp, yp, _ = solvers.pdhg(prob, par, gp, 20000, record=False)
    xa, ya, _ = solvers.admm(prob, par, 3000, record=False)
    scale = np.abs(xa).max()
    np.testing.assert_allclose(tr.x, xa, atol=1e-6 * scale)
    np.testing.assert_allclose(xp, xa, atol=1e-6 * scale)
    np.testing.assert_allclose(tr.u, ya[: prob.m], atol=1e-6 * np.abs(ya[: prob.m]).max())
    y = np.concatenate([tr.u, tr.v])
    r_dual, r_fix = objective.kkt(prob, par, tr.x, y)
    assert r_dual < 1e-6 * np.linalg.norm(prob.Et @ tr.u)
    assert r_fix < 1e-6 * (1 + np.linalg.norm(y))
    # the limit is a minimiser: small perturbations do not lower f
    f0 = objective.objective(prob, xa)
    rng = np.random.default_rng(0)
    for _ in range(20):
        assert objective.objective(prob, xa + 1e-3 * rng.standard_normal(prob.n)) >= f0 - 1e-9 * abs(f0)


def test_monotone_and_summable_lemmas_under_a3():
    # Section 3.2, Lemma (monotone) and Lemma (summable), in the D-seminorm.
    prob = _ct("aniso")
    par = _a3_params(prob)
    mu = problems.eigenvalues(prob, par)
    K = 150
    xs, ys = [np.zeros(prob.n)], [np.zeros(prob.m + 2 * prob.n)]
    x, u, v = xs[0], np.zeros(prob.m), np.zeros(2 * prob.n)
    for _ in range(K):
        tr = solvers.ncs(prob, par, 1, x0=x, u0=u, v0=v, record=False)
        x, u, v = tr.x, tr.u, tr.v
        xs.append(x)
        ys.append(np.concatenate([u, v]))
    star = solvers.ncs(prob, par, 8000, record=False)
    ystar = np.concatenate([star.u, star.v])
    d_step = [objective.d_seminorm_sq(prob, par, mu, xs[k + 1] - xs[k], ys[k + 1] - ys[k]) for k in range(K)]
    d_star = [objective.d_seminorm_sq(prob, par, mu, xs[k] - star.x, ys[k] - ystar) for k in range(K)]
    assert min(d_step) >= -1e-9 * max(d_step)           # A3 makes D a seminorm
    for k in range(K - 1):
        assert d_step[k + 1] <= d_step[k] * (1 + 1e-9) + 1e-12
        assert d_star[k + 1] <= d_star[k] * (1 + 1e-9) + 1e-12
    for k in range(K):
        assert d_step[k] <= d_star[0] / (k + 1) * (1 + 1e-6) + 1e-12


def test_paper_ordering_of_iteration_counts():
    # Section 1.2 / Section 3.1: with M close to alpha A^T A, NCS needs far fewer
    # iterations than PDHG, and ADMM (exact M) fewer still.
    prob = problems.ct_problem(32, 45, 48, 5, 0.01)
    par = problems.Params(0.01, 0.03, 0.3 * 0.01 * operators.default_c_r(32, 45))
    xa, ya, obj_a = solvers.admm(prob, par, 400)
    fstar = np.nanmin(obj_a)
    gp = 1.01 * par.alpha * np.linalg.eigvalsh(solvers.normal_matrix(prob, par))[-1]
    _, _, obj_p = solvers.pdhg(prob, par, gp, 1500)
    obj_n = solvers.ncs(prob, par, 1500).obj
    fstar = min(fstar, np.nanmin(obj_p), np.nanmin(obj_n))

    def first(obj):
        g = (obj - fstar) / abs(fstar)
        idx = np.nonzero(g <= 1e-3)[0]
        return idx[0] + 1 if idx.size else 10 ** 9

    ka, kn, kp = first(obj_a), first(obj_n), first(obj_p)
    assert ka <= kn < kp, (ka, kn, kp)
    assert kp >= 1.5 * kn, (kn, kp)


def test_pet_objective_domain_and_constant():
    prob = _pet()
    x = prob.x_true.copy()
    f = objective.objective(prob, x)
    assert np.isfinite(f)
    # an all-negative image leaves the domain of l on rays with b > 0
    assert objective.objective(prob, -10 * np.ones(prob.n) - x) == np.inf
    # constant: NLL of the exact mean is close to the Poisson entropy, not the raw l
    y = prob.E @ x + prob.bg
    raw = float(np.sum(y - prob.b * np.log(y)))
    assert objective.data_term(prob, prob.E @ x) > raw


def test_tv_of_step_image():
    prob = _ct("aniso", lam=1.0)
    img = np.zeros((N, N))
    img[:, N // 2:] = 2.0                     # one vertical edge of height 2 over N rows
    assert objective.tv(prob, img.ravel()) == pytest.approx(2.0 * N)
    img2 = np.zeros((N, N))
    img2[N // 2:, N // 2:] = 1.0              # corner: N/2 horizontal + N/2 vertical unit jumps
    assert objective.tv(prob, img2.ravel()) == pytest.approx(N)
    prob_iso = _ct("iso", lam=1.0)
    dot = np.zeros((N, N))
    dot[5, 5] = 1.0                           # pixel (5,5) pairs (1, 1); (5,4) and (4,5) one unit each
    assert objective.tv(prob, dot.ravel()) == pytest.approx(4.0)
    assert objective.tv(prob_iso, dot.ravel()) == pytest.approx(2.0 + np.sqrt(2.0))


def test_fixed_point_duals_match_the_ncs_limit():
    # At the limit of NCS the duals are determined where the image has an edge:
    # u* = E x* - b everywhere (CT), v* = s sign(D x*) where |D x*| is not small.
    prob = problems.ct_problem(16, 12, 23, 0, 0.05)
    par = problems.Params(0.05, 0.15, 0.3 * 0.05 * 12 * 16 / np.pi)
    traj = solvers.ncs(prob, par, 20000, record=False)
    u0, v0 = solvers.fixed_point_duals(prob, par, traj.x)
    np.testing.assert_allclose(u0, traj.u, rtol=0, atol=1e-8 * np.abs(traj.u).max())
    edge = np.abs(prob.D @ traj.x) > 1e-3
    assert edge.sum() > 50
    np.testing.assert_allclose(v0[edge], traj.v[edge], rtol=1e-8, atol=1e-10)
    # the ramp agrees with the sign wherever |D x| >= tau
    tau = 1e-2
    _, vr = solvers.fixed_point_duals(prob, par, traj.x, tau)
    big = np.abs(prob.D @ traj.x) >= tau
    np.testing.assert_array_equal(vr[big], v0[big])
    assert np.all(np.abs(vr) <= np.abs(v0) + 1e-15)


def test_pcg_solves_spd_systems():
    # CG reaches the solution in n steps on an n x n SPD system (exact arithmetic),
    # with or without an SPD preconditioner
    rng = np.random.default_rng(12)
    n = 40
    q = rng.standard_normal((n, n))
    a = q @ q.T + n * np.eye(n)
    rhs = rng.standard_normal(n)
    ref = np.linalg.solve(a, rhs)
    d = solvers.pcg(lambda v: a @ v, rhs, n)
    np.testing.assert_allclose(d, ref, rtol=1e-9, atol=1e-12)
    pinv = np.diag(1.0 / np.diag(a))
    d = solvers.pcg(lambda v: a @ v, rhs, n, precond=lambda v: pinv @ v)
    np.testing.assert_allclose(d, ref, rtol=1e-9, atol=1e-12)
    assert np.array_equal(solvers.pcg(lambda v: a @ v, np.zeros(n), 5), np.zeros(n))


@pytest.mark.parametrize("precondition", [True, False])
def test_admm_cg_converged_inner_solves_equal_admm(precondition):
    # with the inner systems solved to convergence ADMM-CG is exact-solve ADMM
    prob = problems.ct_problem(16, 12, 23, 0, 0.05)
    par = problems.Params(0.05, 0.15, 0.3 * 0.05 * 12 * 16 / np.pi)
    x_ref, y_ref, obj_ref = solvers.admm(prob, par, 20)
    x, y, obj = solvers.admm_cg(prob, par, 20, 400, precondition=precondition)
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-8 * np.abs(x_ref).max())
    np.testing.assert_allclose(obj, obj_ref, rtol=1e-9)


def test_preconditioned_cg_needs_fewer_steps():
    # the circulant preconditioner reduces the inner residual faster (Section 4.1:
    # alpha M^+ approximates (A^T A)^-1)
    prob = problems.ct_problem(32, 45, 48, 0, 0.01)
    par = problems.Params(0.01, 0.03, 0.3 * 0.01 * 45 * 32 / np.pi)
    x_ref, _, _ = solvers.admm(prob, par, 30)
    e_pc = np.linalg.norm(solvers.admm_cg(prob, par, 30, 5, True)[0] - x_ref)
    e_cg = np.linalg.norm(solvers.admm_cg(prob, par, 30, 5, False)[0] - x_ref)
    assert e_pc < e_cg


# ---------------------------------------------------------------------------
# Positivity constraint x >= 0 (the remark in Section 4.2): a third block of A
# (rows I) with the indicator of the nonnegative orthant in g.


def _chambolle_pock_nonneg(prob, iters):
    """An independent solver of the constrained problem: the primal-dual method
    of Chambolle and Pock with the constraint on the primal side,
    x+ = max(x - tau K^T p+, 0), K = [E; D], and the conjugate prox of the data
    and TV terms on p; no circulant and no third dual block."""
    K = sp.vstack([prob.E, prob.D]).tocsr()
    Kt = K.T.tocsr()
    tau = sigma = 0.99 / np.sqrt(np.linalg.eigvalsh((Kt @ K).toarray())[-1])
    m, n = prob.m, prob.n
    x = np.zeros(n)
    xb = x.copy()
    p = np.zeros(m + 2 * n)
    for _ in range(iters):
        w = p + sigma * (K @ xb)
        if prob.kind == "ct":   # conjugate of 1/2 |y - b|^2
            p1 = (w[:m] - sigma * prob.b) / (1.0 + sigma)
        else:                   # conjugate of sum l(y + r; b): S(w + sigma r; sigma b)
            z = w[:m] + sigma * prob.bg - 1.0
            p1 = 1.0 + (z - np.sqrt(z * z + 4.0 * sigma * prob.b)) / 2.0
        if prob.tv == "aniso":
            p2 = np.clip(w[m:], -prob.lam, prob.lam)
        else:
            h, v = w[m:m + n], w[m + n:]
            sc = np.maximum(1.0, np.sqrt(h * h + v * v) / prob.lam)
            p2 = np.concatenate([h / sc, v / sc])
        p = np.concatenate([p1, p2])
        xn = np.maximum(x - tau * (Kt @ p), 0.0)
        xb = 2.0 * xn - x
        x = xn
    return x


@pytest.mark.parametrize("kind", ["ct", "pet"])
def test_positivity_limit_is_the_constrained_minimiser(kind):
    prob = _ct() if kind == "ct" else _pet()
    par = _a3_params(prob)
    free = solvers.ncs(prob, par, 3000, record=False).x
    pos = solvers.ncs(prob, par, 20000, record=False, positivity=True)
    ref = _chambolle_pock_nonneg(prob, 20000)
    assert free.min() < -1e-2 * free.max()                # the constraint is active
    assert pos.x.min() >= -1e-6 * pos.x.max()
    assert np.linalg.norm(pos.x - ref) <= 1e-6 * np.linalg.norm(ref)
    assert np.all(pos.t <= 0.0)
    # complementarity of the limit: t < 0 only where x = 0
    assert np.max(np.abs(pos.t) * np.maximum(pos.x, 0.0)) <= 1e-6 * np.abs(pos.t).max() * pos.x.max()
    assert objective.objective(prob, pos.x) >= objective.objective(prob, free) - 1e-9


@pytest.mark.parametrize("kind", ["ct_aniso", "pet_iso"])
def test_positivity_form_is_general_ncs(kind):
    # the third dual block and its coupling: the specialised iteration equals
    # eq. (NCS) on A' = [E; (beta/alpha) D; I] with prox_{alpha g*} from the
    # Moreau identity and M'^+ = F^-1 diag(h') F
    prob = _ct() if kind == "ct_aniso" else _pet()
    par = problems.Params(0.03, 0.09, 20.0)
    h = problems.multiplier(prob, par, positivity=True)
    tr = solvers.ncs(prob, par, 40, positivity=True)
    x, y, _ = solvers.ncs_generic(prob, par, lambda z: operators.apply_circulant(h, z.reshape(N, N)).ravel(), 40,
                                  positivity=True)
    m, n = prob.m, prob.n
    assert np.abs(tr.t).max() > 0
    np.testing.assert_allclose(tr.x, x, rtol=0, atol=1e-10 * np.abs(x).max())
    np.testing.assert_allclose(tr.u, y[:m], rtol=0, atol=1e-10 * np.abs(y[:m]).max())
    np.testing.assert_allclose(tr.t, y[m + 2 * n:], rtol=0, atol=1e-10 * np.abs(y[m + 2 * n:]).max())


def test_positivity_multiplier_meets_the_convergence_condition():
    # NCS converges for M >= alpha A^T A (Section 3): with gamma at the A3
    # threshold of the unconstrained system, M' = M + alpha I meets the
    # condition for A' = [E; (beta/alpha) D; I] and M alone does not.
    prob = _ct("aniso")
    par0 = problems.Params(0.05, 0.1, 0.0)
    par = problems.Params(0.05, 0.1, _gamma_a3(prob, par0) * (1 + 1e-9) + 1e-12)
    ext = par.alpha * (solvers.normal_matrix(prob, par) + np.eye(prob.n))
    gap = np.linalg.eigvalsh(_dense_circulant(problems.eigenvalues(prob, par, positivity=True)) - ext)[0]
    gap0 = np.linalg.eigvalsh(_dense_circulant(problems.eigenvalues(prob, par)) - ext)[0]
    scale = np.abs(ext).max()
    assert gap >= -1e-9 * scale
    assert gap0 < -0.5 * par.alpha


def _d_sq_extended(prob, par, mu, dx, dy):
    """D-seminorm of Section 3.2 for A' = [E; (beta/alpha) D; I] and M with eigenvalues mu."""
    a = par.alpha
    adx = np.concatenate([prob.E @ dx, (par.beta / a) * (prob.D @ dx), dx])
    r = dy - a * adx
    return float(r @ r) + a * objective.quad_M(mu, dx) - a * a * float(adx @ adx)


def test_positivity_iteration_is_monotone_in_the_extended_seminorm():
    # Lemma (monotone) and Lemma (summable) of Section 3.2 for NCS on the
    # extended system; they need M' >= alpha A'^T A', which holds because M' = M + alpha I.
    prob = _ct("aniso")
    par = _a3_params(prob)
    mu = problems.eigenvalues(prob, par, positivity=True)
    K = 150
    x, u, v, t = np.zeros(prob.n), np.zeros(prob.m), np.zeros(2 * prob.n), np.zeros(prob.n)
    xs, ys = [x], [np.concatenate([u, v, t])]
    for _ in range(K):
        tr = solvers.ncs(prob, par, 1, x0=x, u0=u, v0=v, t0=t, record=False, positivity=True)
        x, u, v, t = tr.x, tr.u, tr.v, tr.t
        xs.append(x)
        ys.append(np.concatenate([u, v, t]))
    star = solvers.ncs(prob, par, 8000, record=False, positivity=True)
    ystar = np.concatenate([star.u, star.v, star.t])
    d_step = [_d_sq_extended(prob, par, mu, xs[k + 1] - xs[k], ys[k + 1] - ys[k]) for k in range(K)]
    d_star = [_d_sq_extended(prob, par, mu, xs[k] - star.x, ys[k] - ystar) for k in range(K)]
    assert min(d_step) >= -1e-9 * max(d_step)
    for k in range(K - 1):
        assert d_step[k + 1] <= d_step[k] * (1 + 1e-9) + 1e-12
        assert d_star[k + 1] <= d_star[k] * (1 + 1e-9) + 1e-12
    for k in range(K):
        assert d_step[k] <= d_star[0] / (k + 1) * (1 + 1e-6) + 1e-12
