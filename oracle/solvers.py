"""NCS, PDHG and ADMM iterations (oracle, FP64).

* ``ncs``: the CT and PET forms of NCS in Section 4.1 and Section 4.2,

      x+ = x - (1/alpha) F^-1 diag(h) F (alpha E^T u + beta D^T v)
      u+ = (u + alpha E(2x+ - x) - alpha b) / (1 + alpha)          (CT)
      u+ = S(u + alpha (E(2x+ - x) + r); alpha b)                   (PET)
      v+ = Pi_[-s,s](v + beta D(2x+ - x)),  s = lambda alpha / beta

  (the isotropic variant replaces Pi by the per-pixel l2-ball projection).
  One iteration is one x-update followed by one (u, v)-update; the objective
  recorded at iteration k is f(x^k).  With ``positivity`` the constraint
  x >= 0 of the remark in Section 4.2 enters as a third block of A (rows I,
  the indicator of the nonnegative orthant in g) with its own dual t:

      x+ = x - (1/alpha) F^-1 diag(h') F (alpha E^T u + beta D^T v + alpha t)
      t+ = min(t + alpha (2x+ - x), 0)

  where h' inverts the eigenvalues of M raised by alpha (``problems.eigenvalues``).
  The reported objective leaves out the indicator of x >= 0, which the
  iterates satisfy only in the limit.
* ``ncs_generic``: eq. (NCS) for any M^+ given as a callable, on the stacked
  dual y = [u; v], A = [E; (beta/alpha) D] and prox_{alpha g*} obtained from the
  Moreau identity.  With M^+ = (1/gamma) I it is eq. (PDHG) (``pdhg``); with
  M^+ = (alpha A^T A)^+ it is eq. (ADMM) (``admm``).
* ``admm_classic``: ADMM in the z / x / multiplier form of the appendix
  (Section 7.1), with the primal prox of g (no Moreau identity).

Parity: pinned by special cases (``ncs`` with a constant multiplier equals
``pdhg``; ``admm_classic`` equals ``admm`` after the change of variables of
Section 7.1), by the common limit of the three methods with KKT residuals
tending to zero (Theorem 1), and by Lemma (monotone) under A3.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import operators, prox
from .objective import objective, prox_conj, stacked_A
from .problems import Params, Problem, multiplier


@dataclass
class Trajectory:
    x: np.ndarray
    u: np.ndarray
    v: np.ndarray
    obj: np.ndarray          # obj[k] = f(x^{k+1}), k = 0..iters-1
    x_prev: np.ndarray       # x^{K-1}
    t: np.ndarray | None = None   # positivity dual (positivity runs only)


def ncs(prob: Problem, par: Params, iters: int, x0=None, u0=None, v0=None,
        h: np.ndarray | None = None, record: bool = True, positivity: bool = False,
        t0=None) -> Trajectory:
    n, m, N = prob.n, prob.m, prob.n_side
    a, be = par.alpha, par.beta
    s = prob.lam * a / be
    if h is None:
        h = multiplier(prob, par, positivity)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    u = np.zeros(m) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros(2 * n) if v0 is None else np.array(v0, dtype=np.float64)
    t = (np.zeros(n) if t0 is None else np.array(t0, dtype=np.float64)) if positivity else None
    obj = np.full(iters, np.nan)
    x_prev = x
    for k in range(iters):
        w = a * (prob.Et @ u) + be * (prob.Dt @ v)
        if positivity:
            w = w + a * t
        x_new = x - operators.apply_circulant(h, w.reshape(N, N)).ravel() / a
        xbar = 2.0 * x_new - x
        q = prob.E @ xbar
        if prob.kind == "ct":
            u = prox.conj_quadratic(u + a * q - a * prob.b, a)
        else:
            u = prox.poisson_s(u + a * (q + prob.bg), a * prob.b)
        g = v + be * (prob.D @ xbar)
        if prob.tv == "aniso":
            v = prox.box(g, s)
        else:
            vh, vv = prox.l2_ball(g[:n], g[n:], s)
            v = np.concatenate([vh, vv])
        if positivity:
            t = prox.nonpositive(t + a * xbar)
        x_prev, x = x, x_new
        if record:
            obj[k] = objective(prob, x)
    return Trajectory(x, u, v, obj, x_prev, t)


def ncs_generic(prob: Problem, par: Params, apply_minv, iters: int, x0=None, y0=None,
                record: bool = True, positivity: bool = False):
    """eq. (NCS): x+ = x - M^+ A^T y; y+ = prox_{alpha g*}(y + alpha(A(2x+ - x) - b~))."""
    A, At, btil = stacked_A(prob, par, positivity)
    pc = prox_conj(prob, par, positivity)
    x = np.zeros(prob.n) if x0 is None else np.array(x0, dtype=np.float64)
    y = np.zeros(btil.size) if y0 is None else np.array(y0, dtype=np.float64)
    obj = np.full(iters, np.nan)
    for k in range(iters):
        x_new = x - apply_minv(At(y))
        y = pc(y + par.alpha * (A(2.0 * x_new - x) - btil))
        x = x_new
        if record:
            obj[k] = objective(prob, x)
    return x, y, obj


def pdhg(prob: Problem, par: Params, gamma_p: float, iters: int, **kw):
    """eq. (PDHG): NCS with M = gamma_p I; converges for gamma_p/alpha >= lambda_max(A^T A)."""
    return ncs_generic(prob, par, lambda z: z / gamma_p, iters, **kw)


def normal_matrix(prob: Problem, par: Params) -> np.ndarray:
    """Dense A^T A = E^T E + (beta/alpha)^2 D^T D (small problems only)."""
    ratio = par.beta / par.alpha
    ete = (prob.Et @ prob.E).toarray()
    dtd = (prob.Dt @ prob.D).toarray()
    return ete + ratio * ratio * dtd


def admm_minv(prob: Problem, par: Params):
    """z -> (alpha A^T A)^+ z by Cholesky; eigen-pseudoinverse (cutoff 1e-12 lambda_max)
    when A^T A is not positive definite."""
    ata = normal_matrix(prob, par)
    try:
        cho = sla.cho_factor(ata)
        return lambda z: sla.cho_solve(cho, z) / par.alpha
    except np.linalg.LinAlgError:
        w, q = np.linalg.eigh(ata)
        keep = w > 1e-12 * w.max()
        winv = np.where(keep, 1.0 / np.where(keep, w, 1.0), 0.0)
        return lambda z: q @ (winv * (q.T @ z)) / par.alpha


def admm(prob: Problem, par: Params, iters: int, minv=None, **kw):
    """eq. (ADMM): x+ = x - alpha^-1 (A^T A)^+ A^T y, same y-update as NCS."""
    if minv is None:
        minv = admm_minv(prob, par)
    return ncs_generic(prob, par, minv, iters, **kw)


def admm_classic(prob: Problem, par: Params, iters: int, x0, lam0, ata_pinv_solve):
    """ADMM of Section 7.1 applied to eq. (RCP):

        z+ = prox_{(1/alpha) g}(A x - b~ - l)
        x+ = (A^T A)^+ A^T (z+ + b~ + l)
        l+ = l + z+ - A x+ + b~

    Returns the list of x iterates x^1..x^iters and the first Moreau dual
    y^1 = alpha (A x^0 - b~ - l^0) - alpha z^1 that the change of variables maps
    to the reduced form's initial dual.
    """
    A, At, btil = stacked_A(prob, par)
    m, n = prob.m, prob.n
    a = par.alpha
    s_tv = prob.lam * par.alpha / par.beta

    def prox_g(w, t):
        if prob.kind == "ct":
            zd = prox.prox_quadratic(w[:m], t)
        else:
            zd = prox.prox_poisson(w[:m], prob.b, t)
        if prob.tv == "aniso":
            zt = prox.soft_threshold(w[m:], t * s_tv)
        else:
            wh, wv = w[m:m + n], w[m + n:]
            nrm = np.sqrt(wh * wh + wv * wv)
            sh = np.maximum(nrm - t * s_tv, 0.0) / np.where(nrm > 0, nrm, 1.0)
            zt = np.concatenate([wh * sh, wv * sh])
        return np.concatenate([zd, zt])

    x = np.array(x0, dtype=np.float64)
    lm = np.array(lam0, dtype=np.float64)
    xs = []
    y1 = None
    for k in range(iters):
        arg = A(x) - btil - lm
        z = prox_g(arg, 1.0 / a)
        if k == 0:
            y1 = a * (arg - z)
        x = ata_pinv_solve(At(z + btil + lm))
        lm = lm + z - A(x) + btil
        xs.append(x)
    return xs, y1


def fixed_point_duals(prob: Problem, par: Params, x0: np.ndarray, tau: float = 0.0):
    """Duals (u, v) of a warm start at x0 from the fixed-point relations
    (Section 3.2, lemma on fixed points): at a fixed point u is the gradient of
    the data term at E x (CT: E x - b; PET: 1 - b / (E x + r)), and v lies in
    the subdifferential of s |.|_1 (anisotropic) or s |.|_2 per pixel
    (isotropic) at D x, s = lambda alpha / beta.  Reading: where that
    subdifferential is an interval (D x = 0) v = 0; with tau > 0 the sign is
    replaced by the ramp clamp(D x / tau, -1, 1) (isotropic: D x / max(|D x|, tau)).
    A PET ray outside the domain (E x + r <= 0) gets u = 0."""
    n = prob.n
    y = prob.E @ x0
    if prob.kind == "ct":
        u = y - prob.b
    else:
        yy = y + prob.bg
        u = np.where(yy > 0, 1.0 - prob.b / np.where(yy > 0, yy, 1.0), 0.0)
    g = prob.D @ x0
    s = prob.lam * par.alpha / par.beta
    if prob.tv == "aniso":
        v = s * (np.clip(g / tau, -1.0, 1.0) if tau > 0 else np.sign(g))
    else:
        gh, gv = g[:n], g[n:]
        den = np.maximum(np.sqrt(gh * gh + gv * gv), tau)
        safe = np.where(den > 0, den, 1.0)
        v = np.concatenate([np.where(den > 0, s * gh / safe, 0.0), np.where(den > 0, s * gv / safe, 0.0)])
    return u, v


def pcg(apply_a, rhs: np.ndarray, iters: int, precond=None) -> np.ndarray:
    """Exactly `iters` steps of (preconditioned) conjugate gradients for
    A d = rhs from d = 0 (Hestenes and Stiefel).  A step whose curvature p.A p
    is zero leaves d unchanged (a zero right-hand side gives d = 0)."""
    d = np.zeros_like(rhs)
    r = rhs.copy()
    z = precond(r) if precond is not None else r.copy()
    p = z.copy()
    rz = float(r @ z)
    for _ in range(iters):
        q = apply_a(p)
        pq = float(p @ q)
        a = rz / pq if pq != 0.0 else 0.0
        d = d + a * p
        r = r - a * q
        z = precond(r) if precond is not None else r.copy()
        rz_new = float(r @ z)
        b = rz_new / rz if rz != 0.0 else 0.0
        p = z + b * p
        rz = rz_new
    return d


def admm_cg(prob: Problem, par: Params, iters: int, cg_iters: int, precondition: bool = True, **kw):
    """ADMM (eq. DRS/ADMM in the form x+ = x - alpha^-1 (A^T A)^+ A^T y) with the
    linear system solved approximately by cg_iters CG steps from zero, the
    comparison method of Section 5 (Ramani and Fessler use CG for these
    systems).  With precondition, CG is preconditioned by alpha M^+, the
    method's own circulant (alpha M^+ ~ (A^T A)^-1)."""
    N = prob.n_side
    ratio = par.beta / par.alpha
    h = multiplier(prob, par)

    def apply_a(p):
        return prob.Et @ (prob.E @ p) + ratio * ratio * (prob.Dt @ (prob.D @ p))

    precond = None
    if precondition:
        def precond(r):
            return par.alpha * operators.apply_circulant(h, r.reshape(N, N)).ravel()

    return ncs_generic(prob, par, lambda z: pcg(apply_a, z, cg_iters, precond) / par.alpha, iters, **kw)
