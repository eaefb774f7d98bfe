"""Objective values, KKT residuals and the D-seminorm (oracle, FP64).

* ``tv``: anisotropic |Dx|_1 (Section 4.1) or isotropic sum_p |(Dx)_p|_2.
* ``objective``: CT 1/2 |Ex - b|^2 + lambda TV(x) (Section 4.1); PET the
  Poisson negative log-likelihood sum_i [y_i - b_i log y_i + log Gamma(b_i+1)]
  with y = Ex + r, plus lambda TV(x) (Section 4.2; the log Gamma constant makes
  it the exact negative log-likelihood and does not move the minimiser).
  A ray with b_i > 0 and y_i <= 0 makes the value +inf.  A ray with b_i = 0
  contributes y_i for every sign of y_i: its l is y + indicator(y >= 0), and
  NCS iterates reach y_i < 0 only on such rays, approaching y_i = 0 in the
  limit, so the indicator is dropped when the objective is reported (the value
  is the paper's on the domain).
* ``kkt``: for the pair (eq. RCP, eq. dual) at a primal-dual point (x, y):
  dual feasibility |A^T y| and the fixed-point residual
  |y - prox_{alpha g*}(y + alpha(A x - b~))| (zero exactly at a saddle point).
* ``d_seminorm_sq``: D^2(x, y) = |y - alpha A x|^2 + x^T(alpha M - alpha^2 A^T A) x
  of Section 3.2, with M = F^-1 diag(mu) F.

Parity: pinned through the tests of the solvers (KKT -> 0 at the common
limit of NCS, PDHG and ADMM) and the Lemma (monotone) invariant.
"""
from __future__ import annotations

import numpy as np
from scipy.special import gammaln

from . import prox
from .problems import Params, Problem


def tv(prob: Problem, x: np.ndarray) -> float:
    g = prob.D @ x
    n = prob.n
    if prob.tv == "aniso":
        return float(np.abs(g).sum())
    return float(np.sqrt(g[:n] ** 2 + g[n:] ** 2).sum())


def data_term(prob: Problem, proj: np.ndarray) -> float:
    """g_data(E x) given proj = E x."""
    if prob.kind == "ct":
        r = proj - prob.b
        return 0.5 * float(r @ r)
    y = proj + prob.bg
    b = prob.b
    pos = b > 0
    if np.any(y[pos] <= 0):
        return float("inf")
    # b_i = 0: l = y_i on its domain y_i >= 0, evaluated as y_i for every y_i
    val = np.where(pos, y - b * np.log(np.where(pos, y, 1.0)), y) + gammaln(b + 1.0)
    return float(val.sum())


def objective(prob: Problem, x: np.ndarray) -> float:
    return data_term(prob, prob.E @ x) + prob.lam * tv(prob, x)


def stacked_A(prob: Problem, par: Params, positivity: bool = False):
    """Callables for A = [E; (beta/alpha) D] and A^T, and the offset b~ = [b; 0] (CT)
    or [-r; 0] (PET, where the data block is l(. + r) with zero offset).  With
    ``positivity`` A gains the rows I of the constraint x >= 0 (remark in
    Section 4.2) and b~ a zero block."""
    ratio = par.beta / par.alpha
    m, n = prob.m, prob.n

    def A(x):
        parts = [prob.E @ x, ratio * (prob.D @ x)]
        if positivity:
            parts.append(x)
        return np.concatenate(parts)

    def At(y):
        z = prob.Et @ y[:m] + ratio * (prob.Dt @ y[m:m + 2 * n])
        return z + y[m + 2 * n:] if positivity else z

    head = prob.b if prob.kind == "ct" else -prob.bg
    btil = np.concatenate([head, np.zeros((3 if positivity else 2) * n)])
    return A, At, btil


def prox_conj(prob: Problem, par: Params, positivity: bool = False):
    """prox_{alpha g*} for the stacked g, derived by the Moreau identity
    (Section 2, eq. Moreau) from the primal proximal maps of g (with
    ``positivity``, the indicator of x >= 0 on the third block, whose primal
    prox is max(., 0))."""
    a = par.alpha
    m, n = prob.m, prob.n
    s_tv = prob.lam * par.alpha / par.beta   # weight of |z| in g after scaling D by beta/alpha

    def data_prox(z, t):
        if prob.kind == "ct":
            return prox.prox_quadratic(z, t)
        return prox.prox_poisson(z, prob.b, t)

    def tv_prox(z, t):
        if prob.tv == "aniso":
            return prox.soft_threshold(z, t * s_tv)
        zh, zv = z[:n], z[n:]
        nrm = np.sqrt(zh * zh + zv * zv)
        shrink = np.maximum(nrm - t * s_tv, 0.0) / np.where(nrm > 0, nrm, 1.0)
        return np.concatenate([zh * shrink, zv * shrink])

    def pc(w):
        parts = [prox.moreau_conj(data_prox, w[:m], a), prox.moreau_conj(tv_prox, w[m:m + 2 * n], a)]
        if positivity:
            parts.append(prox.moreau_conj(lambda z, t: np.maximum(z, 0.0), w[m + 2 * n:], a))
        return np.concatenate(parts)

    return pc


def kkt(prob: Problem, par: Params, x: np.ndarray, y: np.ndarray) -> tuple[float, float]:
    A, At, btil = stacked_A(prob, par)
    pc = prox_conj(prob, par)
    r_dual = float(np.linalg.norm(At(y)))
    r_fix = float(np.linalg.norm(y - pc(y + par.alpha * (A(x) - btil))))
    return r_dual, r_fix


def quad_M(mu: np.ndarray, x: np.ndarray) -> float:
    """x^T M x with M = F^-1 diag(mu) F."""
    n_side = mu.shape[0]
    img = x.reshape(n_side, n_side)
    mx = np.real(np.fft.ifft2(mu * np.fft.fft2(img)))
    return float((img * mx).sum())


def d_seminorm_sq(prob: Problem, par: Params, mu: np.ndarray, dx: np.ndarray,
                  dy: np.ndarray) -> float:
    A, _, _ = stacked_A(prob, par)
    a = par.alpha
    adx = A(dx)
    r = dy - a * adx
    return float(r @ r) + a * quad_M(mu, dx) - a * a * float(adx @ adx)
