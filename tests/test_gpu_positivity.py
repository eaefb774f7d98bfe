"""GPU parity of the positivity-constrained iteration (the remark in Section 4.2:
A gains the rows I with the indicator of x >= 0, a dual t updated as
t = min(t + alpha xbar, 0), the backprojection gains alpha t and M is raised
by alpha) against the FP64 oracle, through the C ABI.

Gates are those of the unconstrained trajectories: FP64 rel-L2(x^K) and every
objective within 1e-10; FP32 rel-L2(x^K) <= 1e-4 and objectives within 1e-5.
The dual t is compared at the x gate.  The constraint is active in every
case: the unconstrained iterates go negative on the background.
"""
import numpy as np
import pytest
import torch

from gpu_common import ct_params, ct_problem, log, pet_problem, rel_l2
from oracle import solvers
from paper_1810_13100_amd import ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
DT = {"f32": torch.float32, "f64": torch.float64}
TOL = {"f64": (1e-10, 1e-10), "f32": (1e-4, 1e-5)}


def _case(kind):
    if kind == "ct":
        return ct_problem("c1"), ct_params(64, 90), (64, 90, 92), 200
    return pet_problem("c3"), ct_params(128, 180, alpha=1.0, ratio=3.0, g=1.0), (128, 180, 185), 100


def _params(prob, par, **kw):
    data = ncs.DATA_POISSON if prob.kind == "pet" else ncs.DATA_QUADRATIC
    tv = ncs.TV_ISO if prob.tv == "iso" else ncs.TV_ANISO
    return ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, c_r=par.c_r or 0.0, mu_dc=par.mu_dc or 0.0,
                      data_term=data, tv_term=tv, positivity=1, **kw)


def _solver(prob, p, geom, dtype):
    b = torch.tensor(prob.b, dtype=dtype, device=DEV)
    bg = torch.tensor(prob.bg, dtype=dtype, device=DEV) if prob.kind == "pet" else None
    return ncs.Solver(ncs.Geometry(*geom), p, b=b, bg=bg, dtype=dtype)


_ref = {}


def _oracle(kind):
    if kind not in _ref:
        prob, par, _, K = _case(kind)
        _ref[kind] = (solvers.ncs(prob, par, K, positivity=True), solvers.ncs(prob, par, K))
    return _ref[kind]


@pytest.mark.parametrize("kind", ["ct", "pet"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_positivity_trajectory_matches_oracle(kind, prec):
    prob, par, geom, K = _case(kind)
    ref, free = _oracle(kind)
    log(f"positivity parity {kind} {geom} {prec}, {K} iterations")
    s = _solver(prob, _params(prob, par), geom, DT[prec])
    s.set_init()
    obj = s.iterate(K, record=True)
    x = s.x().double().cpu().numpy()
    t = s.t().double().cpu().numpy()
    s.close()
    assert free.x.min() < -1e-3 * free.x.max() and ref.t.min() < 0   # the constraint is active
    ex, et = rel_l2(x, ref.x), rel_l2(t, ref.t)
    fin = np.isfinite(ref.obj)
    assert np.array_equal(np.isfinite(obj), fin)
    ef = float(np.max(np.abs(obj[fin] - ref.obj[fin]) / np.abs(ref.obj[fin])))
    log(f"  rel-L2 x {ex:.2e}, t {et:.2e}, max rel f {ef:.2e}; min x {x.min():.3e} "
        f"(unconstrained {free.x.min():.3e})")
    tx, tf = TOL[prec]
    assert ex <= tx and et <= tx and ef <= tf
    assert t.max() <= 0.0


def test_positivity_pdhg_matches_oracle():
    # method = PDHG with the constraint: M = gamma I on A' = [E; (beta/alpha) D; I]
    import scipy.sparse.linalg as sla
    prob, par, geom, _ = _case("ct")
    ratio2 = (par.beta / par.alpha) ** 2
    op = sla.LinearOperator((prob.n, prob.n), dtype=np.float64,
                            matvec=lambda v: prob.Et @ (prob.E @ v) + ratio2 * (prob.Dt @ (prob.D @ v)) + v)
    gp = 1.01 * par.alpha * float(sla.eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0])
    K = 150
    x_ref, y_ref, obj_ref = solvers.ncs_generic(prob, par, lambda z: z / gp, K, positivity=True)
    p = ncs.Params(par.alpha, par.beta, gp, prob.lam, method=ncs.METHOD_PDHG, positivity=1)
    s = _solver(prob, p, geom, torch.float64)
    s.set_init()
    obj = s.iterate(K, record=True)
    x = s.x().double().cpu().numpy()
    t = s.t().double().cpu().numpy()
    s.close()
    ex, et = rel_l2(x, x_ref), rel_l2(t, y_ref[prob.m + 2 * prob.n:])
    ef = float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref)))
    log(f"PDHG with x >= 0, f64: rel-L2 x {ex:.2e}, t {et:.2e}, max rel f {ef:.2e}")
    assert ex <= 1e-10 and et <= 1e-10 and ef <= 1e-10


def test_positivity_checkpoint_includes_t():
    prob, par, geom, _ = _case("ct")
    p = _params(prob, par, projector=2, backprojector=1)   # the same kernels in both handles
    a = _solver(prob, p, geom, torch.float32)
    a.set_init()
    a.iterate(30)
    blob = a.get_state()
    a.iterate(30)
    b = _solver(prob, p, geom, torch.float32)
    b.set_state(blob)
    b.iterate(30)
    assert torch.equal(b.x().cpu(), a.x().cpu())
    assert torch.equal(b.t().cpu(), a.t().cpu())
    a.close()
    b.close()


def test_positivity_slice_in_a_batch():
    # one constrained and one unconstrained slice share every launch
    prob, par, geom, K = _case("ct")
    ref, free = _oracle("ct")
    p_pos = _params(prob, par, projector=2, backprojector=2)
    p_free = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, projector=2, backprojector=2)
    b = torch.tensor(prob.b, dtype=torch.float32, device=DEV)
    bat = ncs.Batch([ncs.Geometry(*geom)] * 2, [p_pos, p_free], [b, b.clone()])
    bat.set_init()
    bat.solve(K)
    xs = [bat.slice(i).x().double().cpu().numpy() for i in range(2)]
    t = bat.slice(0).t().double().cpu().numpy()
    bat.close()
    e0, e1, et = rel_l2(xs[0], ref.x), rel_l2(xs[1], free.x), rel_l2(t, ref.t)
    log(f"batch: constrained slice rel-L2 x {e0:.2e}, t {et:.2e}; unconstrained slice {e1:.2e}")
    assert e0 <= 1e-4 and e1 <= 1e-4 and et <= 1e-4


def test_positivity_rejected_with_admm():
    prob, par, geom, _ = _case("ct")
    p = _params(prob, par, method=ncs.METHOD_ADMM_CG)
    with pytest.raises(ncs.NcsError) as e:
        _solver(prob, p, geom, torch.float32)
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    s = _solver(prob, ncs.Params(par.alpha, par.beta, par.gamma, prob.lam), geom, torch.float32)
    with pytest.raises(ncs.NcsError):
        s.t()
    s.close()
