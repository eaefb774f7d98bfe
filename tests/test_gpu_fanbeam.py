"""GPU parity of the fan-beam path against the FP64 oracle, through the C ABI:
the projector and its matched backprojector, the eigenvalues of M with E^T E's
multiplier estimated from probes (eq. H-fan), and whole NCS and PDHG
trajectories.  Gates: FP64 operators rel <= 1e-11, FP32 <= 1e-5 (phantom) and
1e-4 (random data); eigenvalues rel <= 1e-9 (FP64) and 1e-6 (FP32: the probes
of an FP32 handle go through the library's FP64 kernels, so both precisions
run the same M up to the DC entry's FP32 |E 1|^2); trajectories as for the parallel beam: FP64 1e-10, FP32
rel-L2(x) <= 1e-4 and every objective within 1e-5."""
import functools

import numpy as np
import pytest
import torch

import ncs_inputs
from gpu_common import assert_converging, log, rel_l2
from oracle import fanbeam, operators, problems, solvers
from paper_1810_13100_amd import ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
DT = {"f32": torch.float32, "f64": torch.float64}
FAN = {"c64": (64, 60, 128, 120.0),     # 64^2, 60 views x 128 bins
       "ragged": (32, 37, 50, 47.0)}   # odd views, bins not a multiple of 64, source close to the image


@functools.lru_cache(maxsize=None)
def fan_E(key):
    return fanbeam.fan_matrix(fanbeam.FanGeometry(*FAN[key]))


def geometry(key):
    n, nv, nb, rs = FAN[key]
    return ncs.Geometry(n, nv, nb, beam=ncs.BEAM_FAN, source_radius=rs)


def fan_params(n, nv):
    # gamma = alpha N_v N / (2 pi): with the estimated multiplier, 0.3 of it (the
    # parallel-beam choice) makes NCS diverge on these problems
    alpha = 0.01
    c_eq = nv * n / (2.0 * np.pi)    # the views cover every line twice over a full turn
    return problems.Params(alpha, 3 * alpha, alpha * c_eq)


@pytest.mark.parametrize("key", ["c64", "ragged"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fan_operators_match_oracle(key, prec):
    n = FAN[key][0]
    E = fan_E(key)
    log(f"fan operators {key} {FAN[key]} {prec}")
    s = ncs.Solver(geometry(key), ncs.Params(0.01, 0.03, 1.0, 0.01), dtype=DT[prec])
    info = s.info()
    assert info["projector"] == 4 and info["backprojector"] == 4
    img = ncs_inputs.phantom(n, 3).ravel()
    fwd = s.forward(torch.tensor(img, dtype=DT[prec], device=DEV)).double().cpu().numpy()
    e1 = rel_l2(fwd, E @ img)
    y = np.random.default_rng(2).standard_normal(E.shape[0])
    back = s.adjoint(torch.tensor(y, dtype=DT[prec], device=DEV)).double().cpu().numpy()
    e2 = rel_l2(back, E.T @ y)
    log(f"  forward rel-L2 {e1:.2e}, adjoint rel-L2 {e2:.2e}")
    assert e1 <= (1e-11 if prec == "f64" else 1e-5)
    assert e2 <= (1e-11 if prec == "f64" else 1e-4)
    assert info["nnz"] == pytest.approx(E.nnz, rel=5e-3)
    s.close()


def test_fan_pair_is_adjoint():
    s = ncs.Solver(geometry("c64"), ncs.Params(0.01, 0.03, 1.0, 0.01), dtype=torch.float64)
    g = torch.Generator().manual_seed(5)
    x = torch.randn(64 * 64, generator=g, dtype=torch.float64).to(DEV)
    y = torch.randn(60 * 128, generator=g, dtype=torch.float64).to(DEV)
    lhs = float(torch.dot(s.forward(x), y))
    rhs = float(torch.dot(x, s.adjoint(y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    s.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-6)])
def test_fan_eigenvalues_match_the_probe_estimate(prec, tol):
    n, nv, nb, rs = FAN["c64"]
    E = fan_E("c64")
    par = fan_params(n, nv)
    h_e = fanbeam.probe_multiplier(lambda v: E.T @ (E @ v), n, 16)
    prob = problems.Problem("ct", "aniso", n, nv, nb, 0.01, E, operators.diff_2d(n), np.zeros(E.shape[0]),
                            np.zeros(E.shape[0]), np.zeros(n * n))
    ref = problems.eigenvalues(prob, problems.Params(par.alpha, par.beta, par.gamma, h_e=h_e))
    s = ncs.Solver(geometry("c64"), ncs.Params(par.alpha, par.beta, par.gamma, 0.01), dtype=DT[prec])
    mu = s.eigenvalues()
    s.close()
    err = float(np.max(np.abs(mu - ref) / np.abs(ref)))
    log(f"fan eigenvalues {prec}: max rel {err:.2e} (mu in [{ref.min():.3g}, {ref.max():.3g}])")
    assert err <= tol


@functools.lru_cache(maxsize=None)
def _fan_problem():
    n, nv, nb, rs = FAN["c64"]
    return problems.fan_problem(n, nv, nb, rs, 0, 0.01, E=fan_E("c64"))


@functools.lru_cache(maxsize=None)
def _fan_ref(method, iters):
    prob = _fan_problem()
    par0 = fan_params(64, 60)
    h_e = fanbeam.probe_multiplier(lambda v: prob.Et @ (prob.E @ v), 64, 16)
    par = problems.Params(par0.alpha, par0.beta, par0.gamma, h_e=h_e)
    if method == "ncs":
        tr = solvers.ncs(prob, par, iters)
        return tr.x, tr.obj, par
    import scipy.sparse.linalg as sla
    ratio2 = (par.beta / par.alpha) ** 2
    op = sla.LinearOperator((prob.n, prob.n), dtype=np.float64,
                            matvec=lambda v: prob.Et @ (prob.E @ v) + ratio2 * (prob.Dt @ (prob.D @ v)))
    gp = 1.01 * par.alpha * float(sla.eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0])
    x, _, obj = solvers.pdhg(prob, par, gp, iters)
    return x, obj, problems.Params(par.alpha, par.beta, gp)


@pytest.mark.parametrize("method", ["ncs", "pdhg"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fan_trajectory_matches_oracle(method, prec):
    K = 100
    prob = _fan_problem()
    x_ref, obj_ref, par = _fan_ref(method, K)
    assert_converging(obj_ref)
    p = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam,
                   method=ncs.METHOD_NCS if method == "ncs" else ncs.METHOD_PDHG)
    s = ncs.Solver(geometry("c64"), p, b=torch.tensor(prob.b, dtype=DT[prec], device=DEV), dtype=DT[prec])
    s.set_init()
    obj = s.iterate(K, record=True)
    x = s.x().double().cpu().numpy()
    s.close()
    ex = rel_l2(x, x_ref)
    ef = float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref)))
    log(f"fan {method} parity {prec}: rel-L2 x {ex:.2e}, max rel f {ef:.2e}")
    tx, tf = (1e-10, 1e-10) if prec == "f64" else (1e-4, 1e-5)
    assert ex <= tx and ef <= tf


def test_fan_restrictions():
    b = torch.zeros(60 * 128, device=DEV)
    for kw in ({"projector": 2}, {"method": ncs.METHOD_ADMM_CG}):
        with pytest.raises(ncs.NcsError) as e:
            ncs.Solver(geometry("c64"), ncs.Params(0.01, 0.03, 1.0, 0.01, **kw), b=b)
        assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    with pytest.raises(ncs.NcsError) as e:
        ncs.Solver(ncs.Geometry(64, 60, 128, beam=ncs.BEAM_FAN, source_radius=40.0),
                   ncs.Params(0.01, 0.03, 1.0, 0.01), b=b)
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    with pytest.raises(ncs.NcsError) as e:   # a batch mixing fan and parallel slices
        p = ncs.Params(0.01, 0.03, 1.0, 0.01)
        ncs.Batch([geometry("c64"), ncs.Geometry(64, 90, 92)], [p, p], [b, torch.zeros(90 * 92, device=DEV)])
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG


def test_fan_slices_in_a_batch():
    # two fan geometries of different sizes share every launch; each slice
    # follows its own oracle trajectory
    K = 100
    cases = []
    for key, seed in (("c64", 0), ("ragged", 1)):
        n, nv, nb, rs = FAN[key]
        prob = problems.fan_problem(n, nv, nb, rs, seed, 0.01, E=fan_E(key))
        par0 = fan_params(n, nv)
        h_e = fanbeam.probe_multiplier(lambda v, p=prob: p.Et @ (p.E @ v), n, 16)
        par = problems.Params(par0.alpha, par0.beta, par0.gamma, h_e=h_e)
        cases.append((key, prob, par, solvers.ncs(prob, par, K, record=False).x))
    geoms = [geometry(k) for k, _, _, _ in cases]
    params = [ncs.Params(par.alpha, par.beta, par.gamma, prob.lam) for _, prob, par, _ in cases]
    bs = [torch.tensor(prob.b, dtype=torch.float32, device=DEV) for _, prob, _, _ in cases]
    bat = ncs.Batch(geoms, params, bs)
    bat.set_init()
    bat.solve(K)
    errs = [rel_l2(bat.slice(i).x().double().cpu().numpy(), cases[i][3]) for i in range(len(cases))]
    info = bat.slice(0).info()
    bat.close()
    log(f"fan batch: rel-L2 x {errs}")
    assert info["projector"] == 4 and info["backprojector"] == 4
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fan_with_positivity_matches_oracle(prec):
    # the constraint x >= 0 (remark in Section 4.2) on a fan-beam problem: the
    # estimated multiplier raised by alpha, t = min(t + alpha xbar, 0)
    K = 100
    prob = _fan_problem()
    par0 = fan_params(64, 60)
    h_e = fanbeam.probe_multiplier(lambda v: prob.Et @ (prob.E @ v), 64, 16)
    par = problems.Params(par0.alpha, par0.beta, par0.gamma, h_e=h_e)
    ref = solvers.ncs(prob, par, K, positivity=True)
    assert_converging(ref.obj)
    free = solvers.ncs(prob, par, K, record=False)
    p = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, positivity=1)
    s = ncs.Solver(geometry("c64"), p, b=torch.tensor(prob.b, dtype=DT[prec], device=DEV), dtype=DT[prec])
    s.set_init()
    obj = s.iterate(K, record=True)
    x = s.x().double().cpu().numpy()
    t = s.t().double().cpu().numpy()
    s.close()
    assert free.x.min() < 0 and ref.t.min() < 0   # the constraint is active
    ex, et = rel_l2(x, ref.x), rel_l2(t, ref.t)
    ef = float(np.max(np.abs(obj - ref.obj) / np.abs(ref.obj)))
    log(f"fan with x >= 0, {prec}: rel-L2 x {ex:.2e}, t {et:.2e}, max rel f {ef:.2e}")
    if prec == "f64":
        assert max(ex, et, ef) <= 1e-10
    else:
        assert ex <= 1e-4 and et <= 1e-4 and ef <= 1e-5
