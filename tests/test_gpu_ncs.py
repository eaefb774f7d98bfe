"""GPU parity of whole NCS trajectories against the FP64 oracle, through the C ABI,
plus the driver's behaviour (stopping, checkpoints, determinism, errors).

Gates: with the FP64 build of the kernels, rel-L2(x^K) <= 1e-10 and every
objective f(x^k) within 1e-10 relative -- the same arithmetic up to rounding
order.  With FP32 iterates: rel-L2(x^K) <= 1e-4 and |f - f_ref| <= 1e-5 |f_ref|
at every k <= K (the tolerances the method's FP32 build is held to).
"""
import math

import numpy as np
import pytest
import torch

import ncs_inputs
from gpu_common import GEOMS, assert_converging, ct_params, ct_problem, joseph, log, oracle_ncs, pet_problem, rel_l2
from oracle import problems, solvers
from paper_1810_13100_amd import ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
DT = {"f32": torch.float32, "f64": torch.float64}
TOL = {"f64": (1e-10, 1e-10), "f32": (1e-4, 1e-5)}


def make_solver(prob, par, dtype, check_every=50, diverge_checks=0, projector=0, graph_chunk=0, dual_ramp=0.0,
                backprojector=0):
    data = ncs.DATA_POISSON if prob.kind == "pet" else ncs.DATA_QUADRATIC
    tv = ncs.TV_ISO if prob.tv == "iso" else ncs.TV_ANISO
    p = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, c_r=par.c_r or 0.0, mu_dc=par.mu_dc or 0.0,
                   data_term=data, tv_term=tv, check_every=check_every, diverge_checks=diverge_checks,
                   projector=projector, graph_chunk=graph_chunk, dual_ramp=dual_ramp, backprojector=backprojector)
    b = torch.tensor(prob.b, dtype=dtype, device=DEV)
    bg = torch.tensor(prob.bg, dtype=dtype, device=DEV) if prob.kind == "pet" else None
    return ncs.Solver(ncs.Geometry(prob.n_side, prob.n_angles, prob.n_bins), p, b=b, bg=bg, dtype=dtype)


def pet_params(n_side, n_angles):
    return ct_params(n_side, n_angles, alpha=1.0, ratio=3.0, g=1.0)


def check_trajectory(prob, par, iters, prec, **kw):
    ref = oracle_ncs(prob, par, iters)
    assert_converging(ref.obj)
    s = make_solver(prob, par, DT[prec], **kw)
    s.set_init()
    obj = s.iterate(iters, record=True)
    x = s.x().double().cpu().numpy()
    u = s.u().double().cpu().numpy()
    s.close()
    ex = rel_l2(x, ref.x)
    eu = rel_l2(u, ref.u)
    fin = np.isfinite(ref.obj)
    assert np.array_equal(np.isfinite(obj), fin)
    ef = float(np.max(np.abs(obj[fin] - ref.obj[fin]) / np.abs(ref.obj[fin]))) if fin.any() else 0.0
    log(f"  {prec} K={iters}: rel-L2 x {ex:.2e}, u {eu:.2e}, max rel f {ef:.2e}")
    tx, tf = TOL[prec]
    assert ex <= tx, ex
    assert ef <= tf, ef
    return ex, ef


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("projector,backprojector,graph_chunk", [(1, 1, -1), (2, 2, -1), (3, 3, -1), (2, 1, -1),
                                                                 (0, 0, 0), (2, 1, 7), (3, 2, 7), (3, 1, 7)])
def test_ct_64_200_iterations(prec, projector, backprojector, graph_chunk):
    # both projector and backprojector kernels, direct launches and replayed
    # HIP graphs (a largest chunk of 7 keeps graphs of 1, 2 and 4 iterations)
    prob = ct_problem("c1")
    log(f"NCS parity 64^2 CT, 200 iterations, {prec}, projector {projector}, backprojector {backprojector}, "
        f"graph chunk {graph_chunk}")
    check_trajectory(prob, ct_params(64, 90), 200, prec, projector=projector, backprojector=backprojector,
                     graph_chunk=graph_chunk)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ct_ragged_tiny_geometry(prec):
    geom = GEOMS["tiny"]
    prob = problems.ct_problem(*geom, 1, 0.05, E=joseph(*geom))
    log(f"NCS parity tiny {geom}, {prec}")
    check_trajectory(prob, ct_params(geom[0], geom[1], alpha=0.05), 150, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ct_isotropic_tv(prec):
    prob = ct_problem("c1", seed=2, lam=0.5, tv="iso")
    log(f"NCS parity 64^2 CT isotropic TV, {prec}")
    check_trajectory(prob, ct_params(64, 90), 150, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_pet_128(prec):
    prob = pet_problem("c3")
    log(f"NCS parity 128^2 PET, 100 iterations, {prec}")
    check_trajectory(prob, pet_params(128, 180), 100, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ct_256_full_size(prec):
    prob = ct_problem("c2")
    log(f"NCS parity 256^2 CT (360 x 367), 100 iterations, {prec}")
    check_trajectory(prob, ct_params(256, 360, alpha=2.4e-3), 100, prec)


def test_checkpoint_resume_is_bitwise():
    # both handles use the same kernels (the setup timing could pick different ones)
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    a = make_solver(prob, par, torch.float32, projector=2, backprojector=1)
    a.set_init()
    a.iterate(40)
    blob = a.get_state()
    a.iterate(40)
    xa = a.x().cpu()
    b = make_solver(prob, par, torch.float32, projector=2, backprojector=1)
    b.set_state(blob)
    assert b.iteration() == 40
    b.iterate(40)
    assert torch.equal(b.x().cpu(), xa)
    assert torch.equal(b.u().cpu(), a.u().cpu())
    assert b.iteration() == a.iteration() == 80
    a.close()
    b.close()


def test_graph_replay_serves_every_count():
    # the same kernels launched directly and through the power-of-two graphs,
    # over counts that use every graph level and repeats of the largest
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    counts = [1, 2, 3, 5, 20, 31, 33, 64, 7, 1]
    outs = []
    for chunk in (-1, 0, 5):
        s = make_solver(prob, par, torch.float32, projector=2, backprojector=1, graph_chunk=chunk)
        s.set_init()
        obj = np.concatenate([s.iterate(k, record=True) for k in counts])
        assert s.iteration() == sum(counts)
        outs.append((s.x().cpu(), s.u().cpu(), obj))
        s.close()
    for x, u, obj in outs[1:]:
        assert torch.equal(x, outs[0][0])
        assert torch.equal(u, outs[0][1])
        assert np.array_equal(obj, outs[0][2])


def test_runs_are_deterministic():
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    outs = []
    for _ in range(2):   # same kernels in both runs (the setup timing could pick different ones)
        s = make_solver(prob, par, torch.float32, projector=2, backprojector=1)
        s.set_init()
        obj = s.iterate(30, record=True)
        outs.append((s.x().cpu(), obj))
        s.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_solve_stops_at_first_target_crossing():
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    ref = oracle_ncs(prob, par, 200)
    target = float(ref.obj[120]) * (1 + 1e-12)   # above the oracle value: rounding cannot move the crossing
    first = int(np.nonzero(ref.obj <= target)[0][0]) + 1
    s = make_solver(prob, par, torch.float64, check_every=37)
    s.set_init()
    st, iters, f = s.solve(500, target)
    log(f"solve: status {st}, {iters} iterations (oracle {first}), f {f}")
    assert st == ncs.NCS_OK
    assert iters == first
    assert abs(f - ref.obj[first - 1]) <= 1e-10 * abs(f)
    # the chunk continues past the stop without touching the state
    x = s.x().cpu().numpy()
    np.testing.assert_allclose(x, oracle_ncs(prob, par, first).x, rtol=0, atol=1e-9 * np.abs(x).max())
    st2, iters2, _ = s.solve(3, math.nan)
    assert st2 == ncs.NCS_NOT_CONVERGED and iters2 == 3
    assert s.iteration() == first + 3
    s.close()


def test_solve_stops_on_the_fixed_point_residual():
    """fp_residual_tol: the host checks |x^k - x^{k-1}| <= tol |x^k| every
    check_every iterations; the oracle's iterates, continued chunk by chunk,
    fix the first check that passes."""
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    every, checks = 10, 30
    res, x, u, v = [], None, None, None
    for _ in range(checks):
        t = solvers.ncs(prob, par, every, x0=x, u0=u, v0=v, record=False)
        x, u, v = t.x, t.u, t.v
        res.append(float(np.linalg.norm(t.x - t.x_prev) / np.linalg.norm(t.x)))
    res = np.array(res)
    tol = float(res[14]) * (1 + 1e-7)
    first = int(np.nonzero(res <= tol)[0][0])
    assert np.all(np.abs(res[:first] - tol) > 1e-6 * tol)   # no check decided by rounding
    s = make_solver(prob, par, torch.float64, check_every=every)
    s.set_init()
    st, iters, f = s.solve(every * checks, math.nan, tol)
    log(f"residual stop: status {st}, {iters} iterations (oracle {every * (first + 1)}), "
        f"residuals at the checks {res[:first + 1]}")
    assert st == ncs.NCS_OK and iters == every * (first + 1)
    xg = s.x().cpu().numpy()
    np.testing.assert_allclose(xg, oracle_ncs(prob, par, iters).x, rtol=0, atol=1e-9 * np.abs(xg).max())
    # a tolerance no check reaches runs the whole budget; NaN is rejected
    s.set_init()
    st, iters, _ = s.solve(50, math.nan, 1e-300)
    assert st == ncs.NCS_NOT_CONVERGED and iters == 50
    with pytest.raises(ncs.NcsError):
        s.solve(10, math.nan, math.nan)
    s.close()


def test_objective_history_matches_iterate():
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    s = make_solver(prob, par, torch.float64)
    s.set_init()
    obj = s.iterate(25, record=True)
    np.testing.assert_array_equal(s.objectives(0, 25), obj)
    np.testing.assert_array_equal(s.objectives(10, 5), obj[10:15])
    with pytest.raises(ncs.NcsError):
        s.objectives(20, 10)
    s.close()


def test_warm_start_duals_and_progress():
    # Duals from the optimality conditions (Section 3.2, Fact on fixed points):
    # for CT u* = E x* - b exactly; started there NCS stays at the optimal
    # objective to ~1e-4 within 20 iterations, whereas the cold start is still
    # orders of magnitude away.
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    ref = oracle_ncs(prob, par, 2000)
    s = make_solver(prob, par, torch.float64)
    s.set_init(torch.tensor(ref.x, dtype=torch.float64, device=DEV), dual_from_x0=True)
    u0 = s.u().cpu().numpy()
    np.testing.assert_allclose(u0, prob.E @ ref.x - prob.b, rtol=0, atol=1e-10 * np.abs(u0).max())
    warm = s.iterate(20, record=True)
    s.set_init()
    cold = s.iterate(20, record=True)
    fstar = float(np.min(ref.obj))
    log(f"warm start from the limit: gap after 20 {abs(warm[-1] - fstar) / fstar:.2e}, cold {abs(cold[-1] - fstar) / fstar:.2e}")
    assert abs(warm[-1] - fstar) <= 1e-3 * fstar
    assert cold[-1] - fstar > 100 * abs(warm[-1] - fstar)
    s.close()


def test_invalid_arguments_are_rejected():
    par = ct_params(64, 90)
    for geom in ((48, 10, 50), (64, 0, 50), (64, 10, 1), (2048, 4, 8)):
        with pytest.raises(ncs.NcsError) as e:
            ncs.Solver(ncs.Geometry(*geom), ncs.Params(par.alpha, par.beta, par.gamma, 0.01))
        assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    with pytest.raises(ncs.NcsError) as e:
        ncs.Solver(ncs.Geometry(64, 90, 92), ncs.Params(-1.0, 1.0, 1.0, 0.01))
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    s = ncs.Solver(ncs.Geometry(64, 90, 92), ncs.Params(par.alpha, par.beta, par.gamma, 0.01))
    with pytest.raises(ncs.NcsError) as e:
        s.iterate(1)                       # operator-only handle: no data
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        s.forward(torch.zeros(10, device=DEV))
    with pytest.raises(ncs.NcsError):
        s.set_state(b"not a state")
    s.close()


def test_nan_data_reports_nonfinite():
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    b = prob.b.copy()
    b[100] = np.nan
    p = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam)
    s = ncs.Solver(ncs.Geometry(64, 90, 92), p, b=torch.tensor(b, dtype=torch.float32, device=DEV))
    s.set_init()
    with pytest.raises(ncs.NcsError) as e:
        s.solve(100)
    assert e.value.status == ncs.NCS_ERR_NONFINITE
    assert s.iteration() == 1        # stopped on the device after the first NaN objective
    s.close()


def test_a3_violation_is_reported_as_divergence():
    # gamma = 0 leaves M far from dominating alpha A^T A (A3 fails by ~950 alpha
    # at this size); the iterates blow up and the driver says so.
    prob = ct_problem("c1")
    par = problems.Params(0.01, 0.03, 0.0)
    s = make_solver(prob, par, torch.float32, check_every=20, diverge_checks=3)
    s.set_init()
    with pytest.raises(ncs.NcsError) as e:
        s.solve(5000)
    assert e.value.status in (ncs.NCS_ERR_DIVERGED, ncs.NCS_ERR_NONFINITE)
    s.close()


@pytest.mark.parametrize("kind", ["ct", "ct_iso", "pet"])
@pytest.mark.parametrize("tau", [0.0, 0.05])
def test_fixed_point_dual_init(kind, tau):
    # ncs_set_init with dual_from_x0 against the oracle's fixed-point duals
    if kind == "pet":
        prob, par = pet_problem("c3"), pet_params(128, 180)
    else:
        prob = ct_problem("c1") if kind == "ct" else ct_problem("c1", seed=2, lam=0.5, tv="iso")
        par = ct_params(64, 90)
    x0 = ncs_inputs.phantom(prob.n_side, 7).ravel()
    u_ref, v_ref = solvers.fixed_point_duals(prob, par, x0, tau)
    s = make_solver(prob, par, torch.float64, dual_ramp=tau)
    s.set_init(torch.tensor(x0, dtype=torch.float64, device=DEV), dual_from_x0=True)
    u = s.u().cpu().numpy()
    v = s.v().cpu().numpy()
    s.close()
    eu = np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref))
    ev = np.max(np.abs(v - v_ref)) / max(np.max(np.abs(v_ref)), 1e-300)
    log(f"dual init {kind} tau {tau}: max rel err u {eu:.1e}, v {ev:.1e}")
    assert eu <= 1e-10 and ev <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_pdhg_matches_oracle(prec):
    # method = PDHG runs the same kernels with M = gamma I (eq. PDHG)
    import scipy.sparse.linalg as sla
    prob = ct_problem("c1")
    par0 = ct_params(64, 90)
    ata = sla.LinearOperator((prob.n, prob.n), dtype=np.float64,
                             matvec=lambda x: prob.Et @ (prob.E @ x) + (par0.beta / par0.alpha) ** 2 * (prob.Dt @ (prob.D @ x)))
    lmax = float(sla.eigsh(ata, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0])
    gp = 1.01 * par0.alpha * lmax
    K = 200
    x_ref, y_ref, obj_ref = solvers.pdhg(prob, par0, gp, K)
    p = ncs.Params(par0.alpha, par0.beta, gp, prob.lam, method=ncs.METHOD_PDHG)
    dt = DT[prec]
    s = ncs.Solver(ncs.Geometry(64, 90, 92), p, b=torch.tensor(prob.b, dtype=dt, device=DEV), dtype=dt)
    s.set_init()
    obj = s.iterate(K, record=True)
    x = s.x().double().cpu().numpy()
    s.close()
    ex = rel_l2(x, x_ref)
    ef = float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref)))
    log(f"PDHG parity {prec}: rel-L2 x {ex:.2e}, max rel f {ef:.2e}")
    tx, tf = TOL[prec]
    assert ex <= tx and ef <= tf


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("precondition", [1, 0])
def test_admm_cg_matches_oracle(prec, precondition):
    # method = ADMM_CG: cg_iters CG steps per linear solve, the same number as the oracle
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    K, CG = 30, 5
    x_ref, _, obj_ref = solvers.admm_cg(prob, par, K, CG, precondition=bool(precondition))
    p = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, c_r=par.c_r or 0.0, mu_dc=par.mu_dc or 0.0,
                   method=ncs.METHOD_ADMM_CG, cg_iters=CG, cg_precondition=precondition)
    dt = DT[prec]
    b = torch.tensor(prob.b, dtype=dt, device=DEV)
    if prec == "f32" and not precondition:
        # plain CG amplifies FP32 rounding by about the condition number of
        # A^T A (~1e4 here); the library runs it in double precision only
        with pytest.raises(ncs.NcsError) as e:
            ncs.Solver(ncs.Geometry(64, 90, 92), p, b=b, dtype=dt)
        assert e.value.status == ncs.NCS_ERR_INVALID_ARG
        return
    s = ncs.Solver(ncs.Geometry(64, 90, 92), p, b=b, dtype=dt)
    s.set_init()
    obj = s.iterate(K, record=True)
    x = s.x().double().cpu().numpy()
    s.close()
    ex = rel_l2(x, x_ref)
    ef = float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref)))
    log(f"ADMM-CG parity {prec} precondition {precondition}: rel-L2 x {ex:.2e}, max rel f {ef:.2e}")
    tx, tf = (1e-9, 1e-10) if prec == "f64" else TOL[prec]
    assert ex <= tx and ef <= tf


def test_admm_cg_rejected_in_batches():
    prob = ct_problem("c1")
    par = ct_params(64, 90)
    p = ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, method=ncs.METHOD_ADMM_CG)
    b = torch.tensor(prob.b, dtype=torch.float32, device=DEV)
    with pytest.raises(ncs.NcsError) as e:
        ncs.Batch([ncs.Geometry(64, 90, 92)], [p], [b])
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
