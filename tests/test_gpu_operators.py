"""GPU parity of the operators against the FP64 oracle, through the C ABI.

Tolerances.  In FP64 both sides evaluate the same geometry (Definition of the
Joseph model) in a different operation order, so they agree to ~1e-14; the
gate is 1e-11.  In FP32 the sampled coordinate xi of a tap carries an
absolute error of a few ulp of |xi| <= ~600 (<= ~1e-4, typically ~1e-5); the
interpolation weight moves by the same amount, which changes a ray sum only
where neighbouring pixels differ.  For piecewise-constant phantoms that gives
rel-L2 ~1e-6 (gate 1e-5); for white-noise images every tap is an edge (gate
1e-4).  Accumulation over <= 2N taps in FP32 adds ~sqrt(2N) 6e-8.
"""
import numpy as np
import pytest
import torch

from gpu_common import GEOMS, ct_params, ct_problem, joseph, log, pet_problem, rel_l2
from oracle import objective, operators, problems, projector
from paper_1810_13100_amd import ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
DT = {"f32": torch.float32, "f64": torch.float64}


def _solver(geom, dtype, b=None, par=None, data=ncs.DATA_QUADRATIC, tv=ncs.TV_ANISO, lam=0.01, bg=None,
            projector=0, backprojector=0):
    n, na, ns = geom
    if par is None:
        par = ct_params(n, na)
    p = ncs.Params(par.alpha, par.beta, par.gamma, lam, data_term=data, tv_term=tv,
                   c_r=par.c_r or 0.0, mu_dc=par.mu_dc or 0.0, projector=projector, backprojector=backprojector)
    tb = None if b is None else torch.tensor(b, dtype=dtype, device=DEV)
    tbg = None if bg is None else torch.tensor(bg, dtype=dtype, device=DEV)
    return ncs.Solver(ncs.Geometry(n, na, ns), p, b=tb, bg=tbg, dtype=dtype)


def _phantom(n, seed=0):
    import ncs_inputs
    return ncs_inputs.phantom(n, seed).ravel()


@pytest.mark.parametrize("key", ["tiny", "c1", "c4s", "c3", "c4m", "c2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("projector", [1, 2, 3])
def test_forward_matches_oracle(key, prec, projector):
    # the three forward-projector kernels (1: LDS-staged row windows, 2: direct
    # loads, 3: two rays per lane with 16-byte loads)
    geom = GEOMS[key]
    log(f"forward parity {key} {geom} {prec} projector {projector}")
    E = joseph(*geom)
    s = _solver(geom, DT[prec], projector=projector)
    assert s.info()["projector"] == projector
    for img, tol32 in ((_phantom(geom[0]), 1e-5), (np.random.default_rng(1).standard_normal(E.shape[1]), 1e-4)):
        ref = E @ img
        out = s.forward(torch.tensor(img, dtype=DT[prec], device=DEV)).double().cpu().numpy()
        err = rel_l2(out, ref)
        log(f"  rel-L2 {err:.2e}")
        assert err <= (1e-11 if prec == "f64" else tol32), err
    s.close()


@pytest.mark.parametrize("key", ["tiny", "c1", "c4s", "c3", "c4m", "c2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bproj", [1, 2, 3])
def test_adjoint_matches_oracle(key, prec, bproj):
    # the three backprojector kernels (1: LDS-staged detector windows, 2: direct
    # loads, 3: 2 x 2 pixels per lane with 16-byte loads)
    geom = GEOMS[key]
    log(f"adjoint parity {key} {geom} {prec} backprojector {bproj}")
    E = joseph(*geom)
    s = _solver(geom, DT[prec], backprojector=bproj)
    assert s.info()["backprojector"] == bproj
    rng = np.random.default_rng(2)
    for y, tol32 in ((E @ _phantom(geom[0], 3), 1e-5), (rng.standard_normal(E.shape[0]), 1e-4)):
        ref = E.T @ y
        out = s.adjoint(torch.tensor(y, dtype=DT[prec], device=DEV)).double().cpu().numpy()
        err = rel_l2(out, ref)
        log(f"  rel-L2 {err:.2e}")
        assert err <= (1e-11 if prec == "f64" else tol32), err
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("proj,bproj", [(1, 1), (2, 2), (3, 3), (2, 1)])
def test_large_slice_sampled_angles(prec, proj, bproj):
    # 512^2 with 717 x 520 (largest slice of the uneven batch): whole rows of E
    # for sampled angles, including 0, the 45-degree ties and pi/2.
    n, na, ns = 512, 717, 520
    angles = [0, 1, 179, 180, 181, 358, 359, 537, 538, 716]
    log(f"sampled-angle parity 512 {prec} projector {proj} backprojector {bproj}")
    E = projector.joseph_matrix(n, na, ns, angles=angles)
    s = _solver((n, na, ns), DT[prec], projector=proj, backprojector=bproj)
    img = _phantom(n, 5)
    out = s.forward(torch.tensor(img, dtype=DT[prec], device=DEV)).double().cpu().numpy()
    ref = E @ img
    rows = np.concatenate([np.arange(a * ns, (a + 1) * ns) for a in angles])
    err = rel_l2(out[rows], ref[rows])
    log(f"  forward rel-L2 {err:.2e}")
    assert err <= (1e-11 if prec == "f64" else 1e-5)
    y = np.zeros(na * ns)
    y[rows] = np.random.default_rng(3).standard_normal(rows.size)
    back = s.adjoint(torch.tensor(y, dtype=DT[prec], device=DEV)).double().cpu().numpy()
    err = rel_l2(back, E.T @ y)
    log(f"  adjoint rel-L2 {err:.2e}")
    assert err <= (1e-11 if prec == "f64" else 1e-4)
    s.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_gpu_pair_is_adjoint(prec, tol):
    geom = GEOMS["c2"]
    s = _solver(geom, DT[prec])
    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.randn(geom[0] ** 2, generator=g, dtype=torch.float64).to(DEV, DT[prec])
    y = torch.randn(geom[1] * geom[2], generator=g, dtype=torch.float64).to(DEV, DT[prec])
    lhs = float((s.forward(x).double() * y.double()).sum())
    rhs = float((x.double() * s.adjoint(y).double()).sum())
    scale = float(s.forward(x).double().norm() * y.double().norm())
    log(f"adjoint identity {prec}: {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= tol * scale
    s.close()


@pytest.mark.parametrize("key", ["tiny", "c1", "c3", "c2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_circulant_solve_matches_oracle(key, prec):
    geom = GEOMS[key]
    prob = ct_problem(key) if key != "tiny" else problems.ct_problem(*geom, 0, 0.01, E=joseph(*geom))
    par = ct_params(geom[0], geom[1])
    s = _solver(geom, DT[prec], b=prob.b, par=par, lam=prob.lam)
    mu_ref = problems.eigenvalues(prob, par)
    # the DC entry uses |E 1|^2 from the handle's own projector in its own
    # precision (FP32: ~1e-7 relative); every other entry is host double
    np.testing.assert_allclose(s.eigenvalues(), mu_ref, rtol=1e-12 if prec == "f64" else 1e-6)
    np.testing.assert_allclose(s.eigenvalues().ravel()[1:], mu_ref.ravel()[1:], rtol=1e-13)
    h = problems.multiplier(prob, par)
    w = np.random.default_rng(4).standard_normal(geom[0] ** 2)
    ref = operators.apply_circulant(h, w.reshape(geom[0], geom[0])).ravel()
    out = s.apply_minv(torch.tensor(w, dtype=DT[prec], device=DEV)).double().cpu().numpy()
    err = rel_l2(out, ref)
    log(f"M^+ parity {key} {prec}: {err:.2e}")
    assert err <= (1e-12 if prec == "f64" else 2e-6)
    s.close()


def test_circulant_solve_1024():
    n = 1024
    base = ct_params(n, 8)
    par = problems.Params(base.alpha, base.beta, base.gamma, c_r=2000.0, mu_dc=5e4)
    s = _solver((n, 8, 16), torch.float64, par=par)
    mu = operators.ncs_eigenvalues(n, par.alpha, par.beta, par.gamma, par.c_r, par.mu_dc)
    np.testing.assert_allclose(s.eigenvalues(), mu, rtol=1e-13)
    w = np.random.default_rng(5).standard_normal(n * n)
    h = operators.pseudo_inverse_diag(mu)
    ref = operators.apply_circulant(h, w.reshape(n, n)).ravel()
    out = s.apply_minv(torch.tensor(w, dtype=torch.float64, device=DEV)).cpu().numpy()
    assert rel_l2(out, ref) <= 1e-12
    s.close()


@pytest.mark.parametrize("kind", ["ct", "ct_iso", "pet"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_objective_matches_oracle(kind, prec):
    if kind == "pet":
        prob = pet_problem("c3")
        data, tv = ncs.DATA_POISSON, ncs.TV_ISO
    else:
        prob = ct_problem("c1", tv="iso" if kind == "ct_iso" else "aniso")
        data, tv = ncs.DATA_QUADRATIC, ncs.TV_ISO if kind == "ct_iso" else ncs.TV_ANISO
    geom = (prob.n_side, prob.n_angles, prob.n_bins)
    s = _solver(geom, DT[prec], b=prob.b, bg=prob.bg if kind == "pet" else None, data=data, tv=tv, lam=prob.lam)
    for x in (prob.x_true, 0.5 * prob.x_true + 0.1):
        ref = objective.objective(prob, x)
        out = s.objective(torch.tensor(x, dtype=DT[prec], device=DEV))
        log(f"objective {kind} {prec}: {out} vs {ref}")
        assert abs(out - ref) <= (1e-11 if prec == "f64" else 2e-6) * abs(ref)
    s.close()


@pytest.mark.parametrize("key", ["tiny", "c1", "c4s", "c2"])
def test_nonzero_count_matches_oracle(key):
    # nnz(E) counted on the host at setup versus the stored entries of the
    # oracle's CSR E.  Where xi is an integer in exact arithmetic (theta = pi/2,
    # where cos is 6e-17 in double) one side may see f = 0 and the other
    # f = 1e-15, so a tap of weight ~1e-15 is counted by one side only.
    geom = GEOMS[key]
    s = _solver(geom, torch.float32)
    ours, ref = s.info()["nnz"], joseph(*geom).nnz
    assert abs(ours - ref) <= 5e-3 * ref, (ours, ref)
    s.close()


def test_autotuner_times_both_projectors():
    s = _solver(GEOMS["c2"], torch.float32)
    inf = s.info()
    pms = inf["projector_ms"]
    log(f"projector autotune: LDS {pms[0]:.4f} ms, direct {pms[1]:.4f} ms, pairs {pms[2]:.4f} ms "
        f"-> {inf['projector']}")
    assert all(t > 0 for t in pms)
    assert inf["projector"] == 1 + int(np.argmin(pms))
    bms = inf["backprojector_ms"]
    log(f"backprojector autotune: LDS {bms[0]:.4f} ms, direct {bms[1]:.4f} ms, quad {bms[2]:.4f} ms "
        f"-> {inf['backprojector']}")
    assert all(t > 0 for t in bms)
    assert inf["backprojector"] == 1 + int(np.argmin(bms))
    s.close()
