"""GPU parity of the cone-beam path against the FP64 oracle, through the C ABI:
the projector and its voxel-driven adjoint, the eigenvalues of M with E^T E's
multiplier estimated from probes with the 3D DFT (eq. H-fan), the circulant
solve, and whole NCS and PDHG trajectories (x, u, v and every objective).

Gates: FP64 operators rel <= 1e-11 and adjointness to 1e-12; FP32 operators
<= 1e-5 (phantom) and 1e-4 (random data); eigenvalues FP64 <= 1e-9, FP32
<= 1e-6 (the probes of an FP32 handle go through the library's FP64 kernels;
only the DC entry's |E 1|^2 comes from the FP32 projector); trajectories FP64
x, u, v and f <= 1e-10; FP32 x <= 1e-4 and every f within 1e-5.  At the benchmark's size (256^2 x 64,
72 views x 64 rows x 368 bins) the rays of sampled views are compared with
the oracle's rows for those views, and the adjoint with the oracle's block
transpose on data supported on those views."""
import functools
import math

import numpy as np
import pytest
import torch

import ncs_inputs
from gpu_common import assert_converging, log, rel_l2
from oracle import conebeam
from paper_1810_13100_amd import cone, ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
DT = {"f32": torch.float32, "f64": torch.float64}
CONE = {"c32": (32, 16, 24, 48, 11, 60.0),                           # 32^2 x 16, 24 views x 11 rows x 48 bins
        "ragged": (16, 8, 7, 19, 4, 30.0),                           # odd views, even rows, 19 bins
        "wide": (64, 32, 30, 96, 16, 64 / math.sqrt(2.0) + 6.0),     # two bin blocks, slopes up to 2.7
        "flat": (16, 4, 9, 21, 5, 16 / math.sqrt(2.0) + 4.0),        # N_z = 4 (runs of 4 voxels), smallest R_s
        # tall detectors: the adjoint keeps up to 2048 rows' slopes in LDS and
        # reads them from global memory beyond that
        "rows2048": (16, 8, 2, 20, 2048, 24.0),
        "rows2056": (16, 8, 2, 20, 2056, 24.0),
        "rows2056z4": (16, 4, 2, 20, 2056, 24.0),
        "rows2056z16": (16, 16, 2, 20, 2056, 24.0),
        "rows2056z32": (16, 32, 2, 20, 2056, 24.0)}
BENCH = (256, 64, 72, 368, 64, 512.0)


@functools.lru_cache(maxsize=None)
def cone_E(key):
    return conebeam.cone_matrix(conebeam.ConeGeometry(*CONE[key]))


def geometry(key):
    return cone.ConeGeometry(*CONE[key])


def _params(**kw):
    return cone.ConeParams(0.01, 0.03, 1.0, 0.01, **kw)


@pytest.mark.parametrize("key", ["c32", "ragged", "wide", "flat", "rows2048", "rows2056", "rows2056z4", "rows2056z16",
                                 "rows2056z32"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cone_operators_match_oracle(key, prec):
    n, nz = CONE[key][0], CONE[key][1]
    E = cone_E(key)
    log(f"cone operators {key} {CONE[key]} {prec}")
    s = cone.ConeSolver(geometry(key), _params(method=ncs.METHOD_PDHG), dtype=DT[prec])
    vol = ncs_inputs.phantom3d(n, nz, 3).ravel()
    fwd = s.forward(torch.tensor(vol, dtype=DT[prec], device=DEV)).double().cpu().numpy()
    e1 = rel_l2(fwd, E @ vol)
    y = np.random.default_rng(2).standard_normal(E.shape[0])
    back = s.adjoint(torch.tensor(y, dtype=DT[prec], device=DEV)).double().cpu().numpy()
    e2 = rel_l2(back, E.T @ y)
    nnz = s.info()["nnz"]
    s.close()
    log(f"  forward rel-L2 {e1:.2e}, adjoint rel-L2 {e2:.2e}, nnz {nnz} (oracle {E.nnz})")
    assert nnz == pytest.approx(E.nnz, rel=1e-4)
    assert e1 <= (1e-11 if prec == "f64" else 1e-5)
    assert e2 <= (1e-11 if prec == "f64" else 1e-4)


def test_cone_handles_with_different_row_tables_coexist():
    """Two live handles whose adjoints launch the same kernel with different LDS
    (2048 and 4 detector rows in the table): the later setup leaves the earlier
    handle's launches valid."""
    log("cone handles: 2048-row table, then 4-row table, both live")
    big = cone.ConeSolver(geometry("rows2048"), _params(method=ncs.METHOD_PDHG), dtype=torch.float64)
    small = cone.ConeSolver(geometry("ragged"), _params(method=ncs.METHOD_PDHG), dtype=torch.float64)
    rng = np.random.default_rng(4)
    y_big = rng.standard_normal(big.geom.m)
    y_small = rng.standard_normal(small.geom.m)
    back_big = big.adjoint(torch.tensor(y_big, dtype=torch.float64, device=DEV)).cpu().numpy()
    back_small = small.adjoint(torch.tensor(y_small, dtype=torch.float64, device=DEV)).cpu().numpy()
    big.close()
    small.close()
    e_big = rel_l2(back_big, cone_E("rows2048").T @ y_big)
    e_small = rel_l2(back_small, cone_E("ragged").T @ y_small)
    log(f"  adjoint rel-L2 {e_big:.2e} (2048 rows), {e_small:.2e} (4 rows)")
    assert e_big <= 1e-11 and e_small <= 1e-11


def test_cone_pair_is_adjoint():
    g = geometry("c32")
    s = cone.ConeSolver(g, _params(method=ncs.METHOD_PDHG), dtype=torch.float64)
    gen = torch.Generator().manual_seed(5)
    x = torch.randn(g.n, generator=gen, dtype=torch.float64).to(DEV)
    y = torch.randn(g.m, generator=gen, dtype=torch.float64).to(DEV)
    lhs = float(torch.dot(s.forward(x), y))
    rhs = float(torch.dot(x, s.adjoint(y)))
    s.close()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@functools.lru_cache(maxsize=None)
def _problem():
    g = conebeam.ConeGeometry(*CONE["c32"])
    return conebeam.cone_problem(g, 0, 0.01, E=cone_E("c32"))


@functools.lru_cache(maxsize=None)
def _h_e():
    prob = _problem()
    return conebeam.probe_multiplier_3d(lambda v: prob.Et @ (prob.E @ v), prob.geom.shape, 16)


def _gamma():
    # gamma = 3.2 alpha N_v N / (2 pi): with the probe-estimated multiplier a
    # factor of 1 or 2 lets NCS diverge on volumes (M must dominate alpha A^T A)
    n, _, nv = CONE["c32"][:3]
    return 3.2 * 0.01 * nv * n / (2.0 * np.pi)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-6)])
def test_cone_eigenvalues_match_the_probe_estimate(prec, tol):
    prob = _problem()
    ref = conebeam.eigenvalues3d(prob, 0.01, 0.03, _gamma(), _h_e())
    s = cone.ConeSolver(geometry("c32"), cone.ConeParams(0.01, 0.03, _gamma(), 0.01), dtype=DT[prec])
    mu = s.eigenvalues()
    s.close()
    err = float(np.max(np.abs(mu - ref) / np.abs(ref)))
    log(f"cone eigenvalues {prec}: max rel {err:.2e} (mu in [{ref.min():.3g}, {ref.max():.3g}])")
    assert err <= tol


def test_cone_circulant_solve_matches_oracle():
    prob = _problem()
    mu = conebeam.eigenvalues3d(prob, 0.01, 0.03, _gamma(), _h_e())
    w = np.random.default_rng(7).standard_normal(prob.geom.shape)
    ref = np.real(np.fft.ifftn(np.fft.fftn(w) / mu))
    s = cone.ConeSolver(geometry("c32"), cone.ConeParams(0.01, 0.03, _gamma(), 0.01), dtype=torch.float64)
    got = s.apply_minv(torch.tensor(w.ravel(), device=DEV)).cpu().numpy().reshape(w.shape)
    s.close()
    err = rel_l2(got, ref)
    log(f"cone M^+ w, f64: rel-L2 {err:.2e}")
    assert err <= 1e-9


@functools.lru_cache(maxsize=None)
def _ref(method, iters):
    prob = _problem()
    a, be = 0.01, 0.03
    if method == "ncs":
        h = 1.0 / conebeam.eigenvalues3d(prob, a, be, _gamma(), _h_e())
        gam = _gamma()
    else:
        import scipy.sparse.linalg as sla
        ratio2 = (be / a) ** 2
        op = sla.LinearOperator((prob.n, prob.n), dtype=np.float64,
                                matvec=lambda v: prob.Et @ (prob.E @ v) + ratio2 * (prob.Dt @ (prob.D @ v)))
        gam = 1.01 * a * float(sla.eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0])
        h = np.full(prob.geom.shape, 1.0 / gam)
    x, u, v, obj = conebeam.ncs3d(prob, a, be, h, iters)
    return x, u, v, obj, gam


@pytest.mark.parametrize("method", ["ncs", "pdhg"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cone_trajectory_matches_oracle(method, prec):
    K = 60
    prob = _problem()
    x_ref, u_ref, v_ref, obj_ref, gam = _ref(method, K)
    assert_converging(obj_ref)
    p = cone.ConeParams(0.01, 0.03, gam, prob.lam, method=ncs.METHOD_NCS if method == "ncs" else ncs.METHOD_PDHG)
    s = cone.ConeSolver(geometry("c32"), p, b=torch.tensor(prob.b, dtype=DT[prec], device=DEV), dtype=DT[prec])
    s.set_init()
    obj = s.iterate(K, record=True)
    x = s.x().double().cpu().numpy()
    u = s.u().double().cpu().numpy()
    v = s.v().double().cpu().numpy()
    s.close()
    ex, eu, ev = rel_l2(x, x_ref), rel_l2(u, u_ref), rel_l2(v, v_ref)
    ef = float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref)))
    log(f"cone {method} parity {prec}: rel-L2 x {ex:.2e}, u {eu:.2e}, v {ev:.2e}, max rel f {ef:.2e}")
    if prec == "f64":
        assert max(ex, eu, ev, ef) <= 1e-10
    else:
        assert ex <= 1e-4 and ef <= 1e-5


def test_cone_runs_repeat_bit_for_bit():
    prob = _problem()
    b = torch.tensor(prob.b, dtype=torch.float32, device=DEV)
    outs = []
    for _ in range(2):
        s = cone.ConeSolver(geometry("c32"), cone.ConeParams(0.01, 0.03, _gamma(), prob.lam), b=b)
        s.set_init()
        obj = s.iterate(20, record=True)
        outs.append((s.x().cpu(), obj))
        s.close()
    assert torch.equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_cone_warm_start_from_x0():
    # set_init(x0) restarts from x0 with E x0 recomputed: the first objective
    # after K iterations from x0 equals the oracle's run from x0
    prob = _problem()
    x0 = ncs_inputs.phantom3d(32, 16, 0).ravel() * 0.5
    h = 1.0 / conebeam.eigenvalues3d(prob, 0.01, 0.03, _gamma(), _h_e())
    x_ref, _, _, obj_ref = conebeam.ncs3d(prob, 0.01, 0.03, h, 10, x0=x0)
    s = cone.ConeSolver(geometry("c32"), cone.ConeParams(0.01, 0.03, _gamma(), prob.lam),
                        b=torch.tensor(prob.b, device=DEV), dtype=torch.float64)
    s.set_init(torch.tensor(x0, device=DEV))
    obj = s.iterate(10, record=True)
    x = s.x().cpu().numpy()
    s.close()
    assert rel_l2(x, x_ref) <= 1e-10
    assert float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref))) <= 1e-10


def test_cone_benchmark_size_sampled_views():
    g = cone.ConeGeometry(*BENCH)
    og = conebeam.ConeGeometry(*BENCH)
    views = [5, 41]
    E_sub = conebeam.cone_matrix(og, views=views)
    vol = ncs_inputs.phantom3d(g.n_side, g.n_slices, 0).ravel()
    log(f"cone benchmark size {BENCH}: views {views}, {E_sub.nnz} oracle entries")
    s = cone.ConeSolver(g, _params(method=ncs.METHOD_PDHG), dtype=torch.float32)
    y = s.forward(torch.tensor(vol, dtype=torch.float32, device=DEV)).double().cpu().numpy()
    blk = g.n_rows * g.n_bins
    got = np.concatenate([y[a * blk:(a + 1) * blk] for a in views])
    e1 = rel_l2(got, E_sub @ vol)
    ysub = np.random.default_rng(3).standard_normal(len(views) * blk)
    yfull = np.zeros(g.m)
    for i, a in enumerate(views):
        yfull[a * blk:(a + 1) * blk] = ysub[i * blk:(i + 1) * blk]
    back = s.adjoint(torch.tensor(yfull, dtype=torch.float32, device=DEV)).double().cpu().numpy()
    e2 = rel_l2(back, E_sub.T @ ysub)
    s.close()
    log(f"  forward rel-L2 {e1:.2e}, adjoint rel-L2 {e2:.2e}")
    assert e1 <= 1e-5 and e2 <= 1e-4


def test_cone_rejects_bad_arguments():
    bad = [cone.ConeGeometry(32, 16, 24, 48, 11, 25.0),   # source inside the margin
           cone.ConeGeometry(32, 12, 24, 48, 11, 60.0),   # N_z not a power of two
           cone.ConeGeometry(32, 16, 24, 48, 1, 60.0),    # one detector row
           cone.ConeGeometry(32, 16, 24, 4097, 4096, 60.0),   # N_r N_s above 2^24
           cone.ConeGeometry(32, 16, 65536, 48, 11, 60.0)]    # N_v above 65535
    for g in bad:
        with pytest.raises(ncs.NcsError) as e:
            cone.ConeSolver(g, _params())
        assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    with pytest.raises(ncs.NcsError):
        cone.ConeSolver(geometry("c32"), _params(method=ncs.METHOD_ADMM_CG))
    s = cone.ConeSolver(geometry("c32"), _params(method=ncs.METHOD_PDHG))
    with pytest.raises(ncs.NcsError) as e:
        s.iterate(1)
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    s.close()


def test_cone_flat_volume_trajectory_matches_oracle():
    # N_z = 4: the z pass of the DFT has 4 points and the adjoint runs of 4
    # voxels; the source sits at the smallest radius allowed
    g = conebeam.ConeGeometry(*CONE["flat"])
    prob = conebeam.cone_problem(g, 2, 0.01, E=cone_E("flat"))
    a, be = 0.01, 0.03
    gam = 3.2 * a * g.n_views * g.n_side / (2.0 * np.pi)
    h_e = conebeam.probe_multiplier_3d(lambda v: prob.Et @ (prob.E @ v), g.shape, 16)
    h = 1.0 / conebeam.eigenvalues3d(prob, a, be, gam, h_e)
    x_ref, _, v_ref, obj_ref = conebeam.ncs3d(prob, a, be, h, 40)
    s = cone.ConeSolver(geometry("flat"), cone.ConeParams(a, be, gam, prob.lam),
                        b=torch.tensor(prob.b, device=DEV), dtype=torch.float64)
    s.set_init()
    obj = s.iterate(40, record=True)
    x, v = s.x().cpu().numpy(), s.v().cpu().numpy()
    s.close()
    ex, ev = rel_l2(x, x_ref), rel_l2(v, v_ref)
    ef = float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref)))
    log(f"cone flat volume ncs f64: rel-L2 x {ex:.2e}, v {ev:.2e}, max rel f {ef:.2e}")
    assert max(ex, ev, ef) <= 1e-10


def test_cone_probe_count_mu_dc_and_info():
    # 4 probes instead of 16, a given DC eigenvalue, and the setup facts
    prob = _problem()
    a, be, gam = 0.01, 0.03, _gamma()
    h4 = conebeam.probe_multiplier_3d(lambda v: prob.Et @ (prob.E @ v), prob.geom.shape, 4)
    ref = conebeam.eigenvalues3d(prob, a, be, gam, h4, mu_dc=7.5)
    s = cone.ConeSolver(geometry("c32"), cone.ConeParams(a, be, gam, 0.01, mu_dc=7.5, probes=4), dtype=torch.float64)
    mu = s.eigenvalues()
    info = s.info()
    s.close()
    assert float(np.max(np.abs(mu - ref) / np.abs(ref))) <= 1e-9
    assert mu[0, 0, 0] == 7.5 and info["mu_dc"] == 7.5
    e1 = prob.E @ np.ones(prob.n)
    assert info["norm_e1_sq"] == pytest.approx(float(e1 @ e1), rel=1e-12)
    assert info["bin_window"] >= 1


def test_cone_time_phases():
    prob = _problem()
    s = cone.ConeSolver(geometry("c32"), cone.ConeParams(0.01, 0.03, _gamma(), prob.lam),
                        b=torch.tensor(prob.b, dtype=torch.float32, device=DEV))
    s.set_init()
    ph = s.time_phases(3)
    s.close()
    assert list(ph) == cone.PHASES and all(v > 0 and np.isfinite(v) for v in ph.values())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cone_positivity_matches_oracle(prec):
    # x >= 0 as a third block of A (remark in Section 4.2) on a volume
    K = 60
    prob = _problem()
    a, be, gam = 0.01, 0.03, _gamma()
    h = 1.0 / conebeam.eigenvalues3d(prob, a, be, gam, _h_e(), positivity=True)
    x_ref, _, _, obj_ref, t_ref = conebeam.ncs3d(prob, a, be, h, K, positivity=True, with_t=True)
    assert_converging(obj_ref)
    x_free = _ref("ncs", K)[0]
    s = cone.ConeSolver(geometry("c32"), cone.ConeParams(a, be, gam, prob.lam, positivity=1),
                        b=torch.tensor(prob.b, dtype=DT[prec], device=DEV), dtype=DT[prec])
    s.set_init()
    obj = s.iterate(K, record=True)
    x, t = s.x().double().cpu().numpy(), s.t().double().cpu().numpy()
    s.close()
    assert x_free.min() < 0 and t_ref.min() < 0   # the constraint is active
    ex, et = rel_l2(x, x_ref), rel_l2(t, t_ref)
    ef = float(np.max(np.abs(obj - obj_ref) / np.abs(obj_ref)))
    log(f"cone with x >= 0, {prec}: rel-L2 x {ex:.2e}, t {et:.2e}, max rel f {ef:.2e}")
    if prec == "f64":
        assert max(ex, et, ef) <= 1e-10
    else:
        assert ex <= 1e-4 and et <= 1e-4 and ef <= 1e-5
    assert t.max() <= 0.0


def test_cone_t_needs_positivity():
    s = cone.ConeSolver(geometry("c32"), _params(method=ncs.METHOD_PDHG))
    with pytest.raises(ncs.NcsError):
        s.t()
    s.close()


@pytest.mark.parametrize("positivity", [0, 1])
def test_cone_checkpoint_resumes_bit_for_bit(positivity):
    prob = _problem()
    b = torch.tensor(prob.b, dtype=torch.float32, device=DEV)
    p = cone.ConeParams(0.01, 0.03, _gamma(), prob.lam, positivity=positivity)
    a = cone.ConeSolver(geometry("c32"), p, b=b)
    a.set_init()
    a.iterate(20)
    blob = a.get_state()
    obj_a = a.iterate(20, record=True)
    c = cone.ConeSolver(geometry("c32"), p, b=b)
    c.set_state(blob)
    obj_c = c.iterate(20, record=True)
    assert torch.equal(c.x().cpu(), a.x().cpu()) and np.array_equal(obj_a, obj_c)
    if positivity:
        assert torch.equal(c.t().cpu(), a.t().cpu())
    d = cone.ConeSolver(geometry("c32"), cone.ConeParams(0.01, 0.03, _gamma(), prob.lam, positivity=1 - positivity), b=b)
    with pytest.raises(ncs.NcsError):
        d.set_state(blob)
    for s in (a, c, d):
        s.close()
