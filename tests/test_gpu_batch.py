"""Batched slices of uneven size in shared launches, through the C ABI.

Each slice of a batch runs the same kernels as a single-slice solve, reading
its own descriptor, so its trajectory must equal the single-slice run bit for
bit (same projector kernel) and match the FP64 oracle to the usual gates;
every slice stops on its own target.  The iterations between host checks are
replayed HIP graphs; direct launches (graph_chunk < 0) give the same bits.
"""
import numpy as np
import pytest
import torch

from gpu_common import ct_params, joseph, log, oracle_ncs, rel_l2
from oracle import problems
from paper_1810_13100_amd import ncs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)

# (n_side, n_angles, n_bins, seed, kind)
SLICES = [(64, 90, 92, 0, "ct"), (32, 45, 48, 1, "ct"), (128, 179, 130, 2, "ct"),
          (32, 45, 48, 3, "ct"), (64, 90, 92, 4, "pet"), (16, 7, 23, 5, "ct")]


def _problem(n, na, ns, seed, kind):
    if kind == "pet":
        return problems.pet_problem(n, na, ns, seed, 0.02, total_counts=2e5, E=joseph(n, na, ns))
    return problems.ct_problem(n, na, ns, seed, 0.01, E=joseph(n, na, ns))


def _params(prob, projector=2, graph_chunk=0):
    if prob.kind == "pet":
        par = ct_params(prob.n_side, prob.n_angles, alpha=1.0, ratio=3.0, g=1.0)
        return par, ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, data_term=ncs.DATA_POISSON,
                               tv_term=ncs.TV_ISO, projector=projector, backprojector=projector, check_every=10,
                               graph_chunk=graph_chunk)
    par = ct_params(prob.n_side, prob.n_angles)
    return par, ncs.Params(par.alpha, par.beta, par.gamma, prob.lam, projector=projector, backprojector=projector,
                           check_every=10, graph_chunk=graph_chunk)


def _batch(probs, dtype, projector=2, graph_chunk=0):
    geoms, params, bs, bgs = [], [], [], []
    for prob in probs:
        geoms.append(ncs.Geometry(prob.n_side, prob.n_angles, prob.n_bins))
        params.append(_params(prob, projector, graph_chunk)[1])
        bs.append(torch.tensor(prob.b, dtype=dtype, device=DEV))
        bgs.append(torch.tensor(prob.bg, dtype=dtype, device=DEV) if prob.kind == "pet" else None)
    return ncs.Batch(geoms, params, bs, bgs, dtype=dtype), bs, bgs


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_matches_oracle_and_solo(prec):
    dtype = torch.float64 if prec == "f64" else torch.float32
    probs = [_problem(*s) for s in SLICES]
    K = 60
    bt, bs, bgs = _batch(probs, dtype)
    bt.set_init()
    st, iters, f = bt.solve(K)
    assert st == ncs.NCS_NOT_CONVERGED and list(iters) == [K] * len(probs)
    tol_x, tol_f = (1e-10, 1e-10) if prec == "f64" else (1e-4, 1e-5)
    for i, prob in enumerate(probs):
        par, p = _params(prob)
        ref = oracle_ncs(prob, par, K)
        sl = bt.slice(i)
        x = sl.x().double().cpu().numpy()
        obj = sl.objectives(0, K)
        ex = rel_l2(x, ref.x)
        fin = np.isfinite(ref.obj)              # PET objectives are +inf until E x + r > 0 where b > 0
        assert np.array_equal(np.isfinite(obj), fin)
        ef = float(np.max(np.abs(obj[fin] - ref.obj[fin]) / np.abs(ref.obj[fin]))) if fin.any() else 0.0
        log(f"  slice {i} {SLICES[i]} {prec}: rel-L2 x {ex:.2e}, max rel f {ef:.2e}")
        assert ex <= tol_x and ef <= tol_f
        # the same slice solved alone with the same kernels: bit for bit
        solo = ncs.Solver(ncs.Geometry(prob.n_side, prob.n_angles, prob.n_bins), p, b=bs[i], bg=bgs[i], dtype=dtype)
        solo.set_init()
        solo_obj = solo.iterate(K, record=True)
        assert torch.equal(solo.x().cpu(), sl.x().cpu())
        assert np.array_equal(solo_obj, obj)
        solo.close()
    bt.close()


def test_batch_slices_stop_on_their_own_targets():
    probs = [_problem(*s) for s in SLICES if s[4] == "ct"]
    K = 80
    refs = [oracle_ncs(p, _params(p)[0], K) for p in probs]
    picks = [20, 45, 70, 33, 57]
    # just above the oracle's value at the picked iteration, so that rounding
    # (1e-15 here) cannot move the crossing
    targets = np.array([r.obj[k] * (1 + 1e-12) for r, k in zip(refs, picks)])
    firsts = [int(np.nonzero(r.obj <= t)[0][0]) + 1 for r, t in zip(refs, targets)]
    bt, _, _ = _batch(probs, torch.float64)
    bt.set_init()
    st, iters, f = bt.solve(200, targets)
    log(f"batch stops: {list(iters)} (oracle {firsts})")
    assert st == ncs.NCS_OK
    assert list(iters) == firsts
    for i in range(len(probs)):
        assert abs(f[i] - refs[i].obj[firsts[i] - 1]) <= 1e-10 * abs(f[i])
    bt.close()


def test_batch_rejects_bad_slices():
    good = ncs.Params(0.01, 0.03, 1.0, 0.01)
    b = torch.zeros(90 * 92, device=DEV)
    with pytest.raises(ncs.NcsError) as e:
        ncs.Batch([ncs.Geometry(64, 90, 92), ncs.Geometry(48, 90, 92)], [good, good], [b, b])
    assert e.value.status == ncs.NCS_ERR_INVALID_ARG
    assert "slice 1" in str(e.value)


def test_batch_autotuned_kernels():
    # kernels chosen by timing batched iterations; every slice uses the batch's choice
    probs = [_problem(*s) for s in SLICES if s[4] == "ct"]
    K = 40
    bt, _, _ = _batch(probs, torch.float32, projector=0)
    bt.set_init()
    st, iters, f = bt.solve(K)
    assert list(iters) == [K] * len(probs)
    infos = [bt.slice(i).info() for i in range(len(probs))]
    log(f"batch kernels: projector {infos[0]['projector']}, backprojector {infos[0]['backprojector']}")
    assert len({(i["projector"], i["backprojector"]) for i in infos}) == 1
    for i, prob in enumerate(probs):
        ref = oracle_ncs(prob, _params(prob)[0], K)
        ex = rel_l2(bt.slice(i).x().double().cpu().numpy(), ref.x)
        assert ex <= 1e-4, ex
    bt.close()


def test_batch_graph_replay_equals_direct_launches():
    # per-slice stops inside replayed chunks, maps rebuilt (and graphs
    # re-captured) as slices stop: the same iterates and counts as direct launches
    probs = [_problem(*s) for s in SLICES if s[4] == "ct"]
    refs = [oracle_ncs(p, _params(p)[0], 80) for p in probs]
    targets = np.array([r.obj[k] * (1 + 1e-12) for r, k in zip(refs, [20, 45, 70, 33, 57])])
    out = []
    for gc in (-1, 0):
        bt, _, _ = _batch(probs, torch.float32, graph_chunk=gc)
        bt.set_init()
        st, iters, f = bt.solve(200, targets)
        xs = [bt.slice(i).x().cpu() for i in range(len(probs))]
        st2, iters2, _ = bt.solve(37)   # no targets: every slice runs the whole budget, 3 chunks + 7
        xs2 = [bt.slice(i).x().cpu() for i in range(len(probs))]
        out.append((list(iters), xs, list(iters2), xs2))
        bt.close()
    log(f"graph vs direct: stops {out[1][0]} / {out[0][0]}")
    assert out[0][0] == out[1][0] and out[0][2] == out[1][2] == [37] * len(probs)
    for a, b in zip(out[0][1] + out[0][3], out[1][1] + out[1][3]):
        assert torch.equal(a, b)


@pytest.mark.timeout(900)
def test_batch_with_a_512_slice():
    """A 512^2 slice of the uneven batch's geometry (717 angles x 520 bins) with
    a 128^2 and a 256^2 one: 20 FP32 iterations against the FP64 oracle, and
    the 512^2 slice equal bit for bit to its single-slice run."""
    geo = [(512, 717, 520, 7), (128, 179, 130, 8), (256, 358, 260, 9)]
    log("assembling the oracle's 512^2 projector (about a minute)")
    probs = [problems.ct_problem(n, na, ns, seed, 0.005, E=joseph(n, na, ns)) for n, na, ns, seed in geo]
    K = 20
    bt, bs, _ = _batch(probs, torch.float32)
    bt.set_init()
    st, iters, _ = bt.solve(K)
    assert list(iters) == [K] * len(probs)
    for i, prob in enumerate(probs):
        ref = oracle_ncs(prob, _params(prob)[0], K)
        sl = bt.slice(i)
        ex = rel_l2(sl.x().double().cpu().numpy(), ref.x)
        ef = float(np.max(np.abs(sl.objectives(0, K) - ref.obj) / np.abs(ref.obj)))
        log(f"  slice {geo[i]}: rel-L2 x {ex:.2e}, max rel f {ef:.2e}")
        assert ex <= 1e-4 and ef <= 1e-5
    p = _params(probs[0])[1]
    solo = ncs.Solver(ncs.Geometry(512, 717, 520), p, b=bs[0])
    solo.set_init()
    solo.iterate(K)
    assert torch.equal(solo.x().cpu(), bt.slice(0).x().cpu())
    solo.close()
    bt.close()


def test_batch_slice_sits_out_with_minus_infinity_target():
    probs = [_problem(*s) for s in SLICES if s[4] == "ct"]
    bt, _, _ = _batch(probs, torch.float64)
    bt.set_init()
    bt.solve(15)
    before = [bt.slice(i).x().cpu() for i in range(len(probs))]
    t = np.array([-np.inf, np.nan, -np.inf, np.nan, np.nan])
    st, iters, _ = bt.solve(23, t)
    assert list(iters) == [0, 23, 0, 23, 23]
    for i in range(len(probs)):
        after = bt.slice(i).x().cpu()
        assert torch.equal(after, before[i]) == (i in (0, 2))
        assert bt.slice(i).iteration() == (15 if i in (0, 2) else 38)
    # the slices that sat out continue exactly as if never paused
    ref = oracle_ncs(probs[0], _params(probs[0])[0], 30)
    bt.solve(15, np.array([np.nan, -np.inf, -np.inf, -np.inf, -np.inf]))
    assert rel_l2(bt.slice(0).x().cpu().numpy(), ref.x) <= 1e-10
    bt.close()
