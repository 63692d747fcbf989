"""Reduced-precision form: both contractions run on BF16 or FP16 MFMA (FP32
accumulate) on the change of their operand since the previous iteration, with a
full FP32 evaluation every refresh_every iterations and at the last one.
Tolerance: relative Frobenius error <= 1e-3 against the FP64 oracle at equal
iteration counts; observed entries stay bit-exact (lambda = inf)."""
import json
import os

import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import icnnm, inputs

pytestmark = pytest.mark.gpu
TOL_LP = 1e-3
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _case(dims, kdims, pm, seed, b=6):
    prob = inputs.random_problem(dims, kdims, pm, seed)
    V, _ = O.learn(inputs.random_refs(dims, b, seed), kdims)
    return prob, V.astype(np.float32)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("dims,kdims,seed", [((16, 16, 8), (4, 4, 4), 1), ((24, 20, 16), (5, 3, 8), 2),
                                             ((9, 33), (3, 4), 3), ((24, 24, 8), (8, 8, 8), 4),
                                             ((16, 16, 16), (16, 16, 4), 5)])
def test_reduced_precision_parity(lib, prec, dims, kdims, seed):
    prob, V32 = _case(dims, kdims, 0.4, seed)
    iters = 60
    print(f"[gpu] {prec} dims={dims} kdims={kdims}", flush=True)
    L, info = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), kdims, max_iter=iters, precision=prec)
    L = L.cpu().numpy()
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), kdims, iters)
    err = _rel(L, Lo)
    print(f"[gpu] {prec} rel.err {err:.3e}", flush=True)
    assert err <= TOL_LP
    assert np.array_equal(L[prob.mask != 0], prob.M[prob.mask != 0])
    assert info["iters"] == iters


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("lam", [1000.0, 2.0])
def test_reduced_precision_penalized_mode(lib, prec, lam):
    # penalized program (eq:admm): observed entries follow the L-step's weighted mean,
    # so they are checked against the oracle like the rest, within the same tolerance
    prob, V32 = _case((16, 16, 8), (4, 4, 4), 0.4, 6)
    iters = 50
    print(f"[gpu] {prec} lambda={lam}", flush=True)
    L, info = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=iters, precision=prec,
                        lam=lam)
    L = L.cpu().numpy()
    Lo, oi = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, iters, lam=lam)
    err = _rel(L, Lo)
    print(f"[gpu] {prec} lambda={lam} rel.err {err:.3e}", flush=True)
    assert err <= TOL_LP
    obs = prob.mask != 0
    assert _rel(L[obs], Lo[obs]) <= TOL_LP
    assert abs(info["objective"] - oi["objective"]) <= TOL_LP * oi["objective"]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_refresh_every_iteration_is_fp32(lib, prec):
    # refresh_every = 1: every contraction runs in FP32; the reduced-precision forms
    # still keep the multiplier U in 16 bits, so the result matches the FP32 solve to that
    # storage's rounding (far inside the reduced-precision bar) and the oracle likewise,
    # and is closer to both than the delta contractions get
    prob, V32 = _case((16, 16, 8), (4, 4, 4), 0.4, 4)
    L1, _ = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=30, precision=prec,
                      refresh_every=1)
    L0, _ = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=30)
    L10, _ = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=30, precision=prec)
    L0 = L0.cpu().numpy().astype(np.float64)
    d1 = _rel(L1.cpu().numpy(), L0)
    d10 = _rel(L10.cpu().numpy(), L0)
    print(f"[gpu] {prec}: refresh every iteration {d1:.2e}, every 10 {d10:.2e} from the FP32 solve", flush=True)
    assert d1 <= 1e-4
    assert d1 < d10
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, 30)
    assert _rel(L1.cpu().numpy(), Lo) <= 1e-4


def test_refresh_improves_accuracy(lib):
    prob, V32 = _case((16, 16, 8), (4, 4, 4), 0.4, 5)
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, 80)
    errs = {}
    for r in (5, 80):
        L, _ = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=80, precision="bf16",
                         refresh_every=r)
        errs[r] = _rel(L.cpu().numpy(), Lo)
    print(f"[gpu] bf16 rel.err with refresh every 5: {errs[5]:.3e}, without refresh: {errs[80]:.3e}", flush=True)
    # the periodic FP32 evaluation is what keeps the reduced-precision path inside 1e-3
    assert errs[5] <= TOL_LP
    assert errs[80] > 10 * errs[5]


def test_padded_kernel_must_fit_the_tensor(lib):
    # the reduced precisions pad the innermost kernel extent to a multiple of 4; a
    # 3x3x3 kernel on a tensor whose innermost extent is 3 cannot be padded to 4
    prob, V32 = _case((12, 10, 3), (3, 3, 3), 0.4, 6)
    with pytest.raises(icnnm.IcnnmError) as ei:
        lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=5, precision="bf16")
    assert ei.value.code == icnnm.E_INVALID
    L, _ = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=5)  # FP32 runs it as given


# The paper's image and video kernels (Section V: square kernels 13x13 .. 43x43 on
# images, 13x13x13 on videos) in the reduced precisions: the innermost kernel extent
# (13 or 43) is padded to a multiple of 4 with zero rows of V, the L-step keeps the
# true k. Iteration counts include an FP32 refresh in the middle (iteration 11).
PAPER_K = [((64, 64), (13, 13), 0.5, 31, 24), ((64, 64), (43, 43), 0.5, 32, 12),
           ((20, 20, 16), (13, 13, 13), 0.4, 33, 12), ((30, 7), (5, 3), 0.4, 34, 30)]
_ORACLE = {}


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("dims,kdims,pm,seed,iters", PAPER_K)
def test_reduced_precision_paper_kernels(lib, prec, dims, kdims, pm, seed, iters):
    key = (dims, kdims, seed, iters)
    if key not in _ORACLE:
        prob, V32 = _case(dims, kdims, pm, seed, b=2)
        Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), kdims, iters)
        _ORACLE[key] = (prob, V32, Lo)
    prob, V32, Lo = _ORACLE[key]
    print(f"[gpu] {prec} paper kernel dims={dims} kdims={kdims} iters={iters}", flush=True)
    L, info = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), kdims, max_iter=iters, precision=prec)
    L = L.cpu().numpy()
    err = _rel(L, Lo)
    print(f"[gpu] {prec} rel.err {err:.3e}", flush=True)
    assert info["iters"] == iters
    assert err <= TOL_LP
    assert np.array_equal(L[prob.mask != 0], prob.M[prob.mask != 0])
    # the same padded kernel in a joint (batch) launch
    (Lb,), _ = lib.solve_batch([_dev(prob.M)], [_dev(prob.mask)], _dev(V32), kdims, max_iter=iters, precision=prec)
    assert _rel(Lb.cpu().numpy(), Lo) <= TOL_LP


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("name,factory", [("16x16x8", inputs.prediction_16x16x8), ("64x64x16", inputs.video_64x64x16),
                                          ("128x128x32", inputs.interpolation_128x128x32)])
def test_config_reduced_precision_vs_stored_oracle(lib, prec, name, factory):
    if not os.path.exists(os.path.join(GOLD, f"{name}_L.npy")):
        pytest.skip("stored oracle result missing")
    wl = factory(b_refs=0)
    p = wl.problems[0]
    V32 = np.load(os.path.join(GOLD, f"{name}_V.npy"))
    Lo = np.load(os.path.join(GOLD, f"{name}_L.npy"))
    print(f"[gpu] {name} {prec}", flush=True)
    L, info = lib.solve(_dev(p.M), _dev(p.mask), _dev(V32), wl.kdims, max_iter=wl.iters, precision=prec)
    L = L.cpu().numpy()
    err = _rel(L, Lo)
    print(f"[gpu] {name} {prec} rel.err {err:.3e}", flush=True)
    assert err <= TOL_LP
    assert np.array_equal(L[p.mask != 0], p.M[p.mask != 0])


def test_batch_reduced_precision(lib):
    kd = (4, 4, 4)
    shapes = [(16, 12, 8), (24, 16, 8), (12, 12, 4), (20, 9, 16)]
    probs = [inputs.random_problem(d, kd, 0.35, seed=130 + i) for i, d in enumerate(shapes)]
    V, _ = O.learn([inputs.random_refs(shapes[0], 1, seed=140)[0]], kd)
    V32 = V.astype(np.float32)
    Ls, infos = lib.solve_batch([_dev(p.M) for p in probs], [_dev(p.mask) for p in probs], _dev(V32), kd,
                                max_iter=40, precision="bf16")
    for p, L in zip(probs, Ls):
        Lo, _ = O.solve(p.M, p.mask, V32.astype(np.float64), kd, 40)
        assert _rel(L.cpu().numpy(), Lo) <= TOL_LP


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_stopping_checks_keep_the_refresh_schedule(lib, prec):
    # tol > 0 runs the solve in chunks of rounds with a state read between them; a
    # tolerance that never triggers must give bit for bit the result of tol = 0, with
    # the FP32 refreshes (first iteration, every refresh_every-th, the last) in place
    prob, V32 = _case((16, 16, 8), (4, 4, 4), 0.4, 7)
    for iters, every in ((47, 10), (23, 4), (12, 1)):
        print(f"[gpu] {prec} tol chunks iters={iters} refresh_every={every}", flush=True)
        La, ia = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=iters, precision=prec,
                           refresh_every=every)
        Lb, ib = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=iters, precision=prec,
                           refresh_every=every, tol=1e-30)
        assert ia["iters"] == ib["iters"] == iters
        assert np.array_equal(La.cpu().numpy(), Lb.cpu().numpy())
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, 12)
    assert _rel(Lb.cpu().numpy(), Lo) <= TOL_LP


def test_batch_stopping_checks_keep_the_refresh_schedule(lib):
    kd = (4, 4, 4)
    probs = [inputs.random_problem(d, kd, 0.35, seed=80 + i) for i, d in enumerate([(16, 12, 8), (20, 9, 8), (8, 8, 8)])]
    V, _ = O.learn([inputs.random_refs((16, 12, 8), 1, seed=90)[0]], kd)
    V32 = V.astype(np.float32)
    args = ([_dev(p.M) for p in probs], [_dev(p.mask) for p in probs], _dev(V32), kd)
    print("[gpu] bf16 batch tol chunks", flush=True)
    La, ia = lib.solve_batch(*args, max_iter=33, precision="bf16", refresh_every=7)
    Lb, ib = lib.solve_batch(*args, max_iter=33, precision="bf16", refresh_every=7, tol=1e-30)
    for p, a, b, x, y in zip(probs, La, Lb, ia, ib):
        assert x["iters"] == y["iters"] == 33
        a = a.cpu().numpy()
        assert np.array_equal(a, b.cpu().numpy())
        Lo, _ = O.solve(p.M, p.mask, V32.astype(np.float64), kd, 33)
        assert _rel(a, Lo) <= TOL_LP
