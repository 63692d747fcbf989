"""GPU parity of the HIP solver (through the C ABI) against the FP64 oracle.

Tolerances: relative Frobenius error <= 1e-5 for the FP32 path at equal
iteration counts; observed entries bit-exact for lambda = inf; special cases
exact. Inputs are seeded synthetic problems; V is learned by the oracle and
rounded to float32, and both sides consume the same float32 arrays.
"""
import math
import sys

import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import inputs

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _relerr(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _case(dims, kdims, p_missing, seed, b=6):
    prob = inputs.random_problem(dims, kdims, p_missing, seed)
    refs = inputs.random_refs(dims, b, seed)
    V, _ = O.learn(refs, kdims)
    return prob, V.astype(np.float32)


def _gpu_solve(lib, prob, V32, iters, **kw):
    print(f"[gpu] solve dims={prob.dims} kdims={prob.kdims} iters={iters} {kw}", flush=True)
    sys.stdout.flush()
    L, info = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=iters, **kw)
    import torch
    torch.cuda.synchronize()
    return L.cpu().numpy(), info


CASES = [
    ((12, 10, 8), (3, 3, 2), 0.4, 1),      # k = 18 -> padded to 64, several ragged tiles
    ((16, 16, 8), (8, 8, 4), 0.3, 2),      # k = 256, the 16x16x8 shape
    ((13, 11, 7), (4, 3, 2), 0.5, 3),      # odd sizes
    ((9, 33), (4, 5), 0.5, 4),             # order 2
    ((70,), (9,), 0.4, 5),                 # order 1
    ((24, 20, 16), (5, 5, 4), 0.35, 6),    # k = 100, several tiles per dimension
    ((24, 24, 8), (8, 8, 8), 0.4, 7),      # k = 512: the tiled large-kernel adjoint
    ((20, 18, 12), (6, 6, 9), 0.4, 8),     # k = 324 padded to 512, ragged tiles
    ((16, 16, 16), (16, 16, 4), 0.5, 9),   # k = 1024, the 16x16x4 kernel
    ((10, 9, 6), (1, 1, 1), 0.4, 10),      # k = 1: a one-entry kernel
    ((8, 6, 4), (8, 6, 4), 0.4, 11),       # kernel as large as the tensor (k = m = 192)
]


@pytest.mark.parametrize("dims,kdims,pm,seed", CASES)
def test_solve_parity_small(lib, dims, kdims, pm, seed):
    prob, V32 = _case(dims, kdims, pm, seed)
    iters = 30
    L, info = _gpu_solve(lib, prob, V32, iters)
    Lo, oi = O.solve(prob.M, prob.mask, V32.astype(np.float64), kdims, iters)
    assert info["iters"] == iters
    err = _relerr(L, Lo)
    assert err <= TOL32, err
    obs = prob.mask != 0
    assert np.array_equal(L[obs], prob.M[obs])
    assert abs(info["objective"] - oi["objective"]) <= 1e-4 * oi["objective"]
    assert abs(info["theta_final"] - oi["theta_final"]) <= 1e-5 * oi["theta_final"]


# The image and video kernel sizes of the paper's experiments (Section V: square
# kernels up to 43x43 on images, 13x13x13 on videos) on synthetic tensors small
# enough for the oracle: k = 1849 (padded to 2048) and k = 2197 (padded to 2304,
# 9 offset groups, 5120-position halo boxes). Few iterations keep the oracle short.
BIG_K = [
    ((64, 64), (43, 43), 0.5, 21, 8),
    ((20, 20, 16), (13, 13, 13), 0.4, 22, 6),
]


@pytest.mark.parametrize("dims,kdims,pm,seed,iters", BIG_K)
def test_solve_parity_paper_kernel_sizes(lib, dims, kdims, pm, seed, iters):
    prob, V32 = _case(dims, kdims, pm, seed, b=2)
    L, info = _gpu_solve(lib, prob, V32, iters)
    Lo, oi = O.solve(prob.M, prob.mask, V32.astype(np.float64), kdims, iters)
    err = _relerr(L, Lo)
    print(f"[gpu] rel.err {err:.3e}", flush=True)
    assert info["iters"] == iters
    assert err <= TOL32, err
    obs = prob.mask != 0
    assert np.array_equal(L[obs], prob.M[obs])


def test_zero_iterations_is_zero_fill(lib):
    prob, V32 = _case((12, 10, 8), (3, 3, 2), 0.4, 7)
    L, info = _gpu_solve(lib, prob, V32, 0)
    assert np.array_equal(L, np.where(prob.mask != 0, prob.M, 0).astype(np.float32))
    obj = O.objective(np.where(prob.mask != 0, prob.M, 0.0), V32.astype(np.float64), prob.kdims)
    assert abs(info["objective"] - obj) <= 1e-5 * obj


def test_full_sampling_returns_M_bitwise(lib):
    prob, V32 = _case((16, 12, 8), (4, 4, 2), 0.0, 8)
    prob.mask[:] = 1
    L, _ = _gpu_solve(lib, prob, V32, 10)
    assert np.array_equal(L, prob.M)


def test_empty_sampling_returns_zero(lib):
    prob, V32 = _case((16, 12, 8), (4, 4, 2), 0.0, 9)
    prob.mask[:] = 0
    L, info = _gpu_solve(lib, prob, V32, 10)
    assert np.all(L == 0)


def test_identity_bank_gives_zero_fill(lib):
    prob, _ = _case((16, 12, 8), (4, 4, 2), 0.5, 10)
    k = int(np.prod(prob.kdims))
    L, _ = _gpu_solve(lib, prob, np.eye(k, dtype=np.float32), 40)
    obs = prob.mask != 0
    assert np.array_equal(L[obs], prob.M[obs])
    assert np.abs(L[~obs]).max() <= 1e-5 * np.abs(prob.M).max()


@pytest.mark.parametrize("lam", [1000.0, 2.0])
def test_penalized_mode_parity(lib, lam):
    prob, V32 = _case((12, 10, 8), (3, 3, 2), 0.4, 11)
    L, info = _gpu_solve(lib, prob, V32, 40, lam=lam)
    Lo, oi = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, 40, lam=lam)
    assert _relerr(L, Lo) <= TOL32
    # the reported objective is that of the penalized program (eq:admm):
    # ||A_k(L)V||_{2,1} + (lambda k / 2) ||P_Omega(L - M)||^2 at the returned L
    assert abs(info["objective"] - oi["objective"]) <= 1e-4 * oi["objective"]
    obj_gpu_L = O.objective(L.astype(np.float64), V32.astype(np.float64), prob.kdims, M=prob.M,
                            mask=prob.mask, lam=lam)
    assert abs(info["objective"] - obj_gpu_L) <= 1e-5 * obj_gpu_L
    pen = 0.5 * lam * prob.k * float(np.sum(np.where(prob.mask != 0, L.astype(np.float64) - prob.M, 0.0) ** 2))
    assert pen > 0.0


def test_stopping_rule_matches_oracle(lib):
    prob, V32 = _case((12, 10, 8), (3, 3, 2), 0.4, 12)
    L, info = _gpu_solve(lib, prob, V32, 400, tol=1e-4)
    assert info["converged"] == 1
    Lo, oi = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, 400, tol=1e-4)
    assert oi["converged"] and abs(info["iters"] - oi["iters"]) <= 1
    Lr, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, info["iters"])
    assert _relerr(L, Lr) <= TOL32
    assert max(info["r_primal"], info["r_change"]) <= 1e-4


def test_explicit_theta0_and_repeat_call(lib):
    prob, V32 = _case((12, 10, 8), (3, 3, 2), 0.4, 13)
    for _ in range(2):  # the second call reuses the cached plan and state
        L, info = _gpu_solve(lib, prob, V32, 25, theta0=0.05, rho=1.2)
        Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, 25, theta0=0.05, rho=1.2)
        assert _relerr(L, Lo) <= TOL32


def test_invalid_arguments_rejected(lib):
    from paper_2604_17001_amd.icnnm import IcnnmError
    prob, V32 = _case((12, 10, 8), (3, 3, 2), 0.4, 14)
    with pytest.raises(IcnnmError) as ei:  # k_1 = 13 > m_1 = 12, rejected by the library
        lib.solve(_dev(prob.M), _dev(prob.mask), _dev(np.eye(13, dtype=np.float32)), (13, 1, 1), max_iter=1)
    assert ei.value.code == -1
    bad = V32.copy()
    bad[0, 0] += 0.1
    with pytest.raises(IcnnmError):
        lib.solve(_dev(prob.M), _dev(prob.mask), _dev(bad), prob.kdims, max_iter=1, check_v=True)
    L, _ = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=1, check_v=True)


def test_nan_input_reports_numeric_error(lib):
    # a NaN among the observed entries makes the residuals non-finite: the solve stops
    # and reports ICNNM_E_NUMERIC instead of returning a silently wrong result
    from paper_2604_17001_amd import icnnm
    prob, V32 = _case((12, 10, 8), (3, 3, 2), 0.4, 12)
    obs = np.flatnonzero(prob.mask.reshape(-1))
    M = prob.M.copy()
    M.reshape(-1)[obs[0]] = np.nan
    print("[gpu] nan input", flush=True)
    with pytest.raises(icnnm.IcnnmError) as e:
        lib.solve(_dev(M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=10)
    assert e.value.code == icnnm.E_NUMERIC
