"""Split-BF16 refresh of the reduced-precision forms.

Where the tiled adjoint applies (padded k a multiple of 256, 128-row tiles), the
FP32 evaluations that the BF16/FP16 forms make every refresh_every iterations
(Section III-D iteration, with the delta contractions of the reduced-precision
forms in between) run both contractions on BF16 MFMA with the tensor-side operand
(L in the forward, G in the adjoint) split into three BF16 parts and V into two;
five products (all but the 2^-27 one), accumulated in FP32.

Tolerances: the reduced-precision bar against the FP64 oracle (1e-3) with the
observed entries bit-exact; 1e-4 against the same solve with FP32 refreshes
(ICNNM_REFRESH=fp32), the bar the FP32-refresh form meets against the FP32 solve
(U stored in 16 bits in both)."""
import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import inputs

pytestmark = pytest.mark.gpu
TOL_LP = 1e-3
TOL_VS_FP32_REFRESH = 1e-4


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rel(a, b):
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _case(dims, kdims, pm, seed, b=6):
    prob = inputs.random_problem(dims, kdims, pm, seed)
    V, _ = O.learn(inputs.random_refs(dims, b, seed), kdims)
    return prob, V.astype(np.float32)


def _solve(prob, V32, kd, monkeypatch, refresh, **kw):
    # a fresh context per setting: the refresh choice is made when a group is built
    from paper_2604_17001_amd import icnnm
    monkeypatch.setenv("ICNNM_TILE", "4,4,8")
    if refresh == "fp32":
        monkeypatch.setenv("ICNNM_REFRESH", "fp32")
    else:
        monkeypatch.delenv("ICNNM_REFRESH", raising=False)
    solo = icnnm.Library()
    try:
        L, info = solo.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), kd, **kw)
    finally:
        solo.close()
    assert tuple(info["tile"]) == (4, 4, 8)
    return L.cpu().numpy(), info


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_split_bf16_refresh_matches_oracle_and_fp32_refresh(prec, monkeypatch):
    # k = 256 (8x8x4 kernel): one offset group; 60 iterations hold refreshes at 1, 10,
    # 20, ..., 60
    kd = (8, 8, 4)
    prob, V32 = _case((32, 32, 16), kd, 0.4, 71)
    print(f"[gpu] split-BF16 refresh {prec} k=256", flush=True)
    Lx, ix = _solve(prob, V32, kd, monkeypatch, "x3", max_iter=60, precision=prec)
    Lf, if_ = _solve(prob, V32, kd, monkeypatch, "fp32", max_iter=60, precision=prec)
    assert ix["refresh_x3"] == 1 and if_["refresh_x3"] == 0
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), kd, 60)
    e_x, e_f, d = _rel(Lx, Lo), _rel(Lf, Lo), _rel(Lx, Lf)
    print(f"[gpu] {prec} rel.err split-BF16 refresh {e_x:.3e}, FP32 refresh {e_f:.3e}, between {d:.3e}",
          flush=True)
    assert e_x <= TOL_LP
    assert d <= TOL_VS_FP32_REFRESH
    obs = prob.mask != 0
    assert np.array_equal(Lx[obs], prob.M[obs])
    assert ix["iters"] == 60


def test_split_bf16_every_iteration_matches_fp32_solve(monkeypatch):
    # refresh_every = 1: every contraction after the first runs in split BF16, so the
    # result differs from the FP32 solve only by the split products and the 16-bit U
    kd = (8, 8, 4)
    prob, V32 = _case((32, 32, 16), kd, 0.5, 72)
    print("[gpu] split-BF16 every iteration", flush=True)
    Lx, ix = _solve(prob, V32, kd, monkeypatch, "x3", max_iter=30, precision="bf16", refresh_every=1)
    L32, _ = _solve(prob, V32, kd, monkeypatch, "x3", max_iter=30)
    assert ix["refresh_x3"] == 1
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), kd, 30)
    d, e = _rel(Lx, L32), _rel(Lx, Lo)
    print(f"[gpu] split-BF16 every iteration: {d:.3e} from the FP32 solve, {e:.3e} from the oracle", flush=True)
    assert d <= TOL_VS_FP32_REFRESH
    assert e <= TOL_VS_FP32_REFRESH


def test_split_bf16_refresh_several_offset_groups(monkeypatch):
    # k = 1024 (16x16x4 kernel): four 256-wide offset groups in the tiled adjoint and
    # four column groups in the forward
    kd = (16, 16, 4)
    prob, V32 = _case((32, 32, 16), kd, 0.4, 73)
    print("[gpu] split-BF16 refresh bf16 k=1024", flush=True)
    Lx, ix = _solve(prob, V32, kd, monkeypatch, "x3", max_iter=25, precision="bf16")
    Lf, if_ = _solve(prob, V32, kd, monkeypatch, "fp32", max_iter=25, precision="bf16")
    assert ix["refresh_x3"] == 1 and if_["refresh_x3"] == 0
    d = _rel(Lx, Lf)
    print(f"[gpu] k=1024 split-BF16 against FP32 refresh {d:.3e}", flush=True)
    assert d <= TOL_VS_FP32_REFRESH
    obs = prob.mask != 0
    assert np.array_equal(Lx[obs], prob.M[obs])
    assert abs(ix["objective"] - if_["objective"]) <= TOL_VS_FP32_REFRESH * if_["objective"]


def test_split_bf16_refresh_in_a_batch(monkeypatch):
    # two instances of different extents in one joint launch: both report the split
    # refresh and match the same batch with FP32 refreshes
    from paper_2604_17001_amd import icnnm
    kd = (8, 8, 4)
    probs = [inputs.random_problem(d, kd, 0.4, 74 + i) for i, d in enumerate([(32, 32, 16), (32, 16, 16)])]
    V, _ = O.learn(inputs.random_refs((32, 32, 16), 4, 74), kd)
    V32 = V.astype(np.float32)
    monkeypatch.setenv("ICNNM_TILE", "4,4,8")
    outs = {}
    for refresh in ("x3", "fp32"):
        if refresh == "fp32":
            monkeypatch.setenv("ICNNM_REFRESH", "fp32")
        else:
            monkeypatch.delenv("ICNNM_REFRESH", raising=False)
        print(f"[gpu] split-BF16 refresh batch of 2, refresh {refresh}", flush=True)
        lib = icnnm.Library()
        try:
            Ls, infos = lib.solve_batch([_dev(p.M) for p in probs], [_dev(p.mask) for p in probs], _dev(V32), kd,
                                        max_iter=40, precision="bf16")
        finally:
            lib.close()
        outs[refresh] = ([L.cpu().numpy() for L in Ls], infos)
    for i, p in enumerate(probs):
        Lx, ix = outs["x3"][0][i], outs["x3"][1][i]
        Lf, if_ = outs["fp32"][0][i], outs["fp32"][1][i]
        assert ix["refresh_x3"] == 1 and if_["refresh_x3"] == 0
        d = _rel(Lx, Lf)
        print(f"[gpu] batch instance {i} dims {p.dims}: split-BF16 against FP32 refresh {d:.3e}", flush=True)
        assert d <= TOL_VS_FP32_REFRESH
        obs = p.mask != 0
        assert np.array_equal(Lx[obs], p.M[obs])
        assert ix["iters"] == 40
