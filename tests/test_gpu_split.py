"""Split contractions for instances solved alone with few tiles: the four wavefronts of
a workgroup share the kernel offsets (forward, eq:InductiveCNNM's A_k(L)V) or the
eigendirections (adjoint A_k^*) of each 64 x 64 work unit and add their partial sums in
LDS in a fixed order (Section III-D iteration unchanged). Each split solve is checked
against the FP64 oracle and against the unsplit form of the same solve, with the
observed entries bit-exact, in FP32 and BF16, over ragged shapes and both kernel
sizes the split admits (k = 128 in FP32, k = 256 in both)."""
import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 1e-3}
ITERS = 40


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solve_fresh(prob, V32, prec, split, monkeypatch, **kw):
    from paper_2604_17001_amd import icnnm
    monkeypatch.setenv("ICNNM_SPLIT", "1" if split else "0")
    ctx = icnnm.Library()
    try:
        L, info = ctx.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=ITERS, precision=prec,
                            **kw)
        return L.cpu().numpy(), info
    finally:
        ctx.close()


CASES = [
    ((16, 16, 8), (8, 8, 4), "fp32"),   # the 16x16x8 configuration's shapes (32 tiles)
    ((16, 16, 8), (8, 8, 4), "bf16"),
    ((20, 12, 8), (8, 8, 4), "fp32"),   # ragged tiles
    ((20, 12, 8), (8, 8, 4), "bf16"),
    ((24, 16, 8), (8, 4, 4), "fp32"),   # k = 128
    ((12, 10, 7), (4, 8, 4), "fp32"),   # ragged in every dimension, k = 128
]


@pytest.mark.parametrize("dims,kd,prec", CASES)
def test_split_matches_oracle_and_unsplit(dims, kd, prec, monkeypatch):
    prob = inputs.random_problem(dims, kd, 0.4, 70 + dims[0] + kd[1])
    V, _ = O.learn(inputs.random_refs(dims, 3, 71 + dims[1]), kd)
    V32 = V.astype(np.float32)
    print(f"[gpu] split {dims} k={kd} {prec}", flush=True)
    Ls, si = _solve_fresh(prob, V32, prec, True, monkeypatch)
    Lu, ui = _solve_fresh(prob, V32, prec, False, monkeypatch)
    assert si["split"] and not ui["split"]
    assert si["iters"] == ui["iters"] == ITERS
    obs = prob.mask != 0
    assert np.array_equal(Ls[obs], prob.M[obs])
    Lo, oi = O.solve(prob.M, prob.mask, V32.astype(np.float64), kd, ITERS)
    err_s, err_u = _rel(Ls, Lo), _rel(Lu, Lo)
    print(f"[gpu]   rel.err split {err_s:.3e} unsplit {err_u:.3e} split-vs-unsplit {_rel(Ls, Lu):.3e}", flush=True)
    assert err_s <= TOL[prec]
    assert _rel(Ls, Lu) <= TOL[prec]
    assert abs(si["theta_final"] - oi["theta_final"]) <= 1e-5 * oi["theta_final"]
    assert abs(si["objective"] - ui["objective"]) <= (1e-4 if prec == "fp32" else 1e-3) * ui["objective"]


def test_split_is_default_for_few_tiles_and_deterministic(lib):
    from paper_2604_17001_amd import icnnm
    wl = inputs.prediction_16x16x8(b_refs=2)
    p = wl.problems[0]
    V32 = O.learn(wl.refs, wl.kdims)[0].astype(np.float32)
    pl = icnnm.plan(p.dims, wl.kdims)
    assert pl["ntiles"] < 256 and pl["split"]
    assert not icnnm.plan(p.dims, wl.kdims, joint=True)["split"]
    # many tiles: the unsplit form
    assert not icnnm.plan((64, 64, 16), wl.kdims)["split"]
    print("[gpu] split default, repeated", flush=True)
    outs = []
    for _ in range(3):
        L, info = lib.solve(_dev(p.M), _dev(p.mask), _dev(V32), wl.kdims, max_iter=30)
        assert info["split"]
        outs.append((L.cpu().numpy(), info["objective"]))
    for L, obj in outs[1:]:
        assert np.array_equal(L, outs[0][0]) and obj == outs[0][1]


def test_split_penalized_mode(monkeypatch):
    # finite lambda (eq:admm): the L-step's averaging and the objective's penalty term
    # see the split halo partials (four offset groups per tile)
    dims, kd = (16, 16, 8), (8, 8, 4)
    prob = inputs.random_problem(dims, kd, 0.4, 77)
    V, _ = O.learn(inputs.random_refs(dims, 3, 78), kd)
    V32 = V.astype(np.float32)
    print("[gpu] split penalized", flush=True)
    Ls, si = _solve_fresh(prob, V32, "fp32", True, monkeypatch, lam=2.0)
    assert si["split"]
    Lo, oi = O.solve(prob.M, prob.mask, V32.astype(np.float64), kd, ITERS, lam=2.0)
    assert _rel(Ls, Lo) <= 1e-5
    assert abs(si["objective"] - oi["objective"]) <= 1e-4 * oi["objective"]
