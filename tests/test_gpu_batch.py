"""Batched solving (one joint launch per stage and iteration over uneven
instances) against the FP64 oracle and against solving each instance alone."""
import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [(16, 12, 8), (24, 16, 8), (12, 12, 4), (20, 9, 6), (8, 8, 8), (32, 16, 16)]


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _setup(kd=(4, 4, 2)):
    probs = [inputs.random_problem(d, kd, 0.3 + 0.1 * (i % 3), seed=60 + i) for i, d in enumerate(SHAPES)]
    refs = [inputs.random_refs(d, 1, seed=70 + i)[0] for i, d in enumerate(SHAPES[:4])]
    V, _ = O.learn(refs, kd)
    return probs, V.astype(np.float32), kd


def test_batch_matches_oracle_and_single(lib):
    probs, V32, kd = _setup()
    iters = 30
    print(f"[gpu] batch of {len(probs)} iters={iters}", flush=True)
    Ls, infos = lib.solve_batch([_dev(p.M) for p in probs], [_dev(p.mask) for p in probs], _dev(V32), kd,
                                max_iter=iters)
    for p, L, info in zip(probs, Ls, infos):
        L = L.cpu().numpy()
        Lo, _ = O.solve(p.M, p.mask, V32.astype(np.float64), kd, iters)
        assert info["iters"] == iters
        assert np.linalg.norm(L - Lo) / np.linalg.norm(Lo) <= 1e-5
        assert np.array_equal(L[p.mask != 0], p.M[p.mask != 0])
        Ls1, _ = lib.solve(_dev(p.M), _dev(p.mask), _dev(V32), kd, max_iter=iters)
        L1 = Ls1.cpu().numpy()
        assert np.linalg.norm(L - L1) / np.linalg.norm(L1) <= 1e-6


def test_batch_stops_each_instance_on_its_own(lib):
    probs, V32, kd = _setup()
    Ls, infos = lib.solve_batch([_dev(p.M) for p in probs], [_dev(p.mask) for p in probs], _dev(V32), kd,
                                max_iter=300, tol=1e-4)
    its = [i["iters"] for i in infos]
    assert all(i["converged"] == 1 for i in infos)
    for p, L, info in zip(probs, Ls, infos):
        _, one = lib.solve(_dev(p.M), _dev(p.mask), _dev(V32), kd, max_iter=300, tol=1e-4)
        assert abs(one["iters"] - info["iters"]) <= 1
        Lo, _ = O.solve(p.M, p.mask, V32.astype(np.float64), kd, info["iters"])
        assert np.linalg.norm(L.cpu().numpy() - Lo) / np.linalg.norm(Lo) <= 1e-5
    assert len(set(its)) > 1  # the instances really stopped at different iterations


def test_empty_batch(lib):
    _, V32, kd = _setup()
    Ls, infos = lib.solve_batch([], [], _dev(V32), kd, max_iter=10)
    assert Ls == [] and infos == []
