"""Autotuned tile boxes (ICNNM_AUTOTUNE=1): a measured choice among the cost model's
candidates, cached per (shape, kernel, precision) in the context and in the file
ICNNM_AUTOTUNE_CACHE names. The solve stays within the oracle's tolerance, a second
context reads the choice back from the file and reproduces the result bit for bit,
and a batch tunes within the tile class its members share."""
import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import inputs

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture
def tuning(monkeypatch, tmp_path):
    path = tmp_path / "tiles.txt"
    monkeypatch.setenv("ICNNM_AUTOTUNE", "1")
    monkeypatch.setenv("ICNNM_AUTOTUNE_CACHE", str(path))
    return path


def test_default_plan_reports_its_tile(lib):
    prob = inputs.random_problem((40, 24, 16), (8, 8, 4), 0.3, 70)
    V, _ = O.learn(inputs.random_refs(prob.dims, 2, 70), prob.kdims)
    _, info = lib.solve(_dev(prob.M), _dev(prob.mask), _dev(V.astype(np.float32)), prob.kdims, max_iter=3)
    b = info["tile"]
    assert all(x >= 1 for x in b) and np.prod(b) in (64, 128, 256, 512)


def test_autotuned_solve_matches_oracle_and_is_cached(tuning):
    from paper_2604_17001_amd import icnnm
    prob = inputs.random_problem((48, 40, 12), (8, 8, 4), 0.4, 71)
    V, _ = O.learn(inputs.random_refs(prob.dims, 3, 71), prob.kdims)
    V32 = np.ascontiguousarray(V, dtype=np.float32)
    print("[gpu] autotune solve", flush=True)
    a = icnnm.Library()
    try:
        La, ia = a.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=30)
    finally:
        a.close()
    lines = tuning.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert f[0] == "icnnm-tile" and [int(x) for x in f[1:8]] == [48, 40, 12, 8, 8, 4, 0]
    assert tuple(int(x) for x in f[9:12]) == ia["tile"]
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), prob.kdims, 30)
    La = La.cpu().numpy()
    assert np.linalg.norm(La - Lo) <= 1e-5 * np.linalg.norm(Lo)
    # a new context takes the box from the file (no new line) and repeats the result
    b = icnnm.Library()
    try:
        Lb, ib = b.solve(_dev(prob.M), _dev(prob.mask), _dev(V32), prob.kdims, max_iter=30)
    finally:
        b.close()
    assert ib["tile"] == ia["tile"]
    assert len(tuning.read_text().splitlines()) == 1
    assert np.array_equal(Lb.cpu().numpy(), La)


def test_autotuned_batch_matches_oracle(tuning):
    from paper_2604_17001_amd import icnnm
    kd = (4, 4, 4)
    dims_list = [(32, 48, 16), (64, 32, 8), (48, 48, 16)]
    probs = [inputs.random_problem(d, kd, 0.4, 72 + i) for i, d in enumerate(dims_list)]
    V, _ = O.learn(inputs.random_refs((32, 48, 16), 3, 72), kd)
    V32 = np.ascontiguousarray(V, dtype=np.float32)
    print("[gpu] autotune batch", flush=True)
    a = icnnm.Library()
    try:
        Ls, infos = a.solve_batch([_dev(p.M) for p in probs], [_dev(p.mask) for p in probs], _dev(V32), kd,
                                  max_iter=25)
    finally:
        a.close()
    lines = tuning.read_text().splitlines()
    assert len(lines) == len(set(dims_list))
    assert all(line.split()[8] == "1" for line in lines)  # tuned within the batch's tile class
    for p, L, info in zip(probs, Ls, infos):
        Lo, _ = O.solve(p.M, p.mask, V32.astype(np.float64), kd, 25)
        assert np.linalg.norm(L.cpu().numpy() - Lo) <= 1e-5 * np.linalg.norm(Lo)
        assert np.prod(info["tile"]) in (64, 128, 256, 512)
