"""icnnm_solve_noalloc through the C ABI: the allocation-free variant of icnnm_solve
(solver state in the library's fixed per-device scratch) must give the results of
icnnm_solve on the same inputs, observed entries bit-exact, on consecutive calls of
which the second has a smaller instance (the scratch keeps the first call's
contents), and refuse instances above the scratch maximum before any device work."""
import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import icnnm, inputs

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-3)])
def test_noalloc_matches_solve_on_two_calls(lib, prec, tol):
    import torch
    cases = [((64, 64, 16), (8, 8, 4), 0.4, 201, 30), ((20, 18, 12), (4, 4, 4), 0.5, 202, 25)]
    for dims, kd, pm, seed, iters in cases:
        prob = inputs.random_problem(dims, kd, pm, seed)
        V, _ = O.learn(inputs.random_refs((16, 16, 8) if dims[0] > 32 else dims, 2, seed), kd)
        V32 = V.astype(np.float32)
        M, mask, Vd = _dev(prob.M), _dev(prob.mask), _dev(V32)
        print(f"[gpu] noalloc {prec} dims={dims} kdims={kd} iters={iters}", flush=True)
        out = torch.full_like(M, float("nan"))
        Ln, info_n = lib.solve_noalloc(M, mask, Vd, kd, out, max_iter=iters, precision=prec)
        Ls, info_s = lib.solve(M, mask, Vd, kd, max_iter=iters, precision=prec)
        torch.cuda.synchronize()
        Ln, Ls = Ln.cpu().numpy(), Ls.cpu().numpy()
        assert info_n["iters"] == info_s["iters"] == iters
        assert info_n["tile"] == info_s["tile"]
        obs = prob.mask != 0
        assert np.array_equal(Ln[obs], prob.M[obs])
        d = _rel(Ln, Ls)
        print(f"[gpu]   noalloc vs solve {d:.2e} (bit-exact {np.array_equal(Ln, Ls)})", flush=True)
        assert d <= tol * 1e-2
        assert abs(info_n["objective"] - info_s["objective"]) <= 1e-6 * info_s["objective"]
        if dims[0] < 32:  # the small instance is also checked against the oracle
            Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), kd, iters)
            assert _rel(Ln, Lo) <= tol


def test_noalloc_refuses_instances_above_the_scratch(lib):
    import torch
    kd = (8, 8, 4)
    prob = inputs.random_problem((128, 64, 16), kd, 0.4, 203)   # ~270 MB of state
    M, mask = _dev(prob.M), _dev(prob.mask)
    Vd = _dev(np.eye(256, dtype=np.float32))
    out = torch.empty_like(M)
    with pytest.raises(icnnm.IcnnmError) as e:
        lib.solve_noalloc(M, mask, Vd, kd, out, max_iter=3)
    assert e.value.code == icnnm.E_BUDGET
    assert b"scratch" in lib.lib.icnnm_last_error(lib.ctx)
