"""The C ABI used from plain C: paper_2604_17001_amd/examples/solve_c (built by the
package build with gcc, device memory from hipMalloc, no Python on its path) solves
a problem written to raw files; its result matches the FP64 oracle like the Python
binding's (relative error <= 1e-5 in FP32, <= 1e-3 in BF16, observed entries
bit-exact)."""
import os
import subprocess

import numpy as np
import pytest

from oracle import icnnm_ref as O
from paper_2604_17001_amd import inputs

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2604_17001_amd",
                   "examples", "solve_c")


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 1e-3)])
def test_c_client_matches_oracle(tmp_path, prec, tol):
    if not os.path.exists(EXE):
        pytest.fail("examples/solve_c is not built (run python -m paper_2604_17001_amd.build)")
    dims, kd, iters = (16, 12, 8), (4, 4, 4), 25
    prob = inputs.random_problem(dims, kd, 0.4, 51)
    V, _ = O.learn(inputs.random_refs(dims, 4, 51), kd)
    V32 = V.astype(np.float32)
    prob.M.astype(np.float32).tofile(tmp_path / "M.f32")
    prob.mask.astype(np.uint8).tofile(tmp_path / "mask.u8")
    V32.tofile(tmp_path / "V.f32")
    print(f"[gpu] C client precision {prec}", flush=True)
    r = subprocess.run([EXE, str(tmp_path), *map(str, dims), *map(str, kd), str(iters), str(prec)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    it = int(r.stdout.split()[0])
    L = np.fromfile(tmp_path / "L.f32", dtype=np.float32).reshape(dims)
    Lo, _ = O.solve(prob.M, prob.mask, V32.astype(np.float64), kd, iters)
    err = float(np.linalg.norm(L - Lo) / np.linalg.norm(Lo))
    assert it == iters
    assert err <= tol, err
    obs = prob.mask != 0
    assert np.array_equal(L[obs], prob.M[obs])
