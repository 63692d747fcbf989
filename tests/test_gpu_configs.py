"""Full-size parity at the benchmark configurations against stored FP64 oracle
results (tests/golden, written by tests/golden/make_golden.py from the oracle
alone). The solve runs in the same launch configuration the benchmark times."""
import json
import os

import numpy as np
import pytest

from paper_2604_17001_amd import inputs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("name,factory", [("16x16x8", inputs.prediction_16x16x8), ("64x64x16", inputs.video_64x64x16),
                                          ("128x128x32", inputs.interpolation_128x128x32)])
def test_config_matches_stored_oracle(lib, name, factory):
    if not os.path.exists(os.path.join(GOLD, f"{name}_L.npy")):
        pytest.skip("stored oracle result missing")
    wl = factory(b_refs=0)
    p = wl.problems[0]
    V32 = np.load(os.path.join(GOLD, f"{name}_V.npy"))
    Lo = np.load(os.path.join(GOLD, f"{name}_L.npy"))
    meta = json.load(open(os.path.join(GOLD, f"{name}_meta.json")))
    print(f"[gpu] config {name} dims={p.dims} iters={wl.iters}", flush=True)
    L, info = lib.solve(_dev(p.M), _dev(p.mask), _dev(V32), wl.kdims, max_iter=wl.iters)
    L = L.cpu().numpy()
    assert info["iters"] == wl.iters == meta["iters"]
    err = float(np.linalg.norm(L - Lo) / np.linalg.norm(Lo))
    print(f"[gpu] {name} rel.err {err:.3e}", flush=True)
    assert err <= 1e-5
    assert np.array_equal(L[p.mask != 0], p.M[p.mask != 0])
    assert abs(info["theta_final"] - meta["theta_final"]) <= 1e-5 * meta["theta_final"]
    assert abs(info["objective"] - meta["objective"]) <= 1e-4 * meta["objective"]
