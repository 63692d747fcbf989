"""The uneven 64-instance batch (extents {32,48,64,96,128}^2 x {8,16,32}, 8x8x4
kernel, one shared V learned from the workload's 20 references) at full size
and at its 200 iterations, in the launch configuration the batch benchmark
times: every instance keeps its observed entries bit-exact and matches the same
instance solved alone, and the instances with stored FP64 oracle results
(tests/golden/batch_*, written by make_golden.py from the oracle alone; they
span the 48 and 96 extents, 8, 16 and 32 frames and all three mask types) match
them within 1e-5 (FP32) or 1e-3 (BF16)."""
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


# Solved alone, an instance gets the cost model's own tile box, in the batch the box of
# the launch's shared kernel variants: the same iteration with another summation order,
# so the two agree to FP32 rounding accumulated over 200 iterations (1e-5, the FP32
# parity bar), not bit for bit.
@pytest.mark.parametrize("prec,tol_oracle,tol_alone", [("fp32", 1e-5, 1e-5), ("bf16", 1e-3, 1e-4)])
def test_full_batch(lib, prec, tol_oracle, tol_alone):
    meta = json.load(open(os.path.join(GOLD, "batch_meta.json")))
    wl = inputs.batch_uneven(b_refs=0)
    iters = meta["iters"]
    assert iters == wl.iters == 200
    V32 = np.load(os.path.join(GOLD, "batch_V.npy"))
    Vd = _dev(V32)
    probs = wl.problems
    print(f"[gpu] batch {len(probs)} instances, sum m = {sum(p.m for p in probs)}, {prec}", flush=True)
    Ls, infos = lib.solve_batch([_dev(p.M) for p in probs], [_dev(p.mask) for p in probs], Vd, wl.kdims,
                                max_iter=iters, precision=prec)
    worst = 0.0
    for p, L, info in zip(probs, Ls, infos):
        Lh = L.cpu().numpy()
        assert info["iters"] == iters
        assert np.array_equal(Lh[p.mask != 0], p.M[p.mask != 0])
        La, _ = lib.solve(_dev(p.M), _dev(p.mask), Vd, wl.kdims, max_iter=iters, precision=prec)
        La = La.cpu().numpy()
        d = np.linalg.norm(Lh - La) / np.linalg.norm(La)
        worst = max(worst, d)
        assert d <= tol_alone
    print(f"[gpu] worst batch-vs-alone difference {worst:.2e}", flush=True)
    assert len(meta["instances"]) >= 6
    kinds = set()
    for idx, im in meta["instances"].items():
        i = int(idx)
        p = probs[i]
        assert list(p.dims) == im["dims"] and p.meta["mask_kind"] == im["mask_kind"]
        kinds.add(im["mask_kind"])
        Lo = np.load(os.path.join(GOLD, f"batch_{i}_L.npy"))
        err = np.linalg.norm(Ls[i].cpu().numpy() - Lo) / np.linalg.norm(Lo)
        print(f"[gpu] instance {i} dims {p.dims} mask {im['mask_kind']} rel.err {err:.3e}", flush=True)
        assert err <= tol_oracle
        assert abs(infos[i]["objective"] - im["objective"]) <= 10 * tol_oracle * im["objective"]
    assert kinds == {0, 1, 2}
