"""Write the stored oracle results used by the full-size GPU parity tests.

Calls only the FP64 oracle (oracle/icnnm_ref.py) and the seeded input
generators; nothing here touches the GPU library. For each workload it stores

* ``<name>_V.npy``  - the eigenvector bank learned by the oracle from the
  workload's reference tensors (Definition 3), rounded to float32: this exact
  array is the V input of both the GPU solve and the oracle solve;
* ``<name>_L.npy``  - the oracle's iterate after the workload's iteration count
  (float64), computed from the float32 inputs upcast to float64;
* ``<name>_meta.json`` - iterations, theta0, residuals, objective, timings.

For the uneven 64-instance batch (``batch``) it stores the oracle-learned V of
the workload's 20 references (``batch_V.npy``) and, for the instances listed in
``BATCH_GOLDEN`` (chosen to span the 48 and 96 extents, 8, 16 and 32 frames and
all three mask types), ``batch_<idx>_L.npy`` after the workload's 200
iterations, plus ``batch_meta.json``.

Usage: python tests/golden/make_golden.py 16x16x8 64x64x16 [128x128x32] [batch]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import icnnm_ref as O  # noqa: E402
from paper_2604_17001_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
WORKLOADS = {"16x16x8": inputs.prediction_16x16x8, "64x64x16": inputs.video_64x64x16,
             "128x128x32": inputs.interpolation_128x128x32}


# batch instances with stored oracle results: index -> (dims, mask type) as drawn
BATCH_GOLDEN = (2, 1, 16, 49, 29, 24, 3)


def make_batch():
    wl = inputs.batch_uneven()
    t0 = time.time()
    V, w = O.learn(wl.refs, wl.kdims)
    V32 = V.astype(np.float32)
    np.save(os.path.join(HERE, "batch_V.npy"), V32)
    meta = {"workload": wl.name, "kdims": list(wl.kdims), "iters": wl.iters, "refs": len(wl.refs),
            "eig_top": [float(x) for x in w[:4]], "learn_s": time.time() - t0, "instances": {}}
    print("batch V", json.dumps(meta), flush=True)
    for idx in BATCH_GOLDEN:
        p = wl.problems[idx]
        t1 = time.time()
        L, info = O.solve(p.M, p.mask, V32.astype(np.float64), wl.kdims, wl.iters)
        np.save(os.path.join(HERE, f"batch_{idx}_L.npy"), L)
        meta["instances"][str(idx)] = {"dims": list(p.dims), "mask_kind": p.meta["mask_kind"],
                                       "iters": info["iters"], "theta0": info["theta0"],
                                       "r_primal": info["r_primal"], "r_change": info["r_change"],
                                       "objective": info["objective"], "solve_s": time.time() - t1}
        print(idx, json.dumps(meta["instances"][str(idx)]), flush=True)
        with open(os.path.join(HERE, "batch_meta.json"), "w") as f:
            json.dump(meta, f, indent=1)


def make(name):
    if name == "batch":
        return make_batch()
    wl = WORKLOADS[name]()
    prob = wl.problems[0]
    t0 = time.time()
    V, w = O.learn(wl.refs, wl.kdims)
    V32 = V.astype(np.float32)
    t1 = time.time()
    L, info = O.solve(prob.M, prob.mask, V32.astype(np.float64), wl.kdims, wl.iters)
    t2 = time.time()
    np.save(os.path.join(HERE, f"{name}_V.npy"), V32)
    np.save(os.path.join(HERE, f"{name}_L.npy"), L)
    meta = {"workload": wl.name, "dims": list(prob.dims), "kdims": list(wl.kdims), "iters": info["iters"],
            "theta0": info["theta0"], "theta_final": info["theta_final"], "r_primal": info["r_primal"],
            "r_change": info["r_change"], "objective": info["objective"],
            "eig_top": [float(x) for x in w[:4]], "learn_s": t1 - t0, "solve_s": t2 - t1}
    with open(os.path.join(HERE, f"{name}_meta.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(name, json.dumps(meta), flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["16x16x8", "64x64x16"]:
        make(n)
