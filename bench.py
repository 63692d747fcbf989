"""Benchmark of the ICNNM solver on one MI355X.

A step is one complete solve (every ADMM iteration of Section III-D: column
norms and shrinkage, adjoint with col2im, L-step with P_Omega, forward
contraction with the fused dual update) of one synthetic tensor. The default
workload is the 64x64x16 video-shaped tensor with an 8x8x4 kernel (k = 256),
30% random plus 8x8 block missing entries, 200 iterations, FP32. The metric
is solved tensors per second with inputs resident in HBM.

Prints one JSON line with the throughput, per-solve latency percentiles, the
relative error against the stored FP64 oracle result, a roofline entry for
the dominant kernel (stage durations measured with HIP events on the
library's stream in a separate profiled pass) and the FP64 oracle's own rate
on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp32_mfma": 157.3, "bf16_mfma": 2500.0, "fp16_mfma": 2500.0, "hbm_gbs": 8000.0}
METRIC = "solved tensors/s at rel.err\u22641e-3 vs FP64 oracle; p50/p99 latency; vs plain FP32"

# HBM bytes per iterating launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, scaled by
# the same counters on a plain 256 MiB copy (fetch x2.0, write x1.0); valid only for the
# kernel source they were taken on (sha256 prefix of kernels.hip)
TRAFFIC = {
    ("64x64x16", "fp32", "forward"): {"bytes": 284.7e6, "src": "0331dca4bd7903ee"},
    ("64x64x16", "fp32", "adjoint"): {"bytes": 139.3e6, "src": "0331dca4bd7903ee"},
    ("128x128x32", "bf16", "forward"): {"bytes": 9.86e9, "src": "0331dca4bd7903ee"},
    ("128x128x32", "bf16", "adjoint"): {"bytes": 5.63e9, "src": "0331dca4bd7903ee"},
}


def _kernel_src_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_2604_17001_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _workload(name):
    from paper_2604_17001_amd import inputs
    return {"16x16x8": inputs.prediction_16x16x8, "64x64x16": inputs.video_64x64x16,
            "128x128x32": inputs.interpolation_128x128x32, "batch": inputs.batch_uneven}[name]()


def _count_tiles(infos):
    out = {}
    for i in infos:
        key = "x".join(str(x) for x in i["tile"])
        out[key] = out.get(key, 0) + 1
    return out


def _batch_main(args):
    """Batching form: 64 uneven instances (extents {32..128}^2 x {8,16,32}, 8x8x4 kernel,
    one shared V) solved in joint launches; a step is one solve of the whole batch."""
    import torch
    from paper_2604_17001_amd import icnnm
    if not args.no_autotune:
        # tile boxes measured per instance shape during the untimed warm-up
        os.environ["ICNNM_AUTOTUNE"] = "1"
    wl = _workload("batch")
    iters = args.iters or wl.iters
    lib = icnnm.Library.get()
    dev = torch.device("cuda", 0)
    Ms = [torch.from_numpy(p.M).to(dev) for p in wl.problems]
    masks = [torch.from_numpy(p.mask).to(dev) for p in wl.problems]
    outs = [torch.empty_like(x) for x in Ms]
    V, _ = lib.learn_eigvecs([torch.from_numpy(r).to(dev) for r in wl.refs], wl.kdims)
    kw = dict(max_iter=iters, precision=args.precision)
    for _ in range(args.warmup):
        lib.solve_batch(Ms, masks, V, wl.kdims, outs=outs, **kw)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, infos = lib.solve_batch(Ms, masks, V, wl.kdims, outs=outs, **kw)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = len(wl.problems)
    msum = sum(p.m for p in wl.problems)
    # one-at-a-time FP32 solves of the same instances, the baseline form (one untimed
    # pass first: per-shape set-up and, with autotuning, tile measurement)
    for M, mk, o in zip(Ms, masks, outs):
        lib.solve(M, mk, V, wl.kdims, out=o, max_iter=iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for M, mk, o in zip(Ms, masks, outs):
        lib.solve(M, mk, V, wl.kdims, out=o, max_iter=iters)
    torch.cuda.synchronize()
    single = n / (time.perf_counter() - t1)
    flops = 4.0 * msum * wl.problems[0].k ** 2 * iters
    out = {"metric": "solved tensors/s (uneven batch) at rel.err<=1e-3 vs FP64 oracle",
           "value": round(n * args.steps / dt, 3), "unit": "tensors/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else args.precision,
           "data": "synthetic",
           "config": {"workload": wl.name, "instances": n, "sum_m": msum, "kdims": list(wl.kdims),
                      "iters": iters, "precision": args.precision, "autotune": not args.no_autotune},
           "tiles": {k: v for k, v in sorted(_count_tiles(infos).items())},
           "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
           "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
           "tflops_effective": round(flops * args.steps / dt / 1e12, 2),
           "fp32_one_at_a_time_tensors_per_s": round(single, 3),
           "iters_run": [i["iters"] for i in infos][:4]}
    print(json.dumps(out), flush=True)


def _serve_main(args):
    """Serving form: Poisson arrivals of batch-type requests with a share of 128x128x32
    requests at a 16x16x4 kernel; each retired at max(r_primal, r_change) <= tol.
    The first ``--serve-warmup-frac`` of the requests (by arrival) warm the server up
    and are left out: tensors/s counts the other requests from the arrival of the
    first of them to the last retirement, and the latency percentiles
    (arrival to retirement) are over the same requests."""
    import torch
    from paper_2604_17001_amd import icnnm, inputs
    rate, n = args.rate, args.requests
    arrivals, probs = inputs.serve_requests(n, rate, large_frac=args.large_frac)
    lib = icnnm.Library(budget=int(args.budget_gb * (1 << 30)))
    dev = torch.device("cuda", 0)
    banks = {}
    for kd, gen in [((8, 8, 4), inputs.batch_uneven), ((16, 16, 4), inputs.interpolation_128x128x32)]:
        if any(tuple(p.kdims) == kd for p in probs):
            refs = gen(b_refs=4).refs if kd == (16, 16, 4) else gen(count=1).refs
            banks[kd] = lib.learn_eigvecs([torch.from_numpy(r).to(dev) for r in refs], kd)[0]
    Ms = [torch.from_numpy(p.M).to(dev) for p in probs]
    masks = [torch.from_numpy(p.mask).to(dev) for p in probs]
    outs = [torch.empty_like(x) for x in Ms]
    torch.cuda.synchronize()
    kw = dict(max_iter=args.iters or 1000, tol=args.tol, precision=args.precision)
    t0 = time.perf_counter()
    tickets, done, t_ret, iters = {}, {}, {}, {}
    nxt = 0
    while len(done) < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            p = probs[nxt]
            tickets[lib.submit(Ms[nxt], masks[nxt], banks[tuple(p.kdims)], p.kdims, outs[nxt], **kw)] = nxt
            nxt += 1
        for t, i in list(tickets.items()):
            rc, info = lib.poll(t)
            if rc != icnnm.PENDING:
                done[i] = rc
                t_ret[i] = time.perf_counter() - t0
                iters[i] = info["iters"]
                del tickets[t]
        time.sleep(0.0005)
    lib.close()
    n_warm = min(n - 1, int(args.serve_warmup_frac * n))
    meas = range(n_warm, n)
    window = max(t_ret[i] for i in meas) - arrivals[n_warm]
    nm = n - n_warm
    lat_ms = np.array([t_ret[i] - arrivals[i] for i in meas]) * 1e3
    out = {"metric": "served tensors/s at residual <= tol (continuous batching)", "value": round(nm / window, 3),
           "unit": "tensors/s", "n_gpus": 1, "steps": nm, "warmup": n_warm,
           "ms_per_step": round(1e3 * window / nm, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
           "data": "synthetic",
           "config": {"workload": "serve_poisson_mixed_sizes", "rate_req_s": rate, "requests": n,
                      "large_frac": args.large_frac, "tol": args.tol, "budget_gb": args.budget_gb,
                      "warmup_frac": args.serve_warmup_frac},
           "p50_ms": round(float(np.percentile(lat_ms, 50)), 2), "p99_ms": round(float(np.percentile(lat_ms, 99)), 2),
           "ok": int(sum(1 for v in done.values() if v == icnnm.OK)), "requests_total": n,
           "mean_iters": round(float(np.mean([iters[i] for i in meas])), 1)}
    print(json.dumps(out), flush=True)


def _cpu_baseline(prob, V, kdims, iters, sample_iters):
    """The FP64 oracle, untuned, on `sample_iters` iterations of the same solve."""
    from oracle import icnnm_ref as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    t0 = time.perf_counter()
    O.solve(prob.M, prob.mask, V.astype(np.float64), kdims, sample_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / sample_iters
    return {"value": 1.0 / (per_iter * iters), "unit": "tensors/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{sample_iters} of {iters} iterations of one solve ({dt:.1f} s), scaled to a full solve"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="64x64x16", choices=["16x16x8", "64x64x16", "128x128x32", "batch", "serve"],
                    help="16x16x8 prediction, 64x64x16 video (default), 128x128x32 interpolation at k=1024, "
                         "64-instance uneven batch, serving with Poisson arrivals")
    ap.add_argument("--rate", type=float, default=10.0, help="serve: Poisson arrival rate (req/s)")
    ap.add_argument("--requests", type=int, default=256, help="serve: number of requests")
    ap.add_argument("--serve-warmup-frac", type=float, default=0.10,
                    help="serve: share of the first requests left out of the figures")
    ap.add_argument("--large-frac", type=float, default=0.10, help="serve: share of 128x128x32 requests")
    ap.add_argument("--tol", type=float, default=1e-4, help="serve: retirement residual")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: HBM budget of the server")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--no-autotune", action="store_true", help="batch: cost-model tile boxes only")
    ap.add_argument("--cpu-sample-iters", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the other precision form (BF16 vs plain FP32) on the same workload")
    ap.add_argument("--iters", type=int, default=0, help="override the iteration count (short profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent instances shard across GPUs without communication", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return _batch_main(args)
    if args.workload == "serve":
        return _serve_main(args)

    import torch
    from paper_2604_17001_amd import icnnm

    wl = _workload(args.workload)
    if args.iters > 0:
        wl.iters = args.iters
    prob = wl.problems[0]
    kd = wl.kdims
    m, k = prob.m, prob.k
    lib = icnnm.Library.get()
    dev = torch.device("cuda", 0)
    M = torch.from_numpy(prob.M).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    refs = [torch.from_numpy(r).to(dev) for r in wl.refs]
    V, _ = lib.learn_eigvecs(refs, kd)          # pre-step, not timed
    L = torch.empty_like(M)
    kw = dict(max_iter=wl.iters, precision=args.precision)

    for _ in range(args.warmup):
        lib.solve(M, mask, V, kd, out=L, **kw)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, info = lib.solve(M, mask, V, kd, out=L, **kw)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt

    # accuracy against the stored FP64 oracle result (same float32 V)
    rel_err = None
    gV = os.path.join(ROOT, "tests", "golden", f"{args.workload}_V.npy")
    gL = os.path.join(ROOT, "tests", "golden", f"{args.workload}_L.npy")
    if os.path.exists(gV) and os.path.exists(gL) and args.iters == 0:
        Vg = torch.from_numpy(np.ascontiguousarray(np.load(gV))).to(dev)
        Lg, _ = lib.solve(M, mask, Vg, kd, **kw)
        ref = np.load(gL)
        rel_err = float(np.linalg.norm(Lg.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref))

    # stage durations with HIP events on the library stream (separate profiled pass)
    roofline, stages = None, None
    if not args.no_profile:
        lib.stage_times(reset=True)
        lib.set_profiling(True)
        nprof = 2
        for _ in range(nprof):
            lib.solve(M, mask, V, kd, out=L, **kw)
        lib.set_profiling(False)
        st = lib.stage_times(reset=True)
        working = {"colnorm": wl.iters + 1, "adjoint": wl.iters, "lstep": wl.iters + 1, "forward": wl.iters + 1}
        stages = {s: {"avg_us": 1e3 * ms / (nprof * working[s]), "launches": n} for s, (ms, n) in st.items()}
        dom = max(("forward", "adjoint"), key=lambda s: stages[s]["avg_us"])
        flops = 2.0 * m * k * k          # one m x k x k contraction per launch
        sec = stages[dom]["avg_us"] * 1e-6
        # algorithmic state bytes per launch: the forward reads and writes U and Q, the
        # adjoint reads them (FP32, m x kp entries each)
        kp = ((k + 63) // 64) * 64 if k <= 256 else ((k + 255) // 256) * 256
        abytes = (16.0 if dom == "forward" else 8.0) * m * kp
        tr = TRAFFIC.get((args.workload, args.precision, dom))
        traffic = tr["bytes"] if tr and tr["src"] == _kernel_src_hash() and args.iters == 0 else None
        mpeak = PEAKS["fp32_mfma"] if args.precision == "fp32" else PEAKS[f"{args.precision}_mfma"]
        tflops = flops / sec / 1e12
        if flops / abytes >= mpeak * 1e12 / (PEAKS["hbm_gbs"] * 1e9):
            # above the ridge point: the contraction bounds the kernel
            roofline = {"bound": "mfma", "kernel": dom, "achieved": round(tflops, 3), "peak": mpeak,
                        "unit": "TFLOP/s", "frac": round(tflops / mpeak, 4), "traffic": traffic,
                        "flops_per_launch": flops, "algorithmic_bytes_per_launch": abytes}
        else:
            # below it (reduced precision): the U/Q state traffic bounds the kernel
            gbs = abytes / sec / 1e9
            roofline = {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": PEAKS["hbm_gbs"],
                        "unit": "GB/s", "frac": round(gbs / PEAKS["hbm_gbs"], 4), "traffic": traffic,
                        "algorithmic_bytes_per_launch": abytes, "flops_per_launch": flops,
                        "mfma_tflops": round(tflops, 3), "mfma_frac": round(tflops / mpeak, 4)}

    if args.calibrate_copy:
        x = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(prob, V.cpu().numpy(), kd, wl.iters, args.cpu_sample_iters)

    # the same workload in the other form (BF16 against plain FP32 or the reverse), with
    # its own accuracy against the stored oracle result, for the "vs plain FP32" figure
    other = None
    if not args.no_compare and args.workload in ("16x16x8", "64x64x16", "128x128x32") and args.iters == 0:
        oprec = "bf16" if args.precision == "fp32" else "fp32"
        okw = dict(max_iter=wl.iters, precision=oprec)
        for _ in range(args.warmup):
            lib.solve(M, mask, V, kd, out=L, **okw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lib.solve(M, mask, V, kd, out=L, **okw)
        torch.cuda.synchronize()
        ovalue = args.steps / (time.perf_counter() - t0)
        oerr = None
        if os.path.exists(gV) and os.path.exists(gL):
            Lg, _ = lib.solve(M, mask, Vg, kd, **okw)
            oerr = float(np.linalg.norm(Lg.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref))
        fp32_value = value if args.precision == "fp32" else ovalue
        red_value = ovalue if args.precision == "fp32" else value
        other = {"precision": oprec, "value": round(ovalue, 3), "rel_err_vs_oracle": oerr,
                 "reduced_over_plain_fp32": round(red_value / fp32_value, 3)}

    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": round(value, 3), "unit": "tensors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": wl.name, "dims": list(prob.dims), "kdims": list(kd), "k": k,
                   "iters": wl.iters, "precision": args.precision, "lambda": "inf"},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3), "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "iter_us": round(1e3 * dt / args.steps / wl.iters * 1e3, 2),
        "rel_err_vs_oracle": rel_err, "iters_run": info["iters"],
        "roofline": roofline, "stages": stages, "cpu_baseline": cpu, "other_form": other,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
