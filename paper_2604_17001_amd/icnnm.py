"""Python binding of the ICNNM C ABI (include/icnnm.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory and the current stream; tensors are passed to
the library as raw device pointers. The library is loaded from the package
directory (built by ``paper_2604_17001_amd.build``); if it is missing or no
GPU is present, calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libicnnm.so")

OK, PENDING = 0, 1
E_INVALID, E_NOMEM, E_BUDGET, E_DEVICE, E_NUMERIC, E_NOTFOUND = -1, -2, -3, -4, -5, -6
PREC = {"fp32": 0, "bf16": 1, "fp16": 2}

EXPORTS = ["icnnm_params_default", "icnnm_create", "icnnm_destroy", "icnnm_last_error", "icnnm_plan",
           "icnnm_learn_eigvecs", "icnnm_diagnostics", "icnnm_solve", "icnnm_solve_noalloc", "icnnm_solve_batch",
           "icnnm_submit",
           "icnnm_poll",
           "icnnm_set_profiling", "icnnm_stage_times"]
STAGES = ("colnorm", "adjoint", "lstep", "forward")


class Shape(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("m", C.c_int64 * 3), ("kdim", C.c_int64 * 3)]


class Params(C.Structure):
    _fields_ = [("lam", C.c_double), ("theta0", C.c_double), ("rho", C.c_double),
                ("theta_max", C.c_double), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("precision", C.c_int32), ("refresh_every", C.c_int32), ("check_v", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("r_primal", C.c_double),
                ("r_change", C.c_double), ("objective", C.c_double), ("theta_final", C.c_double),
                ("t_queue_s", C.c_double), ("t_device_s", C.c_double), ("tile", C.c_int32 * 3),
                ("split", C.c_int32), ("refresh_x3", C.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["tile"] = tuple(self.tile)
        return d


class PlanInfo(C.Structure):
    _fields_ = [("tile", C.c_int32 * 3), ("tiles_per_dim", C.c_int32 * 3), ("ntiles", C.c_int32),
                ("padded_k", C.c_int32), ("state_bytes", C.c_int64), ("split", C.c_int32)]


class IcnnmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"icnnm error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"ICNNM HIP library not built: {path} is missing "
                           "(run python -m paper_2604_17001_amd.build)")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.icnnm_params_default.argtypes = [C.POINTER(Params)]
    lib.icnnm_params_default.restype = None
    lib.icnnm_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(P)]
    lib.icnnm_create.restype = C.c_int32
    lib.icnnm_destroy.argtypes = [P]
    lib.icnnm_destroy.restype = None
    lib.icnnm_last_error.argtypes = [P]
    lib.icnnm_last_error.restype = C.c_char_p
    lib.icnnm_plan.argtypes = [C.POINTER(Shape), C.POINTER(Params), C.c_int32, C.POINTER(PlanInfo)]
    lib.icnnm_plan.restype = C.c_int32
    lib.icnnm_learn_eigvecs.argtypes = [P, C.POINTER(C.c_int64), C.c_int32, C.POINTER(Shape),
                                        C.POINTER(P), P, C.POINTER(C.c_double), P]
    lib.icnnm_learn_eigvecs.restype = C.c_int32
    lib.icnnm_diagnostics.argtypes = [P, C.POINTER(Shape), P, P, C.c_double, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_double), P]
    lib.icnnm_diagnostics.restype = C.c_int32
    lib.icnnm_solve.argtypes = [P, C.POINTER(Shape), P, P, P, C.POINTER(Params), P, C.POINTER(Info), P]
    lib.icnnm_solve.restype = C.c_int32
    lib.icnnm_solve_noalloc.argtypes = [P, C.POINTER(Shape), P, P, P, C.POINTER(Params), P, C.POINTER(Info), P]
    lib.icnnm_solve_noalloc.restype = C.c_int32
    lib.icnnm_solve_batch.argtypes = [P, C.c_int32, C.POINTER(Shape), C.POINTER(P), C.POINTER(P), P,
                                      C.POINTER(Params), C.POINTER(P), C.POINTER(Info), P]
    lib.icnnm_solve_batch.restype = C.c_int32
    lib.icnnm_submit.argtypes = [P, C.POINTER(Shape), P, P, P, C.POINTER(Params), P, C.POINTER(C.c_uint64)]
    lib.icnnm_submit.restype = C.c_int32
    lib.icnnm_poll.argtypes = [P, C.c_uint64, C.POINTER(Info)]
    lib.icnnm_poll.restype = C.c_int32
    lib.icnnm_set_profiling.argtypes = [P, C.c_int32]
    lib.icnnm_set_profiling.restype = C.c_int32
    lib.icnnm_stage_times.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
    lib.icnnm_stage_times.restype = C.c_int32
    return lib


def make_shape(dims, kdims) -> Shape:
    dims, kdims = tuple(int(d) for d in dims), tuple(int(d) for d in kdims)
    if len(dims) != len(kdims):
        raise ValueError("dims and kdims must have the same length")
    s = Shape()
    s.ndim = len(dims)
    for i, (d, k) in enumerate(zip(dims, kdims)):
        s.m[i] = d
        s.kdim[i] = k
    return s


def make_params(lib, max_iter=100, lam=math.inf, theta0=0.0, rho=1.1, theta_max=1e10, tol=0.0,
                precision="fp32", refresh_every=10, check_v=False) -> Params:
    p = Params()
    lib.icnnm_params_default(C.byref(p))
    p.lam, p.theta0, p.rho, p.theta_max = float(lam), float(theta0), float(rho), float(theta_max)
    p.max_iter, p.tol = int(max_iter), float(tol)
    p.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    p.refresh_every, p.check_v = int(refresh_every), int(bool(check_v))
    return p


def plan(dims, kdims, joint=False, lib=None, **kw):
    """Host-only tile plan of one instance (icnnm_plan; no GPU needed). Returns a dict
    with the tile box, tiles per dimension, tile count, padded k, state bytes and
    whether the contractions take their split form, or raises IcnnmError."""
    lib = lib or load_library()
    shape = make_shape(dims, kdims)
    p = make_params(lib, **kw)
    out = PlanInfo()
    rc = lib.icnnm_plan(C.byref(shape), C.byref(p), int(bool(joint)), C.byref(out))
    if rc != OK:
        raise IcnnmError(rc, "icnnm_plan failed")
    return {"tile": tuple(out.tile), "tiles_per_dim": tuple(out.tiles_per_dim), "ntiles": int(out.ntiles),
            "padded_k": int(out.padded_k), "state_bytes": int(out.state_bytes), "split": bool(out.split)}


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_tensor(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Library:
    """Process-wide handle on libicnnm.so and a default context on the current device."""
    _inst = None

    def __init__(self, device=None, budget=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("ICNNM needs a HIP GPU; none is available")
        self.lib = load_library()
        dev = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        rc = self.lib.icnnm_create(dev, C.c_size_t(int(budget)), C.byref(h))
        if rc != OK:
            raise IcnnmError(rc, "icnnm_create failed")
        self.ctx = h
        self.device = dev

    @classmethod
    def get(cls):
        if cls._inst is None:
            cls._inst = Library()
        return cls._inst

    def close(self):
        if self.ctx:
            self.lib.icnnm_destroy(self.ctx)
            self.ctx = None

    def _raise(self, rc):
        msg = self.lib.icnnm_last_error(self.ctx)
        raise IcnnmError(rc, msg.decode() if msg else "")

    # ------------------------------------------------------------------ API
    def params(self, **kw) -> Params:
        return make_params(self.lib, **kw)

    def learn_eigvecs(self, refs, kdims):
        """Learn the k x k eigenvector bank V from reference tensors (Definition 3)."""
        import torch
        b = len(refs)
        for i, r in enumerate(refs):
            _check_tensor(r, torch.float32, name=f"refs[{i}]")
        kd = tuple(int(x) for x in kdims)
        k = int(np.prod(kd))
        shapes = (Shape * b)(*[make_shape(r.shape, kd) for r in refs])
        ptrs = (C.c_void_p * b)(*[r.data_ptr() for r in refs])
        kk = (C.c_int64 * 3)(*(list(kd) + [1] * (3 - len(kd))))
        V = torch.empty((k, k), dtype=torch.float32, device=refs[0].device)
        w = np.zeros(k, dtype=np.float64)
        rc = self.lib.icnnm_learn_eigvecs(self.ctx, kk, b, shapes, ptrs, _ptr(V),
                                          w.ctypes.data_as(C.POINTER(C.c_double)), _stream())
        if rc != OK:
            self._raise(rc)
        return V, w

    def diagnostics(self, L0, V, kdims, rtol=1e-10):
        """Relative convolution eigenvalues, relative rank and spectral correlation of
        L0 under V (Definition 2, eq:rkL0, eq:alphaK). Returns (sigma, r_K, alpha_K)."""
        import torch
        _check_tensor(L0, torch.float32, name="L0")
        k = int(np.prod(kdims))
        _check_tensor(V, torch.float32, (k, k), name="V")
        shape = make_shape(L0.shape, kdims)
        sigma = np.zeros(k, dtype=np.float64)
        rank = C.c_int32(0)
        alpha = C.c_double(0.0)
        rc = self.lib.icnnm_diagnostics(self.ctx, C.byref(shape), _ptr(L0), _ptr(V), float(rtol),
                                        sigma.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rank),
                                        C.byref(alpha), _stream())
        if rc != OK:
            self._raise(rc)
        return sigma, int(rank.value), float(alpha.value)

    def solve(self, M, mask, V, kdims, out=None, **kw):
        """Complete one tensor. Returns (L, info dict)."""
        import torch
        _check_tensor(M, torch.float32, name="M")
        _check_tensor(mask, torch.uint8, M.shape, name="mask")
        k = int(np.prod(kdims))
        _check_tensor(V, torch.float32, (k, k), name="V")
        L = torch.empty_like(M) if out is None else out
        _check_tensor(L, torch.float32, M.shape, name="out")
        shape = make_shape(M.shape, kdims)
        p = self.params(**kw)
        info = Info()
        rc = self.lib.icnnm_solve(self.ctx, C.byref(shape), _ptr(M), _ptr(mask), _ptr(V), C.byref(p),
                                  _ptr(L), C.byref(info), _stream())
        if rc != OK:
            self._raise(rc)
        return L, info.as_dict()

    def solve_noalloc(self, M, mask, V, kdims, out, **kw):
        """icnnm_solve without device allocation inside the library (the caller passes
        the output buffer; solver state lives in the library's fixed scratch)."""
        import torch
        _check_tensor(M, torch.float32, name="M")
        _check_tensor(mask, torch.uint8, M.shape, name="mask")
        k = int(np.prod(kdims))
        _check_tensor(V, torch.float32, (k, k), name="V")
        _check_tensor(out, torch.float32, M.shape, name="out")
        shape = make_shape(M.shape, kdims)
        p = self.params(**kw)
        info = Info()
        rc = self.lib.icnnm_solve_noalloc(self.ctx, C.byref(shape), _ptr(M), _ptr(mask), _ptr(V), C.byref(p),
                                          _ptr(out), C.byref(info), _stream())
        if rc != OK:
            self._raise(rc)
        return out, info.as_dict()

    def solve_batch(self, Ms, masks, V, kdims, outs=None, **kw):
        import torch
        n = len(Ms)
        k = int(np.prod(kdims))
        _check_tensor(V, torch.float32, (k, k), name="V")
        outs = [torch.empty_like(M) for M in Ms] if outs is None else outs
        for i in range(n):
            _check_tensor(Ms[i], torch.float32, name=f"M[{i}]")
            _check_tensor(masks[i], torch.uint8, Ms[i].shape, name=f"mask[{i}]")
            _check_tensor(outs[i], torch.float32, Ms[i].shape, name=f"out[{i}]")
        shapes = (Shape * n)(*[make_shape(M.shape, kdims) for M in Ms])
        pm = (C.c_void_p * n)(*[M.data_ptr() for M in Ms])
        pk = (C.c_void_p * n)(*[x.data_ptr() for x in masks])
        po = (C.c_void_p * n)(*[x.data_ptr() for x in outs])
        infos = (Info * n)()
        p = self.params(**kw)
        rc = self.lib.icnnm_solve_batch(self.ctx, n, shapes, pm, pk, _ptr(V), C.byref(p), po, infos,
                                        _stream())
        if rc != OK:
            self._raise(rc)
        return outs, [i.as_dict() for i in infos]

    def submit(self, M, mask, V, kdims, out, **kw) -> int:
        import torch
        _check_tensor(M, torch.float32, name="M")
        _check_tensor(mask, torch.uint8, M.shape, name="mask")
        _check_tensor(out, torch.float32, M.shape, name="out")
        shape = make_shape(M.shape, kdims)
        p = self.params(**kw)
        t = C.c_uint64()
        rc = self.lib.icnnm_submit(self.ctx, C.byref(shape), _ptr(M), _ptr(mask), _ptr(V), C.byref(p),
                                   _ptr(out), C.byref(t))
        if rc != OK:
            self._raise(rc)
        return int(t.value)

    def set_profiling(self, on: bool):
        rc = self.lib.icnnm_set_profiling(self.ctx, int(bool(on)))
        if rc != OK:
            self._raise(rc)

    def stage_times(self, reset=True, split=False):
        """{stage: (total_ms, launches)} accumulated while profiling was on; with
        split=True, {(stage, "fp32" | "lowp"): ...}, where "lowp" holds the rounds whose
        contractions both ran as BF16/FP16 deltas and "fp32" the others (FP32 solves,
        initialisation, refresh rounds: FP32 contractions, or split BF16 where the
        solve's info reports refresh_x3)."""
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        rc = self.lib.icnnm_stage_times(self.ctx, ms, n, int(bool(reset)))
        if rc != OK:
            self._raise(rc)
        if split:
            return {(name, part): (ms[4 * j + i], int(n[4 * j + i]))
                    for j, part in enumerate(("fp32", "lowp")) for i, name in enumerate(STAGES)}
        return {name: (ms[i] + ms[4 + i], int(n[i] + n[4 + i])) for i, name in enumerate(STAGES)}

    def poll(self, ticket):
        """Returns (status, info dict); status PENDING while the request runs."""
        info = Info()
        rc = self.lib.icnnm_poll(self.ctx, C.c_uint64(ticket), C.byref(info))
        return rc, info.as_dict()
