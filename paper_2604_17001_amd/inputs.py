"""Seeded synthetic inputs for tensor completion with arbitrary sampling (TCAS).

This module only draws data: target tensors, sampling masks, reference
ensembles and arrival times. It holds none of the method's arithmetic, so both
the FP64 oracle's tests and the GPU path consume the exact same FP32 arrays.

Problem statement: a target tensor L0 of order n and an arbitrary sampling set
Omega of observed entries (Definition 1, Introduction); Omega is carried as a
0/1 ``uint8`` mask (the mask tensor of Section II-B). Percentages below are
*missing* rates, the paper's convention for its image and video experiments
(Section V).

Every random stream is ``numpy.random.default_rng(SeedSequence([cfg, role,
idx]))`` with role 0 = target, 1 = references, 2 = mask, 3 = arrivals. Values
are generated in float64 and rounded to float32 once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROLE_TARGET, ROLE_REFS, ROLE_MASK, ROLE_ARRIVALS = 0, 1, 2, 3


def rng(cfg: int, role: int, idx: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(role), int(idx)]))


# ----------------------------------------------------------------------------- values

def cosine_sum(dims, r, g: np.random.Generator, sigma=0.0, scale01=False,
               separable=False) -> np.ndarray:
    """Sum of ``r`` real cosines on the integer DFT grid plus N(0, sigma) noise.

    * non-separable: cos(2*pi*sum_j u_j x_j / m_j + phi)
    * separable:     prod_j cos(2*pi*u_j x_j / m_j + phi_j)
    with u_j ~ U{0..floor(m_j/2)} and phases ~ U[0, 2*pi). Integer grid
    frequencies make the circular-convolution rank at most 2r (8r separable)
    before noise. ``scale01`` applies min-max scaling after the noise.
    """
    dims = tuple(int(d) for d in dims)
    grids = np.meshgrid(*[np.arange(d, dtype=np.float64) for d in dims], indexing="ij")
    out = np.zeros(dims, dtype=np.float64)
    for _ in range(int(r)):
        u = [int(g.integers(0, d // 2 + 1)) for d in dims]
        if separable:
            term = np.ones(dims, dtype=np.float64)
            for j, d in enumerate(dims):
                phi = g.uniform(0.0, 2.0 * math.pi)
                term = term * np.cos(2.0 * math.pi * u[j] * grids[j] / d + phi)
            out += term
        else:
            phi = g.uniform(0.0, 2.0 * math.pi)
            arg = sum(2.0 * math.pi * u[j] * grids[j] / d for j, d in enumerate(dims))
            out += np.cos(arg + phi)
    if sigma > 0:
        out += g.normal(0.0, sigma, size=dims)
    if scale01:
        lo, hi = out.min(), out.max()
        out = (out - lo) / (hi - lo) if hi > lo else np.zeros_like(out)
    return out.astype(np.float32)


# ----------------------------------------------------------------------------- masks

def mask_frames(dims, observed_frames) -> np.ndarray:
    """Observe whole frames (last axis) listed in ``observed_frames``."""
    m = np.zeros(dims, dtype=np.uint8)
    m[..., list(observed_frames)] = 1
    return m


def mask_trailing_missing(dims, n_missing) -> np.ndarray:
    """Prediction pattern: the last ``n_missing`` frames are unobserved."""
    m = np.ones(dims, dtype=np.uint8)
    if n_missing > 0:
        m[..., dims[-1] - n_missing:] = 0
    return m


def mask_every_other_frame(dims) -> np.ndarray:
    """Interpolation pattern: even frames observed, odd frames missing."""
    return mask_frames(dims, range(0, dims[-1], 2))


def mask_random_missing(dims, p_missing, g: np.random.Generator) -> np.ndarray:
    return (g.random(dims) >= p_missing).astype(np.uint8)


def mask_random_plus_blocks(dims, p_missing, block, block_frac, g) -> np.ndarray:
    """Bernoulli(p_missing) missing entries united with grid-aligned missing blocks.

    The blocks tile the volume on a regular grid; ``round(block_frac * slots)``
    slots are drawn without replacement and removed.
    """
    m = mask_random_missing(dims, p_missing, g)
    nb = [d // b for d, b in zip(dims, block)]
    slots = int(np.prod(nb))
    n_pick = int(round(block_frac * slots))
    picks = g.choice(slots, size=n_pick, replace=False)
    for flat in picks:
        c = np.unravel_index(int(flat), nb)
        sl = tuple(slice(ci * b, (ci + 1) * b) for ci, b in zip(c, block))
        m[sl] = 0
    return m


# ----------------------------------------------------------------------------- problems

@dataclass
class Problem:
    """One completion instance: observed tensor M (= L0 here), mask, kernel size."""
    dims: tuple
    kdims: tuple
    M: np.ndarray            # float32, C-order
    mask: np.ndarray         # uint8, 1 = observed
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return int(np.prod(self.dims))

    @property
    def k(self):
        return int(np.prod(self.kdims))


@dataclass
class Workload:
    name: str
    kdims: tuple
    problems: list
    refs: list               # float32 reference tensors for learning V
    iters: int
    meta: dict = field(default_factory=dict)


def _refs(cfg, gen_one, b):
    return [gen_one(rng(cfg, ROLE_REFS, j)) for j in range(b)]


def prediction_16x16x8(b_refs=20) -> Workload:
    """16x16x8 tensor, 8x8x4 kernel, r=5 separable cosines + N(0,1e-3);
    frames 1-6 observed, 7-8 missing (prediction); 100 iterations."""
    dims, kd = (16, 16, 8), (8, 8, 4)
    gen = lambda g: cosine_sum(dims, 5, g, sigma=1e-3, separable=True)
    M = gen(rng(1, ROLE_TARGET))
    mask = mask_trailing_missing(dims, 2)
    return Workload("prediction_16x16x8_k8x8x4", kd, [Problem(dims, kd, M, mask, "16x16x8")],
                    _refs(1, gen, b_refs), 100)


def video_64x64x16(b_refs=20) -> Workload:
    """64x64x16 tensor, 8x8x4 kernel, r=12 cosines + N(0,1e-2), scaled to [0,1];
    30% random missing plus 8x8x1 missing blocks over 15% of the volume; 200 it."""
    dims, kd = (64, 64, 16), (8, 8, 4)
    gen = lambda g: cosine_sum(dims, 12, g, sigma=1e-2, scale01=True)
    M = gen(rng(2, ROLE_TARGET))
    mask = mask_random_plus_blocks(dims, 0.30, (8, 8, 1), 0.15, rng(2, ROLE_MASK))
    return Workload("video_64x64x16_k8x8x4", kd, [Problem(dims, kd, M, mask, "64x64x16")],
                    _refs(2, gen, b_refs), 200)


def interpolation_128x128x32(b_refs=20) -> Workload:
    """128x128x32 tensor, 16x16x4 kernel, r=20 cosines + N(0,1e-2), scaled [0,1];
    even frames observed (frame interpolation); 100 iterations."""
    dims, kd = (128, 128, 32), (16, 16, 4)
    gen = lambda g: cosine_sum(dims, 20, g, sigma=1e-2, scale01=True)
    M = gen(rng(3, ROLE_TARGET))
    mask = mask_every_other_frame(dims)
    return Workload("interpolation_128x128x32_k16x16x4", kd, [Problem(dims, kd, M, mask, "128x128x32")],
                    _refs(3, gen, b_refs), 100)


BATCH_SPATIAL = (32, 48, 64, 96, 128)
BATCH_FRAMES = (8, 16, 32)


def batch_instance(cfg, idx, kdims=(8, 8, 4)) -> Problem:
    """One instance of the uneven batch: m1, m2 ~ U{32,48,64,96,128}, m3 ~ U{8,16,32};
    values as the 64x64x16 generator; the mask is one of three types drawn uniformly:
    40% random missing / last ceil(m3/4) frames missing / odd frames missing."""
    g = rng(cfg, ROLE_TARGET, idx)
    dims = (int(g.choice(BATCH_SPATIAL)), int(g.choice(BATCH_SPATIAL)), int(g.choice(BATCH_FRAMES)))
    M = cosine_sum(dims, 12, g, sigma=1e-2, scale01=True)
    gm = rng(cfg, ROLE_MASK, idx)
    kind = int(gm.integers(0, 3))
    if kind == 0:
        mask = mask_random_missing(dims, 0.40, gm)
    elif kind == 1:
        mask = mask_trailing_missing(dims, int(math.ceil(dims[2] / 4)))
    else:
        mask = mask_every_other_frame(dims)
    return Problem(dims, tuple(kdims), M, mask, f"batch_{idx}", {"mask_kind": kind})


def batch_uneven(count=64, b_refs=20) -> Workload:
    kd = (8, 8, 4)
    probs = [batch_instance(4, i, kd) for i in range(count)]

    def ref(g):
        dims = (int(g.choice(BATCH_SPATIAL)), int(g.choice(BATCH_SPATIAL)), int(g.choice(BATCH_FRAMES)))
        return cosine_sum(dims, 12, g, sigma=1e-2, scale01=True)
    return Workload("batch_64_uneven_k8x8x4", kd, probs, _refs(4, ref, b_refs), 200)


def serve_requests(n, rate, large_frac=0.10, cfg=5):
    """Serving stream: Poisson arrivals at ``rate`` req/s; each request is a batch-type
    instance, or with probability ``large_frac`` a 128x128x32 interpolation instance
    at kernel 16x16x4. Returns (arrival_times, problems)."""
    ga = rng(cfg, ROLE_ARRIVALS, int(rate * 1000))
    gaps = ga.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    probs = []
    for i in range(n):
        if ga.random() < large_frac:
            dims, kd = (128, 128, 32), (16, 16, 4)
            M = cosine_sum(dims, 20, rng(cfg, ROLE_TARGET, 100000 + i), sigma=1e-2, scale01=True)
            probs.append(Problem(dims, kd, M, mask_every_other_frame(dims), f"s{i}L"))
        else:
            probs.append(batch_instance(cfg, i))
    return t, probs


def random_problem(dims, kdims, p_missing, seed, sigma=1e-2, r=4) -> Problem:
    """Small generic instance for parity sweeps (any order, ragged shapes)."""
    g = rng(900 + seed, ROLE_TARGET)
    M = cosine_sum(dims, r, g, sigma=sigma, scale01=True)
    mask = mask_random_missing(dims, p_missing, rng(900 + seed, ROLE_MASK))
    return Problem(tuple(dims), tuple(kdims), M, mask, f"rand{seed}")


def random_refs(dims, b, seed, sigma=1e-2, r=4):
    return [cosine_sum(dims, r, rng(900 + seed, ROLE_REFS, j), sigma=sigma, scale01=True)
            for j in range(b)]
