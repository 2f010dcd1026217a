"""Seeded synthetic workloads for NNCP.

This module only draws random numbers and assembles test tensors. It holds
none of the decomposition's arithmetic (no MTTKRP, no factor updates, no
fit), so both the FP64 oracle and the GPU path can take their inputs from it
without sharing any of the method. The one norm it computes is the noise
scale of a generated tensor (the clean part's Frobenius norm; for the
slab-wise generator by its closed form over the factors' Gram matrices), a
property of the input, not a step either side takes from here.

Conventions used throughout the package:

* A dense N-way tensor of shape ``(I_1, ..., I_N)`` is stored linearly with
  mode 1 varying fastest, the natural generalisation of column-major order
  (Section IV-C, data distribution). Here every tensor is returned as a
  numpy array in Fortran order, so ``X.ravel(order="F")`` is the device
  layout.
* A factor matrix ``H^(n)`` is ``I_n x R`` and column-major (Fortran order).

Workload recipes (the paper's datasets are not available, so these stand in
for them with the same shapes):

* ``planted``: a sum of R rank-one terms whose factors are drawn from
  U[0, 1), plus Gaussian noise whose Frobenius norm is a given fraction of
  the clean tensor's norm, then clipped at zero (Section V-A describes
  exact-low-rank synthetic tensors; noise is added on top for benchmarks).
* ``hsi_like``: a 4-way hyperspectral time-lapse cube (rows x cols x bands x
  time) built from separable Gaussian spatial bumps, Gaussian spectral
  curves over 400..720 nm in 10 nm steps, and slowly varying temporal
  gains (shape of the Nogueiro scene dataset, Section V-A).
* ``init_factors``: the U[0, 1) starting factors passed to both sides.
"""

from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np


def _as_dims(dims: Sequence[int]) -> Tuple[int, ...]:
    dims = tuple(int(d) for d in dims)
    if len(dims) < 2 or any(d < 1 for d in dims):
        raise ValueError(f"bad tensor shape {dims}")
    return dims


def uniform_factors(dims: Sequence[int], R: int, seed: int) -> List[np.ndarray]:
    """N factor matrices with entries U[0,1), drawn in mode order 1..N."""
    rng = np.random.default_rng(seed)
    return [np.asfortranarray(rng.random((d, R))) for d in _as_dims(dims)]


def init_factors(dims: Sequence[int], R: int, seed: int) -> List[np.ndarray]:
    """Initial factors for a run: all N modes drawn U[0,1) (FP64)."""
    return uniform_factors(dims, R, seed)


def model_tensor(factors: Sequence[np.ndarray], dtype=np.float64) -> np.ndarray:
    """Assemble sum_r H1(:,r) o H2(:,r) o ... o HN(:,r) as a Fortran array.

    The outer products of the first N-1 factors are formed column by column
    (one rank-one term per column, first mode fastest) and contracted with
    the last factor in one matrix product, so the result is built slab by
    slab along the last mode without an N-fold Python loop.
    """
    dims = tuple(f.shape[0] for f in factors)
    R = factors[0].shape[1]
    # outer-product matrix of modes 1..N-1: row index = i_1 + I_1*(i_2 + ...)
    P = np.asarray(factors[0], dtype=np.float64)
    for f in factors[1:-1]:
        P = (f[None, :, :] * P[:, None, :]).reshape(-1, R, order="F")
    last = np.asarray(factors[-1], dtype=np.float64)
    out = np.empty(dims, dtype=dtype, order="F")
    flat = out.reshape(-1, dims[-1], order="F")  # view: column j = slab i_N = j
    step = max(1, (1 << 26) // max(1, P.shape[0]))
    for j0 in range(0, dims[-1], step):
        j1 = min(dims[-1], j0 + step)
        flat[:, j0:j1] = P @ last[j0:j1].T
    return out


def add_noise_clip(Xc: np.ndarray, level: float, seed: int, dtype=np.float64) -> np.ndarray:
    """X = max(0, Xc + level * ||Xc||_F / ||E||_F * E), E ~ N(0,1) i.i.d.

    E is drawn in the tensor's linear (mode-1-fastest) order. ``level`` is the
    noise fraction (0.01 for "1% noise"). Work is done in chunks so a
    multi-GB tensor does not need a second full-size FP64 temporary.
    """
    out = np.empty(Xc.shape, dtype=dtype, order="F")
    if level == 0.0:
        out[...] = np.maximum(Xc, 0)
        return out
    rng = np.random.default_rng(seed)
    src = Xc.reshape(-1, order="F")
    dst = out.reshape(-1, order="F")
    n = src.size
    chunk = 1 << 24
    # pass 1: norms (E is regenerated in pass 2 from the same seed)
    xc2 = 0.0
    e2 = 0.0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        e = rng.standard_normal(b - a)
        xs = src[a:b].astype(np.float64, copy=False)
        xc2 += float(np.dot(xs, xs))
        e2 += float(np.dot(e, e))
    scale = level * math.sqrt(xc2) / math.sqrt(e2)
    rng = np.random.default_rng(seed)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        e = rng.standard_normal(b - a)
        v = src[a:b].astype(np.float64, copy=False) + scale * e
        np.maximum(v, 0.0, out=v)
        dst[a:b] = v
    return out


def planted(dims: Sequence[int], R: int, noise: float, seed: int,
            dtype=np.float64) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Planted nonnegative rank-R tensor plus clipped Gaussian noise.

    Returns (X, truth_factors). Factors are U[0,1) from ``seed``; the noise
    stream uses ``seed + 7919`` so that it is independent of the factors.
    """
    dims = _as_dims(dims)
    truth = uniform_factors(dims, R, seed)
    Xc = model_tensor(truth, dtype=np.float64 if noise else dtype)
    if noise == 0.0:
        return Xc.astype(dtype, copy=False), truth
    X = add_noise_clip(Xc, noise, seed + 7919, dtype=dtype)
    del Xc
    return X, truth


def hsi_factors(dims: Sequence[int], R: int, seed: int) -> List[np.ndarray]:
    """Factors of a hyperspectral time-lapse cube (rows, cols, bands, time).

    * spatial modes: 1-D Gaussian bumps, centre U[0, I), width U[16, 160]
      pixels, plus a 0.01 floor, so each component's spatial map is a
      separable smooth bump;
    * band mode: a Gaussian over the band wavelengths 400, 410, ... nm with
      centre U[400, 720] nm, width U[20, 120] nm, plus a 0.02 baseline;
    * time mode: 1 + 0.5 sin(2 pi f t + phi), f U[0.02, 0.2], phi U[0, 2 pi).
    """
    dims = _as_dims(dims)
    if len(dims) != 4:
        raise ValueError("hsi_factors expects (rows, cols, bands, time)")
    rng = np.random.default_rng(seed)
    out = []
    for d in dims[:2]:
        x = np.arange(d, dtype=np.float64)[:, None]
        c = rng.uniform(0, d, size=(1, R))
        w = rng.uniform(16, 160, size=(1, R))
        out.append(np.asfortranarray(np.exp(-0.5 * ((x - c) / w) ** 2) + 0.01))
    lam = 400.0 + 10.0 * np.arange(dims[2], dtype=np.float64)[:, None]
    c = rng.uniform(400, 720, size=(1, R))
    w = rng.uniform(20, 120, size=(1, R))
    out.append(np.asfortranarray(np.exp(-0.5 * ((lam - c) / w) ** 2) + 0.02))
    t = np.arange(dims[3], dtype=np.float64)[:, None]
    f = rng.uniform(0.02, 0.2, size=(1, R))
    ph = rng.uniform(0, 2 * np.pi, size=(1, R))
    out.append(np.asfortranarray(1.0 + 0.5 * np.sin(2 * np.pi * f * t + ph)))
    return out


def hsi_like(dims: Sequence[int], R: int, noise: float, seed: int,
             dtype=np.float32) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Hyperspectral-shaped planted tensor (rank R) plus clipped noise."""
    truth = hsi_factors(dims, R, seed)
    Xc = model_tensor(truth)
    X = add_noise_clip(Xc, noise, seed + 7919, dtype=dtype)
    del Xc
    return X, truth


def hsi_like_device(dims: Sequence[int], R: int, noise: float, seed: int, device="cuda"):
    """The ``hsi_like`` recipe assembled with torch on a device (the factors are
    the same ``hsi_factors`` draws; the clean tensor is formed in FP32 and the
    N(0,1) noise comes from a seeded torch generator, so the values differ from
    ``hsi_like``). X = max(0, X_c + noise * ||X_c|| / ||E|| * E). Returns the flat
    FP32 tensor, mode 1 fastest."""
    import torch
    dims = _as_dims(dims)
    fs = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(device)
          for f in hsi_factors(dims, R, seed)]
    P = fs[0]
    for f in fs[1:-1]:
        P = (f[:, None, :] * P[None, :, :]).reshape(-1, R)
    X = (fs[-1] @ P.T).reshape(-1)
    del P
    if noise:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) + 7919)
        E = torch.randn(X.numel(), generator=g, device=device, dtype=torch.float32)
        scale = noise * torch.linalg.vector_norm(X.double()) / torch.linalg.vector_norm(E.double())
        X.add_(E, alpha=float(scale))
        del E
        X.clamp_(min=0.0)
    return X


def batch_shapes(n_jobs: int, seed: int, lo: int = 32, hi: int = 256,
                 ranks: Sequence[int] = (8, 16, 32)) -> List[Tuple[Tuple[int, int, int], int]]:
    """Shapes and ranks of a batch of 3-way jobs: dims U{lo..hi}, R from ``ranks``."""
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(n_jobs):
        d = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        R = int(rng.choice(np.asarray(ranks)))
        jobs.append((d, R))
    return jobs


def serving_job_shape(rng: np.random.Generator, min_entries: float = 1e5,
                      max_entries: float = 2e8, orders=(3, 4, 5),
                      ranks=(8, 16, 32, 64), min_dim: int = 4) -> Tuple[Tuple[int, ...], int]:
    """One job of a serving stream: order N, log-uniform size, Dirichlet split.

    log I ~ U[ln min_entries, ln max_entries]; the per-mode shares of log I
    follow a Dirichlet(1) draw; each dim is rounded and at least ``min_dim``.
    """
    N = int(rng.choice(np.asarray(orders)))
    logI = rng.uniform(math.log(min_entries), math.log(max_entries))
    w = rng.dirichlet(np.ones(N))
    dims = tuple(max(min_dim, int(round(math.exp(logI * wi)))) for wi in w)
    R = int(rng.choice(np.asarray(ranks)))
    return dims, R


def planted_device(dims: Sequence[int], R: int, noise: float, seed: int, device="cuda"):
    """The ``planted`` recipe drawn with torch on a device (for large serving
    jobs, where host generation would dominate): factors U[0,1) and N(0,1)
    noise from a seeded torch generator, X = max(0, X_c + noise * ||X_c|| /
    ||E|| * E). Returns the flat FP32 tensor, mode 1 fastest. Its values differ
    from ``planted`` for the same seed (different random streams)."""
    import torch
    dims = _as_dims(dims)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    fs = [torch.rand((d, R), generator=g, device=device, dtype=torch.float32) for d in dims]
    # P[q, r] over modes 1..N-1 with mode 1 fastest, then X[q + Q*iN] = sum_r P[q, r] H_N[iN, r]
    P = fs[0]
    for f in fs[1:-1]:
        P = (f[:, None, :] * P[None, :, :]).reshape(-1, R)
    X = (fs[-1] @ P.T).reshape(-1)
    del P
    if noise:
        E = torch.randn(X.numel(), generator=g, device=device, dtype=torch.float32)
        scale = noise * torch.linalg.vector_norm(X.double()) / torch.linalg.vector_norm(E.double())
        X.add_(E, alpha=float(scale))
        del E
        X.clamp_(min=0.0)
    return X


def planted_device_slabs(dims: Sequence[int], R: int, noise: float, seed: int, dtype: str = "bf16",
                         device="cuda", slab_bytes: int = 1 << 30):
    """The ``planted`` recipe for tensors too large to hold twice in FP32 (the
    30012 x 1200 x 500 fMRI-shaped tensor is 72 GB in FP32): drawn slab by slab
    along the last mode, straight into the storage type ("f32", "bf16", "f16").
    Factors U[0,1) and N(0,1) noise from seeded torch generators; ||X_c||^2 is
    the closed form sum_{r,s} prod_n (F_n^T F_n)[r, s] in FP64, ||E||^2 is
    summed over the slabs in a first pass, and each slab's noise is drawn again
    from its own seed in the second; X = max(0, X_c + noise ||X_c|| / ||E|| E)
    is then rounded to the storage type. Returns the flat tensor, mode 1
    fastest. Its values differ from ``planted`` and ``planted_device``."""
    import torch
    dims = _as_dims(dims)
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    fs = [torch.rand((d, R), generator=g, device=device, dtype=torch.float32) for d in dims]
    gh = torch.ones((R, R), dtype=torch.float64, device=device)
    for f in fs:
        fd = f.double()
        gh *= fd.T @ fd
    xc_norm = math.sqrt(max(0.0, float(gh.sum())))
    P = fs[0]
    for f in fs[1:-1]:
        P = (f[:, None, :] * P[None, :, :]).reshape(-1, R)
    Q, K = P.shape[0], dims[-1]
    per = max(1, int(slab_bytes // (Q * 4)))

    def slab_noise(k0, k1):
        gk = torch.Generator(device=device)
        gk.manual_seed(int(seed) * 1000003 + 7919 * k0 + 1)
        return torch.randn(Q * (k1 - k0), generator=gk, device=device, dtype=torch.float32)

    scale = 0.0
    if noise:
        e2 = 0.0
        for k0 in range(0, K, per):
            E = slab_noise(k0, min(K, k0 + per))
            e2 += float(torch.linalg.vector_norm(E, dtype=torch.float64) ** 2)
            del E
        scale = noise * xc_norm / math.sqrt(e2) if e2 > 0 else 0.0
    out = torch.empty(Q * K, dtype=tdt, device=device)
    for k0 in range(0, K, per):
        k1 = min(K, k0 + per)
        Xs = (fs[-1][k0:k1] @ P.T).reshape(-1)  # (k, q) with q (modes 1..N-1, mode 1 fastest) fastest
        if noise:
            Xs.add_(slab_noise(k0, k1), alpha=scale)
            Xs.clamp_(min=0.0)
        out[k0 * Q:k1 * Q] = Xs.to(tdt)
        del Xs
    return out
