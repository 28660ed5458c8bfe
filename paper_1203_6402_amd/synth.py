"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws data. It holds none of the clustering arithmetic, so both
the FP64 oracle (``oracle/``) and the HIP path can be fed the same bytes from it.

Recipes (all with ``numpy.random.Generator(PCG64(seed))`` on the host, or a seeded
``torch.Generator`` on the device for the multi-GB workloads):

* ``gauss_mixture`` -- the GaussMixture data set of Section 4.1: ``k_true`` centers
  drawn from a spherical Gaussian with per-coordinate variance ``R`` around the
  origin, points drawn from unit-variance Gaussians around uniformly chosen
  centers (equal mixture weights).
* ``heavy_tailed`` -- a synthetic stand-in with the shape of KDDCup1999
  (Section 4.1: 4.8M points in 42 dimensions); the real data set is not used.
  Rows come from ``comps`` mixture components with weights proportional to
  ``1/j**2``; entry (i, c) is ``s[comp(i), c] * exp(sigma * z)`` with
  ``s ~ logU[1, 1e6]`` per (component, column), ``z ~ N(0, 1)``, and each entry
  is zeroed with probability ``zero_frac``.
* ``gauss_mixture_sigma`` -- Gaussian mixture with centers ``N(0, var_c I)`` and a
  per-component isotropic sigma drawn log-uniform in ``[sig_lo, sig_hi]``; its FP8
  variant stores each row as e4m3 codes with the row scale ``max|x| / 448``.
* ``batch_instances`` -- shapes of many independent small instances.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gauss_mixture(n: int, d: int, k_true: int, R: float, seed: int,
                  dtype=np.float32) -> np.ndarray:
    """GaussMixture (Section 4.1): n points, k_true equal-weight unit-variance
    spherical Gaussians whose centers are N(0, R*I)."""
    rng = _rng(seed)
    centers = rng.normal(0.0, math.sqrt(R), size=(k_true, d))
    labels = rng.integers(0, k_true, size=n)
    X = centers[labels] + rng.standard_normal(size=(n, d))
    return np.ascontiguousarray(X.astype(dtype))


def heavy_tailed(n: int, d: int = 42, comps: int = 20, seed: int = 0,
                 sigma: float = 2.0, zero_frac: float = 0.3,
                 chunk: int = 1 << 19, dtype=np.float32) -> np.ndarray:
    """Nonnegative heavy-tailed rows from a skewed mixture (weights 1/j^2)."""
    rng = _rng(seed)
    w = 1.0 / np.arange(1, comps + 1, dtype=np.float64) ** 2
    w /= w.sum()
    scales = np.exp(rng.uniform(0.0, math.log(1e6), size=(comps, d)))
    X = np.empty((n, d), dtype=dtype)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        lab = rng.choice(comps, size=c, p=w)
        z = rng.standard_normal(size=(c, d))
        x = scales[lab] * np.exp(sigma * z)
        x[rng.random(size=(c, d)) < zero_frac] = 0.0
        X[s:s + c] = x.astype(dtype)
    return X


def gauss_mixture_sigma(n: int, d: int, comps: int, seed: int,
                        var_c: float = 25.0, sig_lo: float = 0.5,
                        sig_hi: float = 4.0, chunk: int = 1 << 18,
                        dtype=np.float32) -> np.ndarray:
    """Host variant of the precision workloads at small n (tests)."""
    rng = _rng(seed)
    centers = rng.normal(0.0, math.sqrt(var_c), size=(comps, d))
    sig = np.exp(rng.uniform(math.log(sig_lo), math.log(sig_hi), size=comps))
    X = np.empty((n, d), dtype=dtype)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        lab = rng.integers(0, comps, size=c)
        X[s:s + c] = (centers[lab] + sig[lab, None]
                      * rng.standard_normal(size=(c, d))).astype(dtype)
    return X


def gauss_mixture_sigma_torch(n: int, d: int, comps: int, seed: int,
                              device="cuda", var_c: float = 25.0,
                              sig_lo: float = 0.5, sig_hi: float = 4.0,
                              chunk: int = 1 << 22, out_dtype=None):
    """Device variant of ``gauss_mixture_sigma`` for the multi-GB workloads.

    Returns a float32 tensor unless ``out_dtype`` is given, in which case each
    chunk is rounded (round-to-nearest-even) to that dtype as it is produced."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    centers = torch.randn(comps, d, generator=g, device=device) * math.sqrt(var_c)
    lo, hi = math.log(sig_lo), math.log(sig_hi)
    sig = torch.exp(lo + (hi - lo) * torch.rand(comps, generator=g, device=device))
    X = torch.empty(n, d, device=device, dtype=out_dtype or torch.float32)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        lab = torch.randint(0, comps, (c,), generator=g, device=device)
        x = centers[lab] + sig[lab, None] * torch.randn(c, d, generator=g, device=device)
        X[s:s + c] = x.to(X.dtype)
    return X


def gauss_mixture_sigma_fp8_torch(n: int, d: int, comps: int, seed: int,
                                  device="cuda", var_c: float = 25.0,
                                  sig_lo: float = 0.5, sig_hi: float = 4.0,
                                  chunk: int = 1 << 21):
    """``gauss_mixture_sigma`` stored as OCP e4m3 codes with one FP32 scale
    per row, max|x| / 448 (448 is the largest e4m3 value), each row divided by
    its scale and rounded to nearest even; made chunk by chunk on the device
    so that the FP32 rows never exist all at once.  Returns (codes as an
    n x d uint8 tensor, scales as an n float32 tensor)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    centers = torch.randn(comps, d, generator=g, device=device) * math.sqrt(var_c)
    lo, hi = math.log(sig_lo), math.log(sig_hi)
    sig = torch.exp(lo + (hi - lo) * torch.rand(comps, generator=g, device=device))
    Q = torch.empty(n, d, device=device, dtype=torch.uint8)
    S = torch.empty(n, device=device, dtype=torch.float32)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        lab = torch.randint(0, comps, (c,), generator=g, device=device)
        x = centers[lab] + sig[lab, None] * torch.randn(c, d, generator=g, device=device)
        scale = x.abs().amax(dim=1).clamp_min(1e-30) / 448.0
        Q[s:s + c] = (x / scale[:, None]).to(torch.float8_e4m3fn).view(torch.uint8)
        S[s:s + c] = scale
    return Q, S


def batch_instances(count: int, seed: int, n_lo: int = 2000, n_hi: int = 200000,
                    dims=(32, 64, 128)):
    """Sizes of independent instances: n log-uniform in [n_lo, n_hi], d uniform
    over ``dims``, k = ceil(sqrt(n)/2)."""
    rng = _rng(seed)
    n = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(np.int64)
    d = rng.choice(np.asarray(dims), size=count)
    k = np.ceil(np.sqrt(n) / 2.0).astype(np.int64)
    return n, d, k


def batch_gauss_mixture(ns, ds, ks, seed: int, R: float = 10.0, dtype=np.float32):
    """One GaussMixture instance per (n, d, k): k true centers N(0, R I), n
    unit-variance points (host, for small batches)."""
    return [gauss_mixture(int(n), int(d), int(k), R, seed=seed * 1_000_003 + i, dtype=dtype)
            for i, (n, d, k) in enumerate(zip(ns, ds, ks))]


def batch_gauss_mixture_torch(ns, ds, ks, seed: int, device="cuda", R: float = 10.0,
                              out_dtype=None):
    """Device variant of ``batch_gauss_mixture`` for thousands of instances."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = []
    for n, d, k in zip(ns, ds, ks):
        n, d, k = int(n), int(d), int(k)
        centers = torch.randn(k, d, generator=g, device=device) * math.sqrt(R)
        lab = torch.randint(0, k, (n,), generator=g, device=device)
        x = centers[lab] + torch.randn(n, d, generator=g, device=device)
        out.append(x.to(out_dtype) if out_dtype is not None else x)
    return out
