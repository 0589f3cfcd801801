"""Seeded synthetic inputs (numpy PCG64, generated in FP64, rounded to FP32).

Shared by the tests, the smoke check and the benchmark; holds none of the
transforms' arithmetic.  Seeds follow ``seed = 1000 * workload + case``.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """i.i.d. uniform[lo, hi], FP32."""
    return rng(seed).uniform(lo, hi, size=shape).astype(np.float32)


def normal(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1), FP32."""
    return rng(seed).standard_normal(size=shape).astype(np.float32)


def log_uniform_signed(shape, seed: int, lo: float = 1e-3, hi: float = 1e3) -> np.ndarray:
    """s * 10^u with u ~ U[log10 lo, log10 hi] and random sign s, FP32."""
    g = rng(seed)
    u = g.uniform(np.log10(lo), np.log10(hi), size=shape)
    s = np.where(g.random(size=shape) < 0.5, -1.0, 1.0)
    return (s * np.power(10.0, u)).astype(np.float32)


def five_smooth_even(lo: int = 64, hi: int = 1024) -> list:
    """Even n = 2^a 3^b 5^c in [lo, hi] (50 values for [64, 1024])."""
    out = []
    for n in range(lo, hi + 1):
        if n % 2:
            continue
        m = n
        for f in (2, 3, 5):
            while m % f == 0:
                m //= f
        if m == 1:
            out.append(n)
    return out


def uneven_batch_shapes(count: int, seed: int, lo: int = 64, hi: int = 1024) -> list:
    """(n1, n2) pairs with each side drawn uniformly from five_smooth_even(lo, hi)."""
    sizes = np.asarray(five_smooth_even(lo, hi))
    g = rng(seed)
    return [(int(a), int(b)) for a, b in zip(g.choice(sizes, count), g.choice(sizes, count))]


def gaussian_bumps(n1: int, n2: int, seed: int, count: int = 32) -> np.ndarray:
    """Smooth right-hand side: sum of `count` Gaussians on cell centres of the
    unit square, centres U[0,1]^2, widths U[0.02, 0.1], amplitudes N(0,1)."""
    g = rng(seed)
    yy = (np.arange(n1) + 0.5) / n1
    xx = (np.arange(n2) + 0.5) / n2
    f = np.zeros((n1, n2))
    for _ in range(count):
        cy, cx = g.uniform(0, 1, 2)
        sig = g.uniform(0.02, 0.1)
        amp = g.standard_normal()
        f += amp * np.exp(-(yy[:, None] - cy) ** 2 / (2 * sig * sig)) * \
            np.exp(-(xx[None, :] - cx) ** 2 / (2 * sig * sig))
    return f.astype(np.float32)
