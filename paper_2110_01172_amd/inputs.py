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


def sparse_cosines(n1: int, n2: int, seed: int, groups=((8, 1.0, 2.0), (8, 4.0, 5.0)), noise: float = 1e-3):
    """A synthetic image with a few strong separable cosine components and weak
    noise: sum over components of a * u_p(i) u_q(j) + noise * N(0, 1), where
    u_p(i) = s_p cos(pi p (2 i + 1) / (2 n)), s_0 = sqrt(1/n), s_p = sqrt(2/n)
    (unit-norm cosines), a random sign times U[lo, hi] for each (count, lo, hi)
    group, and distinct random frequencies (p, q).  FP32."""
    g = rng(seed)
    total = sum(c for c, _, _ in groups)
    flat = g.choice(n1 * n2, size=total, replace=False)
    i = np.arange(n1)[:, None]
    j = np.arange(n2)[None, :]
    x = noise * g.standard_normal((n1, n2))
    at = 0
    for count, lo, hi in groups:
        for f in flat[at:at + count]:
            p, q = divmod(int(f), n2)
            a = (1.0 if g.random() < 0.5 else -1.0) * g.uniform(lo, hi)
            sp = np.sqrt((1.0 if p == 0 else 2.0) / n1)
            sq = np.sqrt((1.0 if q == 0 else 2.0) / n2)
            x = x + a * (sp * np.cos(np.pi * p * (2 * i + 1) / (2 * n1))) * (sq * np.cos(np.pi * q * (2 * j + 1) / (2 * n2)))
        at += count
    return x.astype(np.float32)
