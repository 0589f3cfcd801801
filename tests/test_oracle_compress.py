"""Pins of the oracle's threshold compression (Alg. image-compression, Eq.
image-compression) against what the mathematics fixes (CPU only).

A sum of separable unit-norm cosines u_p(i) u_q(j), u_p(i) = s_p cos(pi p
(2i+1) / 2N), has the orthonormal 2-D DCT a at (p, q) and zero elsewhere, and
the raw (backward) DCT a * g_p * g_q with g_0 = sqrt(N), g_p = sqrt(N/2).  So
the compressed image is the sum of the components whose coefficient clears the
threshold, written out here with ``math.cos`` and no transform at all.
"""
import math

import numpy as np
import pytest


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _u(p, n):
    s = math.sqrt((1.0 if p == 0 else 2.0) / n)
    return np.array([s * math.cos(math.pi * p * (2 * i + 1) / (2 * n)) for i in range(n)])


def _g(p, n):
    return math.sqrt(n) if p == 0 else math.sqrt(n / 2.0)


def _components(shape, seed):
    n1, n2 = shape
    g = _rng(seed)
    freqs = [(0, 0), (1, 2), (n1 - 1, n2 - 1), (n1 // 2, 0), (2, n2 // 2), (n1 - 2, 1)]
    amps = [2.5, -0.75, 1.5, -3.0, 0.4, 1.1]
    comps = [(p, q, a * (1.0 + 0.01 * g.standard_normal())) for (p, q), a in zip(freqs, amps)]
    x = sum(a * np.outer(_u(p, n1), _u(q, n2)) for p, q, a in comps)
    return x, comps


@pytest.mark.parametrize("norm", ["ortho", "backward"])
@pytest.mark.parametrize("shape", [(6, 8), (9, 10), (16, 12)])
@pytest.mark.parametrize("cut", [0.0, 0.5, 1.3, 2.0, 2.8])
def test_compression_keeps_the_components_above_the_threshold(orc, norm, shape, cut):
    n1, n2 = shape
    x, comps = _components(shape, 500 + n1 * 10 + n2)
    eps = cut if norm == "ortho" else cut * math.sqrt(n1 * n2) / 2.0
    expect = np.zeros(shape)
    for p, q, a in comps:
        coef = a if norm == "ortho" else a * _g(p, n1) * _g(q, n2)
        if abs(coef) >= eps:
            expect += a * np.outer(_u(p, n1), _u(q, n2))
    np.testing.assert_allclose(orc.compress2d(x, eps, norm), expect, rtol=0, atol=1e-10)


@pytest.mark.parametrize("norm", ["ortho", "backward"])
def test_zero_threshold_is_identity_and_large_threshold_is_zero(orc, norm):
    x = _rng(3).standard_normal((10, 14))
    np.testing.assert_allclose(orc.compress2d(x, 0.0, norm), x, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(orc.compress2d(x, 1e9, norm), np.zeros_like(x))


def test_compression_is_idempotent_and_keeps_the_energy_it_keeps(orc):
    """Applying f_eps twice changes nothing (the kept coefficients are kept
    again, the rest stay zero), and under ortho the output energy equals the
    energy of the kept coefficients (Parseval)."""
    x, comps = _components((12, 10), 77)
    x = x + 1e-3 * _rng(78).standard_normal(x.shape)
    eps = 1.0
    once = orc.compress2d(x, eps)
    twice = orc.compress2d(once, eps)
    np.testing.assert_allclose(twice, once, rtol=0, atol=1e-12)
    kept = sum(a * a for _, _, a in comps if abs(a) >= eps)
    assert abs(float(np.sum(once * once)) - kept) <= 1e-2 * kept


MUTANTS = {
    "inverted_test": lambda orc, x, eps, norm="ortho", sel=None: orc.idctn(
        np.where(np.abs(orc.dctn(x, norm)) < eps, orc.dctn(x, norm), 0.0), norm, sel=sel),
    "signed_test": lambda orc, x, eps, norm="ortho", sel=None: orc.idctn(
        np.where(orc.dctn(x, norm) >= eps, orc.dctn(x, norm), 0.0), norm, sel=sel),
    "inverse_with_other_norm": lambda orc, x, eps, norm="ortho", sel=None: orc.idctn(
        np.where(np.abs(orc.dctn(x, norm)) >= eps, orc.dctn(x, norm), 0.0),
        "backward" if norm == "ortho" else "ortho", sel=sel),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(orc, monkeypatch, name):
    bad = MUTANTS[name]
    monkeypatch.setattr(orc, "compress2d", lambda x, eps, norm="ortho", sel=None: bad(orc, x, eps, norm, sel))
    failed = 0
    for cut in (0.5, 1.3):
        try:
            test_compression_keeps_the_components_above_the_threshold(orc, "ortho", (9, 10), cut)
        except AssertionError:
            failed += 1
    assert failed, f"no pin caught mutant {name}"
