"""Pins of the oracle's IDXST and mixed 2-D transforms (Eq. idxst) against
what the mathematics fixes (CPU only).

The oracle builds IDXST as the equation states it (reverse with a zero in
front, inverse DCT, sign).  The checks below do not: they use the sine sum
that the equation reduces to, cos(pi (N - n)(2k + 1) / 2N) =
(-1)^k sin(pi n (2k + 1) / 2N), written out with ``math.sin``; scipy's DST-III
of the shifted sequence; the fact that x(0) drops out; and brute-force 2-D
double sums that fix which axis each transform acts on (a 1-D transform of a
matrix acts on its columns, so IDCT_IDXST has the sine kernel on axis 0).
"""
import math

import numpy as np
import pytest

NORMS = ["backward", "ortho"]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _sine_weight(n_len, norm):
    # every term has IDCT frequency N - n >= 1: weight 2/N (backward) or sqrt(2/N) (ortho)
    return 2.0 / n_len if norm == "backward" else math.sqrt(2.0 / n_len)


def _cos_weight(m, n_len, norm):
    if norm == "backward":
        return 1.0 / n_len if m == 0 else 2.0 / n_len
    return math.sqrt(1.0 / n_len) if m == 0 else math.sqrt(2.0 / n_len)


def _idxst_sine_sum(x, norm):
    n_len = len(x)
    w = _sine_weight(n_len, norm)
    return np.array([w * sum(float(x[n]) * math.sin(math.pi * n * (2 * k + 1) / (2 * n_len))
                             for n in range(1, n_len)) for k in range(n_len)])


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 9, 15, 16])
def test_idxst_is_a_sine_sum(orc, norm, n):
    x = _rng(100 + n).standard_normal(n)
    np.testing.assert_allclose(orc.idxst_axis(x, 0, norm), _idxst_sine_sum(x, norm), rtol=0, atol=1e-13 * n)


@pytest.mark.parametrize("n", [2, 3, 8, 12])
def test_idxst_matches_scipy_dst3_of_shifted_sequence(orc, n):
    """scipy's unnormalised DST-III of (x1, ..., x_{N-1}, 0) is 2 sum_{n>=1}
    x_n sin(pi n (2k+1) / 2N): N times the backward IDXST."""
    fft = pytest.importorskip("scipy.fft")
    x = _rng(200 + n).standard_normal(n)
    shifted = np.concatenate([x[1:], [0.0]])
    np.testing.assert_allclose(orc.idxst_axis(x, 0), fft.dst(shifted, type=3) / n, rtol=0, atol=1e-12 * n)


def test_idxst_ignores_first_element(orc):
    x = _rng(7).standard_normal((5, 12))
    x2 = x.copy()
    x2[:, 0] = 1e3
    np.testing.assert_array_equal(orc.idxst_axis(x, 1), orc.idxst_axis(x2, 1))
    np.testing.assert_array_equal(orc.idxst_idct2(x), orc.idxst_idct2(x2))
    x3 = x.copy()
    x3[0, :] = -1e3
    np.testing.assert_array_equal(orc.idct_idxst2(x), orc.idct_idxst2(x3))


def _brute_2d(x, row_kernel, col_kernel):
    """y(k1, k2) = sum_{n1, n2} x(n1, n2) A(n1, k1) B(n2, k2) in pure Python."""
    n1, n2 = x.shape
    y = np.zeros((n1, n2))
    for k1 in range(n1):
        for k2 in range(n2):
            acc = 0.0
            for a in range(n1):
                ca = row_kernel(a, k1, n1)
                for b in range(n2):
                    acc += float(x[a, b]) * ca * col_kernel(b, k2, n2)
            y[k1, k2] = acc
    return y


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("shape", [(2, 4), (3, 4), (4, 6), (5, 2), (6, 10)])
def test_mixed_2d_brute_force(orc, norm, shape):
    """IDCT_IDXST: sine kernel on axis 0, cosine kernel on axis 1; IDXST_IDCT
    the other way round.  Non-square shapes catch a swapped axis."""
    x = _rng(300 + shape[0] * 16 + shape[1]).standard_normal(shape)

    def cosk(m, k, n):
        return _cos_weight(m, n, norm) * math.cos(math.pi * m * (2 * k + 1) / (2 * n))

    def sink(m, k, n):
        return 0.0 if m == 0 else _sine_weight(n, norm) * math.sin(math.pi * m * (2 * k + 1) / (2 * n))

    tol = 1e-12 * x.size
    np.testing.assert_allclose(orc.idct_idxst2(x, norm), _brute_2d(x, sink, cosk), rtol=0, atol=tol)
    np.testing.assert_allclose(orc.idxst_idct2(x, norm), _brute_2d(x, cosk, sink), rtol=0, atol=tol)


def test_mixed_2d_selection_matches_full(orc):
    x = _rng(9).standard_normal((12, 10))
    full = orc.idct_idxst2(x)
    np.testing.assert_allclose(orc.idct_idxst2(x, sel={1: [0, 3, 9]}), full[:, [0, 3, 9]], rtol=0, atol=1e-13)
    np.testing.assert_allclose(orc.idct_idxst2(x, sel={0: [1, 11]}), full[[1, 11], :], rtol=0, atol=1e-13)
    full2 = orc.idxst_idct2(x)
    np.testing.assert_allclose(orc.idxst_idct2(x, sel={1: [2, 5]}), full2[:, [2, 5]], rtol=0, atol=1e-13)
    np.testing.assert_allclose(orc.idxst_idct2(x, sel={0: [0, 7]}), full2[[0, 7], :], rtol=0, atol=1e-13)
