"""The paper's stages and the GPU decomposition, modelled in FP64, against the
oracle (CPU only).  These lock the readings of the garbled passages before any
kernel is trusted, and tie the post-processing to the paper's printed counts."""
import os

import numpy as np
import pytest

import stage_model as sm

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SHAPES = [(2, 2), (4, 4), (6, 8), (8, 6), (5, 8), (7, 6), (10, 10), (12, 20), (16, 12), (3, 4)]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _tol(ref):
    return 1e-12 * max(1.0, float(np.abs(ref).max()))


@pytest.mark.parametrize("n", [1, 2, 5, 6, 7, 8, 16])
def test_dct1d_npoint_algorithm(orc, n):
    """Alg. 1d-dct-via-fft (N-point): 2 * raw DCT-II, any n."""
    x = _rng(n).standard_normal(n)
    np.testing.assert_allclose(sm.dct1d_npoint(x), 2 * orc.dctn(x), rtol=0, atol=_tol(x) * n)


@pytest.mark.parametrize("shape", SHAPES)
def test_dct2d_naive_post_modular_reading(orc, shape):
    """Eq. (2d_dct_post) with X(N1, n2) read as X(0, n2) gives 4 * raw."""
    x = _rng(1).standard_normal(shape)
    ref = 4 * orc.dctn(x)
    np.testing.assert_allclose(sm.dct2d_paper_naive(x), ref, rtol=0, atol=_tol(ref))


def test_dct2d_printed_zero_convention_is_wrong(orc):
    """The printed convention X(N1, n2) = 0 halves row k1 = 0 (reading A1)."""
    x = _rng(2).standard_normal((6, 8))
    ref = 4 * orc.dctn(x)
    y = sm.dct2d_paper_naive(x, modular=False)
    np.testing.assert_allclose(y[0], ref[0] / 2, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(y[1:], ref[1:], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape", SHAPES)
def test_four_element_post_writes_each_output_once(orc, shape):
    """Eqs. (four-elements)/(s-t) with the corner mapping: exact, write-once."""
    x = _rng(3).standard_normal(shape)
    y, writes, _ = sm.dct2d_paper_fourelem(x)
    ref = 4 * orc.dctn(x)
    np.testing.assert_allclose(y, ref, rtol=0, atol=_tol(ref))
    assert (writes == 1).all()


@pytest.mark.parametrize("shape", SHAPES)
def test_idct2d_plus_sign_reading(orc, shape):
    """Eq. (2d_idct_pre) with +j exponent + unnormalised C2R + Eq. (2d_idct_post)
    is 4 * raw DCT-III composed over both axes (reading A2)."""
    y = _rng(4).standard_normal(shape)
    raw3 = orc.dct_axis(orc.dct_axis(y, 0, 3), 1, 3)
    out, _ = sm.idct2d_paper(y, +1)
    np.testing.assert_allclose(out, 4 * raw3, rtol=0, atol=_tol(raw3) * 4)


def test_idct2d_printed_minus_sign_is_not_hermitian(orc):
    """The printed -j exponent gives a pre-processed array that is not the half of
    a Hermitian spectrum and a wrong result."""
    n1, n2 = 6, 8
    y = _rng(5).standard_normal((n1, n2))
    _, Xp_plus = sm.idct2d_paper(y, +1)
    _, Xp_minus = sm.idct2d_paper(y, -1)
    # column 0 of a Hermitian half spectrum satisfies X(k1, 0) = conj X(-k1, 0)
    col_p, col_m = Xp_plus[:, 0], Xp_minus[:, 0]
    rev = (-np.arange(n1)) % n1
    np.testing.assert_allclose(col_p, np.conj(col_p[rev]), atol=1e-12)
    assert np.abs(col_m - np.conj(col_m[rev])).max() > 1e-3
    out_m, _ = sm.idct2d_paper(y, -1)
    raw3 = orc.dct_axis(orc.dct_axis(y, 0, 3), 1, 3)
    assert np.abs(out_m - 4 * raw3).max() > 1e-3


@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 6, 8), (6, 4, 10), (3, 4, 4)])
def test_dct3d_four_read_eight_write_post(orc, shape):
    x = _rng(6).standard_normal(shape)
    y, writes = sm.dct3d_paper(x)
    ref = 8 * orc.dctn(x)
    np.testing.assert_allclose(y, ref, rtol=0, atol=_tol(ref))
    assert (writes == 1).all()


@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 6, 8), (6, 4, 10), (3, 4, 4)])
def test_idct3d_eight_read_pre(orc, shape):
    """The separable 3-D extension of Eq. (2d_idct_pre) gives 8 * raw DCT-III."""
    y = _rng(16).standard_normal(shape)
    raw3 = y
    for a in range(3):
        raw3 = orc.dct_axis(raw3, a, 3)
    np.testing.assert_allclose(sm.idct3d_paper(y), 8 * raw3, rtol=0, atol=_tol(raw3) * 8)


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", [(2, 2), (4, 4), (6, 8), (8, 6), (5, 8), (7, 6), (10, 10), (16, 12), (3, 4)])
def test_gpu_decomposition_dct(orc, norm, shape):
    x = _rng(7).standard_normal(shape)
    ref = orc.dctn(x, norm)
    np.testing.assert_allclose(sm.gpu_model_dct2d(x, norm), ref, rtol=0, atol=_tol(ref))


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", [(2, 2), (4, 4), (6, 8), (8, 6), (5, 8), (7, 6), (10, 10), (16, 12), (3, 4)])
def test_gpu_decomposition_idct(orc, norm, shape):
    y = _rng(8).standard_normal(shape)
    ref = orc.idctn(y, norm)
    np.testing.assert_allclose(sm.gpu_model_idct2d(y, norm), ref, rtol=0, atol=_tol(ref))


# ------------------------------------------------------------- golden fixtures
def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line)
    return rows


def test_golden_hermitian_pairs():
    """The paper's N=5 and N=6 conjugate-pair examples hold for the real FFT, and
    match the stored-half reading (columns 0..floor(N/2), the rest conjugated)."""
    for row in _read_golden("hermitian_pairs.txt"):
        n_str, pairs = row.split(":")
        n = int(n_str)
        x = _rng(n).standard_normal(n)
        X = np.fft.fft(x)
        listed = set()
        for pr in pairs.split():
            a, b = (int(v) for v in pr.split("-"))
            np.testing.assert_allclose(X[a], np.conj(X[b]), atol=1e-12)
            listed.add((min(a, b), max(a, b)))
        assert listed == {(m, n - m) for m in range(1, n // 2 + 1)}
        Xh = np.fft.rfft(x)
        for k in range(n):
            v = Xh[k] if k <= n // 2 else np.conj(Xh[n - k])
            np.testing.assert_allclose(v, X[k], atol=1e-12)


class _Count:
    """Complex number that counts real multiplications and additions."""
    mul = 0
    add = 0

    def __init__(self, re, im=0.0):
        self.re, self.im = re, im

    def __mul__(self, o):
        _Count.mul += 4
        _Count.add += 2
        return _Count(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def __add__(self, o):
        _Count.add += 2
        return _Count(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        _Count.add += 2
        return _Count(self.re - o.re, self.im - o.im)

    def conj(self):
        return _Count(self.re, -self.im)

    def mul_real_part(self, o):
        """Re(self * o): 2 multiplications and 1 addition."""
        _Count.mul += 2
        _Count.add += 1
        return self.re * o.re - self.im * o.im


def test_golden_post_operation_counts():
    """Table efficient-processing: per-thread real multiplications / additions of
    the naive post (one output) and of the four-element post (s and t)."""
    rows = {r.split()[0]: [float(v) for v in r.split()[1:]] for r in _read_golden("efficient_post_counts.txt")}
    rng = _rng(9)
    A, B, a, b = (_Count(*rng.standard_normal(2)) for _ in range(4))
    # naive: y = 2 Re(b (a A + conj(a) B)), real part only of the last product
    _Count.mul = _Count.add = 0
    b.mul_real_part(a * A + a.conj() * B)
    assert (_Count.mul, _Count.add) == (rows["naive"][2], rows["naive"][3])
    # four-element: s = b (a A + conj(a) B), t = b (a A - conj(a) B)
    _Count.mul = _Count.add = 0
    aA, aB = a * A, a.conj() * B
    _ = b * (aA + aB), b * (aA - aB)
    assert (_Count.mul, _Count.add) == (rows["ours"][2], rows["ours"][3])
    # thread and read totals for even sizes: (N1/2+1)(N2/2+1) threads ~ N1 N2 / 4,
    # each reading 2 of the N1 (N2/2+1) stored values exactly once
    for (n1, n2) in [(64, 64), (128, 256)]:
        x = rng.standard_normal((n1, n2))
        _, writes, threads = sm.dct2d_paper_fourelem(x)
        assert (writes == 1).all()
        assert abs(threads / (n1 * n2) - rows["ours"][0]) < 4.0 / min(n1, n2)
        reads = 2 * threads - (2 * (n2 // 2 + 1))         # self-paired rows read once
        assert reads == n1 * (n2 // 2 + 1)
        assert abs(reads / (n1 * n2) - rows["ours"][4]) <= 1.0 / n2 + 1e-12   # Nyquist column


def test_golden_memory_stages():
    rows = {r.split()[0]: int(r.split()[1]) for r in _read_golden("memory_stages.txt")}
    per_1d_dct = 3            # pre, RFFT, post (Alg. 1d-dct-via-fft, N-point)
    assert rows["row_column"] == 2 * per_1d_dct + 2
    assert rows["three_stage"] == 3
    assert abs(1 - rows["three_stage"] / rows["row_column"] - 0.625) < 1e-12


@pytest.mark.parametrize("n1", [8, 16, 64, 256])
def test_split_column_order_is_the_column_dft(n1):
    """The split-column order of the tall-array kernels (radix-8 step with the
    W_n1^(qq kp) twiddle, then q-point DFTs; its mirror image for the inverse)
    is the plain length-n1 DFT, forward and unnormalised inverse."""
    g = _rng(31)
    Z = g.standard_normal((n1, 5)) + 1j * g.standard_normal((n1, 5))
    np.testing.assert_allclose(sm.split_column_fft(Z), np.fft.fft(Z, axis=0), rtol=0, atol=1e-12 * n1)
    np.testing.assert_allclose(sm.split_column_fft(Z, inverse=True), np.fft.ifft(Z, axis=0) * n1, rtol=0,
                               atol=1e-12 * n1)
