"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Every check here is independent of the oracle's own code path: closed forms
derived by hand, orthogonality of the cosine basis, brute-force non-separable
sums written with ``math.cos`` (no argument reduction, no shared table), the
round-trip and Parseval identities implied by Eq. (1d-definition), the
transposition equivalence used by the axis-swap dispatch (Section
"Results on 2D DCTs"), and the discrete Laplacian residual of the Poisson solve.
"""
import math
import itertools

import numpy as np
import pytest

SHAPES_2D = [(1, 1), (2, 3), (4, 4), (5, 7), (6, 8), (8, 6), (3, 10)]
SHAPES_3D = [(2, 2, 2), (4, 6, 8), (3, 5, 4), (6, 4, 10)]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("shape", [(7,), (6, 8), (5, 7), (4, 6, 8)])
def test_constant_maps_to_dc(orc, shape):
    """x = c everywhere: raw DCT-II has c * prod(N) at k = 0 and zero elsewhere."""
    c = 1.75
    y = orc.dctn(np.full(shape, c))
    expect = np.zeros(shape)
    expect[(0,) * len(shape)] = c * np.prod(shape)
    np.testing.assert_allclose(y, expect, rtol=0, atol=1e-11 * np.prod(shape))


@pytest.mark.parametrize("shape", [(9,), (6, 8), (5, 7), (8, 5), (4, 6, 8), (3, 5, 4)])
def test_basis_maps_to_delta(orc, shape):
    """x = prod_d cos(pi (2 n_d + 1) p_d / (2 N_d)) gives a delta at k = p with
    value prod_d (N_d if p_d = 0 else N_d / 2)  (orthogonality of the DCT-II
    basis).  Distinct p_d on non-square shapes catch a transposed operand."""
    rng = _rng(11)
    for trial in range(4):
        p = tuple(int(rng.integers(0, n)) for n in shape)
        if trial == 0:
            p = tuple(0 for _ in shape)
        if trial == 1:
            p = tuple(n - 1 for n in shape)
        x = np.ones(shape)
        for d, (n, pd) in enumerate(zip(shape, p)):
            v = np.cos(np.pi * (2 * np.arange(n) + 1) * pd / (2 * n))
            bshape = [1] * len(shape)
            bshape[d] = n
            x = x * v.reshape(bshape)
        y = orc.dctn(x)
        expect = np.zeros(shape)
        expect[p] = np.prod([n if pd == 0 else n / 2 for n, pd in zip(shape, p)])
        np.testing.assert_allclose(y, expect, rtol=0, atol=1e-11 * np.prod(shape))


def _ramp_closed_form(n):
    """sum_m m cos(pi k (2m+1)/(2n)):  n(n-1)/2 at k=0, 0 for even k>0 and
    -cos(a)/(2 sin(a)^2), a = pi k/(2n), for odd k  (derived by differentiating
    sum_m sin((2m+1)a) = sin(n a)^2 / sin(a))."""
    out = np.zeros(n)
    out[0] = n * (n - 1) / 2
    for k in range(1, n):
        if k % 2:
            a = math.pi * k / (2 * n)
            out[k] = -math.cos(a) / (2 * math.sin(a) ** 2)
    return out


@pytest.mark.parametrize("shape", [(12,), (7,), (6, 9), (10, 4)])
def test_ramp_closed_form(orc, shape):
    """x(n1, n2) = n1 * n2 (a separable ramp) against the hand-derived closed form."""
    x = np.ones(shape)
    expect = np.ones(shape)
    for d, n in enumerate(shape):
        bshape = [1] * len(shape)
        bshape[d] = n
        x = x * np.arange(n, dtype=np.float64).reshape(bshape)
        expect = expect * _ramp_closed_form(n).reshape(bshape)
    y = orc.dctn(x)
    np.testing.assert_allclose(y, expect, rtol=1e-12, atol=1e-10)


# ----------------------------------------------------------- brute force sums
def _brute_dct2_nd(x):
    """Non-separable direct sum over all input indices, math.cos, no reduction."""
    shape = x.shape
    out = np.zeros(shape)
    for k in itertools.product(*[range(n) for n in shape]):
        s = 0.0
        for m in itertools.product(*[range(n) for n in shape]):
            w = 1.0
            for kd, md, nd in zip(k, m, shape):
                w *= math.cos(math.pi / nd * (md + 0.5) * kd)
            s += x[m] * w
        out[k] = s
    return out


def _brute_dct3_nd(x):
    """Direct sum of Eq. (1d-definition b) composed over all axes (non-separable loop)."""
    shape = x.shape
    out = np.zeros(shape)
    for k in itertools.product(*[range(n) for n in shape]):
        s = 0.0
        for m in itertools.product(*[range(n) for n in shape]):
            w = 1.0
            for kd, md, nd in zip(k, m, shape):
                w *= 0.5 if md == 0 else math.cos(math.pi / nd * md * (kd + 0.5))
            s += x[m] * w
        out[k] = s
    return out


@pytest.mark.parametrize("shape", SHAPES_2D + SHAPES_3D)
def test_brute_force_nonseparable(orc, shape):
    x = _rng(hash(shape) % 1000).uniform(-1, 1, shape)
    np.testing.assert_allclose(orc.dctn(x), _brute_dct2_nd(x), rtol=0, atol=1e-12 * x.size)
    raw3 = x
    for a in range(x.ndim):
        raw3 = orc.dct_axis(raw3, a, 3)
    np.testing.assert_allclose(raw3, _brute_dct3_nd(x), rtol=0, atol=1e-12 * x.size)


@pytest.mark.parametrize("shape", [(4, 4), (5, 7), (8, 6), (16, 3)])
def test_matrix_product(orc, shape):
    """2-D DCT-II equals C1 X C2^T with C_N[k, n] = cos(pi (2n+1) k / (2N))."""
    n1, n2 = shape
    C1 = np.cos(np.pi * np.outer(np.arange(n1), 2 * np.arange(n1) + 1) / (2 * n1))
    C2 = np.cos(np.pi * np.outer(np.arange(n2), 2 * np.arange(n2) + 1) / (2 * n2))
    x = _rng(5).standard_normal(shape)
    np.testing.assert_allclose(orc.dctn(x), C1 @ x @ C2.T, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------- identities and norms
@pytest.mark.parametrize("shape", [(16,), (6, 8), (5, 7), (4, 6, 8), (3, 5, 4)])
def test_dct3_after_dct2_is_scaled_identity(orc, shape):
    """Raw DCT-III after raw DCT-II along one axis is (N/2) * identity."""
    x = _rng(3).standard_normal(shape)
    for a in range(len(shape)):
        y = orc.dct_axis(orc.dct_axis(x, a, 2), a, 3)
        np.testing.assert_allclose(y, x * shape[a] / 2, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", [(17,), (6, 8), (5, 7), (8, 1), (4, 6, 8), (3, 5, 2)])
def test_roundtrip(orc, norm, shape):
    x = _rng(4).uniform(-1, 1, shape)
    np.testing.assert_allclose(orc.idctn(orc.dctn(x, norm), norm), x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(orc.dctn(orc.idctn(x, norm), norm), x, rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [(6, 8), (5, 7), (4, 6, 8)])
def test_parseval_ortho(orc, shape):
    x = _rng(6).standard_normal(shape)
    y = orc.dctn(x, "ortho")
    assert abs(np.sum(y * y) - np.sum(x * x)) <= 1e-12 * np.sum(x * x)
    z = orc.idctn(x, "ortho")
    assert abs(np.sum(z * z) - np.sum(x * x)) <= 1e-12 * np.sum(x * x)


def test_transposition_equivalence(orc):
    """DCT of the transposed input is the transposed DCT (axis-swap dispatch)."""
    x = _rng(7).standard_normal((6, 10))
    np.testing.assert_allclose(orc.dctn(x.T), orc.dctn(x).T, rtol=1e-13, atol=1e-12)
    x3 = _rng(8).standard_normal((3, 4, 5))
    np.testing.assert_allclose(orc.dctn(x3.transpose(2, 0, 1)),
                               orc.dctn(x3).transpose(2, 0, 1), rtol=1e-13, atol=1e-12)


def test_selected_outputs_match_full(orc):
    x = _rng(9).standard_normal((12, 20))
    full = orc.dctn(x, "ortho")
    part = orc.dctn(x, "ortho", sel={1: [0, 3, 19]})
    np.testing.assert_allclose(part, full[:, [0, 3, 19]], rtol=1e-13, atol=1e-13)
    full3 = orc.idctn(x, "backward")
    part3 = orc.idctn(x, "backward", sel={0: [11, 2], 1: [5]})
    np.testing.assert_allclose(part3, full3[np.ix_([11, 2], [5])], rtol=1e-13, atol=1e-13)


def test_scipy_cross_check(orc):
    """Third-party cross-check only: scipy's type-2 DCT is 2^D times the raw sum."""
    sfft = pytest.importorskip("scipy.fft")
    x = _rng(10).standard_normal((6, 10))
    np.testing.assert_allclose(sfft.dctn(x, type=2), 4 * orc.dctn(x), rtol=1e-12, atol=1e-11)
    np.testing.assert_allclose(sfft.dctn(x, type=2, norm="ortho"), orc.dctn(x, "ortho"),
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sfft.idctn(x, type=2, norm="ortho"), orc.idctn(x, "ortho"),
                               rtol=1e-12, atol=1e-12)
    # scipy's backward idctn inverts its own 2^D-scaled forward transform
    np.testing.assert_allclose(4 * sfft.idctn(x, type=2), orc.idctn(x), rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------- Poisson
def _neumann_laplacian(u, h1, h2):
    """Cell-centred 5-point Laplacian with mirror ghost cells (zero normal flux)."""
    up = np.pad(u, 1, mode="edge")
    return ((up[2:, 1:-1] - 2 * u + up[:-2, 1:-1]) / h1 ** 2
            + (up[1:-1, 2:] - 2 * u + up[1:-1, :-2]) / h2 ** 2)


@pytest.mark.parametrize("shape", [(16, 16), (12, 20), (9, 7)])
def test_poisson_residual(orc, shape):
    n1, n2 = shape
    rng = _rng(12)
    yy, xx = np.meshgrid((np.arange(n1) + 0.5) / n1, (np.arange(n2) + 0.5) / n2, indexing="ij")
    f = np.zeros(shape)
    for _ in range(8):
        c = rng.uniform(0, 1, 2)
        s = rng.uniform(0.05, 0.2)
        f += rng.standard_normal() * np.exp(-((yy - c[0]) ** 2 + (xx - c[1]) ** 2) / (2 * s * s))
    u = orc.poisson2d_neumann(f)
    lap = _neumann_laplacian(u, 1.0 / n1, 1.0 / n2)
    np.testing.assert_allclose(lap, f - f.mean(), rtol=0, atol=1e-9 * np.abs(f).max())
    assert abs(u.mean()) < 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("shape,h1,h2", [((16, 12), 0.3, 0.07), ((9, 14), 2.5, 0.5), ((10, 10), 1e-2, 4e-2)])
def test_poisson_residual_explicit_spacings(orc, shape, h1, h2):
    """The explicit-spacing path of the solve (h1 != h2, neither 1/N): the
    Neumann Laplacian with those spacings, written out as a stencil, gives
    back f - mean(f), and mean(u) = 0.  Planted mistakes in the eigenvalue
    divide (spacings swapped, or squared spacings left out) fail it."""
    n1, n2 = shape
    rng = _rng(13)
    f = rng.standard_normal(shape)
    u = orc.poisson2d_neumann(f, h1, h2)
    lap = _neumann_laplacian(u, h1, h2)
    np.testing.assert_allclose(lap, f - f.mean(), rtol=0, atol=1e-9 * np.abs(f).max())
    assert abs(u.mean()) < 1e-12 * np.abs(u).max()
    # the swapped spacings solve a different equation (the pin can tell them apart)
    u_sw = orc.poisson2d_neumann(f, h2, h1)
    assert np.abs(_neumann_laplacian(u_sw, h1, h2) - (f - f.mean())).max() > 1e-3 * np.abs(f).max()


def test_rel_l2(orc):
    a = np.array([3.0, 4.0])
    assert orc.rel_l2(a, a) == 0.0
    assert abs(orc.rel_l2(a + np.array([0.3, 0.4]), a) - 0.1) < 1e-15
