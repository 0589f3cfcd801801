"""GPU parity of the fused threshold compression (Alg. image-compression,
Eq. image-compression) against the FP64 oracle, through the C ABI.

Inputs are synthetic images of a few strong unit-norm cosine components
(amplitudes in [1, 2] and [4, 5]) over weak noise (sigma 1e-3).  Under the
orthonormal norm their DCT coefficients are the amplitudes themselves, so the
thresholds 0.5 and 3.0 sit in wide gaps and the FP32 kernel and the FP64
oracle keep the same coefficients; under the backward norm the threshold is
placed in the widest gap of the oracle's coefficients.  Tolerance: relative L2
<= 1e-6.  Whole arrays up to 1024^2, whole columns at 2048 and 4096 rows."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_01172_amd as dx
    from paper_2110_01172_amd import inputs
    import oracle
    oracle.build(force=False)
    return torch, dx, inputs, oracle


def _run(env, x_np, eps, norm="ortho"):
    torch, dx, _, _ = env
    print(f"[gpu] compress2d shape={x_np.shape} eps={eps} norm={norm}", flush=True)
    y = dx.compress2d(torch.from_numpy(x_np).cuda(), eps, norm)
    torch.cuda.synchronize()
    return y.cpu().numpy()


FULL = [(48, 90), (250, 486), (81, 54), (6, 10), (256, 256), (512, 128), (1024, 1024)]


@pytest.mark.parametrize("eps", [0.5, 3.0])
@pytest.mark.parametrize("shape", FULL)
def test_compress_full(env, shape, eps):
    _, _, inputs, oracle = env
    x = inputs.sparse_cosines(shape[0], shape[1], 7000 + shape[0] + shape[1])
    y = _run(env, x, eps)
    err = oracle.rel_l2(y, oracle.compress2d(x, eps))
    assert err <= TOL, f"compress {shape} eps={eps}: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape", [(2048, 512), (4096, 1024), (4096, 4096)])
def test_compress_split_columns(env, shape):
    _, _, inputs, oracle = env
    n1, n2 = shape
    x = inputs.sparse_cosines(n1, n2, 7100 + n1 + n2)
    y = _run(env, x, 3.0)
    err = oracle.rel_l2(y, oracle.compress2d(x, 3.0))
    assert err <= TOL, f"compress {shape} whole array: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape", [(96, 160), (256, 512)])
def test_compress_backward_norm(env, shape):
    _, _, inputs, oracle = env
    x = inputs.sparse_cosines(shape[0], shape[1], 7200 + sum(shape))
    mags = np.sort(np.abs(oracle.dctn(x, "backward")).ravel())[::-1][:20]
    i = int(np.argmax(mags[1:17] / mags[2:18])) + 1
    assert mags[i] / mags[i + 1] > 1.2
    eps = float(np.sqrt(mags[i] * mags[i + 1]))
    y = _run(env, x, eps, "backward")
    err = oracle.rel_l2(y, oracle.compress2d(x, eps, "backward"))
    assert err <= TOL, f"compress backward {shape}: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape", [(48, 90), (256, 256), (2048, 512)])
def test_compress_limits(env, shape):
    """eps = 0 keeps everything (a DCT / IDCT round trip); an eps above every
    coefficient zeroes the output exactly."""
    torch, dx, inputs, oracle = env
    x_np = inputs.normal(shape, 7300 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    same = dx.compress2d(x, 0.0)
    zero = dx.compress2d(x, 1e30)
    torch.cuda.synchronize()
    assert oracle.rel_l2(same.cpu().numpy(), x_np) <= TOL
    assert not bool(zero.any())


def test_fused_equals_composed(env):
    """The fused three-pass compression equals DCT, the threshold as a tensor
    operation, and IDCT composed from the plain entry points."""
    torch, dx, inputs, oracle = env
    x = torch.from_numpy(inputs.sparse_cosines(512, 768, 7400)).cuda()
    fused = dx.compress2d(x, 0.5)
    b = dx.dct2d(x, "ortho")
    composed = dx.idct2d(torch.where(b.abs() >= 0.5, b, torch.zeros_like(b)), "ortho")
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm((fused - composed).double()) / torch.linalg.vector_norm(composed.double()))
    assert err <= TOL


@pytest.mark.parametrize("shape,eps", [((8, 14), 0.5), ((8, 8), float("nan")), ((8, 8), float("inf")),
                                       ((8, 8), -1.0)])
def test_compress_errors_enqueue_nothing(env, shape, eps):
    torch, dx, _, _ = env
    x = torch.zeros(shape, device="cuda")
    y = torch.full(shape, 2.0, device="cuda")
    with pytest.raises(dx.DctxError):
        dx.compress2d(x, eps, out=y)
    torch.cuda.synchronize()
    assert bool((y == 2.0).all())


@pytest.mark.parametrize("shape", [(9, 15), (64, 75), (100, 81), (6, 5), (48, 2)])
def test_compress_odd_and_two_last_dimension(env, shape):
    """Odd contiguous dimension (the fused column pass takes column 0 alone)
    and n2 = 2 (a length-1 row FFT): whole arrays against the oracle, outputs
    NaN-poisoned."""
    torch, dx, inputs, oracle = env
    x = inputs.sparse_cosines(shape[0], shape[1], 7300 + sum(shape))
    xt = torch.from_numpy(x).cuda()
    y = torch.full_like(xt, float("nan"))
    print(f"[gpu] compress odd {shape}", flush=True)
    dx.compress2d(xt, 0.5, out=y)
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    err = oracle.rel_l2(yn, oracle.compress2d(x, 0.5))
    assert err <= TOL, f"compress {shape}: rel L2 {err:.3e}"
