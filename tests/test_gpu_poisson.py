"""GPU parity of the fused spectral Neumann Poisson solve against the FP64
oracle (``oracle.poisson2d_neumann``: DCT-II, divide by the 5-point Neumann
Laplacian eigenvalues with U(0,0) = 0, DCT-III), through the C ABI.

Tolerance: relative L2 <= 1e-6 (FP32 data, FP64-built tables).  Whole arrays
against the oracle at every size (2048^2 and the split-form grids included); the
discrete-Laplacian residual at sizes where FP32 rounding of u keeps it
meaningful."""
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


def _solve(env, f, h1=0.0, h2=0.0):
    torch, dx, _, _ = env
    print(f"[gpu] poisson2d shape={f.shape} h=({h1},{h2})", flush=True)
    u = dx.poisson2d(torch.from_numpy(f).cuda(), h1, h2)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _neumann_laplacian(u, h1, h2):
    """Cell-centred 5-point Laplacian with mirrored ghost cells, FP64."""
    u = np.asarray(u, dtype=np.float64)
    p = np.pad(u, 1, mode="edge")
    return ((p[2:, 1:-1] - 2 * u + p[:-2, 1:-1]) / (h1 * h1) +
            (p[1:-1, 2:] - 2 * u + p[1:-1, :-2]) / (h2 * h2))


SHAPES = [(4, 4), (6, 10), (5, 8), (9, 6), (48, 90), (64, 100), (250, 486), (256, 256), (128, 1000), (1024, 1024),
          (2, 4), (3, 6)]


@pytest.mark.parametrize("shape", SHAPES)
def test_poisson_full(env, shape):
    _, _, inputs, oracle = env
    f = inputs.gaussian_bumps(shape[0], shape[1], 5000 + sum(shape))
    u = _solve(env, f)
    ref = oracle.poisson2d_neumann(f)
    err = oracle.rel_l2(u, ref)
    assert err <= TOL, f"poisson {shape}: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape,h", [((96, 80), (0.01, 0.02)), ((256, 128), (1.0, 1.0)), ((30, 40), (0.5, 0.25))])
def test_poisson_spacings(env, shape, h):
    _, _, inputs, oracle = env
    f = inputs.uniform(shape, 5100 + sum(shape))
    u = _solve(env, f, *h)
    ref = oracle.poisson2d_neumann(f, *h)
    err = oracle.rel_l2(u, ref)
    assert err <= TOL, f"poisson {shape} h={h}: rel L2 {err:.3e}"


@pytest.mark.parametrize("n", [2048])
def test_poisson_2048_columns_and_residual(env, n):
    """2048^2 smooth RHS (32 Gaussians): the whole solution against the
    oracle."""
    _, _, inputs, oracle = env
    f = inputs.gaussian_bumps(n, n, 5200)
    u = _solve(env, f)
    err = oracle.rel_l2(u, oracle.poisson2d_neumann(f))
    assert err <= TOL, f"poisson 2048^2 whole array: rel L2 {err:.3e}"
    assert abs(u.astype(np.float64).mean()) <= 1e-6 * np.abs(u).max()


@pytest.mark.parametrize("n", [64, 128, 256])
def test_poisson_residual(env, n):
    """The discrete Neumann Laplacian of u equals f - mean(f).  The Laplacian
    amplifies the FP32 rounding of u by up to 8 n^2 |u| / |f| (about 5e-2 at
    2048^2), so the check runs at sizes where that stays below 1e-2."""
    _, _, inputs, _ = env
    f = inputs.gaussian_bumps(n, n, 5250 + n)
    u = _solve(env, f)
    res = _neumann_laplacian(u, 1.0 / n, 1.0 / n)
    g = f.astype(np.float64) - f.astype(np.float64).mean()
    rres = np.linalg.norm(res - g) / np.linalg.norm(g)
    assert rres <= 1e-2, f"residual {rres:.3e}"
    assert abs(u.astype(np.float64).mean()) <= 1e-6 * np.abs(u).max()


def test_poisson_deterministic_and_fused_equals_composed(env):
    """The fused three-pass solve equals DCT -> divide -> IDCT composed from the
    plain entry points (same tables), to the FP32 tolerance."""
    torch, dx, inputs, oracle = env
    n1, n2 = 512, 768
    f = torch.from_numpy(inputs.gaussian_bumps(n1, n2, 5300)).cuda()
    a = dx.poisson2d(f)
    b = dx.poisson2d(f)
    F = dx.dct2d(f).double()
    lam = torch.from_numpy(oracle.neumann_eigenvalues(n1, n2, 1.0 / n1, 1.0 / n2)).cuda()
    lam[0, 0] = 1.0
    U = (F / lam).float()
    U[0, 0] = 0.0
    c = dx.idct2d(U)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    err = float(torch.linalg.vector_norm((a - c).double()) / torch.linalg.vector_norm(c.double()))
    assert err <= TOL


@pytest.mark.parametrize("shape,h", [((8, 7), (0.0, 0.0)), ((1, 8), (0.0, 0.0)), ((8, 8), (float("nan"), 0.0)),
                                     ((8, 8), (0.0, float("inf")))])
def test_poisson_errors_enqueue_nothing(env, shape, h):
    torch, dx, _, _ = env
    f = torch.zeros(shape, device="cuda")
    u = torch.full(shape, 3.0, device="cuda")
    with pytest.raises(dx.DctxError):
        dx.poisson2d(f, *h, out=u)
    torch.cuda.synchronize()
    assert bool((u == 3.0).all())


@pytest.mark.parametrize("shape", [(2048, 512), (2048, 2048), (4096, 1024), (4096, 4096)])
def test_poisson_split_form(env, shape):
    """Tall power-of-two grids take the split-column kernels (row pass with the
    first radix-8 column step, fused column pass on q-point FFTs): the whole
    solution against the plain kernels (a handle created with DCTX_SPLIT=0)
    and against the oracle.  4096^2 takes the two-unit row
    kernels with their tables in LDS."""
    import os
    torch, dx, inputs, oracle = env
    n1, n2 = shape
    f = inputs.gaussian_bumps(n1, n2, 5400 + n1 + n2)
    ft = torch.from_numpy(f).cuda()
    print(f"[gpu] poisson split {shape}", flush=True)
    us = dx.poisson2d(ft, handle=dx.Handle(0))
    os.environ["DCTX_SPLIT"] = "0"
    try:
        up = dx.poisson2d(ft, handle=dx.Handle(0))
    finally:
        del os.environ["DCTX_SPLIT"]
    torch.cuda.synchronize()
    us_np = us.cpu().numpy()
    assert oracle.rel_l2(us_np, up.cpu().numpy()) <= TOL
    assert oracle.rel_l2(us_np, oracle.poisson2d_neumann(f)) <= TOL


@pytest.mark.parametrize("shape,h", [((9, 15), (0.0, 0.0)), ((64, 75), (0.0, 0.0)), ((100, 81), (0.02, 0.05)),
                                     ((250, 45), (0.0, 0.0)), ((6, 5), (0.0, 0.0)), ((64, 2), (0.0, 0.0))])
def test_poisson_odd_and_two_last_dimension(env, shape, h):
    """Odd contiguous dimension (the fused column pass takes column 0 alone,
    paired with the zero column n2) and n2 = 2: whole solutions against the
    oracle."""
    _, _, inputs, oracle = env
    f = inputs.uniform(shape, 5500 + sum(shape))
    u = _solve(env, f, *h)
    ref = oracle.poisson2d_neumann(f, *(v if v > 0 else None for v in h))
    err = oracle.rel_l2(u, ref)
    assert err <= TOL, f"poisson {shape} h={h}: rel L2 {err:.3e}"
