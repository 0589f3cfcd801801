"""GPU parity of the mixed 2-D transforms IDCT_IDXST and IDXST_IDCT (Eq.
idxst) against the FP64 oracle, through the C ABI.

They run the two IDCT passes with the reversal folded into the inverse pre
and the sign into the row stores, on all three kernel families: the generic
run-time schedules (5-smooth sizes), the power-of-two kernels and the split
column form of tall power-of-two arrays.  Tolerance: relative L2 <= 1e-6, as
for the IDCT.  Whole arrays up to 1024^2; at 2048 and 4096 rows whole output
columns the oracle computes exactly."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-6
FNS = {"idct_idxst2d": "idct_idxst2", "idxst_idct2d": "idxst_idct2"}


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


def _run(env, fn, x_np, norm="backward"):
    torch, dx, _, _ = env
    print(f"[gpu] {fn} shape={x_np.shape} norm={norm}", flush=True)
    y = getattr(dx, fn)(torch.from_numpy(x_np).cuda(), norm)
    torch.cuda.synchronize()
    return y.cpu().numpy()


# generic (5-smooth, odd rows included), power-of-two, and small edge shapes
FULL = [(2, 4), (3, 6), (5, 8), (6, 10), (9, 6), (48, 90), (64, 100), (250, 486), (81, 54), (1024, 6),
        (256, 256), (128, 1024), (1024, 512), (512, 64), (1024, 1024)]


@pytest.mark.parametrize("shape", FULL)
@pytest.mark.parametrize("fn", sorted(FNS))
def test_mixed_full(env, fn, shape):
    _, _, inputs, oracle = env
    x = inputs.uniform(shape, 6000 + 7 * shape[0] + shape[1])
    y = _run(env, fn, x)
    err = oracle.rel_l2(y, getattr(oracle, FNS[fn])(x))
    assert err <= TOL, f"{fn} {shape}: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape", [(6, 10), (256, 256), (250, 486)])
@pytest.mark.parametrize("fn", sorted(FNS))
def test_mixed_ortho(env, fn, shape):
    _, _, inputs, oracle = env
    x = inputs.normal(shape, 6100 + shape[0] + shape[1])
    y = _run(env, fn, x, "ortho")
    err = oracle.rel_l2(y, getattr(oracle, FNS[fn])(x, "ortho"))
    assert err <= TOL, f"{fn} {shape} ortho: rel L2 {err:.3e}"


# the split column form (n1 = 2048 / 4096, power-of-two n2); 4096^2 is the
# paper's largest timed size
SPLIT = [(2048, 512), (4096, 1024), (4096, 4096)]


@pytest.mark.parametrize("shape", SPLIT)
@pytest.mark.parametrize("fn", sorted(FNS))
def test_mixed_split_columns(env, fn, shape):
    _, _, inputs, oracle = env
    n1, n2 = shape
    x = inputs.normal(shape, 6200 + n1 + n2)
    y = _run(env, fn, x)
    err = oracle.rel_l2(y, getattr(oracle, FNS[fn])(x))
    assert err <= TOL, f"{fn} {shape} whole array: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape", [(48, 90), (256, 256), (4096, 1024)])
def test_ignored_line_is_never_read(env, shape):
    """IDXST drops x(0) on its axis: IDCT_IDXST does not read row 0 and
    IDXST_IDCT does not read column 0, so changing them leaves the output
    bitwise equal."""
    torch, dx, inputs, _ = env
    x = torch.from_numpy(inputs.uniform(shape, 6300 + sum(shape))).cuda()
    a = dx.idct_idxst2d(x)
    x2 = x.clone()
    x2[0, :] = 1e3
    b = dx.idct_idxst2d(x2)
    c = dx.idxst_idct2d(x)
    x3 = x.clone()
    x3[:, 0] = -1e3
    d = dx.idxst_idct2d(x3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(c, d)


def test_idct_unchanged_beside_mixed(env):
    """The plain IDCT of the same cached plans is unaffected by the mixed calls."""
    torch, dx, inputs, oracle = env
    x_np = inputs.uniform((256, 512), 6400)
    x = torch.from_numpy(x_np).cuda()
    first = dx.idct2d(x)
    dx.idct_idxst2d(x)
    dx.idxst_idct2d(x)
    second = dx.idct2d(x)
    torch.cuda.synchronize()
    assert torch.equal(first, second)
    assert oracle.rel_l2(second.cpu().numpy(), oracle.idctn(x_np)) <= TOL


@pytest.mark.parametrize("shape", [(6, 5), (9, 15), (64, 75), (100, 81), (27, 125), (512, 375), (3, 3), (10, 2),
                                   (64, 2)])
@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("fn", sorted(FNS))
def test_mixed_odd_and_two_last_dimension(env, fn, norm, shape):
    """Odd contiguous dimension (generic kernels; the column reversal pairs
    column k2 with n2 - k2 and column 0 with the zero column n2, the signs ride
    on the full-length row stores) and n2 = 2: whole arrays against the
    oracle, outputs NaN-poisoned."""
    torch, dx, inputs, oracle = env
    x_np = inputs.uniform(shape, 6400 + 3 * shape[0] + shape[1])
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] {fn} odd {shape} {norm}", flush=True)
    getattr(dx, fn)(x, norm, out=y)
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    err = oracle.rel_l2(yn, getattr(oracle, FNS[fn])(x_np, norm))
    assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


@pytest.mark.parametrize("shape", [(8, 7), (8, 14), (1, 8)])
@pytest.mark.parametrize("fn", sorted(FNS))
def test_unsupported_shapes_rejected(env, fn, shape):
    torch, dx, _, _ = env
    x = torch.zeros(shape, device="cuda")
    y = torch.full(shape, 5.0, device="cuda")
    with pytest.raises(dx.DctxError):
        getattr(dx, fn)(x, out=y)
    torch.cuda.synchronize()
    assert bool((y == 5.0).all())
