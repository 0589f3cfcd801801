"""GPU tests of the allocation-free 2-D entry point (dctx_dct2d_noalloc),
through the C ABI via the binding: its results against the plain entry points
(dctx_dct2d / dctx_idct2d, same kernels: bitwise equal) and against the FP64
oracle (relative L2 <= 1e-6), on calls in a row whose shapes shrink, so a
call finds the previous call's contents in the shared static scratch; device
memory does not change across the calls; shapes beyond the scratch are
refused with DCTX_ERR_TOO_LARGE and leave the output untouched."""
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


# Shapes in call order, each smaller than the one before: 4096^2 (the largest
# the scratch holds; split form, two units per workgroup), 8192 x 40 (long
# columns: row pass, radix-8 step, 1024-point columns), 1000 x 768 (fast
# power-of-two rows, generic columns), 10000 x 100 (transposed route), 250 x 486
# (generic kernels), 48 x 90.
SEQ = [(4096, 4096), (8192, 40), (1000, 768), (10000, 100), (250, 486), (48, 90)]


@pytest.mark.parametrize("norm", ["backward", "ortho"])
def test_noalloc_calls_in_a_row_match_plain(env, norm):
    torch, dx, inputs, oracle = env
    xs = [torch.from_numpy(inputs.normal(s, 7100 + i)).cuda() for i, s in enumerate(SEQ)]
    outs = [[torch.full(s, float("nan"), device="cuda") for _ in range(2)] for s in SEQ]
    refs = []
    for x in xs:
        y = dx.dct2d(x, norm)
        refs.append((y, dx.idct2d(x, norm)))
    torch.cuda.synchronize()
    free0 = None
    for i, (s, x) in enumerate(zip(SEQ, xs)):
        for inv in (False, True):
            print(f"[gpu] dctx_dct2d_noalloc shape={s} norm={norm} inverse={inv}", flush=True)
            dx.dct2d_noalloc(x, outs[i][inv], norm, inverse=inv)
            torch.cuda.synchronize()
            if free0 is None:
                free0 = torch.cuda.mem_get_info()[0]   # after set-up (first call)
            got = outs[i][inv].cpu().numpy()
            want = refs[i][inv].cpu().numpy()
            assert np.array_equal(got, want), f"{s} inverse={inv}: differs from the plain call"
            assert oracle.rel_l2(got, want) <= TOL
    assert torch.cuda.mem_get_info()[0] == free0, "device memory changed across allocation-free calls"
    # the oracle on the smaller shapes (the plain calls' own parity tests cover the rest)
    for i in (4, 5):
        x = xs[i].cpu().numpy()
        for inv, fn in ((False, "dctn"), (True, "idctn")):
            err = oracle.rel_l2(outs[i][inv].cpu().numpy(), getattr(oracle, fn)(x, norm))
            assert err <= TOL, f"{SEQ[i]} inverse={inv}: rel L2 {err:.3e} vs oracle"


def test_noalloc_repeat_same_shape_after_smaller(env):
    """A 4096^2 call after smaller ones (tables of several shapes in the arena)
    still matches the plain call."""
    torch, dx, inputs, _ = env
    for s, seed in (((512, 512), 7201), ((4096, 4096), 7202), ((64, 64), 7203), ((4096, 4096), 7204)):
        print(f"[gpu] dctx_dct2d_noalloc shape={s} seed={seed}", flush=True)
        x = torch.from_numpy(inputs.normal(s, seed)).cuda()
        y = torch.empty_like(x)
        dx.dct2d_noalloc(x, y)
        ref = dx.dct2d(x)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"{s}: differs from the plain call"


@pytest.mark.parametrize("shape", [(4096, 4098), (8192, 4096), (16384, 2048)])
def test_noalloc_too_large(env, shape):
    torch, dx, _, _ = env
    x = torch.zeros(shape, device="cuda")
    y = torch.full(shape, float("nan"), device="cuda")
    with pytest.raises(dx.DctxError) as ei:
        dx.dct2d_noalloc(x, y)
    assert "ERR_TOO_LARGE" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.isnan(y).all()), "a refused call wrote its output"


def test_noalloc_invalid_arguments(env):
    torch, dx, _, _ = env
    x = torch.zeros((64, 77), device="cuda")
    y = torch.empty_like(x)
    lib = dx.lib()
    h = dx.default_handle(0)
    assert lib.dctx_dct2d_noalloc(None, x.data_ptr(), y.data_ptr(), 64, 64, 0, 0, None) == 1
    assert lib.dctx_dct2d_noalloc(h.ptr, x.data_ptr(), y.data_ptr(), 64, 64, 0, 2, None) == 1
    assert lib.dctx_dct2d_noalloc(h.ptr, x.data_ptr(), x.data_ptr(), 64, 64, 0, 0, None) == 1
    assert lib.dctx_dct2d_noalloc(h.ptr, x.data_ptr(), y.data_ptr(), 0, 64, 0, 0, None) == 1
    assert lib.dctx_dct2d_noalloc(h.ptr, x.data_ptr(), y.data_ptr(), 64, 7 * 11, 0, 0, None) == 2
