"""GPU parity of the 2-D three-stage transforms and the row-column baseline
against the FP64 oracle, through the C ABI (via the thin Python binding).

Tolerance: relative L2 error <= 1e-6 over the compared outputs (FP32 data,
FP64-generated tables).  Every array is compared whole against the oracle, the
full-size 1024^2, 2048^2, 4096^2 and 2048x1024 cases included (in the launch
configuration the benchmark times); only the 8192^2 long-column case, outside
the benchmarked sizes, compares whole output rows and columns."""
import sys

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


def _run(env, fn, x_np, norm):
    torch, dx, _, _ = env
    print(f"[gpu] {fn} shape={x_np.shape} norm={norm}", flush=True)
    x = torch.from_numpy(x_np).cuda()
    y = getattr(dx, fn)(x, norm)
    torch.cuda.synchronize()
    return y.cpu().numpy()


FWD = {"dct2d": "dctn", "rc_dct2d": "dctn"}
INV = {"idct2d": "idctn", "rc_idct2d": "idctn"}

SMALL = [(256, 256), (2, 4), (3, 8), (6, 10), (16, 12), (48, 90), (250, 486), (100, 64),
         (64, 100), (128, 1000), (1024, 6), (5, 1024), (81, 54), (2, 2), (6, 2), (64, 2), (1000, 2)]


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("fn", ["dct2d", "idct2d"])
def test_three_stage_small_full(env, fn, shape, norm):
    _, _, inputs, oracle = env
    x = inputs.uniform(shape, 1000 + sum(shape))
    y = _run(env, fn, x, norm)
    ref = getattr(oracle, FWD.get(fn) or INV[fn])(x, norm)
    err = oracle.rel_l2(y, ref)
    assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


ODD = [(6, 5), (2, 3), (3, 3), (9, 15), (64, 75), (100, 81), (27, 125), (48, 225), (250, 45), (16, 135),
       (512, 375)]


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", ODD)
@pytest.mark.parametrize("fn", ["dct2d", "idct2d"])
def test_odd_last_dimension_full(env, fn, shape, norm):
    """Odd contiguous dimension: the row pass runs a full-length complex FFT
    of the real row and keeps columns 0 .. (n2-1)/2 (no packed Nyquist
    column).  Whole arrays against the oracle; outputs start as NaN so every
    element must be written."""
    torch, dx, inputs, oracle = env
    x_np = inputs.uniform(shape, 1700 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] odd {fn} shape={shape} norm={norm}", flush=True)
    getattr(dx, fn)(x, norm, out=y)
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    ref = getattr(oracle, FWD.get(fn) or INV[fn])(x_np, norm)
    err = oracle.rel_l2(yn, ref)
    assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


def test_odd_last_dimension_roundtrip_and_limits(env):
    """IDCT(DCT(x)) = x for an odd contiguous dimension; odd lengths above the
    one-workgroup row FFT are refused (DCTX_ERR_UNSUPPORTED, nothing
    enqueued)."""
    torch, dx, inputs, oracle = env
    x = torch.from_numpy(inputs.normal((360, 405), 1750)).cuda()
    z = dx.idct2d(dx.dct2d(x))
    torch.cuda.synchronize()
    assert float(torch.linalg.vector_norm(z - x) / torch.linalg.vector_norm(x)) <= TOL
    lib = dx.lib()
    h = dx.default_handle(0)
    s = torch.cuda.current_stream().cuda_stream
    # odd n2 above 7680 (here 3 5^5) needs more than one workgroup per row FFT
    xl = torch.ones(2, 9375, device="cuda")
    yl = torch.full((2, 9375), 7.0, device="cuda")
    assert lib.dctx_dct2d(h.ptr, xl.data_ptr(), yl.data_ptr(), 2, 9375, 0, s) == 2
    torch.cuda.synchronize()
    assert torch.all(yl == 7.0)


@pytest.mark.parametrize("shape", [(256, 256), (6, 10), (48, 90), (250, 486), (64, 100), (128, 1000), (9, 15),
                                   (75, 64), (81, 125), (2, 2), (6, 2), (3, 5), (1000, 6)])
@pytest.mark.parametrize("fn", ["rc_dct2d", "rc_idct2d"])
@pytest.mark.parametrize("norm", ["backward", "ortho"])
def test_row_column_small_full(env, fn, shape, norm):
    _, _, inputs, oracle = env
    x = inputs.normal(shape, 2000 + sum(shape))
    y = _run(env, fn, x, norm)
    ref = getattr(oracle, FWD.get(fn) or INV[fn])(x, norm)
    err = oracle.rel_l2(y, ref)
    assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


def test_config1_roundtrip_256(env):
    """256 x 256 uniform[-1,1], seed 1000: DCT then IDCT recovers x; IDCT of an
    N(0,1) array matches the oracle."""
    torch, dx, inputs, oracle = env
    x = inputs.uniform((256, 256), 1000)
    xt = torch.from_numpy(x).cuda()
    back = dx.idct2d(dx.dct2d(xt)).cpu().numpy()
    assert oracle.rel_l2(back, x) <= TOL
    z = inputs.normal((256, 256), 1001)
    assert oracle.rel_l2(_run(env, "idct2d", z, "backward"), oracle.idctn(z)) <= TOL


def _lines(n, rng, count=6):
    picks = {0, 1, n // 2 - 1, n // 2, n // 2 + 1, n - 1}
    picks |= set(int(v) for v in rng.integers(0, n, count))
    return sorted(p for p in picks if 0 <= p < n)


_REF_CACHE = {}


def _full_seed(shape):
    return 2000 + shape[0] // 1024 * 10 + shape[1] // 1024


def _whole_ref(oracle, inputs, direction, shape, seed):
    """Whole-array oracle output (cached: the three-stage and row-column tests
    compare against the same array)."""
    key = (direction, shape, seed)
    if key not in _REF_CACHE:
        x = inputs.normal(shape, seed)
        _REF_CACHE[key] = (oracle.dctn if direction == "dct" else oracle.idctn)(x, "backward")
    return _REF_CACHE[key]


@pytest.mark.parametrize("shape", [(1024, 1024), (2048, 2048), (4096, 4096), (2048, 1024)])
@pytest.mark.parametrize("fn", ["dct2d", "idct2d", "rc_dct2d", "rc_idct2d"])
def test_full_size_whole_array(env, fn, shape):
    """Config-2 sizes, N(0,1): the whole output against the oracle (every
    element, outputs NaN-poisoned first so each must be written)."""
    torch, dx, inputs, oracle = env
    seed = _full_seed(shape)
    x_np = inputs.normal(shape, seed)
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] whole array {fn} {shape}", flush=True)
    getattr(dx, fn)(x, out=y)
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    ref = _whole_ref(oracle, inputs, "dct" if fn in FWD else "idct", shape, seed)
    err = oracle.rel_l2(yn, ref)
    assert err <= TOL, f"{fn} {shape}: whole-array rel L2 {err:.3e}"


def test_roundtrip_4096(env):
    torch, dx, inputs, oracle = env
    x = inputs.normal((4096, 4096), 2099)
    xt = torch.from_numpy(x).cuda()
    for norm in ("backward", "ortho"):
        back = dx.idct2d(dx.dct2d(xt, norm), norm).cpu().numpy()
        assert oracle.rel_l2(back, x) <= 2 * TOL
        back_rc = dx.rc_idct2d(dx.rc_dct2d(xt, norm), norm).cpu().numpy()
        assert oracle.rel_l2(back_rc, x) <= 2 * TOL


def test_every_output_written_once_poisoned(env):
    """Outputs pre-filled with NaN: every element must be overwritten."""
    torch, dx, inputs, _ = env
    for shape in [(6, 10), (250, 486), (1024, 1024)]:
        x = torch.from_numpy(inputs.uniform(shape, 3)).cuda()
        for fn in ("dct2d", "idct2d", "rc_dct2d", "rc_idct2d"):
            out = torch.full(shape, float("nan"), device="cuda")
            getattr(dx, fn)(x, out=out)
            torch.cuda.synchronize()
            assert torch.isfinite(out).all(), f"{fn} {shape} left unwritten outputs"


# (3, 6561): the largest odd 5-smooth length (3^8) a one-workgroup FFT of at
# most 512 threads x 15 values takes
LIMITS = [(8192, 16384), (2, 16384), (8192, 4), (3, 6561), (16, 5625)]


@pytest.mark.parametrize("shape", LIMITS)
@pytest.mark.parametrize("fn", ["dct2d", "idct2d"])
def test_size_limits(env, fn, shape):
    """The largest supported lengths along each axis (n1 = 8192, n2 = 16384,
    odd n2 = 6561): every output written (NaN-poisoned), whole output rows
    against the oracle, and the round trip over the whole array."""
    torch, dx, inputs, oracle = env
    n1, n2 = shape
    x_np = inputs.normal(shape, 1900 + n1 + n2)
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] limits {fn} {shape}", flush=True)
    getattr(dx, fn)(x, out=y)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all())
    rows = sorted({0, 1, n1 // 2, n1 - 1})
    ref = getattr(oracle, FWD.get(fn) or INV[fn])(x_np, sel={0: rows})
    err = oracle.rel_l2(y[rows].cpu().numpy(), ref)
    assert err <= TOL, f"{fn} {shape}: rows rel L2 {err:.3e}"
    back = dx.idct2d(y) if fn == "dct2d" else dx.dct2d(y)
    torch.cuda.synchronize()
    if fn == "dct2d":
        rt = float(torch.linalg.vector_norm((back - x).double()) / torch.linalg.vector_norm(x.double()))
        assert rt <= TOL, f"round trip {shape}: {rt:.3e}"
    del x, y, back
    torch.cuda.empty_cache()


def test_deterministic(env):
    torch, dx, inputs, _ = env
    x = torch.from_numpy(inputs.normal((2048, 2048), 11)).cuda()
    a = dx.dct2d(x)
    b = dx.dct2d(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_errors_enqueue_nothing(env):
    torch, dx, _, _ = env
    lib = dx.lib()
    h = dx.default_handle(0)
    x = torch.ones(64, 64, device="cuda")
    y = torch.full((64, 64), 7.0, device="cuda")
    xp, yp = x.data_ptr(), y.data_ptr()
    s = torch.cuda.current_stream().cuda_stream
    cases = [
        ((h.ptr, xp, yp, 64, 63, 0, s), 2),     # last dimension not 5-smooth (63 = 9 x 7)
        ((h.ptr, xp, yp, 64, 0, 0, s), 1),      # zero dimension
        ((h.ptr, xp, yp, 7, 64, 0, s), 2),      # not 5-smooth
        ((h.ptr, xp, yp, 64, 64, 5, s), 1),     # bad norm
        ((h.ptr, xp, xp, 64, 64, 0, s), 1),     # in place
        ((h.ptr, xp, xp + 4 * 64, 64, 64, 0, s), 1),   # overlap
        ((h.ptr, xp + 4, yp, 32, 64, 0, s), 1),  # misaligned
    ]
    for args, want in cases:
        for name in ("dctx_dct2d", "dctx_idct2d", "dctx_rc_dct2d", "dctx_rc_idct2d"):
            assert getattr(lib, name)(*args) == want, (name, args[3:6])
    # beyond the longest supported length, with buffers of the claimed size
    xb = torch.ones(2, 32768, device="cuda")
    yb = torch.full((2, 32768), 7.0, device="cuda")
    for name in ("dctx_dct2d", "dctx_idct2d", "dctx_rc_dct2d", "dctx_rc_idct2d"):
        assert getattr(lib, name)(h.ptr, xb.data_ptr(), yb.data_ptr(), 2, 32768, 0, s) == 2, name
    torch.cuda.synchronize()
    assert torch.all(y == 7.0)
    assert torch.all(yb == 7.0)


def test_caller_workspace_and_streams(env):
    """The _ws entry points on two streams with two workspaces give the same
    results as the handle's own workspace."""
    torch, dx, inputs, _ = env
    import ctypes
    lib = dx.lib()
    h = dx.default_handle(0)
    shape = (512, 768)
    xs = [torch.from_numpy(inputs.normal(shape, 40 + i)).cuda() for i in range(2)]
    ref = [dx.dct2d(x) for x in xs]
    wsb = dx.workspace_bytes_2d(*shape)
    streams = [torch.cuda.Stream() for _ in range(2)]
    outs = [torch.empty(shape, device="cuda") for _ in range(2)]
    wss = [torch.empty(wsb // 4, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    for i in range(2):
        st = lib.dctx_dct2d_ws(h.ptr, xs[i].data_ptr(), outs[i].data_ptr(), shape[0], shape[1], 0,
                               wss[i].data_ptr(), wsb, ctypes.c_void_p(streams[i].cuda_stream))
        assert st == 0
    assert lib.dctx_dct2d_ws(h.ptr, xs[0].data_ptr(), outs[0].data_ptr(), shape[0], shape[1], 0,
                             wss[0].data_ptr(), wsb - 8, None) == 1
    torch.cuda.synchronize()
    for i in range(2):
        assert torch.equal(outs[i], ref[i])


def test_unaligned_16_bytes(env):
    """Pointers that are 8- but not 16-byte aligned take the 8-byte access path."""
    torch, dx, inputs, oracle = env
    lib = dx.lib()
    h = dx.default_handle(0)
    n1, n2 = 64, 96
    x = inputs.normal((n1, n2), 77)
    buf_x = torch.zeros(n1 * n2 + 2, device="cuda")
    buf_y = torch.zeros(n1 * n2 + 2, device="cuda")
    buf_x[2:] = torch.from_numpy(x.ravel()).cuda()
    s = torch.cuda.current_stream().cuda_stream
    assert lib.dctx_dct2d(h.ptr, buf_x.data_ptr() + 8, buf_y.data_ptr() + 8, n1, n2, 0, s) == 0
    torch.cuda.synchronize()
    y = buf_y[2:].cpu().numpy().reshape(n1, n2)
    assert oracle.rel_l2(y, oracle.dctn(x)) <= TOL
    assert lib.dctx_idct2d(h.ptr, buf_y.data_ptr() + 8, buf_x.data_ptr() + 8, n1, n2, 0, s) == 0
    torch.cuda.synchronize()
    back = buf_x[2:].cpu().numpy().reshape(n1, n2)
    assert oracle.rel_l2(back, x) <= TOL


FAST_SHAPES = [(64, 64), (128, 64), (64, 128), (256, 512), (512, 256), (1024, 128), (128, 1024),
               (64, 4096), (4096, 64), (2048, 256), (256, 2048), (4096, 512)]


@pytest.mark.parametrize("norm", ["backward", "ortho"])
@pytest.mark.parametrize("shape", FAST_SHAPES)
@pytest.mark.parametrize("fn", ["dct2d", "idct2d"])
def test_fast_path_shapes(env, fn, shape, norm):
    """Power-of-two shapes take the compile-time fast kernels (every fast length
    for both the row length n2/2 in [32, 2048] and the column length n1 in
    [64, 4096])."""
    _, _, inputs, oracle = env
    x = inputs.normal(shape, 5000 + shape[0] + 3 * shape[1])
    y = _run(env, fn, x, norm)
    if x.size <= 1 << 20:
        ref = getattr(oracle, FWD.get(fn) or INV[fn])(x, norm)
        err = oracle.rel_l2(y, ref)
    else:
        g = inputs.rng(3)
        cols = _lines(shape[1], g)
        ref = getattr(oracle, FWD.get(fn) or INV[fn])(x, norm, sel={1: cols})
        err = oracle.rel_l2(y[:, cols], ref)
    assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


def test_fast_and_general_paths_agree(env):
    """The same power-of-two transform through the fast kernels and through the
    general kernels (a handle created with DCTX_FAST=0) agree to rounding."""
    import os
    torch, dx, inputs, oracle = env
    x = torch.from_numpy(inputs.normal((512, 1024), 9)).cuda()
    fast = dx.Handle(0)
    os.environ["DCTX_FAST"] = "0"
    try:
        gen = dx.Handle(0)
        a = dx.dct2d(x, handle=gen)
        b = dx.idct2d(x, handle=gen)
    finally:
        del os.environ["DCTX_FAST"]
    c = dx.dct2d(x, handle=fast)
    d = dx.idct2d(x, handle=fast)
    torch.cuda.synchronize()
    assert oracle.rel_l2(c.cpu().numpy(), a.cpu().numpy()) <= TOL
    assert oracle.rel_l2(d.cpu().numpy(), b.cpu().numpy()) <= TOL


def test_unaligned_on_fast_shape(env):
    """8- but not 16-byte aligned pointers on a power-of-two shape run the
    general kernels with the fast plan's tables."""
    torch, dx, inputs, oracle = env
    lib = dx.lib()
    h = dx.default_handle(0)
    n1, n2 = 128, 256
    x = inputs.normal((n1, n2), 78)
    buf_x = torch.zeros(n1 * n2 + 2, device="cuda")
    buf_y = torch.zeros(n1 * n2 + 2, device="cuda")
    buf_x[2:] = torch.from_numpy(x.ravel()).cuda()
    s = torch.cuda.current_stream().cuda_stream
    assert lib.dctx_dct2d(h.ptr, buf_x.data_ptr() + 8, buf_y.data_ptr() + 8, n1, n2, 1, s) == 0
    torch.cuda.synchronize()
    y = buf_y[2:].cpu().numpy().reshape(n1, n2)
    assert oracle.rel_l2(y, oracle.dctn(x, "ortho")) <= TOL
    assert lib.dctx_idct2d(h.ptr, buf_y.data_ptr() + 8, buf_x.data_ptr() + 8, n1, n2, 1, s) == 0
    torch.cuda.synchronize()
    assert oracle.rel_l2(buf_x[2:].cpu().numpy().reshape(n1, n2), x) <= TOL


SPLIT_SHAPES = [(2048, 512), (2048, 4096), (4096, 512), (4096, 1024), (4096, 2048), (2048, 1024), (4096, 4096)]


@pytest.mark.parametrize("shape", SPLIT_SHAPES)
@pytest.mark.parametrize("fn", ["dct2d", "idct2d"])
def test_split_column_form(env, fn, shape):
    """Tall power-of-two shapes (n1 = 2048, 4096) take the split-column
    kernels: the whole array against the oracle, and against the plain column
    kernels (DCTX_SPLIT=0)."""
    import os
    torch, dx, inputs, oracle = env
    n1, n2 = shape
    seed = _full_seed(shape) if shape in ((2048, 1024), (4096, 4096)) else 2300 + n1 + n2
    x = inputs.normal(shape, seed)
    xt = torch.from_numpy(x).cuda()
    print(f"[gpu] split {fn} {shape}", flush=True)
    old = os.environ.get("DCTX_SPLIT")
    try:
        os.environ["DCTX_SPLIT"] = "1"
        y = getattr(dx, fn)(xt)
        os.environ["DCTX_SPLIT"] = "0"
        y0 = getattr(dx, fn)(xt)
    finally:
        if old is None:
            del os.environ["DCTX_SPLIT"]
        else:
            os.environ["DCTX_SPLIT"] = old
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert oracle.rel_l2(yn, y0.cpu().numpy()) <= TOL
    ref = _whole_ref(oracle, inputs, "dct" if fn == "dct2d" else "idct", shape, seed)
    err = oracle.rel_l2(yn, ref)
    assert err <= TOL, f"{fn} {shape}: whole-array rel L2 {err:.3e}"


def test_split_roundtrip_and_written(env):
    torch, dx, inputs, oracle = env
    x = torch.from_numpy(inputs.uniform((4096, 4096), 2400)).cuda()
    y = torch.full_like(x, float("nan"))
    dx.dct2d(x, out=y)
    z = torch.full_like(x, float("nan"))
    dx.idct2d(y, out=z)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all()) and bool(torch.isfinite(z).all())
    err = float(torch.linalg.vector_norm(z - x) / torch.linalg.vector_norm(x))
    assert err <= TOL


TRANSPOSED = [(10000, 100), (16384, 6), (9000, 30), (8640, 2), (12000, 75), (16384, 64), (10240, 9)]


@pytest.mark.parametrize("shape", TRANSPOSED)
@pytest.mark.parametrize("fn", ["dct2d", "idct2d"])
def test_transposed_route(env, fn, shape):
    """Columns longer than one workgroup holds (n1 > 8192): the array is
    transformed as its n2 x n1 transpose with the transposes folded into the
    passes (the row pass reads columns of x, the column pass writes rows of y;
    the paper's 10000 x 100 shape among them).  Whole arrays against the
    oracle, outputs NaN-poisoned, and no transpose kernel runs."""
    torch, dx, inputs, oracle = env
    x = inputs.uniform(shape, 9000 + shape[1])
    xt = torch.from_numpy(x).cuda()
    h = dx.Handle(0)
    for norm in ("backward", "ortho"):
        print(f"[gpu] {fn} axis-order route {shape} {norm}", flush=True)
        y = torch.full_like(xt, float("nan"))
        h.profile(True)
        h.profile_read()
        getattr(dx, fn)(xt, norm, out=y, handle=h)
        prof = h.profile_read()
        h.profile(False)
        torch.cuda.synchronize()
        assert "transpose" not in prof, sorted(prof)
        yn = y.cpu().numpy()
        assert np.isfinite(yn).all()
        ref = getattr(oracle, FWD.get(fn) or INV[fn])(x, norm)
        err = oracle.rel_l2(yn, ref)
        assert err <= TOL, f"{fn} {shape} {norm}: rel L2 {err:.3e}"


@pytest.mark.parametrize("fn,ofn", [("idct_idxst2d", "idct_idxst2"), ("idxst_idct2d", "idxst_idct2")])
def test_transposed_route_mixed(env, fn, ofn):
    """The IDXST axis follows the transpose."""
    _, _, inputs, oracle = env
    x = inputs.uniform((10000, 100), 9100)
    y = _run(env, fn, x, "backward")
    err = oracle.rel_l2(y, getattr(oracle, ofn)(x))
    assert err <= TOL, f"{fn} 10000x100: rel L2 {err:.3e}"


def test_transposed_route_caller_workspace(env):
    """The axis-order route through dctx_dct2d_ws: the reported workspace size
    is the transposed problem's spectrum, the result equals the handle's own
    workspace, and a workspace 16 bytes short is rejected."""
    torch, dx, inputs, _ = env
    import ctypes
    lib = dx.lib()
    h = dx.default_handle(0)
    n1, n2 = 10000, 100
    x = torch.from_numpy(inputs.normal((n1, n2), 9200)).cuda()
    ref = dx.dct2d(x)
    wsb = dx.workspace_bytes_2d(n1, n2)
    assert wsb == n2 * (n1 // 2) * 8
    ws = torch.empty(wsb // 4 + 64, device="cuda")
    out = torch.full((n1, n2), 3.0, device="cuda")
    assert lib.dctx_dct2d_ws(h.ptr, x.data_ptr(), out.data_ptr(), n1, n2, 0, ws.data_ptr(),
                             wsb - 16, None) == 1
    torch.cuda.synchronize()
    assert bool((out == 3.0).all())
    assert lib.dctx_dct2d_ws(h.ptr, x.data_ptr(), out.data_ptr(), n1, n2, 0, ws.data_ptr(), wsb, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


LONG_SHAPES = [(8192, 2), (8192, 6), (8192, 16), (8192, 1000), (8192, 2048), (8192, 8192)]


@pytest.mark.parametrize("shape", LONG_SHAPES)
@pytest.mark.parametrize("fn", ["dct2d", "idct2d"])
def test_long_column_route(env, fn, shape):
    """n1 = 8192 (even n2): plain row pass, the radix-8 column step as a pass
    of its own, then the 1024-point split column kernels.  Whole output rows
    (every residue class mod 8, both ends of each 1024-row block) and columns
    (first, last, Nyquist-adjacent, a ragged tile) against the oracle, and the
    whole array against the plain column kernels (DCTX_SPLIT=0); the whole
    array against the oracle up to 8192 x 2048."""
    import os
    torch, dx, inputs, oracle = env
    n1, n2 = shape
    x = inputs.normal(shape, 2500 + n2)
    xt = torch.from_numpy(x).cuda()
    print(f"[gpu] long columns {fn} {shape}", flush=True)
    old = os.environ.get("DCTX_SPLIT")
    try:
        os.environ["DCTX_SPLIT"] = "1"
        y = getattr(dx, fn)(xt)
        os.environ["DCTX_SPLIT"] = "0"
        y0 = getattr(dx, fn)(xt)
    finally:
        if old is None:
            del os.environ["DCTX_SPLIT"]
        else:
            os.environ["DCTX_SPLIT"] = old
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    assert oracle.rel_l2(yn, y0.cpu().numpy()) <= TOL
    ref_fn = oracle.dctn if fn == "dct2d" else oracle.idctn
    if n2 <= 2048:
        err = oracle.rel_l2(yn, ref_fn(x))
        assert err <= TOL, f"{fn} {shape}: whole-array rel L2 {err:.3e}"
        return
    # 8192^2 (beyond the benchmarked sizes; a whole-array oracle would take
    # minutes): whole output rows in every residue class mod 8 and at both ends
    # of each 1024-row block, and whole columns
    rows = sorted({0, 1, 2, 3, 4, 5, 6, 7, 8, 1023, 1024, 1025, 4095, 4096, 4097, 4100, 7168, 8184, 8188, 8191, 3001})
    cols = sorted({0, 1, n2 // 2 - 1, n2 // 2, n2 - 1, min(n2 - 1, 997)})
    err_r = oracle.rel_l2(yn[rows], ref_fn(x, sel={0: rows}))
    err_c = oracle.rel_l2(yn[:, cols], ref_fn(x, sel={1: cols}))
    assert err_r <= TOL and err_c <= TOL, f"{fn} {shape}: rows {err_r:.3e}, cols {err_c:.3e}"


@pytest.mark.parametrize("fn,ofn", [("idct_idxst2d", "idct_idxst2"), ("idxst_idct2d", "idxst_idct2")])
def test_long_column_route_mixed_and_ortho(env, fn, ofn):
    """The IDXST reversal in the 1024-point pre and the sign in the plain row
    stores, and the orthonormal scale, on the long-column route (whole array
    against the oracle at 8192 x 40)."""
    _, _, inputs, oracle = env
    x = inputs.uniform((8192, 40), 2600)
    y = _run(env, fn, x, "backward")
    err = oracle.rel_l2(y, getattr(oracle, ofn)(x))
    assert err <= TOL, f"{fn} 8192x40: rel L2 {err:.3e}"
    for f in ("dct2d", "idct2d"):
        y = _run(env, f, x, "ortho")
        err = oracle.rel_l2(y, getattr(oracle, FWD.get(f) or INV[f])(x, "ortho"))
        assert err <= TOL, f"{f} 8192x40 ortho: rel L2 {err:.3e}"


@pytest.mark.parametrize("fn,ofn,norm", [("idct_idxst2d", "idct_idxst2", "backward"),
                                         ("idxst_idct2d", "idxst_idct2", "backward"),
                                         ("dct2d", "dctn", "ortho"), ("idct2d", "idctn", "ortho"),
                                         ("idct_idxst2d", "idct_idxst2", "ortho")])
def test_long_column_route_wide_tiles(env, fn, ofn, norm):
    """8192 x 2048 (m >= 1024) runs the 16-column instantiations of the
    1024-point kernels: the mixed transforms (reversal in the pre, sign in the
    row stores) and the orthonormal scale there.  The whole array against the
    plain column kernels (DCTX_SPLIT=0) and whole output rows from every
    residue class mod 8 and both ends of each 1024-row block against the
    oracle."""
    import os
    torch, dx, inputs, oracle = env
    shape = (8192, 2048)
    x = inputs.uniform(shape, 2700)
    xt = torch.from_numpy(x).cuda()
    print(f"[gpu] long columns wide tiles {fn} {norm}", flush=True)
    old = os.environ.get("DCTX_SPLIT")
    try:
        os.environ["DCTX_SPLIT"] = "1"
        y = getattr(dx, fn)(xt, norm)
        os.environ["DCTX_SPLIT"] = "0"
        y0 = getattr(dx, fn)(xt, norm)
    finally:
        if old is None:
            del os.environ["DCTX_SPLIT"]
        else:
            os.environ["DCTX_SPLIT"] = old
    torch.cuda.synchronize()
    yn = y.cpu().numpy()
    assert np.isfinite(yn).all()
    assert oracle.rel_l2(yn, y0.cpu().numpy()) <= TOL
    rows = sorted({0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 1023, 1024, 1025, 4095, 4096, 4097, 7168, 8183, 8188, 8191})
    ref = getattr(oracle, ofn)(x, norm, sel={0: rows})
    err = oracle.rel_l2(yn[rows], ref)
    assert err <= TOL, f"{fn} {norm} 8192x2048 rows: rel L2 {err:.3e}"
