"""Every output word written exactly once: the write-count build of the
library (libdctx_wc.so, the same sources with -DDCTX_WRITE_COUNT) counts each
store of a transform's final output per 4-byte word.  NaN-poisoned outputs in
the parity tests show words never written; these counts also catch words
written twice.  Called through the C ABI of that library with ctypes; the
results are also checked against the FP64 oracle, so the counted build is the
same arithmetic as the product one."""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WC_LIB = os.path.join(ROOT, "paper_2110_01172_amd", "libdctx_wc.so")
TOL = 1e-6


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(WC_LIB):
        raise RuntimeError(f"{WC_LIB} is not built (python -m paper_2110_01172_amd.build --write-count)")
    import paper_2110_01172_amd as dx
    from paper_2110_01172_amd import inputs
    import oracle
    oracle.build(force=False)
    lib = ctypes.CDLL(WC_LIB)
    vp, ci = ctypes.c_void_p, ctypes.c_int
    sigs = {
        "dctx_create": [ci, ctypes.POINTER(vp)], "dctx_destroy": [vp],
        "dctx_debug_write_count": [vp, vp, vp, ctypes.c_size_t],
        "dctx_dct2d": [vp, vp, vp, ci, ci, ci, vp], "dctx_idct2d": [vp, vp, vp, ci, ci, ci, vp],
        "dctx_dct3d": [vp, vp, vp, ci, ci, ci, ci, vp], "dctx_idct3d": [vp, vp, vp, ci, ci, ci, ci, vp],
        "dctx_dct1d": [vp, vp, vp, ci, ci, ci, vp], "dctx_idct1d": [vp, vp, vp, ci, ci, ci, vp],
        "dctx_idct_idxst2d": [vp, vp, vp, ci, ci, ci, vp], "dctx_idxst_idct2d": [vp, vp, vp, ci, ci, ci, vp],
        "dctx_poisson2d": [vp, vp, vp, ci, ci, ctypes.c_double, ctypes.c_double, vp],
        "dctx_compress2d": [vp, vp, vp, ci, ci, ci, ctypes.c_double, vp],
        "dctx_submit_batch": [vp, ctypes.POINTER(dx.Desc), ci, vp, ctypes.POINTER(ci)],
    }
    for name, args in sigs.items():
        getattr(lib, name).restype = ci
        getattr(lib, name).argtypes = args
    h = vp()
    assert lib.dctx_create(0, ctypes.byref(h)) == 0
    yield torch, dx, inputs, oracle, lib, h
    lib.dctx_destroy(h)


def _counted(env, out, call):
    """Runs call() with out's words counted; returns the counts."""
    torch, _, _, _, lib, h = env
    cnt = torch.zeros(out.numel(), dtype=torch.int32, device=out.device)
    torch.cuda.synchronize()
    assert lib.dctx_debug_write_count(h, cnt.data_ptr(), out.data_ptr(), out.numel() * 4) == 0
    try:
        assert call() == 0
        torch.cuda.synchronize()
    finally:
        assert lib.dctx_debug_write_count(h, None, None, 0) == 0
    return cnt.cpu().numpy()


def _once(counts, what):
    bad = np.flatnonzero(counts != 1)
    assert bad.size == 0, (f"{what}: {bad.size} output words not written exactly once "
                           f"(first {bad[:5].tolist()}, counts {counts[bad[:5]].tolist()})")


# the fast (powers of two), split (tall power-of-two), generic (5-smooth),
# odd-last-axis and axis-order (n1 > 8192) 2-D routes
SHAPES_2D = [(512, 256), (2048, 2048), (4096, 4096), (250, 486), (9, 15), (64, 75), (10240, 9), (3, 2)]


@pytest.mark.parametrize("shape", SHAPES_2D)
@pytest.mark.parametrize("fn", ["dctx_dct2d", "dctx_idct2d"])
def test_2d_outputs_written_once(env, fn, shape):
    torch, dx, inputs, oracle, lib, h = env
    x_np = inputs.normal(shape, 8100 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] write count {fn} {shape}", flush=True)
    c = _counted(env, y, lambda: getattr(lib, fn)(h, x.data_ptr(), y.data_ptr(), shape[0], shape[1], 0, None))
    _once(c, f"{fn} {shape}")
    if x_np.size <= 1 << 20:
        ref = oracle.dctn(x_np) if fn == "dctx_dct2d" else oracle.idctn(x_np)
        assert oracle.rel_l2(y.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("shape", [(128, 128, 128), (64, 64, 64), (256, 64, 40), (16, 12, 45), (6, 10, 15),
                                   (64, 128, 100)])
@pytest.mark.parametrize("fn", ["dctx_dct3d", "dctx_idct3d"])
def test_3d_outputs_written_once(env, fn, shape):
    torch, dx, inputs, oracle, lib, h = env
    x_np = inputs.normal(shape, 8200 + sum(shape))
    x = torch.from_numpy(x_np).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] write count {fn} {shape}", flush=True)
    c = _counted(env, y, lambda: getattr(lib, fn)(h, x.data_ptr(), y.data_ptr(), *shape, 0, None))
    _once(c, f"{fn} {shape}")
    ref = oracle.dctn(x_np) if fn == "dctx_dct3d" else oracle.idctn(x_np)
    assert oracle.rel_l2(y.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("n,batch", [(4096, 8), (1000, 5), (32768, 2), (1 << 18, 1), (12, 3)])
@pytest.mark.parametrize("fn", ["dctx_dct1d", "dctx_idct1d"])
def test_1d_outputs_written_once(env, fn, n, batch):
    torch, dx, inputs, oracle, lib, h = env
    x = torch.from_numpy(inputs.normal((batch, n), 8300 + n)).cuda()
    y = torch.full_like(x, float("nan"))
    print(f"[gpu] write count {fn} n={n} batch={batch}", flush=True)
    c = _counted(env, y, lambda: getattr(lib, fn)(h, x.data_ptr(), y.data_ptr(), n, batch, 0, None))
    _once(c, f"{fn} n={n}")


@pytest.mark.parametrize("shape", [(1024, 1024), (2048, 1024), (250, 486), (30, 25)])
def test_spectral_and_idxst_outputs_written_once(env, shape):
    torch, dx, inputs, oracle, lib, h = env
    x = torch.from_numpy(inputs.normal(shape, 8400 + sum(shape))).cuda()
    n1, n2 = shape
    calls = {
        "poisson2d": lambda y: lib.dctx_poisson2d(h, x.data_ptr(), y.data_ptr(), n1, n2, 0.0, 0.0, None),
        "compress2d": lambda y: lib.dctx_compress2d(h, x.data_ptr(), y.data_ptr(), n1, n2, 0, 0.5, None),
        "idct_idxst2d": lambda y: lib.dctx_idct_idxst2d(h, x.data_ptr(), y.data_ptr(), n1, n2, 0, None),
        "idxst_idct2d": lambda y: lib.dctx_idxst_idct2d(h, x.data_ptr(), y.data_ptr(), n1, n2, 0, None),
    }
    for name, call in calls.items():
        y = torch.full_like(x, float("nan"))
        print(f"[gpu] write count {name} {shape}", flush=True)
        _once(_counted(env, y, lambda: call(y)), f"{name} {shape}")


def test_batch_outputs_written_once(env):
    """A mixed batch (persistent passes and grouped compile-time launches):
    the items' outputs sit in one buffer, counted together."""
    torch, dx, inputs, oracle, lib, h = env
    specs = [("dct2d", (512, 512)), ("idct2d", (96, 250)), ("poisson2d", (64, 64)), ("dct2d", (1024, 1024)),
             ("dct2d", (1024, 1024)), ("dct3d", (64, 64, 64)), ("idct2d", (45, 30)), ("dct2d", (100, 81))]
    sizes = [int(np.prod(s)) for _, s in specs]
    offs = np.concatenate([[0], np.cumsum([(n + 63) // 64 * 64 for n in sizes])])
    outbuf = torch.full((int(offs[-1]),), float("nan"), device="cuda")
    items, xs = [], []
    for i, (kind, shape) in enumerate(specs):
        x_np = inputs.uniform(shape, 8500 + i)
        xt = torch.from_numpy(x_np).cuda()
        out = outbuf[int(offs[i]):int(offs[i]) + sizes[i]].view(shape)
        items.append((kind, xt, out))
        xs.append(x_np)
    descs = dx.make_descs(items)
    st = (ctypes.c_int * len(items))()
    print("[gpu] write count batch", flush=True)
    c = _counted(env, outbuf, lambda: lib.dctx_submit_batch(h, descs, len(items), None, st))
    for i in range(len(items)):
        _once(c[int(offs[i]):int(offs[i]) + sizes[i]], f"batch item {i} {specs[i]}")
        assert (c[int(offs[i]) + sizes[i]:int(offs[i + 1])] == 0).all(), f"item {i} wrote past its output"
    for (kind, _, out), x_np in zip(items, xs):
        ref = {"dct2d": oracle.dctn, "idct2d": oracle.idctn, "dct3d": oracle.dctn,
               "poisson2d": oracle.poisson2d_neumann}[kind](x_np)
        assert oracle.rel_l2(out.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("n", [16, 32, 64, 128])
@pytest.mark.parametrize("prec", [0, 1])
def test_small_outputs_written_once(env, n, prec):
    """The small-N matrix path (both precisions, forward and inverse)."""
    torch, dx, inputs, oracle, lib, h = env
    lib.dctx_dct2d_small.restype = ctypes.c_int
    lib.dctx_dct2d_small.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5 + \
        [ctypes.c_void_p]
    batch = 37
    x = torch.from_numpy(inputs.normal((batch, n, n), 8600 + n)).cuda()
    for inverse in (0, 1):
        y = torch.full_like(x, float("nan"))
        print(f"[gpu] write count small n={n} prec={prec} inverse={inverse}", flush=True)
        c = _counted(env, y, lambda: lib.dctx_dct2d_small(h, x.data_ptr(), y.data_ptr(), n, batch, inverse, 0,
                                                            prec, None))
        _once(c, f"small n={n} prec={prec} inverse={inverse}")


@pytest.mark.parametrize("shape", [(64, 100), (9, 15), (256, 256)])
def test_row_column_outputs_written_once(env, shape):
    """The row-column baseline (its last transpose writes the output)."""
    torch, dx, inputs, oracle, lib, h = env
    for fn in ("dctx_rc_dct2d", "dctx_rc_idct2d"):
        getattr(lib, fn).restype = ctypes.c_int
        getattr(lib, fn).argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int] * 3 + [ctypes.c_void_p]
        x = torch.from_numpy(inputs.normal(shape, 8700 + sum(shape))).cuda()
        y = torch.full_like(x, float("nan"))
        print(f"[gpu] write count {fn} {shape}", flush=True)
        c = _counted(env, y, lambda: getattr(lib, fn)(h, x.data_ptr(), y.data_ptr(), shape[0], shape[1], 0, None))
        _once(c, f"{fn} {shape}")
