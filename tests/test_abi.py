"""The C-ABI library loads and exports every symbol its public headers declare
(CPU only: no call here touches a GPU except dctx_create's device count)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dx():
    import paper_2110_01172_amd as dx
    if not dx.available():
        from paper_2110_01172_amd import build
        build.build()
    return dx


def _declared_symbols():
    names = set()
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(dctx_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_entry_points():
    names = _declared_symbols()
    for required in ["dctx_create", "dctx_destroy", "dctx_dct2d", "dctx_idct2d",
                     "dctx_rc_dct2d", "dctx_rc_idct2d", "dctx_status_string"]:
        assert required in names


def test_library_exports_every_declared_symbol(dx):
    lib = ctypes.CDLL(dx.library_path())
    missing = [n for n in _declared_symbols() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_status_strings_and_version(dx):
    lib = dx.lib()
    for code in range(6):
        assert lib.dctx_status_string(code)
    assert lib.dctx_status_string(99) == b"unknown status"
    assert lib.dctx_version() >= 1


def test_butterfly_constants_match_fp64(dx):
    assert dx.selfcheck() < 3e-8


@pytest.mark.parametrize("n,last,ok", [
    (4, True, True), (2, True, True), (6, True, True), (7, True, False), (486, True, True),
    (1000, True, True), (14, True, False), (2, False, True), (3, False, True), (1, False, False),
    (125, False, True), (16384, False, True), (32768, False, False), (0, False, False), (-4, True, False),
    (3, True, True), (6561, True, True), (9375, True, False), (16384, True, True), (10000, False, True),
])
def test_length_supported(dx, n, last, ok):
    """dctx_length_supported is dctx_dct2d's rule along one axis: 5-smooth,
    >= 2, up to 16384; an odd contiguous length only while one workgroup runs
    its full-length row FFT (6561 = 3^8 yes, 9375 = 3 5^5 no)."""
    assert dx.length_supported(n, last) is ok


# (kind, shape, accepted by the plain call): the limits stated per entry point
SHAPES = [
    ("dct2d", (2, 2), True), ("dct2d", (3, 3), True), ("idct2d", (8192, 16384), True),
    ("dct2d", (16384, 6), True), ("dct2d", (16384, 9000), False), ("dct2d", (1, 8), False),
    ("dct2d", (8, 7), False), ("dct2d", (2, 9375), False), ("poisson2d", (64, 75), True),
    ("poisson2d", (16384, 6), False), ("poisson2d", (8192, 8192), True), ("poisson2d", (6, 2), True),
    ("dct3d", (4, 4, 5), True), ("dct3d", (4, 4, 2), True), ("idct3d", (4096, 2, 4), True),
    ("dct3d", (8192, 2, 4), False), ("dct3d", (2, 8192, 4), True), ("dct3d", (2, 16384, 4), False),
    ("dct3d", (4, 4, 9375), False), ("idct3d", (128, 128, 135), True), ("dct3d", (1, 4, 8), False),
]


@pytest.mark.parametrize("kind,shape,ok", SHAPES)
def test_shape_supported(dx, kind, shape, ok):
    assert dx.shape_supported(kind, shape) is ok


def test_workspace_bytes(dx):
    assert dx.workspace_bytes_2d(4096, 4096) == 4096 * 2048 * 8
    assert dx.workspace_bytes_2d(6, 10) == 6 * 5 * 8
    # the axis-order route (n1 > 8192): the spectrum of the n2 x n1 transpose, no transposed copies
    assert dx.workspace_bytes_2d(10000, 100) == 100 * 5000 * 8
    out = ctypes.c_size_t(0)
    assert dx.lib().dctx_workspace_bytes_2d(0, 4, ctypes.byref(out)) == 1
    assert dx.lib().dctx_workspace_bytes_2d(4, 4, None) == 1


def test_null_handle_and_pointers_are_invalid(dx):
    lib = dx.lib()
    assert lib.dctx_dct2d(None, None, None, 8, 8, 0, None) == 1
    assert lib.dctx_idct2d(None, None, None, 8, 8, 0, None) == 1
    assert lib.dctx_rc_dct2d(None, None, None, 8, 8, 0, None) == 1
    assert lib.dctx_idct_idxst2d(None, None, None, 8, 8, 0, None) == 1
    assert lib.dctx_idxst_idct2d(None, None, None, 8, 8, 0, None) == 1
    assert lib.dctx_compress2d(None, None, None, 8, 8, 0, ctypes.c_double(0.5), None) == 1
    assert lib.dctx_dct1d(None, None, None, 8, 1, 0, None) == 1
    assert lib.dctx_idct1d(None, None, None, 8, 1, 0, None) == 1
    assert lib.dctx_destroy(None) == 1
    assert lib.dctx_create(0, None) == 1
    assert lib.dctx_server_cancel(None, 0) == 1
    assert lib.dctx_server_inject_alloc_failures(None, 1) == 1
    assert lib.dctx_status_string(7) == b"request cancelled"
    assert lib.dctx_debug_write_count(None, None, None, 0) == 1


def test_create_without_gpu_reports_device_error(dx):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p(0)
    assert dx.lib().dctx_create(0, ctypes.byref(h)) in (1, 4)
    assert not h.value


def test_transforms_refuse_cpu_tensors(dx):
    torch = pytest.importorskip("torch")
    with pytest.raises(dx.DctxError):
        dx.dct2d(torch.zeros(8, 8))


def test_batch_tile_geometry_all_uneven_shapes(dx):
    """Every n1 x n2 of the uneven batch (both sides over the 50 even 5-smooth
    sizes in [64, 1024]), plus odd and small shapes: for every block size the
    autotuner tries and every batched pass, the LDS the tile bodies touch fits
    the bytes the launch passes and the device's LDS, and the tiles have their
    threads (host-side check; no GPU)."""
    from paper_2110_01172_amd import inputs
    sizes = inputs.five_smooth_even(64, 1024)
    shapes = [(a, b) for a in sizes for b in sizes] + [(2, 3), (3, 2), (5, 125), (1000, 375), (48, 90)]
    msg = ctypes.create_string_buffer(256)
    bad = []
    for n1, n2 in shapes:
        if not dx.lib().dctx_batch_geometry_check(n1, n2, msg, 256):
            bad.append(msg.value.decode())
    assert not bad, bad[:5]


def test_batch_tile_geometry_reports_unplannable(dx):
    msg = ctypes.create_string_buffer(256)
    assert dx.lib().dctx_batch_geometry_check(7 * 11, 64, msg, 256) == 0
    assert b"no plan" in msg.value


def test_write_count_library_loads_and_exports():
    """The write-count variant (libdctx_wc.so, a test aid built by build()) is
    loadable without a GPU and exports every entry point the header declares."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2110_01172_amd",
                        "libdctx_wc.so")
    if not os.path.exists(path):
        pytest.skip("libdctx_wc.so not built")
    wc = ctypes.CDLL(path)
    missing = [n for n in _declared_symbols() if not hasattr(wc, n)]
    assert not missing, missing
    wc.dctx_debug_write_count.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    assert wc.dctx_debug_write_count(None, None, None, 0) == 1
