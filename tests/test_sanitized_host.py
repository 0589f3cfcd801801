"""The library's host code and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no GPU call succeeds here).

`python -m paper_2110_01172_amd.build --sanitize` builds libdctx_san.so with
ASan + UBSan on every host pass (the device code as usual); the oracle's C is
built the same way.  A child process with the sanitizer runtime preloaded then
drives every host-only path: the shape and length queries over thousands of
shapes, the batched passes' tile-geometry check over all uneven-batch shapes,
the self-check, status strings, workspace sizes, the argument checks of every
entry point (null handle, null pointers, bad enums), handle creation without
a device, and the oracle's transforms, Poisson solve and compression on small
arrays.  Any sanitizer report aborts the child with a non-zero status."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2110_01172_amd")
CLANG = "/opt/rocm/lib/llvm/bin/clang"


def _rt(name):
    out = subprocess.run([CLANG, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def _stale(lib, srcs):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(s) > t for s in srcs)


@pytest.fixture(scope="module")
def san_libs():
    if not os.path.exists(CLANG):
        pytest.skip("no clang")
    asan = _rt("libclang_rt.asan-x86_64.so")
    if asan is None:
        pytest.skip("no ASan runtime")
    sys.path.insert(0, ROOT)
    from paper_2110_01172_amd import build
    csrc = [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)]
    if _stale(build.SAN_LIB, csrc + [os.path.join(ROOT, "include", "dctx.h")]):
        build.build_sanitized()
    osrc = os.path.join(ROOT, "oracle", "dct_oracle.c")
    olib = os.path.join(ROOT, "oracle", "liboracle_san.so")
    if _stale(olib, [osrc]):
        subprocess.run([CLANG, "-O1", "-g", "-fPIC", "-shared", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-Wno-source-uses-openmp",
                        "-o", olib, osrc, "-lm"], check=True)
    return build.SAN_LIB, olib, asan


CHILD = textwrap.dedent(r'''
    import ctypes, sys
    sys.path.insert(0, ROOT)
    import numpy as np
    lib = ctypes.CDLL(SAN_LIB)
    c_int, c_void_p, c_size_t = ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    lib.dctx_shape_supported.argtypes = [c_int, c_int, c_int, c_int]
    lib.dctx_batch_geometry_check.argtypes = [c_int, c_int, ctypes.c_char_p, c_int]
    lib.dctx_length_supported.argtypes = [c_int, c_int]
    lib.dctx_status_string.restype = ctypes.c_char_p
    # shape queries: every kind over 2-D and 3-D shapes (supported and not)
    sizes = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 14, 15, 16, 30, 64, 77, 100, 128, 250, 256, 486, 1000, 1024, 4096,
             6561, 7680, 8192, 9000, 10000, 16384, 16385, 32768]
    n = 0
    for kind in range(5):
        for a in sizes:
            for b in sizes:
                n += lib.dctx_shape_supported(kind, a, b, 0)
        for a in (2, 4, 8, 64, 128, 256, 4096):
            for b in (2, 5, 64, 256, 8192):
                for c in (2, 3, 6, 64, 135, 16384):
                    n += lib.dctx_shape_supported(kind, a, b, c)
    for kind in (-5, 7, 99):   # not a dctx_kind
        assert lib.dctx_shape_supported(kind, 8, 8, 8) == 0
    for m in range(0, 20000):
        n += lib.dctx_length_supported(m, m & 1)
    msg = ctypes.create_string_buffer(256)
    from paper_2110_01172_amd import inputs
    for a in inputs.five_smooth_even(64, 1024):
        for b in inputs.five_smooth_even(64, 1024):
            assert lib.dctx_batch_geometry_check(a, b, msg, 256) == 1, msg.value
    assert lib.dctx_batch_geometry_check(77, 64, msg, 256) == 0
    assert lib.dctx_batch_geometry_check(77, 64, None, 0) == 0
    err = ctypes.c_double(0.0)
    assert lib.dctx_selfcheck(ctypes.byref(err)) == 0
    for s in range(-2, 9):
        assert lib.dctx_status_string(s)
    out = c_size_t(0)
    for a, b in ((4096, 4096), (10000, 100), (6, 10), (0, 4), (2, 3)):
        lib.dctx_workspace_bytes_2d(a, b, ctypes.byref(out))
    lib.dctx_workspace_bytes_3d(128, 128, 128, ctypes.byref(out))
    # argument checks of the entry points: null handle / pointers
    z = c_void_p(0)
    for name in ("dctx_dct2d", "dctx_idct2d", "dctx_rc_dct2d", "dctx_rc_idct2d", "dctx_idct_idxst2d",
                 "dctx_idxst_idct2d", "dctx_dct1d", "dctx_idct1d"):
        assert getattr(lib, name)(z, z, z, 8, 8, 0, z) == 1, name
    assert lib.dctx_dct3d(z, z, z, 8, 8, 8, 0, z) == 1
    assert lib.dctx_idct3d(z, z, z, 8, 8, 8, 0, z) == 1
    assert lib.dctx_submit_batch(z, z, 1, z, z) == 1
    assert lib.dctx_destroy(z) == 1
    h = c_void_p(0)
    rc = lib.dctx_create(0, ctypes.byref(h))
    assert rc in (0, 4), rc
    if rc == 0:
        lib.dctx_destroy(h)
    # the oracle
    import oracle
    prev = oracle._swap_library(ORACLE_SAN)
    x = inputs.uniform((6, 10), 1)
    y = oracle.dctn(x); zz = oracle.idctn(y)
    assert np.allclose(zz, x, atol=1e-12)
    x3 = inputs.uniform((3, 5, 4), 2)
    assert np.allclose(oracle.idctn(oracle.dctn(x3, "ortho"), "ortho"), x3, atol=1e-12)
    oracle.dctn(inputs.uniform((1, 257), 3), axes=[1], sel={1: [0, 5, 256]})
    oracle.poisson2d_neumann(inputs.uniform((12, 20), 4))
    oracle.compress2d(inputs.uniform((16, 12), 5), 0.5)
    oracle._restore_library(prev)
    print("SANITIZED-OK", n)
''')


def test_host_code_and_oracle_under_asan_ubsan(san_libs):
    san_lib, olib, asan = san_libs
    code = f"ROOT = {ROOT!r}\nSAN_LIB = {san_lib!r}\nORACLE_SAN = {olib!r}\n" + CHILD
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0 and "SANITIZED-OK" in res.stdout, tail
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, tail
