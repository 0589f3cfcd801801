"""dctx: multi-dimensional DCT-II / DCT-III (IDCT) on AMD MI355X (gfx950).

Thin Python binding over the C ABI in ``include/dctx.h`` (``libdctx.so``, built
by ``python -m paper_2110_01172_amd.build``).  This module only marshals
arguments: PyTorch provides device memory and the current HIP stream, and every
step of every transform runs in the library's HIP kernels.  If the library is
not built, importing works but every transform raises ``DctxError``; there is
no fallback implementation.

Transforms (all FP32, row-major, last dimension contiguous):

* ``dct2d`` / ``idct2d`` — the three-stage method (reorder, real FFT,
  twiddle / symmetric-pair postprocess; Alg. alg:DCT of the paper), two HBM
  passes each;
* ``rc_dct2d`` / ``rc_idct2d`` — the row-column baseline (1-D N-point DCTs
  along each axis with separate pre / FFT / post kernels and transposes).

``norm`` is ``"backward"`` (raw DCT-II sums; the inverse scales by
prod(2/N)) or ``"ortho"`` (orthonormal).
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = ["DctxError", "available", "library_path", "dct2d", "idct2d", "dct1d", "idct1d", "idct_idxst2d", "idxst_idct2d", "dct3d", "idct3d", "rc_dct2d", "rc_idct2d", "workspace_bytes_3d", "poisson2d", "compress2d", "submit_batch", "autotune_batch", "BatchGraph", "dct2d_small", "Server",
           "workspace_bytes_2d", "length_supported", "selfcheck", "Handle", "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdctx.so")

STATUS = {0: "OK", 1: "ERR_INVALID", 2: "ERR_UNSUPPORTED", 3: "ERR_NOMEM", 4: "ERR_DEVICE", 5: "ERR_BUSY",
          6: "ERR_TOO_LARGE", 7: "ERR_CANCELLED"}
_NORMS = {"backward": 0, "ortho": 1}

_lib = None
_lib_lock = threading.Lock()
_handles: dict = {}


class DctxError(RuntimeError):
    """A dctx call returned a non-OK status (or the library is missing)."""

    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


def library_path() -> str:
    return _LIB_PATH


class KernelStat(ctypes.Structure):
    """Mirror of dctx_kernel_stat."""
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


KINDS = {"dct2d": 0, "idct2d": 1, "dct3d": 2, "idct3d": 3, "poisson2d": 4}


class Desc(ctypes.Structure):
    """``dctx_desc`` of include/dctx.h."""
    _fields_ = [("kind", ctypes.c_int), ("ndim", ctypes.c_int), ("dims", ctypes.c_int * 3),
                ("inp", ctypes.c_void_p), ("out", ctypes.c_void_p), ("norm", ctypes.c_int),
                ("h", ctypes.c_double * 2)]


class TuneInfo(ctypes.Structure):
    """``dctx_tune_info`` of include/dctx.h."""
    _fields_ = [("block", ctypes.c_int * 5), ("grid_factor", ctypes.c_int * 5), ("per_cap", ctypes.c_int * 5),
                ("tiles", ctypes.c_int * 5), ("pass_ms", ctypes.c_double * 5), ("default_ms", ctypes.c_double),
                ("tuned_ms", ctypes.c_double)]


PASS_NAMES = ("dct_rows", "dct_cols", "idct_cols", "idct_rows", "poisson_cols")


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int),
                ("nstreams", ctypes.c_int), ("max_batch", ctypes.c_int), ("plain", ctypes.c_int),
                ("min_batch", ctypes.c_int), ("max_wait_us", ctypes.c_int)]


class ReqStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("arrival_s", ctypes.c_double), ("launch_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("latency_ms", ctypes.c_double), ("batch_size", ctypes.c_int)]


class ServerSummary(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("span_s", ctypes.c_double),
                ("req_per_s", ctypes.c_double), ("batches", ctypes.c_int64), ("mean_batch", ctypes.c_double),
                ("peak_pool_bytes", ctypes.c_size_t)]


def _declare(lib):
    c_int, c_void_p, c_size_t = ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    sigs = {
        "dctx_status_string": (ctypes.c_char_p, [c_int]),
        "dctx_version": (c_int, []),
        "dctx_selfcheck": (c_int, [ctypes.POINTER(ctypes.c_double)]),
        "dctx_length_supported": (c_int, [c_int, c_int]),
        "dctx_shape_supported": (c_int, [c_int, c_int, c_int, c_int]),
        "dctx_batch_geometry_check": (c_int, [c_int, c_int, ctypes.c_char_p, c_int]),
        "dctx_create": (c_int, [c_int, ctypes.POINTER(c_void_p)]),
        "dctx_destroy": (c_int, [c_void_p]),
        "dctx_workspace_bytes_2d": (c_int, [c_int, c_int, ctypes.POINTER(c_size_t)]),
        "dctx_workspace_bytes_3d": (c_int, [c_int, c_int, c_int, ctypes.POINTER(c_size_t)]),
        "dctx_dct2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_idct2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_dct1d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_idct1d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_idct_idxst2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_idxst_idct2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_dct2d_ws": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p,
                                  c_size_t, c_void_p]),
        "dctx_idct2d_ws": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p,
                                   c_size_t, c_void_p]),
        "dctx_dct2d_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p]),
        "dctx_dct3d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p]),
        "dctx_idct3d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p]),
        "dctx_poisson2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, ctypes.c_double,
                                   ctypes.c_double, c_void_p]),
        "dctx_compress2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, ctypes.c_double,
                                    c_void_p]),
        "dctx_dct2d_small": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p]),
        "dctx_submit_batch": (c_int, [c_void_p, ctypes.POINTER(Desc), c_int, c_void_p, ctypes.POINTER(c_int)]),
        "dctx_autotune_batch": (c_int, [c_void_p, ctypes.POINTER(Desc), c_int, c_void_p,
                                        ctypes.POINTER(TuneInfo)]),
        "dctx_tune_save": (c_int, [c_void_p, ctypes.c_char_p]),
        "dctx_tune_load": (c_int, [c_void_p, ctypes.c_char_p, ctypes.POINTER(c_int)]),
        "dctx_graph_create": (c_int, [c_void_p, ctypes.POINTER(Desc), c_int, ctypes.POINTER(c_void_p)]),
        "dctx_graph_launch": (c_int, [c_void_p, c_void_p]),
        "dctx_graph_destroy": (c_int, [c_void_p]),
        "dctx_server_create": (c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(c_void_p)]),
        "dctx_server_now": (c_int, [c_void_p, ctypes.POINTER(ctypes.c_double)]),
        "dctx_server_submit": (c_int, [c_void_p, ctypes.POINTER(Desc), ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_uint64)]),
        "dctx_server_poll": (c_int, [c_void_p, ctypes.c_uint64, ctypes.POINTER(ReqStats)]),
        "dctx_server_drain": (c_int, [c_void_p]),
        "dctx_server_summary_get": (c_int, [c_void_p, ctypes.c_uint64, ctypes.POINTER(ServerSummary)]),
        "dctx_server_cancel": (c_int, [c_void_p, ctypes.c_uint64]),
        "dctx_server_inject_alloc_failures": (c_int, [c_void_p, c_int]),
        "dctx_server_destroy": (c_int, [c_void_p]),
        "dctx_rc_dct2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_rc_idct2d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]),
        "dctx_profile_enable": (c_int, [c_void_p, c_int]),
        "dctx_profile_read": (c_int, [c_void_p, ctypes.POINTER(KernelStat), c_int,
                                      ctypes.POINTER(c_int)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def lib():
    """The loaded ``libdctx.so`` (raises DctxError if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise DctxError(f"{_LIB_PATH} is not built; run `python -m paper_2110_01172_amd.build`")
            _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def available() -> bool:
    return os.path.exists(_LIB_PATH)


def _check(status: int, what: str):
    if status != 0:
        text = lib().dctx_status_string(status).decode()
        raise DctxError(f"{what} failed: {STATUS.get(status, status)} ({text})", status)


def selfcheck() -> float:
    err = ctypes.c_double(0.0)
    _check(lib().dctx_selfcheck(ctypes.byref(err)), "dctx_selfcheck")
    return err.value


def length_supported(n: int, last_axis: bool) -> bool:
    return bool(lib().dctx_length_supported(int(n), 1 if last_axis else 0))


def shape_supported(kind: str, shape) -> bool:
    """Whether the plain call of ``kind`` (a KINDS name) accepts ``shape``."""
    dims = [int(v) for v in shape] + [0] * (3 - len(shape))
    return bool(lib().dctx_shape_supported(KINDS[kind], dims[0], dims[1], dims[2]))


def workspace_bytes_2d(n1: int, n2: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().dctx_workspace_bytes_2d(int(n1), int(n2), ctypes.byref(out)), "dctx_workspace_bytes_2d")
    return out.value


class Handle:
    """Owns one ``dctx_handle`` (plan cache + workspace) on one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p(0)
        _check(lib().dctx_create(int(device), ctypes.byref(h)), "dctx_create")
        self._h = h
        self.device = int(device)

    @property
    def ptr(self):
        return self._h

    def profile(self, enable: bool = True):
        """Turn per-kernel event timing on or off for this handle."""
        _check(lib().dctx_profile_enable(self._h, 1 if enable else 0), "dctx_profile_enable")

    def profile_read(self) -> dict:
        """Synchronise, return {kernel: {launches, total_ms, min_ms, max_ms}}, clear."""
        cap = 64
        arr = (KernelStat * cap)()
        n = ctypes.c_int(0)
        _check(lib().dctx_profile_read(self._h, arr, cap, ctypes.byref(n)), "dctx_profile_read")
        return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                       "min_ms": arr[i].min_ms, "max_ms": arr[i].max_ms}
                for i in range(min(n.value, cap))}

    def close(self):
        if self._h and self._h.value:
            lib().dctx_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_handle(device: int) -> Handle:
    h = _handles.get(device)
    if h is None:
        h = Handle(device)
        _handles[device] = h
    return h


def _torch():
    import torch
    return torch


def _prep(x, ndim: int, out):
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not x.is_cuda:
        raise DctxError("dctx transforms need a tensor on a HIP device (no CPU path exists)")
    if x.dtype != torch.float32:
        raise TypeError("dctx transforms take float32 tensors")
    if x.dim() != ndim:
        raise ValueError(f"expected a {ndim}-D tensor, got shape {tuple(x.shape)}")
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    else:
        if out.shape != x.shape or out.dtype != torch.float32 or not out.is_contiguous() \
                or out.device != x.device:
            raise ValueError("out must be a contiguous float32 tensor of the input's shape and device")
    stream = torch.cuda.current_stream(x.device).cuda_stream
    return x, out, stream


def _call2d(name: str, x, norm: str, out, handle):
    if norm not in _NORMS:
        raise ValueError(f"norm must be one of {tuple(_NORMS)}")
    x, out, stream = _prep(x, 2, out)
    h = handle or default_handle(x.device.index or 0)
    n1, n2 = x.shape
    st = getattr(lib(), name)(h.ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              int(n1), int(n2), _NORMS[norm], ctypes.c_void_p(stream))
    _check(st, f"{name}({n1}x{n2})")
    return out


def dct2d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """2-D DCT-II of an n1 x n2 float32 CUDA tensor (three-stage method)."""
    return _call2d("dctx_dct2d", x, norm, out, handle)


def idct2d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """2-D DCT-III, the inverse of :func:`dct2d` under the same norm."""
    return _call2d("dctx_idct2d", x, norm, out, handle)


def dct2d_noalloc(x, out, norm: str = "backward", inverse: bool = False, handle: Handle | None = None):
    """:func:`dct2d` (or :func:`idct2d` with ``inverse``) through the
    allocation-free entry point: ``out`` must be given (nothing is allocated,
    by torch or the library); the workspace and tables sit in the library's
    static device scratch (shapes whose workspace exceeds 64 MiB raise)."""
    if norm not in _NORMS:
        raise ValueError(f"norm must be one of {tuple(_NORMS)}")
    if out is None:
        raise ValueError("dct2d_noalloc needs `out` (it allocates nothing)")
    if not x.is_contiguous():
        raise ValueError("dct2d_noalloc needs a contiguous input (a copy would allocate)")
    x, out, stream = _prep(x, 2, out)
    h = handle or default_handle(x.device.index or 0)
    n1, n2 = x.shape
    st = lib().dctx_dct2d_noalloc(h.ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  int(n1), int(n2), _NORMS[norm], 1 if inverse else 0, ctypes.c_void_p(stream))
    _check(st, f"dctx_dct2d_noalloc({n1}x{n2}, inverse={bool(inverse)})")
    return out


def _call1d(name: str, x, norm: str, out, handle):
    """A 1-D tensor is one row; a 2-D tensor is a batch of rows."""
    if norm not in _NORMS:
        raise ValueError(f"norm must be one of {tuple(_NORMS)}")
    single = getattr(x, "dim", lambda: 0)() == 1
    if single:
        x = x.unsqueeze(0)
        out = None if out is None else out.unsqueeze(0)
    x, out, stream = _prep(x, 2, out)
    h = handle or default_handle(x.device.index or 0)
    batch, n = x.shape
    st = getattr(lib(), name)(h.ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              int(n), int(batch), _NORMS[norm], ctypes.c_void_p(stream))
    _check(st, f"{name}({batch}x{n})")
    return out[0] if single else out


def dct1d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """1-D DCT-II of a length-n float32 CUDA tensor, or of every row of a
    batch x n one (n even, 2^a 3^b 5^c, at most 2^20)."""
    return _call1d("dctx_dct1d", x, norm, out, handle)


def idct1d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """1-D DCT-III of every row, the inverse of :func:`dct1d` under the same norm."""
    return _call1d("dctx_idct1d", x, norm, out, handle)


def idct_idxst2d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """IDCT_IDXST of an n1 x n2 float32 CUDA tensor (Eq. idxst): IDXST along
    the first axis (n1), IDCT along the last (n2, even)."""
    return _call2d("dctx_idct_idxst2d", x, norm, out, handle)


def idxst_idct2d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """IDXST_IDCT of an n1 x n2 float32 CUDA tensor (Eq. idxst): IDCT along
    the first axis (n1), IDXST along the last (n2, even)."""
    return _call2d("dctx_idxst_idct2d", x, norm, out, handle)


def rc_dct2d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """Row-column baseline 2-D DCT-II (8 memory stages)."""
    return _call2d("dctx_rc_dct2d", x, norm, out, handle)


def rc_idct2d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """Row-column baseline 2-D DCT-III."""
    return _call2d("dctx_rc_idct2d", x, norm, out, handle)


def _call3d(name: str, x, norm: str, out, handle):
    if norm not in _NORMS:
        raise ValueError(f"norm must be one of {tuple(_NORMS)}")
    x, out, stream = _prep(x, 3, out)
    h = handle or default_handle(x.device.index or 0)
    n1, n2, n3 = x.shape
    st = getattr(lib(), name)(h.ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              int(n1), int(n2), int(n3), _NORMS[norm], ctypes.c_void_p(stream))
    _check(st, f"{name}({n1}x{n2}x{n3})")
    return out


def dct3d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """3-D DCT-II of an n1 x n2 x n3 float32 CUDA tensor (three-stage method)."""
    return _call3d("dctx_dct3d", x, norm, out, handle)


def idct3d(x, norm: str = "backward", out=None, handle: Handle | None = None):
    """3-D DCT-III, the inverse of :func:`dct3d` under the same norm."""
    return _call3d("dctx_idct3d", x, norm, out, handle)


def workspace_bytes_3d(n1: int, n2: int, n3: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().dctx_workspace_bytes_3d(int(n1), int(n2), int(n3), ctypes.byref(out)), "workspace_bytes_3d")
    return int(out.value)


def poisson2d(f, h1: float = 0.0, h2: float = 0.0, out=None, handle: Handle | None = None):
    """Neumann Poisson solve Lap(u) = f - mean(f), mean(u) = 0, on an n1 x n2
    cell-centred grid (spacings h1, h2; 0 selects 1/n1, 1/n2)."""
    f, out, stream = _prep(f, 2, out)
    h = handle or default_handle(f.device.index or 0)
    n1, n2 = f.shape
    st = lib().dctx_poisson2d(h.ptr, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              int(n1), int(n2), float(h1), float(h2), ctypes.c_void_p(stream))
    _check(st, f"dctx_poisson2d({n1}x{n2})")
    return out


def compress2d(x, eps: float, norm: str = "ortho", out=None, handle: Handle | None = None):
    """Threshold compression of an n1 x n2 float32 CUDA tensor (n2 even):
    idct(f_eps(dct(x))) under ``norm``, where f_eps zeroes the coefficients
    with |B| < eps.  The default orthonormal norm puts the threshold on
    energy-preserving coefficients."""
    if norm not in _NORMS:
        raise ValueError(f"norm must be one of {tuple(_NORMS)}")
    x, out, stream = _prep(x, 2, out)
    h = handle or default_handle(x.device.index or 0)
    n1, n2 = x.shape
    st = lib().dctx_compress2d(h.ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               int(n1), int(n2), _NORMS[norm], float(eps), ctypes.c_void_p(stream))
    _check(st, f"dctx_compress2d({n1}x{n2})")
    return out


def make_descs(items):
    """ctypes array of ``dctx_desc`` from (kind, x, out[, norm[, (h1, h2)]]) tuples;
    kind is one of KINDS' names; x and out are float32 device tensors."""
    arr = (Desc * len(items))()
    for i, it in enumerate(items):
        kind, x, out = it[0], it[1], it[2]
        norm = it[3] if len(it) > 3 and it[3] is not None else "backward"
        hh = it[4] if len(it) > 4 and it[4] is not None else (0.0, 0.0)
        if kind not in KINDS:
            raise ValueError(f"unknown kind {kind!r}")
        if norm not in _NORMS:
            raise ValueError(f"norm must be one of {tuple(_NORMS)}")
        for t in (x, out):
            if not t.is_cuda or t.dtype != _torch().float32 or not t.is_contiguous():
                raise DctxError("batch items take contiguous float32 tensors on a HIP device")
        if tuple(x.shape) != tuple(out.shape):
            raise ValueError("input and output shapes differ")
        d = arr[i]
        d.kind = KINDS[kind]
        d.ndim = x.dim()
        for j in range(min(3, x.dim())):
            d.dims[j] = int(x.shape[j])
        d.inp = x.data_ptr()
        d.out = out.data_ptr()
        d.norm = _NORMS[norm]
        d.h[0], d.h[1] = float(hh[0]), float(hh[1])
    return arr


class Batch:
    """A batch's descriptor array, built once (see make_descs) and submitted
    any number of times; it keeps the item tensors alive."""

    def __init__(self, items):
        self.items = list(items)
        self.descs = make_descs(self.items)
        self.device = self.items[0][1].device if self.items else _torch().device("cuda", 0)
        self._per = (ctypes.c_int * max(1, len(self.items)))()

    def submit(self, handle: Handle | None = None, stream=None):
        h = handle or default_handle(self.device.index or 0)
        s = stream if stream is not None else _torch().cuda.current_stream(self.device).cuda_stream
        n = len(self.items)
        st = lib().dctx_submit_batch(h.ptr, self.descs, n, ctypes.c_void_p(s), self._per)
        if st != 0:
            raise DctxError(f"dctx_submit_batch: {STATUS.get(st, st)}; per item: "
                            f"{[STATUS.get(self._per[i], self._per[i]) for i in range(n)]}", st)


def submit_batch(items, handle: Handle | None = None, stream=None):
    """Enqueue a batch (a list of items, see make_descs, or a Batch) on the
    current stream; returns nothing, raises DctxError (with the per-item
    statuses) if any item is rejected."""
    b = items if isinstance(items, Batch) else Batch(items)
    b.submit(handle, stream)


def autotune_batch(items, handle: Handle | None = None) -> dict:
    """Run the autotuner on a batch (writes the outputs); returns the chosen
    launch geometry and the measured pass times."""
    torch = _torch()
    descs = make_descs(items)
    dev = items[0][1].device
    h = handle or default_handle(dev.index or 0)
    info = TuneInfo()
    st = lib().dctx_autotune_batch(h.ptr, descs, len(items),
                                   ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream), ctypes.byref(info))
    _check(st, "dctx_autotune_batch")
    out = {"default_ms": info.default_ms, "tuned_ms": info.tuned_ms, "passes": {}}
    for k, name in enumerate(PASS_NAMES):
        if info.tiles[k]:
            out["passes"][name] = {"block": info.block[k], "grid_factor": info.grid_factor[k],
                                   "per_cap": info.per_cap[k], "tiles": info.tiles[k], "ms": info.pass_ms[k]}
    return out


def tune_save(path: str, handle: Handle | None = None, device: int = 0):
    """Write the handle's batch tuning cache to a JSON file (keyed by gfx
    architecture and batch signature; other architectures' entries kept)."""
    h = handle or default_handle(device)
    _check(lib().dctx_tune_save(h.ptr, os.fsencode(path)), "dctx_tune_save")


def tune_load(path: str, handle: Handle | None = None, device: int = 0) -> int:
    """Add the file's entries for this device's architecture to the handle's
    tuning cache; returns how many."""
    h = handle or default_handle(device)
    n = ctypes.c_int(0)
    _check(lib().dctx_tune_load(h.ptr, os.fsencode(path), ctypes.byref(n)), "dctx_tune_load")
    return n.value


class BatchGraph:
    """A batch captured into a HIP graph; launch() replays it on a stream."""

    def __init__(self, items, handle: Handle | None = None):
        descs = make_descs(items)
        dev = items[0][1].device
        self._handle = handle or default_handle(dev.index or 0)
        self._items = items   # keep the tensors alive as long as the graph
        g = ctypes.c_void_p()
        _check(lib().dctx_graph_create(self._handle.ptr, descs, len(items), ctypes.byref(g)), "dctx_graph_create")
        self._g = g

    def launch(self, stream=None):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _check(lib().dctx_graph_launch(self._g, ctypes.c_void_p(s)), "dctx_graph_launch")

    def close(self):
        if getattr(self, "_g", None) and self._g.value:
            lib().dctx_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PRECS = {"bf16x3": 0, "fp16": 1}


def dct2d_small(x, prec: str = "bf16x3", inverse: bool = False, norm: str = "backward", out=None,
                handle: Handle | None = None):
    """Batched small-N 2-D DCT-II (or DCT-III) of a (batch, n, n) float32 tensor,
    n in {16, 32, 64, 128}, as C X C^T on the matrix cores in the chosen
    precision ("bf16x3" or "fp16", the scaled FP16 form)."""
    if prec not in PRECS:
        raise ValueError(f"prec must be one of {tuple(PRECS)}")
    if norm not in _NORMS:
        raise ValueError(f"norm must be one of {tuple(_NORMS)}")
    x, out, stream = _prep(x, 3, out)
    b, n1, n2 = x.shape
    if n1 != n2:
        raise ValueError("matrices must be square")
    h = handle or default_handle(x.device.index or 0)
    st = lib().dctx_dct2d_small(h.ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), int(n1),
                                int(b), int(bool(inverse)), _NORMS[norm], PRECS[prec], ctypes.c_void_p(stream))
    _check(st, f"dctx_dct2d_small({b}x{n1}x{n1}, {prec})")
    return out


class Server:
    """Continuous-batching serving loop (see dctx_server_* in include/dctx.h).

    submit() takes one request (kind, x, out[, norm[, (h1, h2)]]) with an
    optional arrival time on the server clock; the tensors must stay alive
    until the request is done (the server keeps a reference until then)."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_inflight: int = 256, nstreams: int = 4,
                 max_batch: int = 0, plain: bool = False, min_batch: int = 0, max_wait_us: int = 0):
        cfg = ServerConfig(int(device), int(hbm_budget), int(max_inflight), int(nstreams), int(max_batch),
                           int(bool(plain)), int(min_batch), int(max_wait_us))
        srv = ctypes.c_void_p()
        _check(lib().dctx_server_create(ctypes.byref(cfg), ctypes.byref(srv)), "dctx_server_create")
        self._s = srv
        self._keep = {}

    def now(self) -> float:
        t = ctypes.c_double()
        _check(lib().dctx_server_now(self._s, ctypes.byref(t)), "dctx_server_now")
        return t.value

    def submit(self, item, arrival: float = -1.0) -> int:
        d = make_descs([item])
        tk = ctypes.c_uint64()
        _check(lib().dctx_server_submit(self._s, d, float(arrival), ctypes.byref(tk)), "dctx_server_submit")
        self._keep[tk.value] = item
        return tk.value

    def poll(self, ticket: int):
        """None while busy, else a dict of the request's statistics."""
        st = ReqStats()
        r = lib().dctx_server_poll(self._s, ctypes.c_uint64(ticket), ctypes.byref(st))
        if r == 5:
            return None
        _check(r, "dctx_server_poll")
        self._keep.pop(ticket, None)
        return {"status": STATUS.get(st.status, st.status), "arrival_s": st.arrival_s, "launch_s": st.launch_s,
                "done_s": st.done_s, "latency_ms": st.latency_ms, "batch_size": st.batch_size}

    def cancel(self, ticket: int) -> bool:
        """True if the request was cancelled (it had not been launched);
        False if it is already on the GPU or done."""
        r = lib().dctx_server_cancel(self._s, ctypes.c_uint64(ticket))
        if r == 5:
            return False
        _check(r, "dctx_server_cancel")
        return True

    def inject_alloc_failures(self, count: int):
        """The next `count` batches fail as an allocation failure would (test aid)."""
        _check(lib().dctx_server_inject_alloc_failures(self._s, int(count)), "dctx_server_inject_alloc_failures")

    def drain(self):
        _check(lib().dctx_server_drain(self._s), "dctx_server_drain")
        self._keep.clear()

    def summary(self, first_ticket: int = 0) -> dict:
        sm = ServerSummary()
        _check(lib().dctx_server_summary_get(self._s, ctypes.c_uint64(first_ticket), ctypes.byref(sm)),
               "dctx_server_summary_get")
        return {f: getattr(sm, f) for f, _ in ServerSummary._fields_}

    def close(self):
        if getattr(self, "_s", None) and self._s.value:
            lib().dctx_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
