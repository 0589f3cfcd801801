"""FP64 CPU oracle for the multi-dimensional DCT-II / DCT-III.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only ``tests/``, the smoke
check in ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product (``paper_2110_01172_amd``) never
imports, links or calls anything here, and nothing here imports the product.

What is computed, with the passage of the paper each part follows:

* raw DCT-II / DCT-III along one axis: Eq. (1d-definition) a and b, in
  ``dct_oracle.c`` (FP64 sums, exact integer argument reduction of the cosine);
* multi-dimensional transforms: the composition of the 1-D transform along every
  axis (Eq. 2d-dct-definition; 3-D by the same composition, Fig. 3d-dct);
* normalisations (the paper states none; see the readings in the design notes):
  ``backward``: dct = raw DCT-II per axis, idct = prod_d(2/N_d) * raw DCT-III,
  so idct(dct(x)) = x;  ``ortho``: the orthonormal DCT-II matrix and its
  transpose, so Parseval holds;
* the spectral Neumann Poisson solve (the spectral method of the DREAMPlace case
  study, Alg. electirc-dreamplace): DCT-II, divide by the eigenvalues of the
  cell-centred 5-point Neumann Laplacian, zero the DC term, backward DCT-III.
* the threshold compression of the image-compression case study (Alg.
  image-compression, Eq. image-compression): B = dctn(x), zero the
  coefficients with |B| < eps, idctn;
* the IDXST and the mixed 2-D transforms IDCT_IDXST / IDXST_IDCT of the same
  case study (Eq. idxst): the IDCT of the sequence reversed with a zero in
  front, times (-1)^k; a 1-D transform of a matrix acts on its columns (as in
  MATLAB), so IDCT(IDXST(x)^T)^T is IDXST along axis 0 and IDCT along axis 1,
  which is also how the paper describes it in words.

Every function takes and returns numpy arrays; inputs are promoted to FP64
exactly (an FP32 array is widened without rounding).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dct_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

NORMS = ("backward", "ortho")


def build(force: bool = True) -> str:
    """Compile ``dct_oracle.c`` into ``liboracle.so`` with gcc + OpenMP."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            lib = ctypes.CDLL(_LIB_PATH)
            lib.oracle_dct_axis_sel.restype = ctypes.c_int
            lib.oracle_dct_axis_sel.argtypes = [
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _swap_library(path):
    """Load the oracle from another shared object (used only by the mutation
    test, which builds deliberately broken copies of ``dct_oracle.c`` to show
    that the pins catch them).  Returns the previously loaded library."""
    global _lib
    old = _load()
    if path is None:
        return old
    lib = ctypes.CDLL(path)
    lib.oracle_dct_axis_sel.restype = ctypes.c_int
    lib.oracle_dct_axis_sel.argtypes = old.oracle_dct_axis_sel.argtypes
    lib.oracle_num_threads.restype = ctypes.c_int
    with _lock:
        _lib = lib
    return old


def _restore_library(lib):
    global _lib
    with _lock:
        _lib = lib


def num_threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().oracle_num_threads())


def dct_axis(x, axis: int, kind: int, sel=None) -> np.ndarray:
    """Raw DCT-II (kind=2) or DCT-III (kind=3) along ``axis``.

    Eq. (1d-definition) a / b of the paper, FP64.  ``sel`` optionally lists the
    output indices to keep along ``axis`` (in the given order).
    """
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim < 1:
        raise ValueError("need at least one axis")
    axis = axis % x.ndim
    dims = np.asarray(x.shape, dtype=np.int32)
    if sel is None:
        nsel, sel_arr, sel_ptr = x.shape[axis], None, None
    else:
        sel_arr = np.ascontiguousarray(np.asarray(sel, dtype=np.int32).ravel())
        nsel, sel_ptr = int(sel_arr.size), sel_arr.ctypes.data
    out_shape = list(x.shape)
    out_shape[axis] = nsel
    out = np.empty(out_shape, dtype=np.float64)
    if x.size == 0 or nsel == 0:
        return out
    rc = _load().oracle_dct_axis_sel(x.ctypes.data, out.ctypes.data, x.ndim,
                                     dims.ctypes.data, axis, kind, nsel, sel_ptr)
    if rc != 0:
        raise ValueError(f"oracle_dct_axis_sel rejected shape={x.shape} axis={axis} kind={kind}")
    return out


def _ortho_scale(n: int) -> np.ndarray:
    s = np.full(n, np.sqrt(2.0 / n))
    s[0] = np.sqrt(1.0 / n)
    return s


def _bcast(v: np.ndarray, ndim: int, axis: int) -> np.ndarray:
    shape = [1] * ndim
    shape[axis] = v.size
    return v.reshape(shape)


def dctn(x, norm: str = "backward", axes=None, sel=None) -> np.ndarray:
    """Multi-dimensional DCT-II: the 1-D DCT-II applied along every axis.

    ``sel`` (optional) maps an axis to the output indices kept along it, so a
    few full output lines of a large array can be computed exactly.
    """
    if norm not in NORMS:
        raise ValueError(f"norm must be one of {NORMS}")
    y = np.asarray(x, dtype=np.float64)
    axes = range(y.ndim) if axes is None else [a % y.ndim for a in axes]
    sel = dict(sel or {})
    # Transform the axes with an output selection first: they shrink the array.
    order = sorted(axes, key=lambda a: (a not in sel, a))
    for a in order:
        keep = sel.get(a)
        n = y.shape[a]
        y = dct_axis(y, a, 2, keep)
        if norm == "ortho":
            s = _ortho_scale(n)
            if keep is not None:
                s = s[np.asarray(keep, dtype=np.int64)]
            y = y * _bcast(s, y.ndim, a)
    return y


def idctn(x, norm: str = "backward", axes=None, sel=None) -> np.ndarray:
    """Multi-dimensional inverse of :func:`dctn` (DCT-III along every axis).

    backward: prod_d (2/N_d) * raw DCT-III (Eq. 1d-definition b) per axis.
    ortho: input scaled by the orthonormal weights, then DCT-III without the
    halving of the first term, i.e. the transpose of the orthonormal DCT-II.
    """
    if norm not in NORMS:
        raise ValueError(f"norm must be one of {NORMS}")
    y = np.asarray(x, dtype=np.float64)
    axes = range(y.ndim) if axes is None else [a % y.ndim for a in axes]
    sel = dict(sel or {})
    order = sorted(axes, key=lambda a: (a not in sel, a))
    for a in order:
        keep = sel.get(a)
        n = y.shape[a]
        if norm == "ortho":
            w = _ortho_scale(n)
            w[0] *= 2.0  # cancels the 1/2 on the first term of the raw DCT-III
            y = y * _bcast(w, y.ndim, a)
            y = dct_axis(y, a, 3, keep)
        else:
            y = dct_axis(y, a, 3, keep) * (2.0 / n)
    return y


def idxst_axis(x, axis: int, norm: str = "backward", sel=None) -> np.ndarray:
    """1-D IDXST along ``axis`` (Eq. idxst): IDXST(x)_k = (-1)^k IDCT({x_{N-n}})_k
    with x_N = 0, where IDCT is :func:`idctn` of ``norm`` along that axis.

    In the order of the equation: the reversed sequence y(n) = x(N - n) with
    y(0) = x(N) = 0, its IDCT, the sign (-1)^k.  ``sel`` optionally lists the
    output indices k to keep.
    """
    x = np.asarray(x, dtype=np.float64)
    axis = axis % x.ndim
    n = x.shape[axis]
    src = np.array([0] + list(range(n - 1, 0, -1)), dtype=np.int64)   # y(m) = x(n - m), m >= 1
    y = np.take(x, src, axis=axis)
    first = [slice(None)] * x.ndim
    first[axis] = 0
    y[tuple(first)] = 0.0                                               # y(0) = x(N) = 0
    keep = None if sel is None else [int(k) for k in sel]
    z = idctn(y, norm, axes=[axis], sel=None if keep is None else {axis: keep})
    k = np.arange(n) if keep is None else np.asarray(keep, dtype=np.int64)
    return z * _bcast(np.where(k % 2 == 0, 1.0, -1.0), z.ndim, axis)


def idct_idxst2(x, norm: str = "backward", sel=None) -> np.ndarray:
    """IDCT_IDXST(x) = IDCT(IDXST(x)^T)^T of a 2-D array (Eq. idxst): IDXST
    along axis 0 (the columns), then IDCT along axis 1 (the rows).  ``sel``
    maps an axis to the output indices kept along it."""
    sel = dict(sel or {})
    y = idxst_axis(x, 0, norm, sel.get(0))
    return idctn(y, norm, axes=[1], sel={1: sel[1]} if 1 in sel else None)


def idxst_idct2(x, norm: str = "backward", sel=None) -> np.ndarray:
    """IDXST_IDCT(x) = IDXST(IDCT(x)^T)^T of a 2-D array (Eq. idxst): IDCT
    along axis 0, then IDXST along axis 1."""
    sel = dict(sel or {})
    y = idctn(x, norm, axes=[0], sel={0: sel[0]} if 0 in sel else None)
    return idxst_axis(y, 1, norm, sel.get(1))


def compress2d(x, eps: float, norm: str = "ortho", sel=None) -> np.ndarray:
    """Alg. image-compression: B = 2-D DCT of x under ``norm``; C = f_eps(B),
    which keeps B(i, j) when |B(i, j)| >= eps and zeroes it otherwise (Eq.
    image-compression); the result is the 2-D IDCT of C under the same norm.
    ``sel`` selects output lines as in :func:`idctn`."""
    b = dctn(x, norm)
    c = np.where(np.abs(b) >= eps, b, 0.0)
    return idctn(c, norm, sel=sel)


def neumann_eigenvalues(n1: int, n2: int, h1: float, h2: float) -> np.ndarray:
    """Eigenvalues of the cell-centred 5-point Neumann Laplacian on an n1 x n2
    grid: lam(k1,k2) = (2cos(pi k1/n1) - 2)/h1^2 + (2cos(pi k2/n2) - 2)/h2^2.
    The DCT-II basis vectors cos(pi k (i + 1/2)/n) are its eigenvectors."""
    k1 = np.arange(n1, dtype=np.float64)[:, None]
    k2 = np.arange(n2, dtype=np.float64)[None, :]
    return (2.0 * np.cos(np.pi * k1 / n1) - 2.0) / (h1 * h1) + \
           (2.0 * np.cos(np.pi * k2 / n2) - 2.0) / (h2 * h2)


def poisson2d_neumann(f, h1: float | None = None, h2: float | None = None) -> np.ndarray:
    """Spectral solve of  Lap(u) = f - mean(f)  with homogeneous Neumann
    boundaries on a cell-centred grid, normalised by mean(u) = 0.

    Steps: F = raw DCT-II of f; U = F / lam with U[0,0] = 0; u = backward
    DCT-III of U.  Default spacing h_d = 1/N_d (unit square).
    """
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 2:
        raise ValueError("poisson2d_neumann expects a 2-D array")
    n1, n2 = f.shape
    h1 = 1.0 / n1 if h1 is None else float(h1)
    h2 = 1.0 / n2 if h2 is None else float(h2)
    F = dctn(f, "backward")
    lam = neumann_eigenvalues(n1, n2, h1, h2)
    lam[0, 0] = 1.0
    U = F / lam
    U[0, 0] = 0.0
    return idctn(U, "backward")


def rel_l2(y, y_ref) -> float:
    """||y - y_ref||_2 / ||y_ref||_2 in FP64 over the whole array."""
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    den = float(np.linalg.norm(y_ref.ravel()))
    num = float(np.linalg.norm((y - y_ref).ravel()))
    return num / den if den > 0 else num
