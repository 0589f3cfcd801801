"""FP64 numpy model of the paper's three-stage DCT / IDCT (test-only).

This is NOT the oracle (the oracle is the plain definition in ``oracle/``).  It
models, step by step in FP64 with numpy's FFT, the stages the paper describes
and the decomposition the GPU kernels implement, so the readings of garbled or
silent passages can be checked against the oracle before any kernel runs:

* Alg. alg:DCT, 2D_DCT: Eq. (2d_dct_pre) reorder, 2D real FFT, Eq. (2d_dct_post)
  with the partner index read modulo N1 (the printed zero convention at
  k1 = 0 halves row 0);
* the four-element postprocess of Eqs. (four-elements) and (s-t) with the
  corner-thread mapping that writes every output exactly once;
* Alg. alg:DCT, 2D_IDCT: Eq. (2d_idct_pre) with the twiddle exponent read as
  +j (the printed -j form is not Hermitian), unnormalised inverse real FFT,
  Eq. (2d_idct_post) inverse reorder;
* Alg. 1d-dct-via-fft, "DCT using N FFT": Eq. (n_pre), real FFT, Eq. (n_post_update);
* the 3-D form (Section "Other Transforms and Platforms"): 3-D reorder, 3-D
  real FFT, post reading four spectrum values and writing eight outputs;
* the GPU decomposition: half-length complex FFT of each reordered row with the
  even/odd split, DC and Nyquist columns packed into one complex column, column
  FFT, unpack, four-element post with scale factors folded into the twiddles,
  and the mirror image for the inverse.
"""
import numpy as np


def perm(n):
    """p(m) of Eq. (2d_dct_pre) / (n_pre): 2m for m <= floor((n-1)/2), else 2n-2m-1."""
    m = np.arange(n)
    return np.where(m <= (n - 1) // 2, 2 * m, 2 * n - 2 * m - 1)


# ------------------------------------------------------------------ 1-D, N FFT
def dct1d_npoint(x):
    """Alg. 1d-dct-via-fft, N-point variant: returns 2 * raw DCT-II."""
    n = x.size
    xp = x[perm(n)]
    X = np.fft.rfft(xp)                       # ceil((n+1)/2) values
    y = np.empty(n)
    for k in range(n):
        w = np.exp(-1j * np.pi * k / (2 * n))
        if k <= n // 2:                        # k <= ceil((n-1)/2)
            y[k] = 2 * (w * X[k]).real
        else:
            y[k] = 2 * (w * np.conj(X[n - k])).real
    return y


# ------------------------------------------------------------ paper, 2-D DCT
def dct2d_paper_naive(x, modular=True):
    """Eq. (2d_dct_pre) + RFFT2 + Eq. (2d_dct_post), one output at a time.

    Returns 4 * raw DCT-II.  ``modular=False`` applies the printed convention
    X(N1, n2) = 0, which is wrong for row 0."""
    n1, n2 = x.shape
    xp = x[perm(n1)][:, perm(n2)]
    V = np.fft.fft2(xp)                      # full spectrum; RFFT2 holds its left half
    y = np.empty((n1, n2))
    for k1 in range(n1):
        for k2 in range(n2):
            a = np.exp(-1j * np.pi * k1 / (2 * n1))
            b = np.exp(-1j * np.pi * k2 / (2 * n2))
            if k1 == 0 and not modular:
                partner = 0.0
            else:
                partner = V[(n1 - k1) % n1, k2]
            y[k1, k2] = 2 * (b * (a * V[k1, k2] + np.conj(a) * partner)).real
    return y


def half_spectrum_read(Xh, n1, n2, k1, k2):
    """Read X(k1, k2) of the full 2-D spectrum from the stored half (columns
    0..floor(n2/2)); columns beyond are conj X(-k1 mod n1, n2 - k2)."""
    if k2 <= n2 // 2:
        return Xh[k1 % n1, k2]
    return np.conj(Xh[(-k1) % n1, n2 - k2])


def dct2d_paper_fourelem(x):
    """Eqs. (four-elements), (s-t) on the half spectrum; returns (4*raw, writes).

    Each "thread" is a pair of rows (k1, N1-k1 mod N1) and a stored column k2;
    row 0 and row N1/2 pair with themselves, columns 0 and N2/2 have no mirror.
    ``writes`` counts how often each output was written (must be all ones)."""
    n1, n2 = x.shape
    xp = x[perm(n1)][:, perm(n2)]
    Xh = np.fft.rfft2(xp)
    y = np.zeros((n1, n2))
    writes = np.zeros((n1, n2), dtype=int)
    threads = 0
    for k1 in range(n1 // 2 + 1):
        k1p = (n1 - k1) % n1
        for k2 in range(n2 // 2 + 1):
            threads += 1
            A = half_spectrum_read(Xh, n1, n2, k1, k2)
            B = half_spectrum_read(Xh, n1, n2, k1p, k2)
            a = np.exp(-1j * np.pi * k1 / (2 * n1))
            b = np.exp(-1j * np.pi * k2 / (2 * n2))
            s = b * (a * A + np.conj(a) * B)
            t = b * (a * A - np.conj(a) * B)
            outs = [(k1, k2, 2 * s.real)]
            if 0 < k2 and 2 * k2 != n2:
                outs.append((k1, n2 - k2, -2 * s.imag))
            if k1p != k1:
                outs.append((k1p, k2, -2 * t.imag))
                if 0 < k2 and 2 * k2 != n2:
                    outs.append((k1p, n2 - k2, -2 * t.real))
            for (i, j, v) in outs:
                y[i, j] = v
                writes[i, j] += 1
    return y, writes, threads


# ----------------------------------------------------------- paper, 2-D IDCT
def idct2d_paper(y, sign=+1):
    """Eq. (2d_idct_pre) with twiddle exponent sign*j, unnormalised inverse
    real FFT (exponent +j), Eq. (2d_idct_post).  Returns 4 * raw DCT-III (per
    axis, composed) for sign=+1.  y(N1, .) = y(., N2) = 0."""
    n1, n2 = y.shape

    def Y(i, j):
        return 0.0 if (i >= n1 or j >= n2) else y[i, j]

    Xp = np.zeros((n1, n2 // 2 + 1), dtype=complex)
    for k1 in range(n1):
        for k2 in range(n2 // 2 + 1):
            tw = np.exp(sign * 1j * np.pi * k1 / (2 * n1)) * np.exp(sign * 1j * np.pi * k2 / (2 * n2))
            Xp[k1, k2] = tw * ((Y(k1, k2) - Y(n1 - k1, n2 - k2)) - 1j * (Y(n1 - k1, k2) + Y(k1, n2 - k2)))
    v = np.fft.irfft2(Xp, s=(n1, n2)) * (n1 * n2)
    out = np.empty((n1, n2))
    out[np.ix_(perm(n1), perm(n2))] = v      # Eq. (2d_idct_post) is the inverse reorder
    return out, Xp


# ------------------------------------------------------------------- 3-D DCT
def dct3d_paper(x):
    """3-D reorder + 3-D RFFT + post reading V(+-k1, +-k2, k3) (4 values) and
    writing y(+-k1, +-k2, k3) and y(+-k1, +-k2, N3-k3) (8 values).
    Returns (8 * raw DCT-II, writes)."""
    n1, n2, n3 = x.shape
    xp = x[perm(n1)][:, perm(n2)][:, :, perm(n3)]
    Xh = np.fft.rfftn(xp)                    # n1 x n2 x (n3//2 + 1)
    a = np.exp(-1j * np.pi * np.arange(n1) / (2 * n1))
    b = np.exp(-1j * np.pi * np.arange(n2) / (2 * n2))
    c = np.exp(-1j * np.pi * np.arange(n3) / (2 * n3))
    y = np.zeros((n1, n2, n3))
    writes = np.zeros((n1, n2, n3), dtype=int)
    for k1 in range(n1 // 2 + 1):
        for k2 in range(n2 // 2 + 1):
            for k3 in range(n3 // 2 + 1):
                vals = {}
                for s1 in (k1, (n1 - k1) % n1):
                    for s2 in (k2, (n2 - k2) % n2):
                        vals[(s1, s2)] = Xh[s1, s2, k3]          # the four reads
                targets = set()
                for o1 in (k1, (n1 - k1) % n1):
                    for o2 in (k2, (n2 - k2) % n2):
                        for o3 in (k3, (n3 - k3) % n3):
                            targets.add((o1, o2, o3))
                for (o1, o2, o3) in targets:
                    acc = 0.0
                    for sg1 in (1, -1):
                        for sg2 in (1, -1):
                            p1 = o1 if sg1 > 0 else (n1 - o1) % n1
                            p2 = o2 if sg2 > 0 else (n2 - o2) % n2
                            ta = a[o1] if sg1 > 0 else np.conj(a[o1])
                            tb = b[o2] if sg2 > 0 else np.conj(b[o2])
                            if o3 == k3:
                                v = vals[(p1, p2)]
                            else:   # V(p1, p2, N3-k3) = conj V(-p1, -p2, k3)
                                v = np.conj(vals[((n1 - p1) % n1, (n2 - p2) % n2)])
                            acc = acc + ta * tb * v
                    val = 2 * (c[o3] * acc).real
                    y[o1, o2, o3] = val
                    writes[o1, o2, o3] += 1
    return y, writes


# ------------------------------------------------------ GPU decomposition, 2-D
def tables_dct(n1, n2, norm):
    """Post twiddles with every scale folded in (the kernels' FP64-built tables):
    a'[k1] = g1(k1) e^{-j pi k1/2N1},  b'[k2] = 2 * (1/4) * g2(k2) e^{-j pi k2/2N2},
    g = 1 (backward) or the orthonormal weights."""
    g1 = np.ones(n1)
    g2 = np.ones(n2 // 2 + 1)
    if norm == "ortho":
        g1[:] = np.sqrt(2.0 / n1)
        g1[0] = np.sqrt(1.0 / n1)
        g2[:] = np.sqrt(2.0 / n2)
        g2[0] = np.sqrt(1.0 / n2)
    a = g1 * np.exp(-1j * np.pi * np.arange(n1) / (2 * n1))
    b = 0.5 * g2 * np.exp(-1j * np.pi * np.arange(n2 // 2 + 1) / (2 * n2))
    return a, b


def tables_idct(n1, n2, norm):
    """Pre twiddles for the inverse with scale folded in:
    A'[k1] = f1(k1) e^{+j pi k1/2N1}, B'[k2] = f2(k2) e^{+j pi k2/2N2};
    backward f = 1/N, ortho f(0) = sqrt(1/N), f(k>0) = sqrt(2/N)/2."""
    def f(n, m):
        if norm == "ortho":
            v = np.full(m, np.sqrt(2.0 / n) / 2)
            v[0] = np.sqrt(1.0 / n)
            return v
        return np.full(m, 1.0 / n)
    A = f(n1, n1) * np.exp(1j * np.pi * np.arange(n1) / (2 * n1))
    B = f(n2, n2 // 2 + 1) * np.exp(1j * np.pi * np.arange(n2 // 2 + 1) / (2 * n2))
    return A, B


def gpu_model_dct2d(x, norm="backward"):
    """Row pass (reorder, half-length complex FFT, split, pack DC + j*Nyquist into
    column 0) then column pass (complex FFT over rows, unpack column 0, four-element
    post with folded scale).  n2 must be even."""
    n1, n2 = x.shape
    m = n2 // 2
    xp = x[perm(n1)][:, perm(n2)]
    z = xp[:, 0::2] + 1j * xp[:, 1::2]
    Z = np.fft.fft(z, axis=1)
    k = np.arange(m + 1)
    Zk, Zmk = Z[:, k % m], np.conj(Z[:, (m - k) % m])
    X = 0.5 * (Zk + Zmk) - 0.5j * np.exp(-2j * np.pi * k / n2) * (Zk - Zmk)
    P = X[:, :m].copy()
    P[:, 0] = X[:, 0].real + 1j * X[:, m].real          # workspace: n1 x m complex
    W = np.fft.fft(P, axis=0)
    a, b = tables_dct(n1, n2, norm)
    y = np.zeros((n1, n2))
    for k1 in range(n1 // 2 + 1):
        k1p = (n1 - k1) % n1
        for k2 in range(m):
            if k2 == 0:
                cols = [(0, 0.5 * (W[k1, 0] + np.conj(W[k1p, 0])), 0.5 * (W[k1p, 0] + np.conj(W[k1, 0]))),
                        (m, -0.5j * (W[k1, 0] - np.conj(W[k1p, 0])), -0.5j * (W[k1p, 0] - np.conj(W[k1, 0])))]
            else:
                cols = [(k2, W[k1, k2], W[k1p, k2])]
            for (c, A, B) in cols:
                s = b[c] * (a[k1] * A + np.conj(a[k1]) * B)
                t = b[c] * (a[k1] * A - np.conj(a[k1]) * B)
                y[k1, c] = s.real
                if 0 < c < m:
                    y[k1, n2 - c] = -s.imag
                if k1p != k1:
                    y[k1p, c] = -t.imag
                    if 0 < c < m:
                        y[k1p, n2 - c] = -t.real
    return y


def gpu_model_idct2d(y, norm="backward"):
    """Column pass (four-read pre with folded scale, pack column 0 with column
    N2/2, inverse complex FFT over rows) then row pass (unpack, inverse split,
    half-length inverse complex FFT, inverse reorder).  n2 must be even."""
    n1, n2 = y.shape
    m = n2 // 2
    A, B = tables_idct(n1, n2, norm)

    def Y(i, j):
        return 0.0 if (i >= n1 or j >= n2) else y[i, j]

    Xp = np.zeros((n1, m + 1), dtype=complex)
    for k1 in range(n1):
        for k2 in range(m + 1):
            Xp[k1, k2] = A[k1] * B[k2] * ((Y(k1, k2) - Y(n1 - k1, n2 - k2)) - 1j * (Y(n1 - k1, k2) + Y(k1, n2 - k2)))
    P = Xp[:, :m].copy()
    P[:, 0] = Xp[:, 0] + 1j * Xp[:, m]
    U = np.fft.ifft(P, axis=0) * n1                      # unnormalised inverse
    Uf = np.zeros((n1, m + 1), dtype=complex)
    Uf[:, :m] = U
    Uf[:, 0] = U[:, 0].real
    Uf[:, m] = U[:, 0].imag
    k = np.arange(m)
    Uk, Umk = Uf[:, k], np.conj(Uf[:, m - k])
    Z = (Uk + Umk) + 1j * np.exp(2j * np.pi * k / n2) * (Uk - Umk)
    z = np.fft.ifft(Z, axis=1) * m
    v = np.empty((n1, n2))
    v[:, 0::2] = z.real
    v[:, 1::2] = z.imag
    out = np.empty_like(v)
    out[np.ix_(perm(n1), perm(n2))] = v
    return out


def idct3d_paper(y):
    """3-D form of Eq. (2d_idct_pre): per axis the factor (1 - j S_d) with S_d the
    reflection k_d -> N_d - k_d (zero at N_d), i.e. eight reads
        y - j(y1 + y2 + y3) - (y12 + y13 + y23) + j y123,
    times prod_d e^{+j pi k_d / 2N_d}; unnormalised 3-D inverse real FFT; inverse
    reorder on every axis.  Returns 8 * raw DCT-III composed over the axes."""
    n1, n2, n3 = y.shape
    m3 = n3 // 2

    def Y(i, j, k):
        return 0.0 if (i >= n1 or j >= n2 or k >= n3) else y[i, j, k]

    Xp = np.zeros((n1, n2, m3 + 1), dtype=complex)
    for k1 in range(n1):
        for k2 in range(n2):
            for k3 in range(m3 + 1):
                b1, b2, b3 = n1 - k1, n2 - k2, n3 - k3
                v = (Y(k1, k2, k3) - 1j * (Y(b1, k2, k3) + Y(k1, b2, k3) + Y(k1, k2, b3))
                     - (Y(b1, b2, k3) + Y(b1, k2, b3) + Y(k1, b2, b3)) + 1j * Y(b1, b2, b3))
                tw = (np.exp(1j * np.pi * k1 / (2 * n1)) * np.exp(1j * np.pi * k2 / (2 * n2))
                      * np.exp(1j * np.pi * k3 / (2 * n3)))
                Xp[k1, k2, k3] = tw * v
    v = np.fft.irfftn(Xp, s=(n1, n2, n3), axes=(0, 1, 2)) * (n1 * n2 * n3)
    out = np.empty_like(v)
    out[np.ix_(perm(n1), perm(n2), perm(n3))] = v
    return out


def split_column_fft(Z, inverse=False):
    """Length-n1 DFT along axis 0 (unnormalised both ways) in the split-column
    order of the tall-array kernels, n1 = 8 q, n = qq + q r, k = kp + 8 kq:
    forward, the radix-8 step (8-point DFT across r, then the twiddle
    W_n1^(qq kp)) gives workspace row kp q + qq, and a q-point DFT over qq
    gives output row kp + 8 kq; inverse, a q-point inverse DFT over kq, then
    the conjugate twiddle and the inverse 8-point DFT across kp."""
    n1 = Z.shape[0]
    q = n1 // 8
    sgn = 1.0 if inverse else -1.0
    e8 = np.exp(sgn * 2j * np.pi * np.outer(np.arange(8), np.arange(8)) / 8)      # [kp, r]
    tw = np.exp(sgn * 2j * np.pi * np.outer(np.arange(8), np.arange(q)) / n1)     # [kp, qq]
    if not inverse:
        A = Z.reshape(8, q, -1)                                    # A[r, qq] = Z(qq + q r)
        ws = np.einsum("kr,rqc->kqc", e8, A) * tw[:, :, None]      # row kp q + qq
        C = np.fft.fft(ws, axis=1)                                 # C[kp, kq] = X(kp + 8 kq)
        return C.transpose(1, 0, 2).reshape(Z.shape)
    Y = Z.reshape(q, 8, -1).transpose(1, 0, 2)                     # Y[kp, kq] = Z(kp + 8 kq)
    ws = np.fft.ifft(Y, axis=1) * q                                # row kp q + qq
    out = np.einsum("kr,kqc->rqc", e8, ws * tw[:, :, None])        # out[r, qq] = x(qq + q r)
    return out.reshape(Z.shape)
