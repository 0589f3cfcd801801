// Tile bodies of the generic (any 5-smooth length, run-time radix schedule)
// 2-D three-stage passes, shared by the per-transform kernels and the
// persistent batched kernels.  Each body processes one tile with the calling
// workgroup; threads beyond the tile's rows x T (or C x T) only join the
// barriers.
//
// 2-D DCT-II / DCT-III by the three-stage method, two HBM passes each.
//
// Forward (Alg. alg:DCT, "2D_DCT"):
//   rows    : load row p1(n1) of x coalesced, apply the Eq. (2d_dct_pre) reorder
//             inside LDS, run the length-n2 real FFT as a length-m = n2/2
//             complex FFT of z(q) = x'(2q) + j x'(2q+1) followed by the
//             even/odd split, and store the half spectrum with the real DC and
//             Nyquist values packed into column 0 as X(0) + j X(m).
//   columns : load a tile of packed columns for all n1 rows, run the length-n1
//             complex FFT down each column, unpack column 0 and apply the
//             four-element postprocess of Eqs. (four-elements) and (s-t) on the
//             row pairs (k1, n1-k1 mod n1), writing output columns k2 and n2-k2.
// Inverse (Alg. alg:DCT, "2D_IDCT"):
//   columns : the Eq. (2d_idct_pre) preprocess (exponent +j, four reads per
//             pair of outputs, y(n1, .) = y(., n2) = 0) on a tile of columns
//             k2 and their mirrors n2-k2, column 0 packed with column m, then
//             the inverse length-n1 FFT down each column.
//   rows    : unpack, inverse split, inverse length-m complex FFT, and the
//             Eq. (2d_idct_post) inverse reorder applied in LDS before a
//             coalesced store of output row p1(n1).
// Every scale factor (normalisation, the factor 2 of the post, the 4 of the
// unnormalised inverse) is folded into the FP64-built twiddle tables.
#pragma once

#include "fft_core.h"

namespace dctx {


// All global loads and stores below run in fully unrolled loops over a
// compile-time number of slots (guarded by the runtime sizes), so every load of
// a thread is in flight before the first one is used.  Bounds: a sequence of
// length L has T >= L / kEmax threads, so a thread owns at most kEmax elements.
constexpr int kSlots = kEmax;            // elements per thread
constexpr int kHalf = kEmax / 2;         // float4 pairs per thread
constexpr int kPairs = kEmax / 2 + 1;    // (k, L - k) pairs per thread

// ------------------------------------------------------------- forward rows
// Row tile `tile` (rows tile*rpb ..) of the forward row pass; blockDim >= rpb * T.
__device__ __forceinline__ void dct2_rows_body(const Plan2D &p, int rpb, int tile, const float *__restrict__ x,
                                               float2 *__restrict__ ws, float2 *lds) {
    const int T = p.row.T;
    const int r = threadIdx.x / T;
    const int t = threadIdx.x - r * T;
    const int n1 = tile * rpb + r;
    const bool active = (r < rpb) && (n1 < p.n1);
    const int M = p.m, N2 = p.n2;
    if (p.odd) {
        // odd n2: the reordered real row as a length-n2 complex sequence, its
        // FFT, and columns 0 .. m of the spectrum (no even/odd packing)
        float2 *row = lds + (r < rpb ? r : 0) * lpad_len(N2);
        if (active) {
            const float *srow = x + (size_t)src_row(n1, p.n1, p.nsub) * N2;
            float v[kSlots];
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int i = t + e * T;
                if (i < N2) v[e] = srow[i];
            }
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int i = t + e * T;
                if (i < N2) row[lpad((i & 1) ? N2 - 1 - (i >> 1) : (i >> 1))] = make_float2(v[e], 0.f);
            }
        }
        lds_sync();
        fft_lds<false>(row, 1, active ? t : T, T, p.row);
        if (active) {
            float2 *out = ws + (size_t)n1 * (M + 1);
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int k = t + e * T;
                if (k <= M) out[k] = row[lpad(k)];
            }
        }
        return;
    }
    float2 *base = lds + (r < rpb ? r : 0) * lpad_len(M);
    float *bf = reinterpret_cast<float *>(base);

    if (active) {
        // x'(n) = x(p(n)) (Eq. 2d_dct_pre): source element i lands at x' index
        // pinv(i), pinv(2q) = q, pinv(2q + 1) = n2 - 1 - q.
        const float *srow = x + (size_t)src_row(n1, p.n1, p.nsub) * N2;
        if (p.trans) {
            // transposed input: element i of row r at x[i n1 + r]
            const float *scol = x + src_row(n1, p.n1, p.nsub);
            float v[2 * kSlots];
#pragma unroll
            for (int e = 0; e < 2 * kSlots; ++e) {
                const int i = t + e * T;
                if (i < N2) v[e] = scol[(size_t)i * p.n1];
            }
#pragma unroll
            for (int e = 0; e < 2 * kSlots; ++e) {
                const int i = t + e * T;
                if (i < N2) bf[xq_off((i & 1) ? N2 - 1 - (i >> 1) : (i >> 1))] = v[e];
            }
        } else if ((N2 & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
            // x[4q .. 4q+3] gives z(q) = (x[4q], x[4q+2]) and z(m-1-q) = (x[4q+3], x[4q+1])
            const float4 *src = reinterpret_cast<const float4 *>(srow);
            float4 v[kHalf];
#pragma unroll
            for (int e = 0; e < kHalf; ++e) {
                const int q = t + e * T;
                if (q < M / 2) v[e] = src[q];
            }
#pragma unroll
            for (int e = 0; e < kHalf; ++e) {
                const int q = t + e * T;
                if (q < M / 2) {
                    base[lpad(q)] = make_float2(v[e].x, v[e].z);
                    base[lpad(M - 1 - q)] = make_float2(v[e].w, v[e].y);
                }
            }
        } else {
            const float2 *src = reinterpret_cast<const float2 *>(srow);
            float2 v[kSlots];
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int q = t + e * T;
                if (q < M) v[e] = src[q];
            }
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int q = t + e * T;
                if (q < M) {
                    bf[xq_off(q)] = v[e].x;
                    bf[xq_off(N2 - 1 - q)] = v[e].y;
                }
            }
        }
    }
    lds_sync();
    fft_lds<false>(base, 1, active ? t : T, T, p.row);

    if (active) {
        float2 *out = ws + (size_t)n1 * M;
        float2 wk[kPairs], wm[kPairs];
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k = t + i * T;
            if (k >= 1 && k <= M / 2) {
                wk[i] = p.split[k];
                wm[i] = p.split[M - k];
            }
        }
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k = t + i * T;
            if (k > M / 2) continue;
            const float2 zk = base[lpad(k)];
            if (k == 0) {
                // X(0) = Re Z(0) + Im Z(0), X(m) = Re Z(0) - Im Z(0), both real
                out[0] = make_float2(zk.x + zk.y, zk.x - zk.y);
                continue;
            }
            const int km = M - k;
            float2 xk, xm;
            rsplit_pair(zk, base[lpad(km)], wk[i], wm[i], xk, xm);
            out[k] = xk;
            if (km != k) out[km] = xm;
        }
    }
}

// Four outputs of the post for the row pair (k1, k1p) and stored column col:
// s = b (a A + conj(a) B), t = b (a A - conj(a) B);
// y(k1, col) = Re s, y(k1, n2-col) = -Im s, y(k1p, col) = -Im t, y(k1p, n2-col) = -Re t.
// The factor 2 and the normalisation are inside the tables a, b.
// Element (r, c) of the output lives at y[r sr + c sc]: (sr, sc) = (n2, 1), or
// (1, n1) for a transposed output.
__device__ __forceinline__ void post_store(float *__restrict__ y, size_t sr, size_t sc, int N2, int k1, int k1p,
                                           int col, bool mirror, float2 a, float2 b, float2 A, float2 B) {
    const float2 aA = cmul(a, A);
    const float2 aB = cmulc(B, a);
    const float2 s = cmul(b, cadd(aA, aB));
    out_store(&y[k1 * sr + col * sc], s.x);
    if (mirror) out_store(&y[k1 * sr + (N2 - col) * sc], -s.y);
    if (k1p != k1) {
        const float2 tt = cmul(b, csub(aA, aB));
        out_store(&y[k1p * sr + col * sc], -tt.y);
        if (mirror) out_store(&y[k1p * sr + (N2 - col) * sc], -tt.x);
    }
}

// ---------------------------------------------------------- forward columns
// Column tile `tile` (packed columns tile*C ..) of the forward column pass +
// post; blockDim >= C * T.
__device__ __forceinline__ void dct2_cols_body(const Plan2D &p, int C, int tile, const float2 *__restrict__ ws,
                                               float *__restrict__ y, float2 *lds) {
    const int T = p.col.T;
    const int c = threadIdx.x % C;
    const int t = threadIdx.x / C;
    const int M = p.m, N1 = p.n1, N2 = p.n2, MW = ws_cols(p);
    const int c0 = tile * C;
    const int k2 = c0 + c;
    const bool act = (t < T) && (k2 < MW);

    {
        float2 v[kSlots];
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int row = t + e * T;
            if (act && row < N1) v[e] = ws[(size_t)row * MW + k2];
        }
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int row = t + e * T;
            if (t < T && row < N1) lds[lslot(row, C) + c] = act ? v[e] : make_float2(0.f, 0.f);
        }
    }
    lds_sync();
    fft_lds<false>(lds + c, C, t < T ? t : T, T, p.col);

    if (act) {
        float2 a[kPairs];
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k1 = t + i * T;
            if (k1 <= N1 / 2) a[i] = p.ta[k1];
        }
        const float2 b = p.tb[k2];
        const float2 bm = p.tb[M];
        const size_t sr = p.trans ? 1 : (size_t)N2, sc = p.trans ? (size_t)N1 : 1;
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k1 = t + i * T;
            if (k1 > N1 / 2) continue;
            const int k1p = (k1 == 0) ? 0 : N1 - k1;
            const float2 A = lds[lslot(k1, C) + c];
            const float2 B = lds[lslot(k1p, C) + c];
            if (k2 == 0 && p.odd) {
                post_store(y, sr, sc, N2, k1, k1p, 0, false, a[i], b, A, B);   // no Nyquist column
            } else if (k2 == 0) {
                // unpack W = V(., 0) + j V(., m):  V0(k) = (W(k) + conj W(-k)) / 2,
                // Vm(k) = -j (W(k) - conj W(-k)) / 2
                const float2 v0a = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
                const float2 v0b = make_float2(0.5f * (B.x + A.x), 0.5f * (B.y - A.y));
                const float2 vma = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
                const float2 vmb = make_float2(0.5f * (B.y + A.y), -0.5f * (B.x - A.x));
                post_store(y, sr, sc, N2, k1, k1p, 0, false, a[i], b, v0a, v0b);
                post_store(y, sr, sc, N2, k1, k1p, M, false, a[i], bm, vma, vmb);
            } else {
                post_store(y, sr, sc, N2, k1, k1p, k2, true, a[i], b, A, B);
            }
        }
    }
}

// ---------------------------------------------------------- inverse columns
// Column tile of the inverse column pass (pre + inverse column FFT).
// XST: the IDXST axes (the p.xst bits) fixed at compile time.
template <int XST>
__device__ __forceinline__ void idct2_cols_body(const Plan2D &p, int C, int tile, const float *__restrict__ x,
                                                float2 *__restrict__ ws, float2 *lds) {
    const int T = p.col.T;
    const int c = threadIdx.x % C;
    const int t = threadIdx.x / C;
    const int M = p.m, N1 = p.n1, N2 = p.n2, MW = ws_cols(p);
    const int c0 = tile * C;
    const int k2 = c0 + c;
    const bool act = (t < T) && (k2 < MW);
    // mirror column: n2 - k2; column 0 pairs with m (even n2, packed) or with
    // the zero column n2 (odd n2)
    const bool zero_mirror = p.odd && k2 == 0;
    const int mcol = (k2 == 0) ? (p.odd ? 0 : M) : N2 - k2;

    // (x(k1, k2), x(k1, mirror)) for the rows k1 = t + e T (element (r, c) at
    // x[r sr + c sc]; transposed input: sr = 1, sc = n1)
    {
        const size_t sr = p.trans ? 1 : (size_t)N2, sc = p.trans ? (size_t)N1 : 1;
        float vx[kSlots], vm[kSlots];
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int row = t + e * T;
            if (act && row < N1) {
                vx[e] = x[row * sr + k2 * sc];
                vm[e] = zero_mirror ? 0.f : x[row * sr + mcol * sc];
            }
        }
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int row = t + e * T;
            if (t < T && row < N1)
                lds[lslot(row, C) + c] = act ? make_float2(vx[e], vm[e]) : make_float2(0.f, 0.f);
        }
    }
    lds_sync();

    // Eq. (2d_idct_pre): X'(k1,k2) = A(k1) B(k2) [(x(k1,k2) - x(N1-k1,N2-k2)) - j (x(N1-k1,k2) + x(k1,N2-k2))]
    float2 pre[kSlots];
    {
        float2 a[kSlots];
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int k1 = t + e * T;
            if (act && k1 < N1) a[e] = p.ta[k1];
        }
        const float2 b = p.tb[k2];
        const float2 bm = p.tb[M];
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int k1 = t + e * T;
            pre[e] = make_float2(0.f, 0.f);
            if (act && k1 < N1) {
                float2 P = lds[lslot(k1, C) + c];
                float2 Q = (k1 == 0) ? make_float2(0.f, 0.f) : lds[lslot(N1 - k1, C) + c];
                if (XST) xst_reverse(XST, k1, k2, P, Q);
                if (k2 == 0 && !p.odd) {
                    const float2 x0 = cmul(cmul(a[e], b), make_float2(P.x, -Q.x));
                    const float2 xm = cmul(cmul(a[e], bm), make_float2(P.y - Q.y, -(Q.y + P.y)));
                    pre[e] = make_float2(x0.x - xm.y, x0.y + xm.x);   // X'(k1,0) + j X'(k1,m)
                } else {
                    pre[e] = cmul(cmul(a[e], b), make_float2(P.x - Q.y, -(Q.x + P.y)));
                }
            }
        }
    }
    lds_sync();
#pragma unroll
    for (int e = 0; e < kSlots; ++e) {
        const int k1 = t + e * T;
        if (act && k1 < N1) lds[lslot(k1, C) + c] = pre[e];
    }
    lds_sync();
    fft_lds<true>(lds + c, C, t < T ? t : T, T, p.col);

#pragma unroll
    for (int e = 0; e < kSlots; ++e) {
        const int row = t + e * T;
        if (act && row < N1) ws[(size_t)row * MW + k2] = lds[lslot(row, C) + c];
    }
}

// ------------------------------------------------------------- inverse rows
// Row tile of the inverse row pass (inverse split + FFT + inverse reorder).
__device__ __forceinline__ void idct2_rows_body(const Plan2D &p, int rpb, int tile, const float2 *__restrict__ ws,
                                                float *__restrict__ y, float2 *lds) {
    const int T = p.row.T;
    const int r = threadIdx.x / T;
    const int t = threadIdx.x - r * T;
    const int n1 = tile * rpb + r;
    const bool active = (r < rpb) && (n1 < p.n1);
    const int M = p.m, N2 = p.n2;
    if (p.odd) {
        // odd n2: columns 0 .. m extended by Hermitian symmetry to the whole
        // length-n2 spectrum, its inverse FFT, and the Eq. (2d_idct_post)
        // reorder of the real part
        float2 *row = lds + (r < rpb ? r : 0) * lpad_len(N2);
        if (active) {
            const float2 *src = ws + (size_t)n1 * (M + 1);
            float2 v[kSlots];
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int k = t + e * T;
                if (k <= M) v[e] = src[k];
            }
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int k = t + e * T;
                if (k <= M) {
                    row[lpad(k)] = v[e];
                    if (k >= 1) row[lpad(N2 - k)] = make_float2(v[e].x, -v[e].y);
                }
            }
        }
        lds_sync();
        fft_lds<true>(row, 1, active ? t : T, T, p.row);
        if (active) {
            const int orow = src_row(n1, p.n1, p.nsub);
            float *drow = y + (size_t)orow * N2;
            // IDXST signs (-1)^row and (-1)^col (Eq. idxst), exact
            const float srow = ((p.xst & 1) && (orow & 1)) ? -1.f : 1.f;
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int i = t + e * T;
                if (i < N2) {
                    const float sg = ((p.xst & 2) && (i & 1)) ? -srow : srow;
                    out_store(&drow[i], sg * row[lpad((i & 1) ? N2 - 1 - (i >> 1) : (i >> 1))].x);
                }
            }
        }
        return;
    }
    float2 *base = lds + (r < rpb ? r : 0) * lpad_len(M);
    float *bf = reinterpret_cast<float *>(base);

    if (active) {
        const float2 *src = ws + (size_t)n1 * M;
        float2 v[kSlots];
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int k = t + e * T;
            if (k < M) v[e] = src[k];
        }
#pragma unroll
        for (int e = 0; e < kSlots; ++e) {
            const int k = t + e * T;
            if (k < M) base[lpad(k)] = v[e];
        }
    }
    lds_sync();

    // inverse split: Z(k) = (U(k) + conj U(m-k)) + j e^{+2 pi j k/n2} (U(k) - conj U(m-k)),
    // with U(0) = Re P(0), U(m) = Im P(0) (both real).
    float2 zk[kPairs], zm[kPairs];
    if (active) {
        float2 wk[kPairs], wm[kPairs];
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k = t + i * T;
            if (k >= 1 && k <= M / 2) {
                wk[i] = p.split[k];
                wm[i] = p.split[M - k];
            }
        }
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k = t + i * T;
            if (k > M / 2) continue;
            if (k == 0) {
                const float2 p0 = base[0];
                zk[i] = make_float2(p0.x + p0.y, p0.x - p0.y);
            } else {
                irsplit_pair(base[lpad(k)], base[lpad(M - k)], wk[i], wm[i], zk[i], zm[i]);
            }
        }
    }
    lds_sync();
    if (active) {
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k = t + i * T;
            if (k <= M / 2) {
                base[lpad(k)] = zk[i];
                if (k != 0 && M - k != k) base[lpad(M - k)] = zm[i];
            }
        }
    }
    lds_sync();
    fft_lds<true>(base, 1, active ? t : T, T, p.row);

    if (active) {
        // Eq. (2d_idct_post): y(p1(n1), p2(n)) = x'(n1, n); output element i
        // takes x' index pinv(i): pinv(2q) = q, pinv(2q + 1) = n2 - 1 - q.
        const int orow = src_row(n1, p.n1, p.nsub);
        float *drow = y + (size_t)orow * N2;
        if (p.trans) {
            // transposed output: element i of row r at y[i n1 + r]
            float *dcol = y + orow;
            const float srow = ((p.xst & 1) && (orow & 1)) ? -1.f : 1.f;
#pragma unroll
            for (int e = 0; e < 2 * kSlots; ++e) {
                const int i = t + e * T;
                if (i < N2) {
                    const float sg = ((p.xst & 2) && (i & 1)) ? -srow : srow;
                    out_store(&dcol[(size_t)i * p.n1], sg * bf[xq_off((i & 1) ? N2 - 1 - (i >> 1) : (i >> 1))]);
                }
            }
        } else if ((N2 & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
            float4 *dst = reinterpret_cast<float4 *>(drow);
#pragma unroll
            for (int e = 0; e < kHalf; ++e) {
                const int q = t + e * T;
                if (q < M / 2) {
                    const float2 a = base[lpad(q)], b = base[lpad(M - 1 - q)];
                    out_store(&dst[q], xst_sign4(p.xst, orow, make_float4(a.x, b.y, a.y, b.x)));
                }
            }
        } else {
            float2 *dst = reinterpret_cast<float2 *>(drow);
#pragma unroll
            for (int e = 0; e < kSlots; ++e) {
                const int q = t + e * T;
                if (q < M) out_store(&dst[q], xst_sign2(p.xst, orow, make_float2(bf[xq_off(q)], bf[xq_off(N2 - 1 - q)])));
            }
        }
    }
}

}  // namespace dctx
