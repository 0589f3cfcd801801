// Spectral solve of the cell-centred Neumann Poisson problem on an n1 x n2
// grid (Section "DREAMPlace": the electric potential is obtained by a DCT, a
// division by the Laplacian eigenvalues and an inverse DCT):
//   F = DCT-II(f);  U(k1, k2) = F(k1, k2) / lam(k1, k2), U(0, 0) = 0;
//   u = DCT-III(U) (backward scale, so u has zero mean),
//   lam(k1, k2) = (2 cos(pi k1 / n1) - 2) / h1^2 + (2 cos(pi k2 / n2) - 2) / h2^2.
//
// Three HBM passes instead of the four of a DCT followed by an IDCT:
//   (1) the DCT row pass (reorder + row real FFT) into the packed half spectrum;
//   (2) this kernel, one column pair per workgroup slot: forward column FFT,
//       the four-element post (Eqs. four-elements, s-t) giving F at
//       (k1, k2), (k1, n2-k2), (n1-k1, k2), (n1-k1, n2-k2), the divide, then
//       the four-read IDCT pre (Eq. 2d_idct_pre) of exactly those four values
//       for rows k1 and n1-k1, and the inverse column FFT, written back in
//       place;
//   (3) the IDCT row pass (inverse real FFT + inverse reorder).
// The spectrum F never reaches HBM: the post's four outputs are the pre's four
// inputs.
#pragma once

#include "fft_core.h"
#include "poisson.h"

namespace dctx {



constexpr int kSlotsP = kEmax;
constexpr int kPairsP = kEmax / 2 + 1;

// DCT values of the post for the row pair (k1, k1p) from spectrum values A =
// V(k1), B = V(k1p) of one stored column: (y(k1, col), y(k1, n2-col),
// y(k1p, col), y(k1p, n2-col)) = (Re s, -Im s, -Im t, -Re t).
__device__ __forceinline__ float4 post4(float2 a, float2 b, float2 A, float2 B) {
    const float2 aA = cmul(a, A);
    const float2 aB = cmulc(B, a);
    const float2 s = cmul(b, cadd(aA, aB));
    const float2 t = cmul(b, csub(aA, aB));
    return make_float4(s.x, -s.y, -t.y, -t.x);
}

// The pointwise step on one DCT coefficient v at (k1, k2) (see PoissonTabs):
// the Poisson divide (zero at DC), or the compression threshold f_eps.  MODE
// is the table's mode fixed at compile time (a run-time branch inside the
// unrolled post would cost time).
template <int MODE>
__device__ __forceinline__ float spec_op(const PoissonTabs &q, float v, float l1, float l2, bool dc) {
    if (MODE == 1) return fabsf(v) >= q.eps ? v : 0.f;
    return dc ? 0.f : v / (l1 + l2);
}

// Eq. (2d_idct_pre) for one row: P = (U(r, col), U(r, n2-col)), Q = the same
// at the reflected row (zero for row 0).
__device__ __forceinline__ float2 pre1(float2 ab, float2 P, float2 Q) {
    return cmul(ab, make_float2(P.x - Q.y, -(Q.x + P.y)));
}

// Column 0 packs columns 0 and m: P = (U(r, 0), U(r, m)), Q at the reflected row.
__device__ __forceinline__ float2 pre1_dc(float2 ab0, float2 abm, float2 P, float2 Q) {
    const float2 x0 = cmul(ab0, make_float2(P.x, -Q.x));
    const float2 xm = cmul(abm, make_float2(P.y - Q.y, -(Q.y + P.y)));
    return make_float2(x0.x - xm.y, x0.y + xm.x);
}

// Column tile `tile` (packed columns tile*C ..) of the fused Poisson column
// pass, in place on the workspace (the packed half spectrum, or for odd n2
// columns 0 .. (n2-1)/2 with column 0 alone); blockDim >= C * T.
template <int MODE>
__device__ __forceinline__ void poisson_cols_body(const Plan2D &p, const PoissonTabs &q, int C, int tile,
                                                  float2 *__restrict__ ws, float2 *lds) {
    const int T = p.col.T;
    const int c = threadIdx.x % C;
    const int t = threadIdx.x / C;
    const int M = p.m, N1 = p.n1, N2 = p.n2, MW = ws_cols(p);
    const int k2 = tile * C + c;
    const bool act = (t < T) && (k2 < MW);

    {
        float2 v[kSlotsP];
#pragma unroll
        for (int e = 0; e < kSlotsP; ++e) {
            const int row = t + e * T;
            if (act && row < N1) v[e] = ws[(size_t)row * MW + k2];
        }
#pragma unroll
        for (int e = 0; e < kSlotsP; ++e) {
            const int row = t + e * T;
            if (t < T && row < N1) lds[lslot(row, C) + c] = act ? v[e] : make_float2(0.f, 0.f);
        }
    }
    lds_sync();
    fft_lds<false>(lds + c, C, t < T ? t : T, T, p.col);

    // post -> divide -> pre for the pairs (k1, n1 - k1), k1 = t + i T <= n1 / 2
    float2 xa[kPairsP], xb[kPairsP];
    if (act) {
        const float2 b = p.tb[k2], bm = p.tb[M];
        const float2 bi = q.tbi[k2], bim = q.tbi[M];
        const int k2r = (k2 == 0) ? M : N2 - k2;   // second column of the group
        const float l2a = q.l2[k2], l2b = q.l2[k2r];
#pragma unroll
        for (int i = 0; i < kPairsP; ++i) {
            const int k1 = t + i * T;
            if (k1 > N1 / 2) continue;
            const int k1p = (k1 == 0) ? 0 : N1 - k1;
            const float2 A = lds[lslot(k1, C) + c];
            const float2 B = lds[lslot(k1p, C) + c];
            const float2 a = p.ta[k1];
            const float l1a = q.l1[k1], l1b = q.l1[k1p];
            // U at (k1, k2), (k1, k2r), (k1p, k2), (k1p, k2r)
            float4 U;
            if (k2 == 0 && p.odd) {
                // odd n2: column 0 pairs with the zero column n2 (no Nyquist column)
                const float4 f = post4(a, b, A, B);   // .x = F(k1, 0), .z = F(k1p, 0)
                const float2 P = make_float2(spec_op<MODE>(q, f.x, l1a, l2a, k1 == 0), 0.f);
                const float2 Q = make_float2(spec_op<MODE>(q, f.z, l1b, l2a, k1p == 0), 0.f);
                const float2 R = (k1 == 0) ? make_float2(0.f, 0.f) : (k1p == k1 ? P : Q);
                xa[i] = pre1(cmul(q.tai[k1], bi), P, R);
                if (k1p != k1) xb[i] = pre1(cmul(q.tai[k1p], bi), Q, P);
            } else if (k2 == 0) {
                const float2 v0a = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
                const float2 v0b = make_float2(0.5f * (B.x + A.x), 0.5f * (B.y - A.y));
                const float2 vma = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
                const float2 vmb = make_float2(0.5f * (B.y + A.y), -0.5f * (B.x - A.x));
                const float4 f0 = post4(a, b, v0a, v0b);    // .x = F(k1, 0), .z = F(k1p, 0)
                const float4 fm = post4(a, bm, vma, vmb);   // .x = F(k1, m), .z = F(k1p, m)
                U = make_float4(spec_op<MODE>(q, f0.x, l1a, l2a, k1 == 0), spec_op<MODE>(q, fm.x, l1a, l2b, false),
                                spec_op<MODE>(q, f0.z, l1b, l2a, k1p == 0), spec_op<MODE>(q, fm.z, l1b, l2b, false));
                const float2 ai = q.tai[k1];
                const float2 P = make_float2(U.x, U.y), Q = make_float2(U.z, U.w);
                // reflected row: none for row 0, the row itself for n1/2
                const float2 R = (k1 == 0) ? make_float2(0.f, 0.f) : (k1p == k1 ? P : Q);
                xa[i] = pre1_dc(cmul(ai, bi), cmul(ai, bim), P, R);
                if (k1p != k1) {
                    const float2 aip = q.tai[k1p];
                    xb[i] = pre1_dc(cmul(aip, bi), cmul(aip, bim), Q, P);
                }
            } else {
                const float4 f = post4(a, b, A, B);
                U = make_float4(spec_op<MODE>(q, f.x, l1a, l2a, false), spec_op<MODE>(q, f.y, l1a, l2b, false),
                                spec_op<MODE>(q, f.z, l1b, l2a, false), spec_op<MODE>(q, f.w, l1b, l2b, false));
                const float2 P = make_float2(U.x, U.y), Q = make_float2(U.z, U.w);
                const float2 R = (k1 == 0) ? make_float2(0.f, 0.f) : (k1p == k1 ? P : Q);
                xa[i] = pre1(cmul(q.tai[k1], bi), P, R);
                if (k1p != k1) xb[i] = pre1(cmul(q.tai[k1p], bi), Q, P);
            }
        }
    }
    lds_sync();
    if (act) {
#pragma unroll
        for (int i = 0; i < kPairsP; ++i) {
            const int k1 = t + i * T;
            if (k1 > N1 / 2) continue;
            const int k1p = (k1 == 0) ? 0 : N1 - k1;
            lds[lslot(k1, C) + c] = xa[i];
            if (k1p != k1) lds[lslot(k1p, C) + c] = xb[i];
        }
    }
    lds_sync();
    fft_lds<true>(lds + c, C, t < T ? t : T, T, p.col);
#pragma unroll
    for (int e = 0; e < kSlotsP; ++e) {
        const int row = t + e * T;
        if (act && row < N1) ws[(size_t)row * MW + k2] = lds[lslot(row, C) + c];
    }
}

}  // namespace dctx
