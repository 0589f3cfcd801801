// 3-D DCT-II / DCT-III by the three-stage method (Section "Other Transforms and
// Platforms": 3-D reorder, 3-D real FFT, a postprocess that reads four spectrum
// values and writes eight outputs; the inverse mirrors it).
//
// Three HBM passes each way on an n1 x n2 x n3 array (n3 contiguous):
//   forward : (1) n3 rows: reorder on all three axes + real FFT along n3, packed
//             half spectrum (the 2-D row kernels with a two-level row map);
//             (2) complex FFT along n2 inside every n1-plane;
//             (3) complex FFT along n1 of the columns (k2, k3) and (n2-k2, k3)
//             together, then the post: from V(+-k1, +-k2, k3) the eight outputs
//             y(+-k1, +-k2, k3) and y(+-k1, +-k2, n3-k3), using
//             V(p, q, n3-k3) = conj V(-p, -q, k3) (Hermitian symmetry).
//   inverse : (3') the separable 3-D form of Eq. (2d_idct_pre): per output
//             prod_d e^{+j pi k_d/2N_d} [y - j(y1+y2+y3) - (y12+y13+y23) + j y123]
//             (y_S: reflected k_d -> N_d - k_d on the axes in S, zero at N_d),
//             eight reads per pair of outputs, then the inverse FFT along n1;
//             (2') inverse FFT along n2; (1') inverse real FFT along n3 + the
//             inverse reorder (the 2-D inverse row kernels).
// The k3 = 0 column of the workspace holds the k3 = 0 and k3 = n3/2 values
// packed as X(., ., 0) + j X(., ., m3) (both 2-D Hermitian after the n3 pass).
// Scale factors live in the FP64-built tables ta, tb, tc.
#include <algorithm>

#include "fast_chain.h"

namespace dctx {

namespace {

constexpr int kSlots3 = kEmax;

template <int V>
struct IC {
    static constexpr int value = V;
};

// ------------------------------------------------------------ n2 direction
// Workgroup: plane a = n1 index, C consecutive k3 columns; thread (c, t).
template <bool INV>
__global__ void __launch_bounds__(kMaxBlock) k3_mid(Plan3D p, float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    const int C = p.cols2;
    const int T = p.f2.T;
    const int c = threadIdx.x % C;
    const int t = threadIdx.x / C;
    const int W3 = ws3_cols(p);
    const int tiles = (W3 + C - 1) / C;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= p.n1 * tiles) return;
    const int a = unit / tiles;
    const int k3 = (unit - a * tiles) * C + c;
    const bool act = (t < T) && (k3 < W3);
    float2 *plane = ws + (size_t)a * p.n2 * W3;
    {
        float2 v[kSlots3];
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int r = t + e * T;
            if (act && r < p.n2) v[e] = plane[(size_t)r * W3 + k3];
        }
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int r = t + e * T;
            if (t < T && r < p.n2) lds[lpad(r) * C + c] = act ? v[e] : make_float2(0.f, 0.f);
        }
    }
    lds_sync();
    fft_lds<INV>(lds + c, C, t < T ? t : T, T, p.f2);
#pragma unroll
    for (int e = 0; e < kSlots3; ++e) {
        const int r = t + e * T;
        if (act && r < p.n2) plane[(size_t)r * W3 + k3] = lds[lpad(r) * C + c];
    }
}

// Sequence slot sc = s * C + c of a unit: s = 0 is column (u, k3), s = 1 is
// column (n2 - u, k3).  LDS element n1 of slot sc at lds[lpad(n1) * 2C + sc].
struct Unit3 {
    int u, ubar, c0;
};

__device__ __forceinline__ Unit3 unit3(const Plan3D &p, int unit) {
    const int tiles = (ws3_cols(p) + p.cols1 - 1) / p.cols1;
    Unit3 r;
    r.u = unit / tiles;
    r.ubar = (r.u == 0) ? 0 : p.n2 - r.u;
    r.c0 = (unit - r.u * tiles) * p.cols1;
    return r;
}

// y(o1, o2, o3) = Re(tc[o3] S) for the four values v[i1][i2] = V(k1 or k1p,
// k2 or k2p, k3): S = sum over sign choices of a^(+-) b^(+-) V(+-o1, +-o2, o3).
// Used for the packed column k3 = 0 (o3 = 0 and m3); other columns use
// post3_sums.
template <int i1, int i2>
__device__ __forceinline__ float post3_value(const float2 (&v)[2][2], float2 a, float2 b, float2 cz) {
    const float2 ab = cmul(a, b), anb = cmulc(b, a), abn = cmulc(a, b);
    const float2 anbn = conjf2(ab);
    const float2 S = cadd(cadd(cmul(ab, v[i1][i2]), cmul(anb, v[1 - i1][i2])),
                          cadd(cmul(abn, v[i1][1 - i2]), cmul(anbn, v[1 - i1][1 - i2])));
    const float2 r = cmul(cz, S);
    return r.x;
}

// All four sums S(i1, i2) of post3_value (non-conj side) at once, with
// a[i] = ta(k1 or k1p) and b[i] = tb(k2 or k2p):
//   S(i1, i2) = a Q(i1, i2) + conj(a) Q(1 - i1, i2),
//   Q(i, i2)  = b v[i][i2] + conj(b) v[i][1 - i2]   (b = b[i2], a = a[i1]).
// The conj side (o3 = n3 - k3) sums to conj(S(i1, i2)), so
//   y(o1, o2, k3) = Re(tc[k3] S),  y(o1, o2, n3 - k3) = Re(tc[n3 - k3] conj S).
__device__ __forceinline__ void post3_sums(const float2 (&v)[2][2], const float2 (&a)[2], const float2 (&b)[2],
                                           float2 (&S)[2][2]) {
    float2 Q[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int i2 = 0; i2 < 2; ++i2) {
            const float2 x = v[i][i2], xp = v[i][1 - i2], bb = b[i2];
            Q[i][i2] = make_float2(bb.x * (x.x + xp.x) - bb.y * (x.y - xp.y), bb.x * (x.y + xp.y) + bb.y * (x.x - xp.x));
        }
#pragma unroll
    for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
        for (int i2 = 0; i2 < 2; ++i2) {
            const float2 P = Q[i1][i2], Pp = Q[1 - i1][i2], aa = a[i1];
            S[i1][i2] = make_float2(aa.x * (P.x + Pp.x) - aa.y * (P.y - Pp.y), aa.x * (P.y + Pp.y) + aa.y * (P.x - Pp.x));
        }
}

// ------------------------------------------------------ n1 direction + post
__global__ void __launch_bounds__(kMaxBlock) k3_cols_fwd(Plan3D p, const float2 *__restrict__ ws,
                                                          float *__restrict__ y) {
    extern __shared__ float2 lds[];
    const int C = p.cols1;
    const int C2 = 2 * C;
    const int T = p.f1.T;
    const int sc = threadIdx.x % C2;
    const int t = threadIdx.x / C2;
    const int s = sc / C, c = sc - (sc / C) * C;
    const int W3 = ws3_cols(p);
    const int tiles = (W3 + C - 1) / C;
    const int nunits = (p.n2 / 2 + 1) * tiles;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= nunits) return;
    const Unit3 U = unit3(p, unit);
    const int N1 = p.n1, N2 = p.n2, N3 = p.n3, M3 = p.m3;
    {
        const int k2 = s == 0 ? U.u : U.ubar;
        const int k3 = U.c0 + c;
        const bool act = (t < T) && (k3 < W3);
        float2 v[kSlots3];
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int n1 = t + e * T;
            if (act && n1 < N1) v[e] = ws[((size_t)n1 * N2 + k2) * W3 + k3];
        }
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int n1 = t + e * T;
            if (t < T && n1 < N1) lds[lpad(n1) * C2 + sc] = act ? v[e] : make_float2(0.f, 0.f);
        }
    }
    lds_sync();
    fft_lds<false>(lds + sc, C2, t < T ? t : T, T, p.f1);

    // post: items (k1 pair i, column c) spread over the whole workgroup
    const int items = (N1 / 2 + 1) * C;
    const bool k2self = (U.u == 0) || (2 * U.u == N2);
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int i = it / C, cc = it - (it / C) * C;
        const int k3 = U.c0 + cc;
        if (k3 >= W3) continue;
        const int k1 = i, k1p = (i == 0) ? 0 : N1 - i;
        const bool k1self = (k1 == k1p);
        float2 W[2][2];
        W[0][0] = lds[lpad(k1) * C2 + cc];
        W[1][0] = lds[lpad(k1p) * C2 + cc];
        // when k2 is self-paired the second sequence is the same column
        W[0][1] = lds[lpad(k1) * C2 + C + cc];
        W[1][1] = lds[lpad(k1p) * C2 + C + cc];
        if (k3 == 0 && p.odd) {
            // odd n3: column k3 = 0 alone, self-paired (no n3 - k3 output)
            const float2 c0 = p.tc[0];
            const float2 a[2] = {p.ta[k1], p.ta[k1p]}, b[2] = {p.tb[U.u], p.tb[U.ubar]};
            float2 S[2][2];
            post3_sums(W, a, b, S);
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < 2; ++i2) {
                    if ((i1 == 1 && k1self) || (i2 == 1 && k2self)) continue;
                    const int o1 = i1 ? k1p : k1, o2 = i2 ? U.ubar : U.u;
                    const float2 v = S[i1][i2];
                    out_store(&y[((size_t)o1 * N2 + o2) * N3], c0.x * v.x - c0.y * v.y);
                }
        } else if (k3 == 0) {
            // unpack X(., ., 0) + j X(., ., m3): V0 = (W + conj W(-,-)) / 2, Vm = -j (W - conj W(-,-)) / 2
            float2 V0[2][2], Vm[2][2];
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < 2; ++i2) {
                    const float2 w = W[i1][i2], wn = W[1 - i1][1 - i2];
                    V0[i1][i2] = make_float2(0.5f * (w.x + wn.x), 0.5f * (w.y - wn.y));
                    Vm[i1][i2] = make_float2(0.5f * (w.y + wn.y), -0.5f * (w.x - wn.x));
                }
            const float2 c0 = p.tc[0], cm = p.tc[M3];
            auto put = [&](auto I1, auto I2) {
                constexpr int i1 = decltype(I1)::value, i2 = decltype(I2)::value;
                if ((i1 == 1 && k1self) || (i2 == 1 && k2self)) return;
                const int o1 = i1 ? k1p : k1, o2 = i2 ? U.ubar : U.u;
                const float2 a = p.ta[o1], b = p.tb[o2];
                float *row = y + ((size_t)o1 * N2 + o2) * N3;
                out_store(&row[0], post3_value<i1, i2>(V0, a, b, c0));
                out_store(&row[M3], post3_value<i1, i2>(Vm, a, b, cm));
            };
            put(IC<0>(), IC<0>());
            put(IC<0>(), IC<1>());
            put(IC<1>(), IC<0>());
            put(IC<1>(), IC<1>());
        } else {
            const float2 cf = p.tc[k3], cr = p.tc[N3 - k3];
            const float2 a[2] = {p.ta[k1], p.ta[k1p]}, b[2] = {p.tb[U.u], p.tb[U.ubar]};
            float2 S[2][2];
            post3_sums(W, a, b, S);
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < 2; ++i2) {
                    if ((i1 == 1 && k1self) || (i2 == 1 && k2self)) continue;
                    const int o1 = i1 ? k1p : k1, o2 = i2 ? U.ubar : U.u;
                    float *row = y + ((size_t)o1 * N2 + o2) * N3;
                    const float2 v = S[i1][i2];
                    out_store(&row[k3], cf.x * v.x - cf.y * v.y);
                    out_store(&row[N3 - k3], cr.x * v.x + cr.y * v.y);
                }
        }
    }
}

// ----------------------------------------------------- pre + n1 direction
// LDS staging: float4 per (n1, c) = (y(n1,u,k3), y(n1,u,k3r), y(n1,ub,k3), y(n1,ub,k3r))
// with ub = n2 - u (zero column for u = 0) and k3r = n3 - k3; for k3 = 0 the
// second and fourth entries hold k3 = m3 instead (the packed partner column).
template <int S, bool K3Z, bool SELF3>
__device__ __forceinline__ float2 pre3_value_t(float2 t3, const float4 &F0, const float4 &F1) {
    // Y(a1, a2, a3): a1 selects F0 (row k1) / F1 (row n1 - k1); for sequence S
    // the direct k2 is u (S = 0) or ub (S = 1); a3 = 1 is the k3 reflection.
    // All indices are compile-time, so every Y is a register.
    auto Y = [&](auto A1, auto A2, auto A3) -> float {
        constexpr int a1 = decltype(A1)::value, a2 = decltype(A2)::value, a3 = decltype(A3)::value;
        const float4 &F = a1 ? F1 : F0;
        constexpr int col = (S == 0) ? a2 : 1 - a2;   // 0: u, 1: ub
        if constexpr (K3Z && a3 == 1) return 0.f;     // reflection of k3 = 0 is n3 -> 0
        constexpr int k = SELF3 ? 1 : a3;             // k3 = m3 reflects onto itself (slot 1)
        constexpr int idx = 2 * col + (K3Z ? 0 : k);
        return idx == 0 ? F.x : idx == 1 ? F.y : idx == 2 ? F.z : F.w;
    };
    using I0 = IC<0>;
    using I1 = IC<1>;
    const float re = Y(I0(), I0(), I0()) - (Y(I1(), I1(), I0()) + Y(I1(), I0(), I1()) + Y(I0(), I1(), I1()));
    const float im = -(Y(I1(), I0(), I0()) + Y(I0(), I1(), I0()) + Y(I0(), I0(), I1())) + Y(I1(), I1(), I1());
    return cmul(t3, make_float2(re, im));
}

__device__ __forceinline__ float2 pre3_value(float2 t3, const float4 &F0, const float4 &F1, int s, bool k3zero_side,
                                             bool self3) {
    if (s == 0) {
        if (k3zero_side) return pre3_value_t<0, true, false>(t3, F0, F1);
        return self3 ? pre3_value_t<0, false, true>(t3, F0, F1) : pre3_value_t<0, false, false>(t3, F0, F1);
    }
    if (k3zero_side) return pre3_value_t<1, true, false>(t3, F0, F1);
    return self3 ? pre3_value_t<1, false, true>(t3, F0, F1) : pre3_value_t<1, false, false>(t3, F0, F1);
}

__global__ void __launch_bounds__(kMaxBlock) k3_cols_inv(Plan3D p, const float *__restrict__ x,
                                                          float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    const int C = p.cols1;
    const int C2 = 2 * C;
    const int T = p.f1.T;
    const int sc = threadIdx.x % C2;
    const int t = threadIdx.x / C2;
    const int s = sc / C, c = sc - (sc / C) * C;
    const int W3 = ws3_cols(p);
    const int tiles = (W3 + C - 1) / C;
    const int nunits = (p.n2 / 2 + 1) * tiles;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= nunits) return;
    const Unit3 U = unit3(p, unit);
    const int N1 = p.n1, N2 = p.n2, N3 = p.n3, M3 = p.m3;
    const int k3 = U.c0 + c;
    const bool col_ok = k3 < W3;
    // stage the y values: slot pair (2 float2 = one float4) per (n1, c)
    float4 *stage = reinterpret_cast<float4 *>(lds);
    {
        // threads with s = 0 load the u-column pair, s = 1 the ub-column pair
        const int k3r = (k3 == 0) ? M3 : N3 - k3;
        const bool zero_col = (s == 1 && U.u == 0);
        float va[kSlots3], vb[kSlots3];
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int n1 = t + e * T;
            va[e] = vb[e] = 0.f;
            if (t < T && col_ok && !zero_col && n1 < N1) {
                const float *row = x + ((size_t)n1 * N2 + (s == 0 ? U.u : U.ubar)) * N3;
                va[e] = row[k3];
                vb[e] = row[k3r];
            }
        }
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int n1 = t + e * T;
            if (t < T && n1 < N1) {
                float2 *q = reinterpret_cast<float2 *>(&stage[lpad(n1) * C + c]);
                q[s] = make_float2(va[e], vb[e]);
            }
        }
    }
    lds_sync();
    // X' for sequence s at rows k1 = t + e T
    float2 pre[kSlots3];
    {
        const int k2 = (s == 0) ? U.u : U.ubar;
        const bool seq_ok = col_ok && (t < T) && !(s == 1 && (U.u == 0 || 2 * U.u == N2));
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int k1 = t + e * T;
            pre[e] = make_float2(0.f, 0.f);
            if (seq_ok && k1 < N1) {
                const float4 F0 = stage[lpad(k1) * C + c];
                const float4 F1 = (k1 == 0) ? make_float4(0.f, 0.f, 0.f, 0.f) : stage[lpad(N1 - k1) * C + c];
                const float2 ab = cmul(p.ta[k1], p.tb[k2]);
                if (k3 == 0 && p.odd) {
                    // odd n3: column k3 = 0 alone (its reflection n3 is zero)
                    pre[e] = pre3_value(cmul(ab, p.tc[0]), F0, F1, s, true, false);
                } else if (k3 == 0) {
                    const float2 x0 = pre3_value(cmul(ab, p.tc[0]), F0, F1, s, true, false);
                    const float2 xm = pre3_value(cmul(ab, p.tc[M3]), F0, F1, s, false, true);
                    pre[e] = make_float2(x0.x - xm.y, x0.y + xm.x);   // X'(.,.,0) + j X'(.,.,m3)
                } else {
                    pre[e] = pre3_value(cmul(ab, p.tc[k3]), F0, F1, s, false, false);
                }
            }
        }
    }
    lds_sync();
#pragma unroll
    for (int e = 0; e < kSlots3; ++e) {
        const int n1 = t + e * T;
        if (t < T && n1 < N1) lds[lpad(n1) * C2 + sc] = pre[e];
    }
    lds_sync();
    fft_lds<true>(lds + sc, C2, t < T ? t : T, T, p.f1);
    {
        const int k2 = (s == 0) ? U.u : U.ubar;
        const bool seq_ok = col_ok && (t < T) && !(s == 1 && (U.u == 0 || 2 * U.u == N2));
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int n1 = t + e * T;
            if (seq_ok && n1 < N1) ws[((size_t)n1 * N2 + k2) * W3 + k3] = lds[lpad(n1) * C2 + sc];
        }
    }
}

static inline int round_up8(int v) { return (v + 7) & ~7; }

// ------------------------------------------------------------- plane passes
// Two-pass route for even n3 when an n1-plane's packed half spectrum is small
// (the n1 pass then follows as in the three-pass route).  Forward: workgroup
// (plane a, k3 columns c0 .. c0 + CW): every row b of source plane p1(a) is
// loaded with the Eq. (2d_dct_pre) reorder on all three axes, its length-n3
// real FFT runs as a length-m3 complex FFT plus the even/odd split, and the
// split values of the workgroup's k3 columns go to a column tile in LDS; the
// length-n2 FFTs of those columns then run in the tile and the result is
// written to the workspace rows (a, k2).  The workgroups of one plane share
// its rows through the L2 and repeat the row FFTs (m3 / CW times).
__global__ void __launch_bounds__(kMaxBlock) k3_plane_fwd(Plan3D p, Io io) {
    extern __shared__ float2 lds[];
    const float *__restrict__ x = io_src<float>(io);
    float2 *__restrict__ ws = io_dst<float2>(io);
    const int CW = p.plane_cw, M3 = p.m3, N2 = p.n2, N3 = p.n3;
    const int T3 = p.f3.T, RB = min((int)blockDim.x / T3, N2), RL = lpad_len(M3);
    const int tiles = M3 / CW;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= p.n1 * tiles) return;   // uniform over the workgroup
    const int a = unit / tiles, c0 = (unit - a * tiles) * CW;
    float2 *rows = lds;              // RB rows of RL slots
    float2 *tile = lds + RB * RL;    // lpad_len(n2) x CW
    const int r = threadIdx.x / T3, t = threadIdx.x - r * T3;
    const float *plane = x + (size_t)perm_fwd(a, p.n1) * N2 * N3;
    const bool vec = (N3 & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    for (int b0 = 0; b0 < N2; b0 += RB) {
        const int b = b0 + r;
        const bool active = (r < RB) && (b < N2);
        float2 *base = rows + (r < RB ? r : 0) * RL;
        if (active) {
            const float *srow = plane + (size_t)perm_fwd(b, N2) * N3;
            if (vec) {
                // x[4q .. 4q+3] gives z(q) = (x[4q], x[4q+2]) and z(m3-1-q) = (x[4q+3], x[4q+1])
                const float4 *src = reinterpret_cast<const float4 *>(srow);
                float4 v[kSlots3 / 2];
#pragma unroll
                for (int e = 0; e < kSlots3 / 2; ++e) {
                    const int q = t + e * T3;
                    if (q < M3 / 2) v[e] = src[q];
                }
#pragma unroll
                for (int e = 0; e < kSlots3 / 2; ++e) {
                    const int q = t + e * T3;
                    if (q < M3 / 2) {
                        base[lpad(q)] = make_float2(v[e].x, v[e].z);
                        base[lpad(M3 - 1 - q)] = make_float2(v[e].w, v[e].y);
                    }
                }
            } else {
                // x'(n) = x(p(n)): source element i lands at x' index 2q -> q, 2q + 1 -> n3 - 1 - q
                const float2 *src = reinterpret_cast<const float2 *>(srow);
                float *bf = reinterpret_cast<float *>(base);
                float2 v[kSlots3];
#pragma unroll
                for (int e = 0; e < kSlots3; ++e) {
                    const int q = t + e * T3;
                    if (q < M3) v[e] = src[q];
                }
#pragma unroll
                for (int e = 0; e < kSlots3; ++e) {
                    const int q = t + e * T3;
                    if (q < M3) {
                        bf[xq_off(q)] = v[e].x;
                        bf[xq_off(N3 - 1 - q)] = v[e].y;
                    }
                }
            }
        }
        lds_sync();
        fft_lds<false>(base, 1, active ? t : T3, T3, p.f3);
        if (active) {
            // X(k), k in the tile: X(0) + j X(m3) packed in k = 0
#pragma unroll
            for (int e = 0; e < kSlots3; ++e) {
                const int k = c0 + t + e * T3;
                if (t + e * T3 >= CW) continue;
                const float2 zk = base[lpad(k)];
                float2 xk;
                if (k == 0) {
                    xk = make_float2(zk.x + zk.y, zk.x - zk.y);
                } else {
                    float2 xm;
                    rsplit_pair(zk, base[lpad(M3 - k)], p.split3[k], p.split3[M3 - k], xk, xm);
                }
                tile[lpad(b) * CW + (k - c0)] = xk;
            }
        }
        lds_sync();   // the next rows overwrite the row buffers
    }
    // length-n2 FFTs of the tile's columns
    const int T2 = p.f2.T;
    const int c = threadIdx.x % CW, t2 = threadIdx.x / CW;
    fft_lds<false>(tile + c, CW, t2 < T2 ? t2 : T2, T2, p.f2);
    if (t2 < T2) {
#pragma unroll
        for (int e = 0; e < kSlots3; ++e) {
            const int k2 = t2 + e * T2;
            if (k2 < N2) ws[((size_t)a * N2 + k2) * M3 + c0 + c] = tile[lpad(k2) * CW + c];
        }
    }
}

// Inverse plane pass: workgroup (plane a, n2 rows r0 .. r0 + RW): the inverse
// length-n2 FFTs of all m3 packed columns of the plane (CG columns at a time,
// the workspace written by the inverse n1 pass), rows r0 .. r0 + RW of the
// result kept in a row tile; then per row the inverse split, the inverse
// length-m3 complex FFT and the Eq. (2d_idct_post) inverse reorder on all
// three axes fused into the stores.  The workgroups of one plane repeat the
// column FFTs (n2 / RW times).
__global__ void __launch_bounds__(kMaxBlock) k3_plane_inv(Plan3D p, Io io) {
    extern __shared__ float2 lds[];
    const float2 *__restrict__ ws = io_src<float2>(io);
    float *__restrict__ y = io_dst<float>(io);
    const int RW = p.plane_rw, M3 = p.m3, N2 = p.n2, N3 = p.n3;
    const int T2 = p.f2.T, T3 = p.f3.T, RL = lpad_len(M3);
    const int CG = min((int)blockDim.x / T2, M3);
    const int tiles = N2 / RW;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= p.n1 * tiles) return;   // uniform over the workgroup
    const int a = unit / tiles, r0 = (unit - a * tiles) * RW;
    float2 *colb = lds;                             // lpad_len(n2) x CG
    float2 *rowt = lds + lpad_len(N2) * CG;         // RW rows of RL slots
    const float2 *plane = ws + (size_t)a * N2 * M3;
    {
        const int c = threadIdx.x % CG, t2 = threadIdx.x / CG;
        for (int k0 = 0; k0 < M3; k0 += CG) {
            const int k3 = k0 + c;
            const bool act = t2 < T2 && k3 < M3;
            float2 v[kSlots3];
#pragma unroll
            for (int e = 0; e < kSlots3; ++e) {
                const int k2 = t2 + e * T2;
                if (act && k2 < N2) v[e] = plane[(size_t)k2 * M3 + k3];
            }
#pragma unroll
            for (int e = 0; e < kSlots3; ++e) {
                const int k2 = t2 + e * T2;
                if (t2 < T2 && k2 < N2) colb[lpad(k2) * CG + c] = act ? v[e] : make_float2(0.f, 0.f);
            }
            lds_sync();
            fft_lds<true>(colb + c, CG, t2 < T2 ? t2 : T2, T2, p.f2);
            for (int i = threadIdx.x; i < RW * CG; i += blockDim.x) {
                const int rr = i / CG, cc = i - rr * CG;
                if (k0 + cc < M3) rowt[rr * RL + lpad(k0 + cc)] = colb[lpad(r0 + rr) * CG + cc];
            }
            lds_sync();   // the next columns overwrite the column buffer
        }
    }
    const int RB = (int)blockDim.x / T3;
    const int r = threadIdx.x / T3, t = threadIdx.x - r * T3;
    const int orow0 = perm_fwd(a, p.n1) * N2;
    const bool vec = (N3 & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0;
    for (int rb = 0; rb < RW; rb += RB) {
        const int rr = rb + r;
        const bool active = (r < RB) && (rr < RW);
        float2 *base = rowt + (active ? rr : 0) * RL;
        // inverse split: Z(k) = (U(k) + conj U(m3-k)) + j e^{+2 pi j k/n3} (U(k) - conj U(m3-k)),
        // U(0) = Re P(0), U(m3) = Im P(0)
        float2 zk[kSlots3 / 2 + 1], zm[kSlots3 / 2 + 1];
        if (active) {
#pragma unroll
            for (int i = 0; i < kSlots3 / 2 + 1; ++i) {
                const int k = t + i * T3;
                if (k > M3 / 2) continue;
                if (k == 0) {
                    const float2 p0 = base[0];
                    zk[i] = make_float2(p0.x + p0.y, p0.x - p0.y);
                } else {
                    irsplit_pair(base[lpad(k)], base[lpad(M3 - k)], p.split3[k], p.split3[M3 - k], zk[i], zm[i]);
                }
            }
        }
        lds_sync();
        if (active) {
#pragma unroll
            for (int i = 0; i < kSlots3 / 2 + 1; ++i) {
                const int k = t + i * T3;
                if (k <= M3 / 2) {
                    base[lpad(k)] = zk[i];
                    if (k != 0 && M3 - k != k) base[lpad(M3 - k)] = zm[i];
                }
            }
        }
        lds_sync();
        fft_lds<true>(base, 1, active ? t : T3, T3, p.f3);
        if (active) {
            float *drow = y + (size_t)(orow0 + perm_fwd(r0 + rr, N2)) * N3;
            if (vec) {
                float4 *dst = reinterpret_cast<float4 *>(drow);
#pragma unroll
                for (int e = 0; e < kSlots3 / 2; ++e) {
                    const int q = t + e * T3;
                    if (q < M3 / 2) {
                        const float2 u = base[lpad(q)], w = base[lpad(M3 - 1 - q)];
                        out_store(&dst[q], make_float4(u.x, w.y, u.y, w.x));
                    }
                }
            } else {
                const float *bf = reinterpret_cast<const float *>(base);
                float2 *dst = reinterpret_cast<float2 *>(drow);
#pragma unroll
                for (int e = 0; e < kSlots3; ++e) {
                    const int q = t + e * T3;
                    if (q < M3) out_store(&dst[q], make_float2(bf[xq_off(q)], bf[xq_off(N3 - 1 - q)]));
                }
            }
        }
        lds_sync();   // the next rows' split reads other rows of the tile only; keep rounds apart
    }
}

}  // namespace

size_t plane_fwd_lds(const Plan3D &p) {
    const int RB = std::min(p.plane_block / p.f3.T, p.n2);
    return ((size_t)RB * lpad_len(p.m3) + (size_t)lpad_len(p.n2) * p.plane_cw) * sizeof(float2);
}

size_t plane_inv_lds(const Plan3D &p) {
    const int CG = std::min(p.plane_block / p.f2.T, p.m3);
    return ((size_t)lpad_len(p.n2) * CG + (size_t)p.plane_rw * lpad_len(p.m3)) * sizeof(float2);
}

hipError_t launch_plane3_fwd(const Plan3D &p, const Io &io, hipStream_t s) {
    const size_t lds = plane_fwd_lds(p);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k3_plane_fwd),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int units = p.n1 * (p.m3 / p.plane_cw);
    hipLaunchKernelGGL(k3_plane_fwd, dim3(round_up8(units), io.n), dim3(p.plane_block), lds, s, p, io);
    return hipGetLastError();
}

hipError_t launch_plane3_inv(const Plan3D &p, const Io &io, hipStream_t s) {
    const size_t lds = plane_inv_lds(p);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k3_plane_inv),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int units = p.n1 * (p.n2 / p.plane_rw);
    hipLaunchKernelGGL(k3_plane_inv, dim3(round_up8(units), io.n), dim3(p.plane_block), lds, s, p, io);
    return hipGetLastError();
}

hipError_t launch_dct3_mid(const Plan3D &p, float2 *ws, hipStream_t s) {
    if (p.fast) return launch_fast3_mid(p, ws, s);
    const int C = p.cols2;
    const int units = p.n1 * ((ws3_cols(p) + C - 1) / C);
    const size_t lds = (size_t)lpad_len(p.n2) * C * sizeof(float2);
    if (p.inverse)
        hipLaunchKernelGGL(k3_mid<true>, dim3(round_up8(units)), dim3(C * p.f2.T), lds, s, p, ws);
    else
        hipLaunchKernelGGL(k3_mid<false>, dim3(round_up8(units)), dim3(C * p.f2.T), lds, s, p, ws);
    return hipGetLastError();
}

hipError_t launch_dct3_cols(const Plan3D &p, const float2 *ws, float *y, hipStream_t s) {
    if (p.fast) return launch_fast3_cols(p, ws, y, s);
    const int C = p.cols1;
    const int units = (p.n2 / 2 + 1) * ((ws3_cols(p) + C - 1) / C);
    const size_t lds = (size_t)lpad_len(p.n1) * 2 * C * sizeof(float2);
    hipLaunchKernelGGL(k3_cols_fwd, dim3(round_up8(units)), dim3(2 * C * p.f1.T), lds, s, p, ws, y);
    return hipGetLastError();
}

hipError_t launch_idct3_cols(const Plan3D &p, const float *x, float2 *ws, hipStream_t s) {
    if (p.fast) return launch_fast3_icols(p, x, ws, s);
    const int C = p.cols1;
    const int units = (p.n2 / 2 + 1) * ((ws3_cols(p) + C - 1) / C);
    const size_t lds = (size_t)lpad_len(p.n1) * 2 * C * sizeof(float2);
    hipLaunchKernelGGL(k3_cols_inv, dim3(round_up8(units)), dim3(2 * C * p.f1.T), lds, s, p, x, ws);
    return hipGetLastError();
}

// ===================================================== compile-time kernels
// Power-of-two n1, n2 in [64, 256]: the n2 and n1 FFTs run with compile-time
// schedules (fast_chain.h) instead of the run-time ones; the pre / post
// arithmetic is the same as above.
namespace {

using fast::fft_run;
using fast::kCyclic;
using fast::kMirror;
using fast::kReverse;
using fast::RL;
using fast::StageK;

template <int L> struct F3;
template <> struct F3<256> { using type = RL<16, 16>; static constexpr int T = 16; };
template <> struct F3<128> { using type = RL<8, 16>; static constexpr int T = 8; };
template <> struct F3<64> { using type = RL<8, 8>; static constexpr int T = 4; };
constexpr int kC3 = 16;   // k3 columns per workgroup (128-byte segments)
// Schedules of the n1 pass (k3f_cols / k3f_icols): 8 values per thread up to
// n1 = 128, so that twice the threads of the n2 pass share each column and
// each thread's chain of loads, FFT stages and post items is shorter.
template <int L> struct F3c;
template <> struct F3c<256> { using type = RL<16, 16>; static constexpr int T = 16; };
template <> struct F3c<128> { using type = RL<8, 4, 4>; static constexpr int T = 16; };
template <> struct F3c<64> { using type = RL<8, 8>; static constexpr int T = 8; };

// LDS of the n2 and n1 passes: the column buffers, then the FFT's stage
// twiddles (fast::TwTab layout).
template <int L>
struct MidLds {
    using L_ = typename F3<L>::type;
    static constexpr int TWOFF = kC3 * fast::buf_len<L_>(L);                       // float2, even
    static constexpr size_t bytes = TWOFF * sizeof(float2) + fast::TwTab<L_>::size * sizeof(float4);
    static_assert(TWOFF % 2 == 0, "float4 alignment of the tables");
};
template <int L>
struct ColsLds {
    using L_ = typename F3c<L>::type;
    static constexpr int FFT = 2 * kC3 * fast::buf_len<L_>(L), STG = 2 * L * kC3;   // float2
    static constexpr int TWOFF = FFT > STG ? FFT : STG;                              // even
    static constexpr size_t bytes = TWOFF * sizeof(float2) + fast::TwTab<L_>::size * sizeof(float4);
    static_assert(TWOFF % 2 == 0, "float4 alignment of the tables");
};

// n2 pass: plane a, kC3 columns k3; in place.
template <int L, bool INV>
__device__ __forceinline__ void k3f_mid_b(const Plan3D &p, float2 *__restrict__ ws) {
    using L_ = typename F3<L>::type;
    constexpr int T = F3<L>::T, C = kC3;
    using S0 = StageK<L_, L, T, 0, kCyclic, kCyclic>;
    using SL = StageK<L_, L, T, L_::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int tiles = (p.m3 + C - 1) / C;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= p.n1 * tiles) return;
    const int a = unit / tiles;
    const int k3 = (unit - a * tiles) * C + c;
    const bool act = k3 < p.m3;
    float2 *plane = ws + (size_t)a * p.n2 * p.m3;
    fast::TwCopy<L_, T * C> twc;
    twc.fetch(p.f2f);
    float2 v0[S0::NB][S0::R];
#pragma unroll
    for (int b = 0; b < S0::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < S0::R; ++rr) {
            const int r = t + (b + rr * S0::NB) * T;
            v0[b][rr] = act ? plane[(size_t)r * p.m3 + k3] : make_float2(0.f, 0.f);
        }
    float4 *tab = reinterpret_cast<float4 *>(lds + MidLds<L>::TWOFF);
    twc.store(tab);   // published by the FFT's first barrier
    float2 v[SL::NB][SL::R];
    fft_run<L_, L, T, kCyclic, kCyclic, INV>(lds, C, c, t, v0, v, p.f2f, fast::TwTab<L_>::view(tab));
    if (!act) return;
#pragma unroll
    for (int b = 0; b < SL::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < SL::R; ++rr) plane[(size_t)(t + (b + rr * SL::NB) * T) * p.m3 + k3] = v[b][rr];
}
template <int L, bool INV>
__global__ void __launch_bounds__(F3<L>::T * kC3) k3f_mid(Plan3D p, Io io) {
    k3f_mid_b<L, INV>(p, io_dst<float2>(io));
}

// n1 pass + post: unit (u, kC3 columns k3); half s of the workgroup runs the
// FFT of column (u or n2 - u, k3) into its own buffer, the results go back in
// natural order, and the post reads V(+-k1, u / n2-u, k3) from both buffers.
template <int L>
__device__ __forceinline__ void k3f_cols_b(const Plan3D &p, const float2 *__restrict__ ws, float *__restrict__ y) {
    using L_ = typename F3c<L>::type;
    constexpr int T = F3c<L>::T, C = kC3, BUF = fast::buf_len<L_>(L);
    using S0 = StageK<L_, L, T, 0, kCyclic, kCyclic>;
    using SL = StageK<L_, L, T, L_::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int s = threadIdx.x / (C * T), ht = threadIdx.x % (C * T);
    const int c = ht % C, t = ht / C;
    const int tiles = (p.m3 + C - 1) / C;
    const int nunits = (p.n2 / 2 + 1) * tiles;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= nunits) return;
    const int N1 = p.n1, N2 = p.n2, N3 = p.n3, M3 = p.m3;
    const int u = unit / tiles, c0 = (unit - u * tiles) * C;
    const int ubar = (u == 0) ? 0 : N2 - u;
    const int k2 = s == 0 ? u : ubar;
    float2 *buf = lds + s * C * BUF;
    // the post's factors, fetched before the FFT so that their latency
    // overlaps it: tb of the two columns (the workgroup's), tc of the thread's
    // post column (the same in every post item of the thread, since the block
    // size is a multiple of C), ta of the rows of each post item
    constexpr int NTH = 2 * T * C, ITEMS = (L / 2 + 1) * C, NIT = (ITEMS + NTH - 1) / NTH;
    static_assert(NTH % C == 0, "one post column per thread");
    const int pc = threadIdx.x % C, pk3 = c0 + pc;
    const float2 tbu = p.tb[u], tbb = p.tb[ubar];
    const float2 cf = p.tc[pk3 < M3 ? pk3 : 0], cr = p.tc[pk3 < M3 && pk3 != 0 ? N3 - pk3 : M3];
    float2 tak[NIT], tap[NIT];
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int i = (threadIdx.x + j * NTH) / C;
        const int k1 = i <= L / 2 ? i : 0, k1p = (k1 == 0) ? 0 : N1 - k1;
        tak[j] = p.ta[k1];
        tap[j] = p.ta[k1p];
    }
    fast::TwCopy<L_, NTH> twc;
    twc.fetch(p.f1f);
    float4 *tab = reinterpret_cast<float4 *>(lds + ColsLds<L>::TWOFF);
    {
        const int k3 = c0 + c;
        const bool act = k3 < M3;
        float2 v0[S0::NB][S0::R];
#pragma unroll
        for (int b = 0; b < S0::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < S0::R; ++rr) {
                const int n1 = t + (b + rr * S0::NB) * T;
                v0[b][rr] = act ? ws[((size_t)n1 * N2 + k2) * M3 + k3] : make_float2(0.f, 0.f);
            }
        twc.store(tab);   // published by the FFT's first barrier
        float2 v[SL::NB][SL::R];
        fft_run<L_, L, T, kCyclic, kCyclic, false>(buf, C, c, t, v0, v, p.f1f, fast::TwTab<L_>::view(tab));
        lds_sync();   // the last stage has read its inputs
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) buf[(t + (b + rr * SL::NB) * T) * C + c] = v[b][rr];
    }
    lds_sync();
    const float2 *b0 = lds, *b1 = lds + C * BUF;
    const bool k2self = (u == 0) || (2 * u == N2);
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int it = threadIdx.x + j * NTH;
        if (it >= ITEMS) continue;
        const int i = it / C, cc = pc;
        const int k3 = pk3;
        if (k3 >= M3) continue;
        const int k1 = i, k1p = (i == 0) ? 0 : N1 - i;
        const bool k1self = (k1 == k1p);
        float2 W[2][2];
        W[0][0] = b0[k1 * C + cc];
        W[1][0] = b0[k1p * C + cc];
        W[0][1] = b1[k1 * C + cc];
        W[1][1] = b1[k1p * C + cc];
        if (k3 == 0) {
            float2 V0[2][2], Vm[2][2];
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < 2; ++i2) {
                    const float2 w = W[i1][i2], wn = W[1 - i1][1 - i2];
                    V0[i1][i2] = make_float2(0.5f * (w.x + wn.x), 0.5f * (w.y - wn.y));
                    Vm[i1][i2] = make_float2(0.5f * (w.y + wn.y), -0.5f * (w.x - wn.x));
                }
            const float2 cz = cf, cm = cr;   // tc(0) and tc(m3) for the packed column
            auto put = [&](auto I1, auto I2) {
                constexpr int i1 = decltype(I1)::value, i2 = decltype(I2)::value;
                if ((i1 == 1 && k1self) || (i2 == 1 && k2self)) return;
                const int o1 = i1 ? k1p : k1, o2 = i2 ? ubar : u;
                const float2 a = i1 ? tap[j] : tak[j], b = i2 ? tbb : tbu;
                float *row = y + ((size_t)o1 * N2 + o2) * N3;
                out_store(&row[0], post3_value<i1, i2>(V0, a, b, cz));
                out_store(&row[M3], post3_value<i1, i2>(Vm, a, b, cm));
            };
            put(IC<0>(), IC<0>());
            put(IC<0>(), IC<1>());
            put(IC<1>(), IC<0>());
            put(IC<1>(), IC<1>());
        } else {
            const float2 a[2] = {tak[j], tap[j]}, b[2] = {tbu, tbb};
            float2 S[2][2];
            post3_sums(W, a, b, S);
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < 2; ++i2) {
                    if ((i1 == 1 && k1self) || (i2 == 1 && k2self)) continue;
                    const int o1 = i1 ? k1p : k1, o2 = i2 ? ubar : u;
                    float *row = y + ((size_t)o1 * N2 + o2) * N3;
                    const float2 v = S[i1][i2];
                    out_store(&row[k3], cf.x * v.x - cf.y * v.y);
                    out_store(&row[N3 - k3], cr.x * v.x + cr.y * v.y);
                }
        }
    }
}
template <int L>
__global__ void __launch_bounds__(2 * F3c<L>::T * kC3) k3f_cols(Plan3D p, Io io) {
    k3f_cols_b<L>(p, io_src<float2>(io), io_dst<float>(io));
}

// pre + n1 inverse FFT: y values staged in LDS as float4 per (n1, c) =
// (y(n1,u,k3), y(n1,u,k3r), y(n1,ub,k3), y(n1,ub,k3r)) in natural order; half s
// builds the pre values of sequence s in its stage-0 slots, then (after a
// barrier, the LDS reused) runs the inverse FFT.
template <int L>
__device__ __forceinline__ void k3f_icols_b(const Plan3D &p, const float *__restrict__ x, float2 *__restrict__ ws) {
    using L_ = typename F3c<L>::type;
    constexpr int T = F3c<L>::T, C = kC3, BUF = fast::buf_len<L_>(L);
    using S0 = StageK<L_, L, T, 0, kCyclic, kCyclic>;
    using SL = StageK<L_, L, T, L_::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int s = threadIdx.x / (C * T), ht = threadIdx.x % (C * T);
    const int c = ht % C, t = ht / C;
    const int tiles = (p.m3 + C - 1) / C;
    const int nunits = (p.n2 / 2 + 1) * tiles;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= nunits) return;
    const int N1 = p.n1, N2 = p.n2, N3 = p.n3, M3 = p.m3;
    const int u = unit / tiles, c0 = (unit - u * tiles) * C;
    const int ubar = (u == 0) ? 0 : N2 - u;
    const int k3 = c0 + c;
    const bool col_ok = k3 < M3;
    float4 *stage = reinterpret_cast<float4 *>(lds);
    const int k2 = (s == 0) ? u : ubar;
    const bool seq_ok = col_ok && !(s == 1 && (u == 0 || 2 * u == N2));
    // the pre's factors, fetched ahead of the staging barrier: tb(k2) tc(k3)
    // is the same for all of the thread's values (tc(0) and tc(m3) for the
    // packed column k3 = 0), ta(k1) one per value
    const float2 tbk = p.tb[k2];
    const float2 bc = cmul(tbk, p.tc[k3 == 0 ? 0 : (k3 < M3 ? k3 : 0)]), bcm = cmul(tbk, p.tc[M3]);
    float2 tav[S0::NB][S0::R];
#pragma unroll
    for (int b = 0; b < S0::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < S0::R; ++rr) tav[b][rr] = p.ta[t + (b + rr * S0::NB) * T];
    fast::TwCopy<L_, 2 * C * T> twc;
    twc.fetch(p.f1f);
    float4 *tab = reinterpret_cast<float4 *>(lds + ColsLds<L>::TWOFF);
    {
        const int k3r = (k3 == 0) ? M3 : N3 - k3;
        const bool zero_col = (s == 1 && u == 0);
        const int col = s == 0 ? u : ubar;
        // all loads of the thread in flight before the first store (n1 = L here);
        // rows t + e T are a fixed stride apart
        float2 vv[L / T];
        const float *row0 = x + ((size_t)t * N2 + col) * N3;
        const size_t rstep = (size_t)T * N2 * N3;
#pragma unroll
        for (int e = 0; e < L / T; ++e) {
            vv[e] = make_float2(0.f, 0.f);
            if (col_ok && !zero_col) {
                const float *row = row0 + e * rstep;
                vv[e] = make_float2(row[k3], row[k3r]);
            }
        }
#pragma unroll
        for (int e = 0; e < L / T; ++e) reinterpret_cast<float2 *>(&stage[(t + e * T) * C + c])[s] = vv[e];
        twc.store(tab);
    }
    lds_sync();
    float2 v0[S0::NB][S0::R];
    // s is uniform over each half (whole wavefronts): one branch per half
    auto fill = [&](auto SS) {
        constexpr int S_ = decltype(SS)::value;
#pragma unroll
        for (int b = 0; b < S0::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < S0::R; ++rr) {
                const int k1 = t + (b + rr * S0::NB) * T;
                float2 pv = make_float2(0.f, 0.f);
                if (seq_ok) {
                    const float4 F0 = stage[k1 * C + c];
                    const float4 F1 = (k1 == 0) ? make_float4(0.f, 0.f, 0.f, 0.f) : stage[(N1 - k1) * C + c];
                    const float2 a = tav[b][rr];
                    if (k3 == 0) {
                        const float2 x0 = pre3_value_t<S_, true, false>(cmul(a, bc), F0, F1);
                        const float2 xm = pre3_value_t<S_, false, true>(cmul(a, bcm), F0, F1);
                        pv = make_float2(x0.x - xm.y, x0.y + xm.x);
                    } else {
                        pv = pre3_value_t<S_, false, false>(cmul(a, bc), F0, F1);
                    }
                }
                v0[b][rr] = pv;
            }
    };
    static_assert((C * T) % 64 == 0, "each half is whole wavefronts");
    if (s == 0)
        fill(IC<0>());
    else
        fill(IC<1>());
    float2 *buf = lds + s * C * BUF;
    float2 v[SL::NB][SL::R];
    fft_run<L_, L, T, kCyclic, kCyclic, true>(buf, C, c, t, v0, v, p.f1f,
                                             fast::TwTab<L_>::view(tab));   // barrier before its first write
    if (!seq_ok) return;
#pragma unroll
    for (int b = 0; b < SL::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < SL::R; ++rr) {
            const int n1 = t + (b + rr * SL::NB) * T;
            ws[((size_t)n1 * N2 + k2) * M3 + k3] = v[b][rr];
        }
}
template <int L>
__global__ void __launch_bounds__(2 * F3c<L>::T * kC3) k3f_icols(Plan3D p, Io io) {
    k3f_icols_b<L>(p, io_src<float>(io), io_dst<float2>(io));
}

// ---------------------------------------------------- compile-time plane pass
// Two-pass route for the small power-of-two planes (packed half-spectrum plane
// of n2 x m3 complex values, m3 = n3 / 2, in LDS): one workgroup per n1-plane.
//   forward : phase 1, thread (b, t) of row b loads row p2(b) of source plane
//             p1(a) with 16-byte loads (the Eq. 2d_dct_pre reorder on all three
//             axes, kReverse first stage), runs the length-m3 complex FFT in
//             its row's exchange buffer (wavefront barriers: T3 divides 64) and
//             the even/odd split (kMirror last stage: X(k) and X(m3 - k) in one
//             thread); after a workgroup barrier (the plane aliases the row
//             buffers) the split values go to plane row b, X(0) + j X(m3)
//             packed in column 0.  Phase 2, thread (c, t) runs the length-n2
//             FFT of plane column c with the plane as its exchange buffer (row
//             pitch P) and writes workspace row (a, k2) with whole-row stores.
//   inverse : the mirror order: the inverse n2 FFTs of the plane's columns
//             (the workspace written by the inverse n1 pass), then per row the
//             inverse split (kMirror first stage), the inverse m3 FFT and the
//             Eq. (2d_idct_post) inverse reorder as 16-byte stores (kReverse).
// Same arithmetic as the row kernel plus the n2 kernel it replaces.
template <int N2, int M3> struct FPlane;
template <> struct FPlane<128, 64> { using R3 = RL<4, 4, 4>; static constexpr int T3 = 8; };
template <> struct FPlane<128, 32> { using R3 = RL<4, 4, 2>; static constexpr int T3 = 4; };
template <> struct FPlane<64, 64> { using R3 = RL<4, 4, 4>; static constexpr int T3 = 8; };
template <> struct FPlane<64, 32> { using R3 = RL<4, 4, 2>; static constexpr int T3 = 4; };

template <int N2, int M3>
struct FPlaneGeo {
    using R3 = typename FPlane<N2, M3>::R3;
    using R2 = typename F3c<N2>::type;
    static constexpr int T3 = FPlane<N2, M3>::T3, T2 = F3c<N2>::T;
    static constexpr int NTH = N2 * T3;                 // one row per T3 threads
    static constexpr int P = M3 + 1;                    // plane row pitch (complex)
    static constexpr int RB3 = fast::buf_len<R3>(M3);   // row exchange buffer
    static constexpr int SLOTS2 = fast::buf_len<R2>(N2);
    // tables after the plane / row buffers: the two FFTs' stage twiddles
    // (LdsTw layout) and the split factors exp(-2 pi j k / n3), k <= m3
    static constexpr int TWOFF = ((SLOTS2 * P > N2 * RB3 ? SLOTS2 * P : N2 * RB3) + 1) & ~1;   // float2
    static constexpr int TW3 = fast::TwTab<R3>::size, TW2 = fast::TwTab<R2>::size;        // float4
    static constexpr int SPW = (M3 + 2) / 2;                                                // float4
    static constexpr int NW = TW3 + TW2 + SPW, NTV = (NW + NTH - 1) / NTH;
    static constexpr size_t LDS = ((size_t)TWOFF + 2 * (size_t)NW) * sizeof(float2);
    static_assert(NTH == M3 * T2, "both phases use every thread");
    static_assert(NTH <= 1024 && NTH % 64 == 0, "whole wavefronts");
    static_assert(64 % T3 == 0, "each row FFT lies inside one wavefront");
};

// The plane kernels' tables: every thread fetches its words (before the
// kernel's data loads, so that waiting for them does not wait for the data)
// and later stores them to LDS.  Words past the tables go to the start of the
// plane, which is written only after a workgroup barrier that follows.
template <class G>
__device__ __forceinline__ void plane_tabs_fetch(const Plan3D &p, float4 (&tv)[G::NTV]) {
#pragma unroll
    for (int i = 0; i < G::NTV; ++i) {
        const int d = threadIdx.x + i * G::NTH;
        const float4 *src;
        if (d < G::TW3)
            src = fast::TwTab<typename G::R3>::src(p.f3f, d);
        else if (d < G::TW3 + G::TW2)
            src = fast::TwTab<typename G::R2>::src(p.f2c, d - G::TW3);
        else
            src = reinterpret_cast<const float4 *>(p.split3) + min(d - G::TW3 - G::TW2, G::SPW - 1);
        tv[i] = *src;
    }
}
template <class G>
__device__ __forceinline__ void plane_tabs_store(float2 *lds, const float4 (&tv)[G::NTV]) {
    float4 *tab = reinterpret_cast<float4 *>(lds + G::TWOFF);
#pragma unroll
    for (int i = 0; i < G::NTV; ++i) {
        const int d = threadIdx.x + i * G::NTH;
        float4 *dst = d < G::NW ? tab + d : reinterpret_cast<float4 *>(lds) + (d - G::NW);
        *dst = tv[i];
    }
}

template <int N2, int M3>
__device__ __forceinline__ void k3f_plane_fwd_b(const Plan3D &p, const float *__restrict__ x,
                                                float2 *__restrict__ ws) {
    using G = FPlaneGeo<N2, M3>;
    using R3 = typename G::R3;
    using R2 = typename G::R2;
    constexpr int T3 = G::T3, T2 = G::T2, P = G::P, N3 = 2 * M3;
    using A0 = StageK<R3, M3, T3, 0, kReverse, kMirror>;
    using AL = StageK<R3, M3, T3, R3::n - 1, kReverse, kMirror>;
    using B0 = StageK<R2, N2, T2, 0, kCyclic, kCyclic>;
    using BL = StageK<R2, N2, T2, R2::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int a = xcd_tile(blockIdx.x, gridDim.x);
    if (a >= p.n1) return;   // whole workgroup
    float4 tv[G::NTV];
    plane_tabs_fetch<G>(p, tv);
    const float4 *tabs = reinterpret_cast<const float4 *>(lds + G::TWOFF);
    const fast::LdsTw tw3 = fast::TwTab<R3>::view(tabs), tw2 = fast::TwTab<R2>::view(tabs + G::TW3);
    const float2 *split = reinterpret_cast<const float2 *>(tabs + G::TW3 + G::TW2);
    {
        const int b = threadIdx.x / T3, t = threadIdx.x % T3;
        const float4 *src =
            reinterpret_cast<const float4 *>(x + ((size_t)perm_fwd(a, p.n1) * N2 + perm_fwd(b, N2)) * N3);
        // float4 j + r Nb of the row holds z(q) (input r of slot j) and z(m3-1-q)
        float2 v0[A0::NB][A0::R];
        constexpr int H0 = A0::NB / 2;
#pragma unroll
        for (int s = 0; s < A0::NB; ++s) {
            const int ps = s < H0 ? s + H0 : s - H0;
#pragma unroll
            for (int rr = 0; rr < A0::R / 2; ++rr) {
                const float4 f = nt_load4(src + A0::j(t, s) + rr * A0::Nb);   // input read once
                v0[s][rr] = make_float2(f.x, f.z);
                v0[ps][A0::R - 1 - rr] = make_float2(f.w, f.y);
            }
        }
        plane_tabs_store<G>(lds, tv);
        lds_sync();   // the tables are in LDS (the row loads stay in flight)
        constexpr int H = AL::NB / 2, R = AL::R, Nb = AL::Nb;
        // the split factors of the thread's pairs, read ahead of the FFT
        float2 wsp[H][R], wsh[R / 2];
#pragma unroll
        for (int s = 0; s < H; ++s)
#pragma unroll
            for (int rr = 0; rr < R; ++rr) wsp[s][rr] = split[AL::j(t, s) + rr * Nb];
#pragma unroll
        for (int rr = 0; rr < R / 2; ++rr) wsh[rr] = split[Nb / 2 + rr * Nb];
        float2 v2[AL::NB][AL::R];
        fft_run<R3, M3, T3, kReverse, kMirror, false, true>(lds + b * G::RB3, 1, 0, t, v0, v2, p.f3f, tw3);
        lds_sync();   // every row FFT has read its buffer: the plane overwrites them
        float2 *row = lds + b * P;
        auto sp = [&](int k, float2 wk, float2 zk, float2 zm) {
            float2 xk, xm;
            rsplit_pair(zk, zm, wk, make_float2(-wk.x, wk.y), xk, xm);
            row[k] = xk;
            if (M3 - k != k) row[M3 - k] = xm;
        };
#pragma unroll
        for (int s = 0; s < H; ++s) {
            const int jj = AL::j(t, s);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int k = jj + rr * Nb;
                if (s == 0 && t == 0) {
                    if (rr > R / 2) continue;
                    if (rr == 0) {
                        const float2 z0 = v2[0][0];
                        row[0] = make_float2(z0.x + z0.y, z0.x - z0.y);   // X(0) + j X(m3)
                        continue;
                    }
                    sp(k, wsp[0][rr], v2[0][rr], v2[0][R - rr]);
                } else {
                    sp(k, wsp[s][rr], v2[s][rr], v2[s + H][R - 1 - rr]);
                }
            }
        }
        if (t == 0) {
#pragma unroll
            for (int rr = 0; rr < R / 2; ++rr) sp(Nb / 2 + rr * Nb, wsh[rr], v2[H][rr], v2[H][R - 1 - rr]);
        }
    }
    lds_sync();
    {
        const int c = threadIdx.x % M3, t = threadIdx.x / M3;
        float2 v0[B0::NB][B0::R];
#pragma unroll
        for (int s = 0; s < B0::NB; ++s)
#pragma unroll
            for (int rr = 0; rr < B0::R; ++rr) v0[s][rr] = lds[(t + (s + rr * B0::NB) * T2) * P + c];
        float2 v[BL::NB][BL::R];
        fft_run<R2, N2, T2, kCyclic, kCyclic, false>(lds, P, c, t, v0, v, p.f2c, tw2);   // barrier before its first write
        float2 *out = ws + (size_t)a * N2 * M3 + c;
#pragma unroll
        for (int s = 0; s < BL::NB; ++s)
#pragma unroll
            for (int rr = 0; rr < BL::R; ++rr) out[(size_t)(t + (s + rr * BL::NB) * T2) * M3] = v[s][rr];
    }
}

template <int N2, int M3>
__device__ __forceinline__ void k3f_plane_inv_b(const Plan3D &p, const float2 *__restrict__ ws,
                                                float *__restrict__ y) {
    using G = FPlaneGeo<N2, M3>;
    using R3 = typename G::R3;
    using R2 = typename G::R2;
    constexpr int T3 = G::T3, T2 = G::T2, P = G::P, N3 = 2 * M3;
    using A0 = StageK<R3, M3, T3, 0, kMirror, kReverse>;
    using AL = StageK<R3, M3, T3, R3::n - 1, kMirror, kReverse>;
    using B0 = StageK<R2, N2, T2, 0, kCyclic, kCyclic>;
    using BL = StageK<R2, N2, T2, R2::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int a = xcd_tile(blockIdx.x, gridDim.x);
    if (a >= p.n1) return;   // whole workgroup
    float4 tv[G::NTV];
    plane_tabs_fetch<G>(p, tv);
    const float4 *tabs = reinterpret_cast<const float4 *>(lds + G::TWOFF);
    const fast::LdsTw tw3 = fast::TwTab<R3>::view(tabs), tw2 = fast::TwTab<R2>::view(tabs + G::TW3);
    const float2 *split = reinterpret_cast<const float2 *>(tabs + G::TW3 + G::TW2);
    {
        const int c = threadIdx.x % M3, t = threadIdx.x / M3;
        const float2 *in = ws + (size_t)a * N2 * M3 + c;
        float2 v0[B0::NB][B0::R];
#pragma unroll
        for (int s = 0; s < B0::NB; ++s)
#pragma unroll
            for (int rr = 0; rr < B0::R; ++rr) v0[s][rr] = in[(size_t)(t + (s + rr * B0::NB) * T2) * M3];
        plane_tabs_store<G>(lds, tv);   // published by the FFT's first barrier
        float2 v[BL::NB][BL::R];
        fft_run<R2, N2, T2, kCyclic, kCyclic, true>(lds, P, c, t, v0, v, p.f2c, tw2);
        lds_sync();   // the last stage has read its inputs
#pragma unroll
        for (int s = 0; s < BL::NB; ++s)
#pragma unroll
            for (int rr = 0; rr < BL::R; ++rr) lds[(t + (s + rr * BL::NB) * T2) * P + c] = v[s][rr];
    }
    lds_sync();
    const int b = threadIdx.x / T3, t = threadIdx.x % T3;
    // inverse split on the pairs (k, m3 - k) of plane row b: Z(k) from U(k),
    // U(m3 - k), with U(0) = Re P(0), U(m3) = Im P(0) packed in column 0
    float2 v0[A0::NB][A0::R];
    {
        const float2 *row = lds + b * P;
        constexpr int H = A0::NB / 2, R = A0::R, Nb = A0::Nb;
        auto isp = [&](int k, float2 &zk, float2 &zm) {
            if (k == 0) {
                const float2 p0 = row[0];
                zk = zm = make_float2(p0.x + p0.y, p0.x - p0.y);
                return;
            }
            const float2 wk = split[k];
            irsplit_pair(row[k], row[M3 - k], wk, make_float2(-wk.x, wk.y), zk, zm);
        };
#pragma unroll
        for (int s = 0; s < H; ++s) {
            const int jj = A0::j(t, s);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int k = jj + rr * Nb;
                float2 f, g;
                if (s == 0 && t == 0) {
                    if (rr > R / 2) continue;
                    isp(k, f, g);
                    v0[0][rr] = f;
                    if (rr != 0 && rr != R / 2) v0[0][(R - rr) % R] = g;
                } else {
                    isp(k, f, g);
                    v0[s][rr] = f;
                    v0[s + H][R - 1 - rr] = g;
                }
            }
        }
        if (t == 0) {
#pragma unroll
            for (int rr = 0; rr < R / 2; ++rr) {
                float2 f, g;
                isp(Nb / 2 + rr * Nb, f, g);
                v0[H][rr] = f;
                v0[H][R - 1 - rr] = g;
            }
        }
    }
    lds_sync();   // every row has read the plane: the row buffers overwrite it
    float2 v2[AL::NB][AL::R];
    fft_run<R3, M3, T3, kMirror, kReverse, true, true>(lds + b * G::RB3, 1, 0, t, v0, v2, p.f3f, tw3);
    // Eq. (2d_idct_post) on all three axes: output float4 q = j + r Nb of row
    // p2(b) of plane p1(a) is (z(q).x, z(m3-1-q).y, z(q).y, z(m3-1-q).x)
    float4 *dst = reinterpret_cast<float4 *>(y + ((size_t)perm_fwd(a, p.n1) * N2 + perm_fwd(b, N2)) * N3);
    constexpr int H2 = AL::NB / 2;
#pragma unroll
    for (int s = 0; s < AL::NB; ++s) {
        const int jj = AL::j(t, s);
        const int ps = s < H2 ? s + H2 : s - H2;
#pragma unroll
        for (int rr = 0; rr < AL::R / 2; ++rr) {
            const float2 u = v2[s][rr], m = v2[ps][AL::R - 1 - rr];
            nt_store4(dst + jj + rr * AL::Nb, make_float4(u.x, m.y, u.y, m.x));   // output written once
        }
    }
}

template <int N2, int M3>
__global__ void __launch_bounds__((FPlaneGeo<N2, M3>::NTH)) k3f_plane_fwd(Plan3D p, Io io) {
    k3f_plane_fwd_b<N2, M3>(p, io_src<float>(io), io_dst<float2>(io));
}
template <int N2, int M3>
__global__ void __launch_bounds__((FPlaneGeo<N2, M3>::NTH)) k3f_plane_inv(Plan3D p, Io io) {
    k3f_plane_inv_b<N2, M3>(p, io_src<float2>(io), io_dst<float>(io));
}

template <class K>
inline void set_lds3(K kernel, size_t bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int L>
hipError_t mid_n(const Plan3D &p, const Io &io, hipStream_t s) {
    constexpr int T = F3<L>::T, C = kC3;
    const size_t lds = MidLds<L>::bytes;
    const int units = p.n1 * ((p.m3 + C - 1) / C);
    if (p.inverse)
        hipLaunchKernelGGL((k3f_mid<L, true>), dim3(round_up8(units), io.n), dim3(T * C), lds, s, p, io);
    else
        hipLaunchKernelGGL((k3f_mid<L, false>), dim3(round_up8(units), io.n), dim3(T * C), lds, s, p, io);
    return hipGetLastError();
}

template <int L>
hipError_t cols_n(const Plan3D &p, const Io &io, hipStream_t s) {
    constexpr int T = F3c<L>::T, C = kC3;
    const size_t lds = ColsLds<L>::bytes;
    set_lds3(k3f_cols<L>, lds);
    const int units = (p.n2 / 2 + 1) * ((p.m3 + C - 1) / C);
    hipLaunchKernelGGL(k3f_cols<L>, dim3(round_up8(units), io.n), dim3(2 * T * C), lds, s, p, io);
    return hipGetLastError();
}

template <int L>
hipError_t icols_n(const Plan3D &p, const Io &io, hipStream_t s) {
    constexpr int T = F3c<L>::T, C = kC3;
    const size_t lds = ColsLds<L>::bytes;
    set_lds3(k3f_icols<L>, lds);
    const int units = (p.n2 / 2 + 1) * ((p.m3 + C - 1) / C);
    hipLaunchKernelGGL(k3f_icols<L>, dim3(round_up8(units), io.n), dim3(2 * T * C), lds, s, p, io);
    return hipGetLastError();
}

template <class L_>
int copy_rad3(int *rad) {
    for (int i = 0; i < L_::n; ++i) rad[i] = L_::r[i];
    return L_::n;
}

template <int N2, int M3>
hipError_t fplane_n(const Plan3D &p, const Io &io, hipStream_t s) {
    using G = FPlaneGeo<N2, M3>;
    const dim3 grid(round_up8(p.n1), io.n);
    if (p.inverse) {
        set_lds3(k3f_plane_inv<N2, M3>, G::LDS);
        hipLaunchKernelGGL((k3f_plane_inv<N2, M3>), grid, dim3(G::NTH), G::LDS, s, p, io);
    } else {
        set_lds3(k3f_plane_fwd<N2, M3>, G::LDS);
        hipLaunchKernelGGL((k3f_plane_fwd<N2, M3>), grid, dim3(G::NTH), G::LDS, s, p, io);
    }
    return hipGetLastError();
}

}  // namespace

bool fplane3_supported(int n2, int m3) { return (n2 == 64 || n2 == 128) && (m3 == 32 || m3 == 64); }

size_t fplane3_lds(int n2, int m3) {
    if (n2 == 128) return m3 == 64 ? FPlaneGeo<128, 64>::LDS : FPlaneGeo<128, 32>::LDS;
    if (n2 == 64) return m3 == 64 ? FPlaneGeo<64, 64>::LDS : FPlaneGeo<64, 32>::LDS;
    return 0;
}

int fplane3_radices(int m3, int *rad) {
    if (m3 == 64) return copy_rad3<FPlane<128, 64>::R3>(rad);
    if (m3 == 32) return copy_rad3<FPlane<128, 32>::R3>(rad);
    return 0;
}

hipError_t launch_fplane3(const Plan3D &p, const Io &io, hipStream_t s) {
    if (p.n2 == 128 && p.m3 == 64) return fplane_n<128, 64>(p, io, s);
    if (p.n2 == 128 && p.m3 == 32) return fplane_n<128, 32>(p, io, s);
    if (p.n2 == 64 && p.m3 == 64) return fplane_n<64, 64>(p, io, s);
    if (p.n2 == 64 && p.m3 == 32) return fplane_n<64, 32>(p, io, s);
    return hipErrorInvalidValue;
}

bool fast3_supported(int n) { return n == 64 || n == 128 || n == 256; }

int fast3c_radices(int n, int *rad) {
    switch (n) {
        case 256: return copy_rad3<F3c<256>::type>(rad);
        case 128: return copy_rad3<F3c<128>::type>(rad);
        case 64: return copy_rad3<F3c<64>::type>(rad);
    }
    return 0;
}

int fast3_radices(int n, int *rad) {
    switch (n) {
        case 256: return copy_rad3<F3<256>::type>(rad);
        case 128: return copy_rad3<F3<128>::type>(rad);
        case 64: return copy_rad3<F3<64>::type>(rad);
    }
    return 0;
}

hipError_t launch_fast3_mid(const Plan3D &p, const Io &io, hipStream_t s) {
    switch (p.n2) {
        case 256: return mid_n<256>(p, io, s);
        case 128: return mid_n<128>(p, io, s);
        case 64: return mid_n<64>(p, io, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fast3_cols(const Plan3D &p, const Io &io, hipStream_t s) {
    switch (p.n1) {
        case 256: return cols_n<256>(p, io, s);
        case 128: return cols_n<128>(p, io, s);
        case 64: return cols_n<64>(p, io, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fast3_icols(const Plan3D &p, const Io &io, hipStream_t s) {
    switch (p.n1) {
        case 256: return icols_n<256>(p, io, s);
        case 128: return icols_n<128>(p, io, s);
        case 64: return icols_n<64>(p, io, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace dctx
