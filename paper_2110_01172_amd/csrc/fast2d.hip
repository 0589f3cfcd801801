// Fast path of the 2-D three-stage DCT-II / DCT-III for power-of-two sizes:
// compile-time FFT schedules (fast_core.h) with the pre- and post-processing
// done in registers by the paired butterfly maps.
//
// Forward (Alg. alg:DCT, "2D_DCT"):
//   rows    : stage 0 in kReverse map, whose inputs are exactly the 16-byte
//             loads x[4q .. 4q+3] of row p1(n1) (Eq. 2d_dct_pre reorder, with the
//             even/odd packing z(q) = x'(2q) + j x'(2q+1) of the real FFT);
//             last stage in kMirror map, so Z(k) and Z(m - k) meet in one thread
//             for the real-FFT split; the half spectrum is stored with the real
//             DC and Nyquist values packed in column 0 as X(0) + j X(m).
//   columns : cyclic loads of a tile of packed columns, last stage in kMirror
//             map so rows k1 and n1 - k1 meet in one thread for the
//             four-element post of Eqs. (four-elements) and (s-t).
// Inverse (Alg. alg:DCT, "2D_IDCT"):
//   columns : stage 0 in kMirror map: the four reads of Eq. (2d_idct_pre)
//             (rows k1, n1 - k1; columns k2, n2 - k2) give the two values the
//             thread owns; column 0 packed with column m; cyclic stores.
//   rows    : stage 0 in kMirror map for the inverse real-FFT split, last stage
//             in kReverse map so the Eq. (2d_idct_post) reorder is one 16-byte
//             store of output row p1(n1).
// Scale factors are folded into the FP64-built tables exactly as on the
// general path (plan.cpp).
#include "fast_core.h"
#include "dct1d.h"

namespace dctx {

using fast::kCyclic;
using fast::kMirror;
using fast::kReverse;
using fast::Stage;

namespace {

template <int L>
struct Sched {
    static constexpr FastCfg cf = fast_cfg(L);
    static constexpr int T = cf.T, R0 = cf.R0, R1 = cf.R1, R2 = cf.R2, C = cf.C;
    static constexpr int BUF = fast_buf(L);
    static_assert(T > 0 && R0 * R1 * R2 == L, "no fast schedule for this length");
};

// Runs stages 1 and 2 after stage 0 (values in v0, already transformed):
// exchange, stage 1, exchange, read stage-2 inputs, stage 2 (values in v2).
template <class S0, class S1, class S2, bool INV>
__device__ __forceinline__ void middle_and_last(float2 *buf, int stride, int c, int t,
                                                float2 (&v0)[S0::NB][S0::R],
                                                float2 (&v2)[S2::NB][S2::R], const float2 *tw1,
                                                const float2 *tw2) {
    fast::write_out<S0>(buf, stride, c, v0, t);
    lds_sync();
    float2 v1[S1::NB][S1::R];
    fast::read_in<S1, S0::D>(buf, stride, c, v1, t);
    fast::butterflies<S1, INV>(v1, t, tw1);
    lds_sync();
    fast::write_out<S1>(buf, stride, c, v1, t);
    lds_sync();
    fast::read_in<S2, S1::D>(buf, stride, c, v2, t);
    fast::butterflies<S2, INV>(v2, t, tw2);
}

// ------------------------------------------------------------- forward rows
template <int L>
__device__ __forceinline__ void dct2_rows_fast(const Plan2D &p, const float *__restrict__ x,
                                               float2 *__restrict__ ws) {
    using Sc = Sched<L>;
    constexpr int T = Sc::T, RPB = 64 / T;
    using S0 = Stage<L, T, Sc::R0, 1, kReverse>;
    using S1 = Stage<L, T, Sc::R1, Sc::R0, kCyclic>;
    using S2 = Stage<L, T, Sc::R2, Sc::R0 * Sc::R1, kMirror>;
    extern __shared__ float2 lds[];
    const int r = threadIdx.x / T;
    const int t = threadIdx.x % T;
    const int n1 = blockIdx.x * RPB + r;
    const bool active = n1 < p.n1;
    float2 *buf = lds + r * Sc::BUF;

    // stage-0 inputs: float4 q = j + r Nb holds z(q) (input r of slot j) and
    // z(L-1-q) (input R0-1-r of the slot Nb-1-j).
    float2 v0[S0::NB][S0::R];
    constexpr int H0 = S0::NB / 2;
    if (active) {
        const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)src_row(n1, p.n1, p.nsub) * p.n2);
#pragma unroll
        for (int b = 0; b < S0::NB; ++b) {
            const int jj = S0::j(t, b);
            const int pb = b < H0 ? b + H0 : b - H0;
#pragma unroll
            for (int rr = 0; rr < S0::R / 2; ++rr) {
                const float4 f = nt_load4(src + jj + rr * S0::Nb);   // input read once
                v0[b][rr] = make_float2(f.x, f.z);
                v0[pb][S0::R - 1 - rr] = make_float2(f.w, f.y);
            }
        }
    }
    fast::butterflies<S0, false>(v0, t, nullptr);
    float2 v2[S2::NB][S2::R];
    middle_and_last<S0, S1, S2, false>(buf, 1, 0, t, v0, v2, p.row.tw + p.row.twoff[1],
                                       p.row.tw + p.row.twoff[2]);

    // real-FFT split on the pairs (k, L - k); W^(L-k) = -conj(W^k), W = e^{-2 pi j / 2L}.
    // Slot b < H pairs with slot b + H (r with R-1-r); thread 0's slot 0 (j = 0)
    // and slot H (j = Nb/2) pair within themselves.  The results go to the row's
    // LDS buffer in natural order and then to memory as whole-row 16-byte
    // stores (the pairs themselves are scattered 8-byte values).
    constexpr int H = S2::NB / 2, R = S2::R, Nb = S2::Nb;
    lds_sync();   // stage 2 has read its inputs (the workgroup is one wavefront)
    float2 *out = buf;
    auto split_store = [&](int k, float2 zk, float2 zm) {
        const float2 wk = p.split[k];
        const float2 wm = make_float2(-wk.x, wk.y);
        float2 xk, xm;
        rsplit_pair(zk, zm, wk, wm, xk, xm);
        out[k] = xk;
        if (L - k != k) out[L - k] = xm;
    };
    if (active) {
#pragma unroll
        for (int b = 0; b < H; ++b) {
            const int jj = S2::j(t, b);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int k = jj + rr * Nb;
                if (b == 0 && t == 0) {
                    if (rr > R / 2) continue;
                    if (rr == 0) {
                        const float2 z0 = v2[0][0];
                        out[0] = make_float2(z0.x + z0.y, z0.x - z0.y);   // X(0) + j X(m), both real
                        continue;
                    }
                    split_store(k, v2[0][rr], v2[0][(R - rr) % R]);
                } else {
                    split_store(k, v2[b][rr], v2[b + H][R - 1 - rr]);
                }
            }
        }
        if (t == 0) {
#pragma unroll
            for (int rr = 0; rr < R / 2; ++rr) split_store(Nb / 2 + rr * Nb, v2[H][rr], v2[H][R - 1 - rr]);
        }
    }
    lds_sync();
    if (!active) return;
    float4 *dst = reinterpret_cast<float4 *>(ws + (size_t)n1 * L);
    static_assert(L % (2 * T) == 0, "whole 16-byte words per thread");
#pragma unroll
    for (int e = 0; e < L / (2 * T); ++e) {
        const int i = t + e * T;
        const float2 a = buf[2 * i], b = buf[2 * i + 1];
        dst[i] = make_float4(a.x, a.y, b.x, b.y);
    }
}

// ------------------------------------------------------------- 1-D rows
// Batched 1-D DCT-II of rows of length n = 2L on the compile-time schedule:
// the loads, FFT and split of kf_dct2_rows (the split staged in LDS in natural
// order, X(0) + j X(L) in slot 0), then the Eq. (n_post_update) postprocess on
// whole 16-byte output words: word w covers y(4w .. 4w+3), all below L
// (y(j) = Re(t(j) X(j))) or all from L on (y(L) = Re t(L) X(L), and
// y(j) = -Im(t(n-j) X(n-j)) above it).
template <int L>
__global__ void __launch_bounds__(64) kf_dct1d(Plan1D p, int batch, const float *__restrict__ x,
                                               float *__restrict__ y) {
    using Sc = Sched<L>;
    constexpr int T = Sc::T, RPB = 64 / T;
    using S0 = Stage<L, T, Sc::R0, 1, kReverse>;
    using S1 = Stage<L, T, Sc::R1, Sc::R0, kCyclic>;
    using S2 = Stage<L, T, Sc::R2, Sc::R0 * Sc::R1, kMirror>;
    extern __shared__ float2 lds[];
    const int r = threadIdx.x / T;
    const int t = threadIdx.x % T;
    const int row = blockIdx.x * RPB + r;
    const bool active = row < batch;
    float2 *buf = lds + r * Sc::BUF;

    float2 v0[S0::NB][S0::R];
    constexpr int H0 = S0::NB / 2;
    if (active) {
        const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)row * 2 * L);
#pragma unroll
        for (int b = 0; b < S0::NB; ++b) {
            const int jj = S0::j(t, b);
            const int pb = b < H0 ? b + H0 : b - H0;
#pragma unroll
            for (int rr = 0; rr < S0::R / 2; ++rr) {
                const float4 f = nt_load4(src + jj + rr * S0::Nb);   // input read once
                v0[b][rr] = make_float2(f.x, f.z);
                v0[pb][S0::R - 1 - rr] = make_float2(f.w, f.y);
            }
        }
    }
    fast::butterflies<S0, false>(v0, t, nullptr);
    float2 v2[S2::NB][S2::R];
    middle_and_last<S0, S1, S2, false>(buf, 1, 0, t, v0, v2, p.row.tw + p.row.twoff[1],
                                       p.row.tw + p.row.twoff[2]);
    constexpr int H = S2::NB / 2, R = S2::R, Nb = S2::Nb;
    lds_sync();   // stage 2 has read its inputs (the workgroup is one wavefront)
    auto split_store = [&](int k, float2 zk, float2 zm) {
        const float2 wk = p.split[k];
        const float2 wm = make_float2(-wk.x, wk.y);
        float2 xk, xm;
        rsplit_pair(zk, zm, wk, wm, xk, xm);
        buf[k] = xk;
        if (L - k != k) buf[L - k] = xm;
    };
    if (active) {
#pragma unroll
        for (int b = 0; b < H; ++b) {
            const int jj = S2::j(t, b);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int k = jj + rr * Nb;
                if (b == 0 && t == 0) {
                    if (rr > R / 2) continue;
                    if (rr == 0) {
                        const float2 z0 = v2[0][0];
                        buf[0] = make_float2(z0.x + z0.y, z0.x - z0.y);   // X(0) + j X(L), both real
                        continue;
                    }
                    split_store(k, v2[0][rr], v2[0][(R - rr) % R]);
                } else {
                    split_store(k, v2[b][rr], v2[b + H][R - 1 - rr]);
                }
            }
        }
        if (t == 0) {
#pragma unroll
            for (int rr = 0; rr < R / 2; ++rr) split_store(Nb / 2 + rr * Nb, v2[H][rr], v2[H][R - 1 - rr]);
        }
    }
    lds_sync();
    if (!active) return;
    float4 *dst = reinterpret_cast<float4 *>(y + (size_t)row * 2 * L);
    static_assert(L % (2 * T) == 0 && L % 4 == 0, "whole 16-byte words per thread, none across y(L)");
#pragma unroll
    for (int e = 0; e < L / (2 * T); ++e) {
        const int w = t + e * T;
        const int j0 = 4 * w;
        float o[4];
        if (j0 < L) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u;
                const float2 X = buf[j], tj = p.tw[j];
                o[u] = (j == 0) ? tj.x * X.x : tj.x * X.x - tj.y * X.y;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u;
                const int k = (j == L) ? 0 : 2 * L - j;
                const float2 X = buf[k], tk = p.tw[j == L ? L : k];
                o[u] = (j == L) ? tk.x * X.y : -(tk.x * X.y + tk.y * X.x);
            }
        }
        nt_store4(dst + w, make_float4(o[0], o[1], o[2], o[3]));   // output written once
    }
}

// Batched 1-D DCT-III of rows of length n = 2L on the compile-time schedule:
// the pre U(k) = t'(k) (y(k) - j y(n - k)), y(n) = 0, read straight from the
// row in place of kf_idct2_rows' spectrum loads, then its inverse split,
// inverse FFT and inverse-reorder stores.
template <int L>
__global__ void __launch_bounds__(64) kf_idct1d(Plan1D p, int batch, const float *__restrict__ x,
                                                float *__restrict__ y) {
    using Sc = Sched<L>;
    constexpr int T = Sc::T, RPB = 64 / T;
    using S0 = Stage<L, T, Sc::R0, 1, kMirror>;
    using S1 = Stage<L, T, Sc::R1, Sc::R0, kCyclic>;
    using S2 = Stage<L, T, Sc::R2, Sc::R0 * Sc::R1, kReverse>;
    extern __shared__ float2 lds[];
    const int r = threadIdx.x / T;
    const int t = threadIdx.x % T;
    const int row = blockIdx.x * RPB + r;
    const bool active = row < batch;
    float2 *buf = lds + r * Sc::BUF;

    float2 v0[S0::NB][S0::R];
    constexpr int H = S0::NB / 2, R = S0::R, Nb = S0::Nb;
    const float *src = x + (size_t)(active ? row : 0) * 2 * L;
    auto isplit_pair = [&](int k, float2 &zk, float2 &zm) {
        if (!active) {
            zk = zm = make_float2(0.f, 0.f);
            return;
        }
        if (k == 0) {
            // U(0) and U(L) are real
            const float u0 = p.tw[0].x * src[0];
            const float uL = cmul(p.tw[L], make_float2(src[L], -src[L])).x;
            zk = zm = make_float2(u0 + uL, u0 - uL);
            return;
        }
        const float2 uk = cmul(p.tw[k], make_float2(src[k], -src[2 * L - k]));
        const float2 um = cmul(p.tw[L - k], make_float2(src[L - k], -src[L + k]));
        const float2 wk = p.split[k];
        irsplit_pair(uk, um, wk, make_float2(-wk.x, wk.y), zk, zm);
    };
#pragma unroll
    for (int b = 0; b < H; ++b) {
        const int jj = S0::j(t, b);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int k = jj + rr * Nb;
            float2 f, g;
            if (b == 0 && t == 0) {
                if (rr > R / 2) continue;
                isplit_pair(k, f, g);
                v0[0][rr] = f;
                if (rr != 0 && rr != R / 2) v0[0][(R - rr) % R] = g;
            } else {
                isplit_pair(k, f, g);
                v0[b][rr] = f;
                v0[b + H][R - 1 - rr] = g;
            }
        }
    }
    if (t == 0) {
#pragma unroll
        for (int rr = 0; rr < R / 2; ++rr) {
            float2 f, g;
            isplit_pair(Nb / 2 + rr * Nb, f, g);
            v0[H][rr] = f;
            v0[H][R - 1 - rr] = g;
        }
    }
    fast::butterflies<S0, true>(v0, t, nullptr);
    float2 v2[S2::NB][S2::R];
    middle_and_last<S0, S1, S2, true>(buf, 1, 0, t, v0, v2, p.row.tw + p.row.twoff[1],
                                      p.row.tw + p.row.twoff[2]);
    if (!active) return;
    // Eq. (n_pre) inverted: output float4 q = j + r Nb is (z(q).x, z(L-1-q).y, z(q).y, z(L-1-q).x)
    float4 *dst = reinterpret_cast<float4 *>(y + (size_t)row * 2 * L);
    constexpr int H2 = S2::NB / 2;
#pragma unroll
    for (int b = 0; b < S2::NB; ++b) {
        const int jj = S2::j(t, b);
        const int pb = b < H2 ? b + H2 : b - H2;
#pragma unroll
        for (int rr = 0; rr < S2::R / 2; ++rr) {
            const float2 a = v2[b][rr];
            const float2 m = v2[pb][S2::R - 1 - rr];
            nt_store4(dst + jj + rr * S2::Nb, make_float4(a.x, m.y, a.y, m.x));   // output written once
        }
    }
}

// Four outputs of the post for the row pair (k1, k1p) and stored column col:
// s = b (a A + conj(a) B), t = b (a A - conj(a) B);
// y(k1, col) = Re s, y(k1, n2-col) = -Im s, y(k1p, col) = -Im t, y(k1p, n2-col) = -Re t.
__device__ __forceinline__ void post4(float *__restrict__ y, int N2, int k1, int k1p, int col, bool mirror,
                                      float2 a, float2 b, float2 A, float2 B) {
    const float2 aA = cmul(a, A);
    const float2 aB = cmulc(B, a);
    const float2 s = cmul(b, cadd(aA, aB));
    out_store(&y[(size_t)k1 * N2 + col], s.x);
    if (mirror) out_store(&y[(size_t)k1 * N2 + (N2 - col)], -s.y);
    if (k1p != k1) {
        const float2 tt = cmul(b, csub(aA, aB));
        out_store(&y[(size_t)k1p * N2 + col], -tt.y);
        if (mirror) out_store(&y[(size_t)k1p * N2 + (N2 - col)], -tt.x);
    }
}

// ---------------------------------------------------------- forward columns
template <int L>
__device__ __forceinline__ void dct2_cols_fast(const Plan2D &p, const float2 *__restrict__ ws,
                                               float *__restrict__ y) {
    using Sc = Sched<L>;
    constexpr int T = Sc::T, C = Sc::C;
    using S0 = Stage<L, T, Sc::R0, 1, kCyclic>;
    using S1 = Stage<L, T, Sc::R1, Sc::R0, kCyclic>;
    using S2 = Stage<L, T, Sc::R2, Sc::R0 * Sc::R1, kMirror>;
    extern __shared__ float2 lds[];
    const int c = threadIdx.x % C;
    const int t = threadIdx.x / C;
    const int M = p.m, N2 = p.n2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile * C >= M) return;  // whole workgroup leaves together
    const int k2 = tile * C + c;
    const bool act = k2 < M;

    float2 v0[S0::NB][S0::R];
#pragma unroll
    for (int b = 0; b < S0::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < S0::R; ++rr) {
            const int row = t + (b + rr * S0::NB) * T;
            v0[b][rr] = act ? ws[(size_t)row * M + k2] : make_float2(0.f, 0.f);
        }
    fast::butterflies<S0, false>(v0, t, nullptr);
    float2 v2[S2::NB][S2::R];
    middle_and_last<S0, S1, S2, false>(lds, C, c, t, v0, v2, p.col.tw + p.col.twoff[1],
                                       p.col.tw + p.col.twoff[2]);
    if (!act) return;

    const float2 bk = p.tb[k2];
    const float2 bm = p.tb[M];
    constexpr int H = S2::NB / 2, R = S2::R, Nb = S2::Nb;
    auto post_pair = [&](int k1, float2 A, float2 B) {
        const int k1p = (k1 == 0) ? 0 : L - k1;
        const float2 a = p.ta[k1];
        if (k2 == 0) {
            // unpack W = V(., 0) + j V(., m):  V0(k) = (W(k) + conj W(-k)) / 2,
            // Vm(k) = -j (W(k) - conj W(-k)) / 2
            const float2 v0a = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
            const float2 v0b = make_float2(0.5f * (B.x + A.x), 0.5f * (B.y - A.y));
            const float2 vma = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
            const float2 vmb = make_float2(0.5f * (B.y + A.y), -0.5f * (B.x - A.x));
            post4(y, N2, k1, k1p, 0, false, a, bk, v0a, v0b);
            post4(y, N2, k1, k1p, M, false, a, bm, vma, vmb);
        } else {
            post4(y, N2, k1, k1p, k2, true, a, bk, A, B);
        }
    };
    // rows k1 and n1 - k1: slot b < H with slot b + H (r with R-1-r); thread 0's
    // slot 0 (k1 = r Nb) and slot H (k1 = Nb/2 + r Nb) pair within themselves.
#pragma unroll
    for (int b = 0; b < H; ++b) {
        const int jj = S2::j(t, b);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int k1 = jj + rr * Nb;
            if (b == 0 && t == 0) {
                if (rr > R / 2) continue;
                post_pair(k1, v2[0][rr], v2[0][(R - rr) % R]);
            } else {
                post_pair(k1, v2[b][rr], v2[b + H][R - 1 - rr]);
            }
        }
    }
    if (t == 0) {
#pragma unroll
        for (int rr = 0; rr < R / 2; ++rr) post_pair(Nb / 2 + rr * Nb, v2[H][rr], v2[H][R - 1 - rr]);
    }
}

// Eq. (2d_idct_pre) for row k1 of column k2 (P = (x(k1,k2), x(k1,mirror)),
// Q = the same for row n1 - k1, zero for k1 = 0); column 0 packs X'(k1,0) + j X'(k1,m).
__device__ __forceinline__ float2 pre_value(int k2, float2 a, float2 b, float2 bm, float2 P, float2 Q) {
    if (k2 == 0) {
        const float2 x0 = cmul(cmul(a, b), make_float2(P.x, -Q.x));
        const float2 xm = cmul(cmul(a, bm), make_float2(P.y - Q.y, -(Q.y + P.y)));
        return make_float2(x0.x - xm.y, x0.y + xm.x);
    }
    return cmul(cmul(a, b), make_float2(P.x - Q.y, -(Q.x + P.y)));
}

// ---------------------------------------------------------- inverse columns
// XST: the IDXST axes of the plan (the p.xst bits), fixed at compile time.
template <int L, int XST>
__device__ __forceinline__ void idct2_cols_fast(const Plan2D &p, const float *__restrict__ x,
                                                float2 *__restrict__ ws) {
    using Sc = Sched<L>;
    constexpr int T = Sc::T, C = Sc::C;
    using S0 = Stage<L, T, Sc::R0, 1, kMirror>;
    using S1 = Stage<L, T, Sc::R1, Sc::R0, kCyclic>;
    using S2 = Stage<L, T, Sc::R2, Sc::R0 * Sc::R1, kCyclic>;
    extern __shared__ float2 lds[];
    const int c = threadIdx.x % C;
    const int t = threadIdx.x / C;
    const int M = p.m, N2 = p.n2;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile * C >= M) return;
    const int k2 = tile * C + c;
    const bool act = k2 < M;
    const int mcol = (k2 == 0) ? M : N2 - k2;

    float2 v0[S0::NB][S0::R];
    constexpr int H = S0::NB / 2, R = S0::R, Nb = S0::Nb;
    const float2 bk = act ? p.tb[k2] : make_float2(0.f, 0.f);
    const float2 bm = p.tb[M];
    // four reads (rows k1, n1 - k1; columns k2 and its mirror) give the values of
    // element k1 (first) and n1 - k1 (second); row n1 is zero.
    auto pre_pair = [&](int k1, float2 &first, float2 &second) {
        if (!act) {
            first = second = make_float2(0.f, 0.f);
            return;
        }
        const float *xr = x + (size_t)k1 * N2;
        float2 P = make_float2(xr[k2], xr[mcol]);
        float2 Q = make_float2(0.f, 0.f);
        if (k1 != 0) {
            const float *xq = x + (size_t)(L - k1) * N2;
            Q = make_float2(xq[k2], xq[mcol]);
        }
        if (XST) xst_reverse(XST, k1, k2, P, Q);   // compile-time: no branch in the IDCT
        first = pre_value(k2, p.ta[k1], bk, bm, P, Q);
        second = (k1 != 0) ? pre_value(k2, p.ta[L - k1], bk, bm, Q, P) : first;
    };
#pragma unroll
    for (int b = 0; b < H; ++b) {
        const int jj = S0::j(t, b);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int k1 = jj + rr * Nb;
            float2 f, g;
            if (b == 0 && t == 0) {
                if (rr > R / 2) continue;
                pre_pair(k1, f, g);
                v0[0][rr] = f;
                if (rr != 0 && rr != R / 2) v0[0][(R - rr) % R] = g;
            } else {
                pre_pair(k1, f, g);
                v0[b][rr] = f;
                v0[b + H][R - 1 - rr] = g;
            }
        }
    }
    if (t == 0) {
#pragma unroll
        for (int rr = 0; rr < R / 2; ++rr) {
            float2 f, g;
            pre_pair(Nb / 2 + rr * Nb, f, g);
            v0[H][rr] = f;
            v0[H][R - 1 - rr] = g;
        }
    }
    fast::butterflies<S0, true>(v0, t, nullptr);
    float2 v2[S2::NB][S2::R];
    middle_and_last<S0, S1, S2, true>(lds, C, c, t, v0, v2, p.col.tw + p.col.twoff[1],
                                      p.col.tw + p.col.twoff[2]);
    if (!act) return;
#pragma unroll
    for (int b = 0; b < S2::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < S2::R; ++rr) {
            const int row = t + (b + rr * S2::NB) * T;
            ws[(size_t)row * M + k2] = v2[b][rr];
        }
}

// ------------------------------------------------------------- inverse rows
template <int L>
__device__ __forceinline__ void idct2_rows_fast(const Plan2D &p, const float2 *__restrict__ ws,
                                                float *__restrict__ y) {
    using Sc = Sched<L>;
    constexpr int T = Sc::T, RPB = 64 / T;
    using S0 = Stage<L, T, Sc::R0, 1, kMirror>;
    using S1 = Stage<L, T, Sc::R1, Sc::R0, kCyclic>;
    using S2 = Stage<L, T, Sc::R2, Sc::R0 * Sc::R1, kReverse>;
    extern __shared__ float2 lds[];
    const int r = threadIdx.x / T;
    const int t = threadIdx.x % T;
    const int n1 = blockIdx.x * RPB + r;
    const bool active = n1 < p.n1;
    float2 *buf = lds + r * Sc::BUF;

    // inverse split on the pairs (k, L - k): Z(k) from U(k), U(L - k), with
    // U(0) = Re P(0), U(L) = Im P(0) packed in column 0.
    float2 v0[S0::NB][S0::R];
    constexpr int H = S0::NB / 2, R = S0::R, Nb = S0::Nb;
    const float2 *src = ws + (size_t)n1 * L;
    auto isplit_pair = [&](int k, float2 &zk, float2 &zm) {
        if (!active) {
            zk = zm = make_float2(0.f, 0.f);
            return;
        }
        if (k == 0) {
            const float2 p0 = src[0];
            zk = zm = make_float2(p0.x + p0.y, p0.x - p0.y);
            return;
        }
        const float2 wk = p.split[k];
        irsplit_pair(src[k], src[L - k], wk, make_float2(-wk.x, wk.y), zk, zm);
    };
#pragma unroll
    for (int b = 0; b < H; ++b) {
        const int jj = S0::j(t, b);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int k = jj + rr * Nb;
            float2 f, g;
            if (b == 0 && t == 0) {
                if (rr > R / 2) continue;
                isplit_pair(k, f, g);
                v0[0][rr] = f;
                if (rr != 0 && rr != R / 2) v0[0][(R - rr) % R] = g;
            } else {
                isplit_pair(k, f, g);
                v0[b][rr] = f;
                v0[b + H][R - 1 - rr] = g;
            }
        }
    }
    if (t == 0) {
#pragma unroll
        for (int rr = 0; rr < R / 2; ++rr) {
            float2 f, g;
            isplit_pair(Nb / 2 + rr * Nb, f, g);
            v0[H][rr] = f;
            v0[H][R - 1 - rr] = g;
        }
    }
    fast::butterflies<S0, true>(v0, t, nullptr);
    float2 v2[S2::NB][S2::R];
    middle_and_last<S0, S1, S2, true>(buf, 1, 0, t, v0, v2, p.row.tw + p.row.twoff[1],
                                      p.row.tw + p.row.twoff[2]);
    if (!active) return;
    // Eq. (2d_idct_post): output float4 q = j + r Nb of row p1(n1) is
    // (x'(2q), x'(2m-1-2q)... ) = (z(q).x, z(L-1-q).y, z(q).y, z(L-1-q).x).
    const int orow = src_row(n1, p.n1, p.nsub);
    float4 *dst = reinterpret_cast<float4 *>(y + (size_t)orow * p.n2);
    constexpr int H2 = S2::NB / 2;
#pragma unroll
    for (int b = 0; b < S2::NB; ++b) {
        const int jj = S2::j(t, b);
        const int pb = b < H2 ? b + H2 : b - H2;
#pragma unroll
        for (int rr = 0; rr < S2::R / 2; ++rr) {
            const float2 a = v2[b][rr];
            const float2 m = v2[pb][S2::R - 1 - rr];
            nt_store4(dst + jj + rr * S2::Nb,
                      xst_sign4(p.xst, orow, make_float4(a.x, m.y, a.y, m.x)));   // output written once
        }
    }
}

// Kernels: blockIdx.y selects the transform of a grouped launch.
template <int L>
__global__ void __launch_bounds__(64) kf_dct2_rows(Plan2D p, Io io) {
    dct2_rows_fast<L>(p, io_src<float>(io), io_dst<float2>(io));
}
template <int L>
__global__ void __launch_bounds__(Sched<L>::T * Sched<L>::C) kf_dct2_cols(Plan2D p, Io io) {
    dct2_cols_fast<L>(p, io_src<float2>(io), io_dst<float>(io));
}
template <int L, int XST>
__global__ void __launch_bounds__(Sched<L>::T * Sched<L>::C) kf_idct2_cols(Plan2D p, Io io) {
    idct2_cols_fast<L, XST>(p, io_src<float>(io), io_dst<float2>(io));
}
template <int L>
__global__ void __launch_bounds__(64) kf_idct2_rows(Plan2D p, Io io) {
    idct2_rows_fast<L>(p, io_src<float2>(io), io_dst<float>(io));
}

template <class K>
inline void set_lds(K kernel, size_t bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int L>
hipError_t rows_fwd(const Plan2D &p, const Io &io, hipStream_t s) {
    constexpr int RPB = 64 / Sched<L>::T;
    const size_t lds = (size_t)RPB * Sched<L>::BUF * sizeof(float2);
    hipLaunchKernelGGL(kf_dct2_rows<L>, dim3((p.n1 + RPB - 1) / RPB, io.n), dim3(64), lds, s, p, io);
    return hipGetLastError();
}

template <int L>
hipError_t rows_inv(const Plan2D &p, const Io &io, hipStream_t s) {
    constexpr int RPB = 64 / Sched<L>::T;
    const size_t lds = (size_t)RPB * Sched<L>::BUF * sizeof(float2);
    hipLaunchKernelGGL(kf_idct2_rows<L>, dim3((p.n1 + RPB - 1) / RPB, io.n), dim3(64), lds, s, p, io);
    return hipGetLastError();
}

template <int L>
hipError_t cols_fwd(const Plan2D &p, const Io &io, hipStream_t s) {
    constexpr int C = Sched<L>::C;
    const size_t lds = (size_t)C * Sched<L>::BUF * sizeof(float2);
    set_lds(kf_dct2_cols<L>, lds);
    const int tiles = (p.m + C - 1) / C;
    hipLaunchKernelGGL(kf_dct2_cols<L>, dim3((tiles + 7) & ~7, io.n), dim3(C * Sched<L>::T), lds, s, p, io);
    return hipGetLastError();
}

template <int L, int XST>
hipError_t cols_inv_x(const Plan2D &p, const Io &io, hipStream_t s) {
    constexpr int C = Sched<L>::C;
    const size_t lds = (size_t)C * Sched<L>::BUF * sizeof(float2);
    set_lds(kf_idct2_cols<L, XST>, lds);
    const int tiles = (p.m + C - 1) / C;
    hipLaunchKernelGGL((kf_idct2_cols<L, XST>), dim3((tiles + 7) & ~7, io.n), dim3(C * Sched<L>::T), lds, s, p,
                       io);
    return hipGetLastError();
}

template <int L>
hipError_t cols_inv(const Plan2D &p, const Io &io, hipStream_t s) {
    switch (p.xst) {
        case 0: return cols_inv_x<L, 0>(p, io, s);
        case 1: return cols_inv_x<L, 1>(p, io, s);
        case 2: return cols_inv_x<L, 2>(p, io, s);
        case 3: return cols_inv_x<L, 3>(p, io, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool fast_rows_supported(int m) {
    return m >= 32 && m <= 2048 && (m & (m - 1)) == 0;
}

bool fast_supported(int n1, int m) {
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    return pow2(m) && m >= 32 && m <= 2048 && pow2(n1) && n1 >= 64 && n1 <= 4096;
}

#define DCTX_FAST_ROWS(FN, CALL)                              \
    switch (p.m) {                                            \
        case 2048: return FN<2048> CALL;                      \
        case 1024: return FN<1024> CALL;                      \
        case 512: return FN<512> CALL;                        \
        case 256: return FN<256> CALL;                        \
        case 128: return FN<128> CALL;                        \
        case 64: return FN<64> CALL;                          \
        case 32: return FN<32> CALL;                          \
    }                                                         \
    return hipErrorInvalidValue

template <int L>
hipError_t dct1d_fast(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s) {
    constexpr int RPB = 64 / Sched<L>::T;
    const size_t lds = (size_t)RPB * Sched<L>::BUF * sizeof(float2);
    hipLaunchKernelGGL(kf_dct1d<L>, dim3((batch + RPB - 1) / RPB), dim3(64), lds, s, p, batch, x, y);
    return hipGetLastError();
}

template <int L>
hipError_t idct1d_fast(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s) {
    constexpr int RPB = 64 / Sched<L>::T;
    const size_t lds = (size_t)RPB * Sched<L>::BUF * sizeof(float2);
    hipLaunchKernelGGL(kf_idct1d<L>, dim3((batch + RPB - 1) / RPB), dim3(64), lds, s, p, batch, x, y);
    return hipGetLastError();
}

#define DCTX_FAST_COLS(FN, CALL)                              \
    switch (p.n1) {                                           \
        case 4096: return FN<4096> CALL;                      \
        case 2048: return FN<2048> CALL;                      \
        case 1024: return FN<1024> CALL;                      \
        case 512: return FN<512> CALL;                        \
        case 256: return FN<256> CALL;                        \
        case 128: return FN<128> CALL;                        \
        case 64: return FN<64> CALL;                          \
    }                                                         \
    return hipErrorInvalidValue

hipError_t launch_fast_dct2_rows(const Plan2D &p, const Io &io, hipStream_t s) {
    DCTX_FAST_ROWS(rows_fwd, (p, io, s));
}
hipError_t launch_fast_idct2_rows(const Plan2D &p, const Io &io, hipStream_t s) {
    DCTX_FAST_ROWS(rows_inv, (p, io, s));
}
hipError_t launch_fast_dct1d(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s) {
    DCTX_FAST_ROWS(dct1d_fast, (p, batch, x, y, s));
}
hipError_t launch_fast_idct1d(const Plan1D &p, int batch, const float *x, float *y, hipStream_t s) {
    DCTX_FAST_ROWS(idct1d_fast, (p, batch, x, y, s));
}
hipError_t launch_fast_dct2_cols(const Plan2D &p, const Io &io, hipStream_t s) {
    DCTX_FAST_COLS(cols_fwd, (p, io, s));
}
hipError_t launch_fast_idct2_cols(const Plan2D &p, const Io &io, hipStream_t s) {
    DCTX_FAST_COLS(cols_inv, (p, io, s));
}

}  // namespace dctx
