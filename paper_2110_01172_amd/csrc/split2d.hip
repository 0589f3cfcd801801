// Split-column form of the 2-D three-stage DCT-II / DCT-III (tall arrays,
// n1 = 8 q).  The length-n1 column FFT is factored as n1 = 8 x q
// (Cooley-Tukey, n = qq + q r, k = kp + 8 kq):
//   X(kp + 8 kq) = sum_qq W_q^(qq kq) [ W_n1^(qq kp) sum_r W_8^(r kp) x(qq + q r) ].
// The bracket is computed in the row pass: one workgroup takes the eight
// rows qq, qq + q, ..., qq + 7q, runs their real FFTs side by side (the
// reorder of Eq. 2d_dct_pre fused into the loads, the split into the last
// stage) leaving the half spectra in LDS, applies the 8-point DFT across them
// and the twiddle W_n1^(qq kp), and writes workspace row kp q + qq.  The column pass then runs only q-point FFTs, so its tiles are
// 16 columns wide (128-byte segments of the packed spectrum instead of 16).
//
// The four-element post (Eqs. four-elements, s-t) needs rows k1 and n1 - k1:
// for k1 = kp + 8 kq the partner is (8 - kp) + 8 (q - 1 - kq) (kp > 0) or
// 8 (q - kq) (kp = 0).  A column workgroup therefore takes the sequence pair
// {kp, 8 - kp} (kp = 1, 2, 3) or {0, 4}.  Forward: the two q-point FFTs run
// side by side and the post reads the partners from LDS.  Inverse: the pre
// fills both sequences in registers and the two FFTs run one after the other,
// with first-stage maps that put every partner in the same thread:
//   {kp, 8-kp}: kCyclic / kRevCyclic (element i with q - 1 - i),
//   {0, 4}    : kMirror (i with q - i) / kReverse (i with q - 1 - i).
// The inverse runs the mirror image: the four-read pre of Eq. (2d_idct_pre)
// fills both sequences of a pair, two inverse q-point FFTs, then the row pass
// applies conj twiddles and the inverse 8-point DFT (into LDS) and the inverse
// real FFT of each of its eight rows with the Eq. (2d_idct_post) reorder
// fused into the stores.  Tables and scale factors are those of the plain form.
#include "fast_chain.h"
#include "poisson_body.h"
#include "split2d.h"

namespace dctx {

using fast::buf_len;
using fast::fft_run;
using fast::kCyclic;
using fast::kMirror;
using fast::kRevCyclic;
using fast::kReverse;
using fast::RL;
using fast::Stage;
using fast::StageK;

namespace {


// Row schedules: T threads per row (one group per row), three stages; the
// first and last stages have two or more butterflies per thread (paired maps).
template <int M> struct RowRL;
template <> struct RowRL<2048> { using type = RL<16, 16, 8>; static constexpr int T = 64; };
template <> struct RowRL<1024> { using type = RL<8, 16, 8>; static constexpr int T = 64; };
template <> struct RowRL<512> { using type = RL<8, 8, 8>; static constexpr int T = 32; };
template <> struct RowRL<256> { using type = RL<8, 4, 8>; static constexpr int T = 16; };

// Column schedules: 16 values per thread, C columns per workgroup.
template <int Q> struct ColRL;
template <> struct ColRL<512> {
    using type = RL<8, 8, 8>;
    static constexpr int T = 32, C = 16;
};
template <> struct ColRL<1024> {   // 8 columns: two 1024-point buffers fill 128 KB of LDS
    using type = RL<8, 16, 8>;
    static constexpr int T = 64, C = 8;
};
// Kernels that keep one FFT buffer (the inverse columns, and the forward
// columns' single-buffer form ks_dct_cols_seq) can take 16-column tiles at
// q = 1024 (W = 1: 64-byte segments of the real rows, 128-byte segments of
// the workspace rows, 147 KB of LDS) where the array has enough columns to
// fill the chip with such tiles; W = 0 keeps 8.
template <int Q, int W> struct ColRLInv : ColRL<Q> {};
template <> struct ColRLInv<1024, 1> : ColRL<1024> { static constexpr int C = 16; };
template <> struct ColRL<256> {
    using type = RL<4, 8, 8>;
    static constexpr int T = 16, C = 16;
};

// Workspace element (row, k2) of a packed half spectrum with row pitch m.
template <class V>
__device__ __forceinline__ V *ws_at(V *ws, int row, int m, int k2) {
    return at_b(ws, row_b(row, 8u * (unsigned)m) + 8u * (unsigned)k2);
}

// Four outputs of the post for rows (k1, k1p) of stored column col:
// s = b (a A + conj(a) B), t = b (a A - conj(a) B);
// y(k1, col) = Re s, y(k1, n2-col) = -Im s, y(k1p, col) = -Im t, y(k1p, n2-col) = -Re t.
__device__ __forceinline__ void post4s(float *__restrict__ y, int N2, int k1, int k1p, int col, bool mirror,
                                       float2 a, float2 b, float2 A, float2 B) {
    const float2 aA = cmul(a, A);
    const float2 aB = cmulc(B, a);
    const float2 s = cmul(b, cadd(aA, aB));
    const unsigned pb = 4u * (unsigned)N2, cb = 4u * (unsigned)col, mb = 4u * (unsigned)(N2 - col);
    const unsigned r0 = row_b(k1, pb);
    out_store(at_b(y, r0 + cb), s.x);
    if (mirror) out_store(at_b(y, r0 + mb), -s.y);
    if (k1p != k1) {
        const float2 tt = cmul(b, csub(aA, aB));
        const unsigned r1 = row_b(k1p, pb);
        out_store(at_b(y, r1 + cb), -tt.y);
        if (mirror) out_store(at_b(y, r1 + mb), -tt.x);
    }
}

// Post for output rows k1 and n1 - k1 of column k2 from A = V(k1), B = V(n1 - k1),
// with a = ta(k1), bk = tb(k2) and bm = tb(m).
__device__ __forceinline__ void post_rows_v(const PlanSplit &p, float *__restrict__ y, int k1, int k2, float2 A,
                                            float2 B, float2 a, float2 bk, float2 bm) {
    const int N1 = p.n1, N2 = p.n2, M = p.m;
    const int k1p = (k1 == 0) ? 0 : N1 - k1;
    if (k2 == 0) {
        // unpack W = V(., 0) + j V(., m): V0(k) = (W(k) + conj W(-k)) / 2, Vm(k) = -j (W(k) - conj W(-k)) / 2
        const float2 v0a = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
        const float2 v0b = make_float2(0.5f * (B.x + A.x), 0.5f * (B.y - A.y));
        const float2 vma = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
        const float2 vmb = make_float2(0.5f * (B.y + A.y), -0.5f * (B.x - A.x));
        post4s(y, N2, k1, k1p, 0, false, a, bk, v0a, v0b);
        post4s(y, N2, k1, k1p, M, false, a, bm, vma, vmb);
    } else {
        post4s(y, N2, k1, k1p, k2, true, a, bk, A, B);
    }
}

__device__ __forceinline__ void post_rows(const PlanSplit &p, float *__restrict__ y, int k1, int k2, float2 A,
                                          float2 B) {
    post_rows_v(p, y, k1, k2, A, B, *at_b(p.ta, 8u * (unsigned)k1), p.tb[k2], p.tb[p.m]);
}

// Eq. (2d_idct_pre) for row k1 of column k2 (P = (x(k1,k2), x(k1,mirror)),
// Q = the same for row n1 - k1, zero for k1 = 0); column 0 packs X'(k1,0) + j X'(k1,m).
__device__ __forceinline__ float2 pre_val(int k2, float2 a, float2 b, float2 bm, float2 P, float2 Q) {
    if (k2 == 0) {
        const float2 x0 = cmul(cmul(a, b), make_float2(P.x, -Q.x));
        const float2 xm = cmul(cmul(a, bm), make_float2(P.y - Q.y, -(Q.y + P.y)));
        return make_float2(x0.x - xm.y, x0.y + xm.x);
    }
    return cmul(cmul(a, b), make_float2(P.x - Q.y, -(Q.x + P.y)));
}

// The pre values of rows k1 (first) and n1 - k1 (second) of column k2.
template <int XST>
__device__ __forceinline__ void pre_rows(const PlanSplit &p, const float *__restrict__ x, int k1, int k2,
                                         float2 &first, float2 &second) {
    const int N1 = p.n1, N2 = p.n2, M = p.m;
    const int mcol = (k2 == 0) ? M : N2 - k2;
    const unsigned pb = 4u * (unsigned)N2, kb = 4u * (unsigned)k2, mb = 4u * (unsigned)mcol;
    const unsigned r0 = row_b(k1, pb);
    float2 P = make_float2(*at_b(x, r0 + kb), *at_b(x, r0 + mb));
    float2 Q = make_float2(0.f, 0.f);
    if (k1 != 0) {
        const unsigned r1 = row_b(N1 - k1, pb);
        Q = make_float2(*at_b(x, r1 + kb), *at_b(x, r1 + mb));
    }
    if (XST) xst_reverse(XST, k1, k2, P, Q);   // compile-time: no branch in the IDCT
    const float2 b = p.tb[k2], bm = p.tb[M];
    first = pre_val(k2, *at_b(p.ta, 8u * (unsigned)k1), b, bm, P, Q);
    second = (k1 != 0) ? pre_val(k2, *at_b(p.ta, 8u * (unsigned)(N1 - k1)), b, bm, Q, P) : first;
}

// ------------------------------------------------------------- forward rows
// One workgroup per qq, one group of T threads per row: group g runs the real
// FFT of row qq + q g (reorder fused into the loads, split in the last stage)
// in its own LDS buffer and leaves the half spectrum there; after a barrier
// every thread takes positions k = tid, tid + 8T, ... and applies the 8-point
// DFT across the eight buffers and the twiddle W_n1^(qq kp), writing workspace
// row kp q + qq with whole-row coalesced stores.
// Tables of the row passes.  RowTabsG reads the plan's tables in global
// memory.  RowTabsL reads an LDS copy made once per workgroup: the stage
// twiddles (records transposed, see LdsTw) and a two-level table for the
// split twiddle W_n2^k and the column twiddle W_n1^e,
//   W^e = A[e mod 64] B[e / 64],  A[a] = W^a, B[b] = W^(64 b)  (FP64-built),
// so that the body issues no global loads besides its row data (a wait for
// a younger global load would also wait for every prefetched row, since
// loads complete in issue order).
struct RowTabsG {
    const PlanSplit *p;
    template <class H>
    __device__ __forceinline__ fast::GlobalTwHook<H> tw(const H &h) const { return fast::GlobalTwHook<H>{{}, h}; }
    __device__ __forceinline__ float2 split(int k) const { return p->split[k]; }
    __device__ __forceinline__ float2 xtw(int qq, int kp) const { return p->xtw[qq * 8 + kp]; }
};

struct RowTabsL {
    fast::LdsTw t;
    const float2 *two;   // A_split[64], B_split[64], A_col[64], B_col[64]
    int n1;
    template <class H>
    __device__ __forceinline__ fast::LdsTwHook<H> tw(const H &h) const { return fast::LdsTwHook<H>{t, h}; }
    __device__ __forceinline__ float2 split(int k) const { return cmul(two[k & 63], two[64 + (k >> 6)]); }
    __device__ __forceinline__ float2 xtw(int qq, int kp) const {
        const int e = (qq * kp) & (n1 - 1);
        return cmul(two[128 + (e & 63)], two[192 + (e >> 6)]);
    }
};

// LDS copy of the row tables behind the eight row buffers (float4 units).
template <int M>
struct RowLdsTabs {
    using L_ = typename RowRL<M>::type;
    static constexpr int n = L_::n;
    // float4 offset of stage K's table (K >= 1); stage 0 has no twiddles
    static constexpr int off(int K) {
        int o = 0;
        for (int i = 1; i < K; ++i) o += L_::ns(i) * tw_record(L_::r[i]) / 2;
        return o;
    }
    static constexpr int TW = off(n);          // all stage tables
    static constexpr int F = TW + 128;         // plus the 256-entry two-level table
    static constexpr size_t bytes() { return (size_t)8 * buf_len<L_>(M) * sizeof(float2) + (size_t)F * 16; }
    static_assert(bytes() <= 160 * 1024, "row buffers and tables must fit the LDS");
    static_assert(M / 64 <= 64, "two-level table covers k <= m");
    static_assert(8 * buf_len<L_>(M) * sizeof(float2) >= 16 * 8 * RowRL<M>::T, "spill words fit a row buffer");

    // Global source of LDS word d (d < F): record k, word h of a stage table,
    // or word d - TW of the two-level table.  One unconditional load per word
    // (words d >= F read word 0 of the two-level table and are not stored).
    __device__ __forceinline__ static float4 src(const PlanSplit &p, int d) {
        const float4 *ptr = reinterpret_cast<const float4 *>(p.tl);
        int idx = (d >= TW && d < F) ? d - TW : 0;
#pragma unroll
        for (int K = 1; K < n; ++K) {
            constexpr int unused = 0;
            (void)unused;
            const int NS = L_::ns(K), H = tw_record(L_::r[K]) / 2;
            const bool in = d >= off(K) && d < off(K + 1);
            const int dd = d - off(K);
            ptr = in ? reinterpret_cast<const float4 *>(p.row.tw + p.row.twoff[K]) : ptr;
            idx = in ? (dd % NS) * H + dd / NS : idx;
        }
        return ptr[idx];
    }
    __device__ __forceinline__ static RowTabsL view(const float2 *lds, int n1) {
        const float4 *base = reinterpret_cast<const float4 *>(lds + 8 * buf_len<L_>(M));
        RowTabsL r;
#pragma unroll
        for (int K = 0; K < kMaxStages; ++K) r.t.tab[K] = base + (K >= 1 && K < n ? off(K) : 0);
        r.two = reinterpret_cast<const float2 *>(base + TW);
        r.n1 = n1;
        return r;
    }
};

template <int M>
struct RowFwd {
    using L_ = typename RowRL<M>::type;
    static constexpr int T = RowRL<M>::T;
    static constexpr int BUF = buf_len<L_>(M);
    using S0 = StageK<L_, M, T, 0, kReverse, kMirror>;
    using SL = StageK<L_, M, T, L_::n - 1, kReverse, kMirror>;
    static constexpr int NL = S0::NB * (S0::R / 2);   // 16-byte loads per thread
};

// Stage-0 inputs of row qq + q g: float4 j + r Nb of row p1(n1) holds z(q) and z(m-1-q).
// Words [lo, hi) of the NL per thread.
template <int M>
__device__ __forceinline__ void dct_rows_load(const PlanSplit &p, const float *__restrict__ x, int qq, int g, int t,
                                              float4 (&f)[RowFwd<M>::NL], int lo = 0, int hi = RowFwd<M>::NL) {
    using S0 = typename RowFwd<M>::S0;
    const float4 *src = reinterpret_cast<const float4 *>(x + (size_t)perm_fwd(qq + p.q * g, p.n1) * p.n2);
#pragma unroll
    for (int b = 0; b < S0::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < S0::R / 2; ++rr) {
            const int i = b * (S0::R / 2) + rr;
            if (i >= lo && i < hi) f[i] = nt_load4(src + S0::j(t, b) + rr * S0::Nb);
        }
}

// FFT, split and 8-point DFT of one qq from the loaded inputs.  The first LDS
// write sits behind a barrier, so consecutive calls may reuse the buffers.
// hook(K) runs after FFT stage K (K < stages) and after the split (K = stages).
template <int M, class TB, class HK>
__device__ __forceinline__ void dct_rows_body(const PlanSplit &p, const TB &tb, const HK &hook, float2 *lds, int qq,
                                              int g, int t, const float4 (&f)[RowFwd<M>::NL],
                                              float2 *__restrict__ ws) {
    using F = RowFwd<M>;
    using L_ = typename F::L_;
    using S0 = typename F::S0;
    using SL = typename F::SL;
    constexpr int T = F::T, BUF = F::BUF;
    static_assert(64 % T == 0, "each row FFT lies inside one wavefront");
    const int Q = p.q;
    float2 *buf = lds + g * BUF;
    lds_sync();   // a previous call's 8-point stage may still read every buffer
    {
        float2 v0[S0::NB][S0::R];
        constexpr int H0 = S0::NB / 2;
#pragma unroll
        for (int b = 0; b < S0::NB; ++b) {
            const int pb = b < H0 ? b + H0 : b - H0;
#pragma unroll
            for (int rr = 0; rr < S0::R / 2; ++rr) {
                const float4 v = f[b * (S0::R / 2) + rr];
                v0[b][rr] = make_float2(v.x, v.z);
                v0[pb][S0::R - 1 - rr] = make_float2(v.w, v.y);
            }
        }
        float2 v2[SL::NB][SL::R];
        fft_run<L_, M, T, kReverse, kMirror, false, true>(buf, 1, 0, t, v0, v2, p.row, tb.tw(hook));
        fast::stage_sync<true>();   // the exchange buffer now receives the half spectrum
        constexpr int H = SL::NB / 2, R = SL::R, Nb = SL::Nb;
        auto sp = [&](int k, float2 zk, float2 zm) {
            const float2 wk = tb.split(k);
            float2 xk, xm;
            rsplit_pair(zk, zm, wk, make_float2(-wk.x, wk.y), xk, xm);
            buf[k] = xk;
            if (M - k != k) buf[M - k] = xm;
        };
#pragma unroll
        for (int b = 0; b < H; ++b) {
            const int jj = SL::j(t, b);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int k = jj + rr * Nb;
                if (b == 0 && t == 0) {
                    if (rr > R / 2) continue;
                    if (rr == 0) {
                        const float2 z0 = v2[0][0];
                        buf[0] = make_float2(z0.x + z0.y, z0.x - z0.y);   // X(0) + j X(m)
                        continue;
                    }
                    sp(k, v2[0][rr], v2[0][R - rr]);
                } else {
                    sp(k, v2[b][rr], v2[b + H][R - 1 - rr]);
                }
            }
        }
        if (t == 0) {
#pragma unroll
            for (int rr = 0; rr < R / 2; ++rr) sp(Nb / 2 + rr * Nb, v2[H][rr], v2[H][R - 1 - rr]);
        }
    }
    hook(L_::n);
    lds_sync();
    float2 w8[8];
#pragma unroll
    for (int kp = 0; kp < 8; ++kp) w8[kp] = tb.xtw(qq, kp);
    // positions k, k + 1 per thread: one 16-byte store per output row
    static_assert(M % (16 * T) == 0, "whole position pairs per thread");
#pragma unroll
    for (int e = 0; e < M / (16 * T); ++e) {
        const int k = 2 * threadIdx.x + e * 16 * T;
        float2 v[8], u[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            v[r] = lds[r * BUF + k];
            u[r] = lds[r * BUF + k + 1];
        }
        Dft<8, false>::run(v);
        Dft<8, false>::run(u);
#pragma unroll
        for (int kp = 0; kp < 8; ++kp) {
            const float2 a = cmul(v[kp], w8[kp]), b = cmul(u[kp], w8[kp]);
            *reinterpret_cast<float4 *>(ws + (size_t)(kp * Q + qq) * M + k) = make_float4(a.x, a.y, b.x, b.y);
        }
    }
}

template <int M>
__device__ __forceinline__ void ks_dct_rows_b(const PlanSplit &p, const float *__restrict__ x, float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    constexpr int T = RowRL<M>::T;
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    float4 f[RowFwd<M>::NL];
    dct_rows_load<M>(p, x, blockIdx.x, g, t, f);
    dct_rows_body<M>(p, RowTabsG{&p}, [](int) {}, lds, blockIdx.x, g, t, f, ws);
}
template <int M>
__global__ void __launch_bounds__(8 * RowRL<M>::T) ks_dct_rows(PlanSplit p, Io io) {
    ks_dct_rows_b<M>(p, io_src<float>(io), io_dst<float2>(io));
}

// Two qq per workgroup (qq = blockIdx.x and blockIdx.x + gridDim.x), for
// shapes whose row workgroup fills a CU's LDS alone: the tables are copied
// to LDS first, then the inputs of both qq are loaded into registers, so the
// second qq's rows arrive while the first is computed and the body waits on
// nothing but its own rows.
template <int M>
__device__ __forceinline__ void ks_dct_rows_p_b(const PlanSplit &p, const float *__restrict__ x, float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    using LT = RowLdsTabs<M>;
    constexpr int T = RowRL<M>::T, NL = RowFwd<M>::NL, NTH = 8 * T;
    constexpr int NTAB = (LT::F + NTH - 1) / NTH;
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    float4 tv[NTAB];
#pragma unroll
    for (int i = 0; i < NTAB; ++i) tv[i] = LT::src(p, threadIdx.x + i * NTH);
    float4 f0[NL], f1[NL];
    dct_rows_load<M>(p, x, blockIdx.x, g, t, f0);
    float4 *tab = reinterpret_cast<float4 *>(lds + 8 * buf_len<typename RowRL<M>::type>(M));
    // words past the tables land in row buffer 0, which is first written
    // after the body's opening barrier (an unconditional store keeps the
    // compiler from sinking the table loads behind the row loads)
#pragma unroll
    for (int i = 0; i < NTAB; ++i) {
        const int d = threadIdx.x + i * NTH;
        float4 *dst = d < LT::F ? tab + d : reinterpret_cast<float4 *>(lds) + (d - LT::F);
        *dst = tv[i];
    }
    const RowTabsL tb = LT::view(lds, p.n1);   // the body's first barrier publishes the tables
    // the second qq's rows are loaded a quarter at a time over the first's
    // FFT stages and split: all at once, the loads would fill the CU's
    // memory queue and hold every wavefront at the load instructions
    constexpr int NP = RowRL<M>::type::n + 1, CH = (NL + NP - 1) / NP;
    const int qq1 = blockIdx.x + gridDim.x;
    auto pf = [&](int K) { dct_rows_load<M>(p, x, qq1, g, t, f1, K * CH, (K + 1) * CH); };
    dct_rows_body<M>(p, tb, pf, lds, blockIdx.x, g, t, f0, ws);
    dct_rows_body<M>(p, tb, [](int) {}, lds, qq1, g, t, f1, ws);
}
template <int M>
__global__ void __launch_bounds__(8 * RowRL<M>::T) ks_dct_rows_p(PlanSplit p, Io io) {
    ks_dct_rows_p_b<M>(p, io_src<float>(io), io_dst<float2>(io));
}

// ---------------------------------------------------------- forward columns
// The two q-point FFTs of a sequence pair run side by side, each on half of
// the workgroup with its own LDS buffer (more wavefronts in flight than one
// after the other); their outputs go back to the buffers in natural order and
// the post then runs over all threads, reading the partners from LDS:
//   pair {kp, 8-kp}: element kq of A with q - 1 - kq of B, k1 = kp + 8 kq;
//   pair {0, 4}    : kq of sequence 0 with q - kq (k1 = 8 kq, kq <= q/2), and
//                    kq of sequence 4 with q - 1 - kq (k1 = 4 + 8 kq, kq < q/2).
template <int Q>
__device__ __forceinline__ void ks_dct_cols_b(const PlanSplit &p, const float2 *__restrict__ ws, float *__restrict__ y) {
    using CR = ColRL<Q>;
    using L_ = typename CR::type;
    constexpr int T = CR::T, C = CR::C, BUF = buf_len<L_>(Q);
    using S0 = StageK<L_, Q, T, 0, kCyclic, kCyclic>;
    using SL = StageK<L_, Q, T, L_::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int half = threadIdx.x / (C * T), ht = threadIdx.x % (C * T);
    const int c = ht % C, t = ht / C;
    const int M = p.m;
    const int ntiles = (M + C - 1) / C;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= 4 * ntiles) return;  // whole workgroup leaves together
    const int pg = unit / ntiles, tile = unit - pg * ntiles;
    const int kpA = pg == 0 ? 0 : pg, kpB = pg == 0 ? 4 : 8 - pg;
    const int kp = half == 0 ? kpA : kpB;
    const int k2 = tile * C + c;
    const bool act = k2 < M;
    float2 *buf = lds + half * C * BUF;
    {
        float2 v0[S0::NB][S0::R];
#pragma unroll
        for (int b = 0; b < S0::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < S0::R; ++rr) {
                const int q = t + (b + rr * S0::NB) * T;
                v0[b][rr] = act ? *ws_at(ws, kp * Q + q, M, k2) : make_float2(0.f, 0.f);
            }
        float2 v[SL::NB][SL::R];
        fft_run<L_, Q, T, kCyclic, kCyclic, false>(buf, C, c, t, v0, v, p.col);
        lds_sync();   // the last stage has read its inputs
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) buf[(t + (b + rr * SL::NB) * T) * C + c] = v[b][rr];
    }
    lds_sync();
    const float2 *bA = lds, *bB = lds + C * BUF;
    const int ntask = (pg == 0) ? Q + 1 : Q;
    for (int i = threadIdx.x; i < ntask * C; i += blockDim.x) {
        const int cc = i % C, task = i / C;
        const int kk2 = tile * C + cc;
        if (kk2 >= M) continue;
        int k1;
        float2 A, B;
        if (pg != 0) {
            k1 = kpA + 8 * task;
            A = bA[task * C + cc];
            B = bB[(Q - 1 - task) * C + cc];
        } else if (task <= Q / 2) {
            k1 = 8 * task;
            A = bA[task * C + cc];
            B = bA[((Q - task) & (Q - 1)) * C + cc];
        } else {
            const int kq = task - (Q / 2 + 1);
            k1 = 4 + 8 * kq;
            A = bB[kq * C + cc];
            B = bB[(Q - 1 - kq) * C + cc];
        }
        post_rows(p, y, k1, kk2, A, B);
    }
}
template <int Q>
__global__ void __launch_bounds__(2 * ColRL<Q>::T * ColRL<Q>::C) ks_dct_cols(PlanSplit p, Io io) {
    ks_dct_cols_b<Q>(p, io_src<float2>(io), io_dst<float>(io));
}

// Forward column pass with one FFT buffer (q = 1024, 16-column tiles): the
// two sequences of the unit run one after the other.  Pair {kp, 8 - kp}: A's
// outputs stay in registers, B goes to LDS in natural order, and the thread
// holding A(kq) reads its partner B(q - 1 - kq).  Pair {0, 4}: each sequence
// pairs with itself, so each goes to LDS and is posted before the next FFT
// reuses the buffer.  Same tasks, so each output is written once, as in
// ks_dct_cols.
template <int Q>
__device__ __forceinline__ void ks_dct_cols_seq_b(const PlanSplit &p, const float2 *__restrict__ ws, float *__restrict__ y) {
    using CR = ColRLInv<Q, 1>;
    using L_ = typename CR::type;
    constexpr int T = CR::T, C = CR::C;
    using S0 = StageK<L_, Q, T, 0, kCyclic, kCyclic>;
    using SL = StageK<L_, Q, T, L_::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int M = p.m;
    const int ntiles = (M + C - 1) / C;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= 4 * ntiles) return;  // whole workgroup leaves together
    const int pg = unit / ntiles, tile = unit - pg * ntiles;
    const int kpA = pg == 0 ? 0 : pg, kpB = pg == 0 ? 4 : 8 - pg;
    const int k2 = tile * C + c;
    const bool act = k2 < M;
    // every thread runs both FFTs and both LDS copies (they hold barriers)
    auto fft = [&](int kp, float2(&v)[SL::NB][SL::R]) {
        float2 v0[S0::NB][S0::R];
#pragma unroll
        for (int b = 0; b < S0::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < S0::R; ++rr) {
                const int q = t + (b + rr * S0::NB) * T;
                v0[b][rr] = act ? *ws_at(ws, kp * Q + q, M, k2) : make_float2(0.f, 0.f);
            }
        fft_run<L_, Q, T, kCyclic, kCyclic, false>(lds, C, c, t, v0, v, p.col);
    };
    auto to_lds = [&](const float2(&v)[SL::NB][SL::R]) {
        lds_sync();   // the last stage has read its inputs
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) lds[(t + (b + rr * SL::NB) * T) * C + c] = v[b][rr];
        lds_sync();
    };
    float2 va[SL::NB][SL::R];
    fft(kpA, va);
    if (pg != 0) {
        float2 vb[SL::NB][SL::R];
        fft(kpB, vb);
        to_lds(vb);
        if (!act) return;
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) {
                const int kq = t + (b + rr * SL::NB) * T;
                post_rows(p, y, kpA + 8 * kq, k2, va[b][rr], lds[(Q - 1 - kq) * C + c]);
            }
        return;
    }
    // sequence 0: kq with q - kq (k1 = 8 kq, kq <= q/2)
    to_lds(va);
    if (act) {
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) {
                const int kq = t + (b + rr * SL::NB) * T;
                if (kq <= Q / 2) post_rows(p, y, 8 * kq, k2, va[b][rr], lds[((Q - kq) & (Q - 1)) * C + c]);
            }
    }
    // sequence 4: kq with q - 1 - kq (k1 = 4 + 8 kq, kq < q/2); the FFT's
    // first exchange waits at a barrier until the posts above are done
    float2 vb[SL::NB][SL::R];
    fft(kpB, vb);
    to_lds(vb);
    if (!act) return;
#pragma unroll
    for (int b = 0; b < SL::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < SL::R; ++rr) {
            const int kq = t + (b + rr * SL::NB) * T;
            if (kq < Q / 2) post_rows(p, y, 4 + 8 * kq, k2, vb[b][rr], lds[(Q - 1 - kq) * C + c]);
        }
}
template <int Q>
__global__ void __launch_bounds__((ColRLInv<Q, 1>::T * ColRLInv<Q, 1>::C)) ks_dct_cols_seq(PlanSplit p, Io io) {
    ks_dct_cols_seq_b<Q>(p, io_src<float2>(io), io_dst<float>(io));
}

// Two units per workgroup (unit = xcd_tile(blockIdx.x + i gridDim.x) over
// 2 gridDim.x units), for shapes whose column workgroup fills a CU's LDS
// alone.  The column FFT twiddles live in LDS for the whole kernel and each
// unit's post factors (ta of its rows, tb of its columns) are copied to LDS
// before its FFT; the second unit's inputs are loaded over the first unit's
// FFT stages, so no wait on a younger load holds them up.
template <int Q>
struct ColLds {
    using CR = ColRL<Q>;
    using L_ = typename CR::type;
    static constexpr int C = CR::C, T = CR::T, BUF = buf_len<L_>(Q), n = L_::n;
    static constexpr int BUFS = 2 * C * BUF;   // float2
    static constexpr int off(int K) {
        int o = 0;
        for (int i = 1; i < K; ++i) o += L_::ns(i) * tw_record(L_::r[i]) / 2;
        return o;
    }
    static constexpr int TW = off(n);          // float4
    static constexpr int NTA = Q + 1, NTB = C + 2;
    // two factor sets, one per unit
    static constexpr size_t bytes() { return (size_t)BUFS * 8 + (size_t)TW * 16 + (size_t)2 * (NTA + NTB) * 8; }
    static_assert(BUFS % 2 == 0, "float4 alignment of the tables");
    static_assert(bytes() <= 160 * 1024, "buffers and tables must fit the LDS");
};

// Row k1 of post task `task` of sequence group pg.
__device__ __forceinline__ int col_task_k1(int pg, int task, int Q) {
    if (pg != 0) return pg + 8 * task;
    return task <= Q / 2 ? 8 * task : 4 + 8 * (task - (Q / 2 + 1));
}

// Loads value i (i = b + rr NB) of the thread's column sequence for words [lo, hi).
template <int Q, class S0>
__device__ __forceinline__ void cols_load(const PlanSplit &p, const float2 *__restrict__ ws, int kp, int k2, bool act,
                                          int t, float2 (&v)[S0::NB][S0::R], int lo, int hi) {
    constexpr int T = ColRL<Q>::T;
#pragma unroll
    for (int b = 0; b < S0::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < S0::R; ++rr) {
            const int i = b * S0::R + rr;
            if (i < lo || i >= hi) continue;
            const int q = t + (b + rr * S0::NB) * T;
            v[b][rr] = act ? *ws_at(ws, kp * Q + q, p.m, k2) : make_float2(0.f, 0.f);
        }
}

template <int Q>
__device__ __forceinline__ void ks_dct_cols_p_b(const PlanSplit &p, const float2 *__restrict__ ws, float *__restrict__ y) {
    using LC = ColLds<Q>;
    using L_ = typename LC::L_;
    constexpr int T = LC::T, C = LC::C, BUF = LC::BUF, NTH = 2 * C * T;
    using S0 = StageK<L_, Q, T, 0, kCyclic, kCyclic>;
    using SL = StageK<L_, Q, T, L_::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    float4 *twl = reinterpret_cast<float4 *>(lds + LC::BUFS);
    float2 *lta = reinterpret_cast<float2 *>(twl + LC::TW);   // factor sets of units 0 and 1
    const int half = threadIdx.x / (C * T), ht = threadIdx.x % (C * T);
    const int c = ht % C, t = ht / C;
    const int M = p.m, ntiles = M / C;
    float2 *buf = lds + half * C * BUF;

    struct U {
        int pg, tile, kpA, kp, k2;
    };
    auto unit_of = [&](int i) {
        U u;
        const int unit = xcd_tile(blockIdx.x + i * gridDim.x, 2 * gridDim.x);
        u.pg = unit / ntiles;
        u.tile = unit - u.pg * ntiles;
        u.kpA = u.pg == 0 ? 0 : u.pg;
        u.kp = half == 0 ? u.kpA : (u.pg == 0 ? 4 : 8 - u.pg);
        u.k2 = u.tile * C + c;
        return u;
    };
    // post factors of a unit: ta for its tasks, tb for its columns, tb(0), tb(m)
    constexpr int NF = (LC::NTA + LC::NTB + NTH - 1) / NTH;
    auto fac_load = [&](const U &u, float2 (&f)[NF]) {
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int d = threadIdx.x + i * NTH;
            int idx;
            const float2 *src;
            if (d < LC::NTA) {
                const int task = d < ((u.pg == 0) ? Q + 1 : Q) ? d : 0;
                src = p.ta;
                idx = col_task_k1(u.pg, task, Q);
            } else {
                const int e = d - LC::NTA;
                src = p.tb;
                idx = e < C ? u.tile * C + e : (e == C ? 0 : M);
                idx = idx <= M ? idx : M;
            }
            f[i] = src[idx];
        }
    };
    auto fac_store = [&](const float2 (&f)[NF], int set) {
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int d = threadIdx.x + i * NTH;
            if (d < LC::NTA + LC::NTB) lta[set * (LC::NTA + LC::NTB) + d] = f[i];
        }
    };

    const U u0 = unit_of(0), u1 = unit_of(1);
    // column FFT twiddles (transposed records) and unit 0's factors, then its data
    constexpr int NTW = (LC::TW + NTH - 1) / NTH;
    float4 tw[NTW];
#pragma unroll
    for (int i = 0; i < NTW; ++i) {
        const int d = threadIdx.x + i * NTH;
        const float4 *ptr = reinterpret_cast<const float4 *>(p.col.tw);
        int idx = 0;
#pragma unroll
        for (int K = 1; K < L_::n; ++K) {
            constexpr int unused = 0;
            (void)unused;
            const int NS = L_::ns(K), H = tw_record(L_::r[K]) / 2;
            const bool in = d >= LC::off(K) && d < LC::off(K + 1);
            const int dd = d - LC::off(K);
            ptr = in ? reinterpret_cast<const float4 *>(p.col.tw + p.col.twoff[K]) : ptr;
            idx = in ? (dd % NS) * H + dd / NS : idx;
        }
        tw[i] = ptr[idx];
    }
    float2 f0[NF], f1[NF];
    fac_load(u0, f0);
    fac_load(u1, f1);
    float2 v0[S0::NB][S0::R], v1[S0::NB][S0::R];
    cols_load<Q, S0>(p, ws, u0.kp, u0.k2, true, t, v0, 0, S0::NB * S0::R);
#pragma unroll
    for (int i = 0; i < NTW; ++i) {
        const int d = threadIdx.x + i * NTH;
        if (d < LC::TW) twl[d] = tw[i];
    }
    fac_store(f0, 0);
    fac_store(f1, 1);
    fast::LdsTw tabs;
#pragma unroll
    for (int K = 0; K < kMaxStages; ++K) tabs.tab[K] = twl + (K >= 1 && K < L_::n ? LC::off(K) : 0);

    auto unit_run = [&](const U &u, int set, float2 (&vin)[S0::NB][S0::R], auto hook) {
        const float2 *ta = lta + set * (LC::NTA + LC::NTB), *tbv = ta + LC::NTA;
        {
            float2 v[SL::NB][SL::R];
            fft_run<L_, Q, T, kCyclic, kCyclic, false>(buf, C, c, t, vin, v, p.col,
                                                        fast::LdsTwHook<decltype(hook)>{tabs, hook});
            hook(L_::n);
            lds_sync();   // the last stage has read its inputs
#pragma unroll
            for (int b = 0; b < SL::NB; ++b)
#pragma unroll
                for (int rr = 0; rr < SL::R; ++rr) buf[(t + (b + rr * SL::NB) * T) * C + c] = v[b][rr];
        }
        lds_sync();
        const float2 *bA = lds, *bB = lds + C * BUF;
        const int ntask = (u.pg == 0) ? Q + 1 : Q;
        const float2 bm = tbv[C + 1];
#pragma unroll
        for (int it = 0; it < ((Q + 1) * C + NTH - 1) / NTH; ++it) {
            const int i = threadIdx.x + it * NTH;
            if (i >= ntask * C) continue;
            const int cc = i % C, task = i / C;
            const int kk2 = u.tile * C + cc;
            float2 A, B;
            if (u.pg != 0) {
                A = bA[task * C + cc];
                B = bB[(Q - 1 - task) * C + cc];
            } else if (task <= Q / 2) {
                A = bA[task * C + cc];
                B = bA[((Q - task) & (Q - 1)) * C + cc];
            } else {
                const int kq = task - (Q / 2 + 1);
                A = bB[kq * C + cc];
                B = bB[(Q - 1 - kq) * C + cc];
            }
            post_rows_v(p, y, col_task_k1(u.pg, task, Q), kk2, A, B, ta[task], tbv[cc], bm);
        }
    };
    // the second unit's inputs, a part after each FFT stage of the first
    // (all before the first unit's stores)
    constexpr int NP = L_::n + 1, CH = (S0::NB * S0::R + NP - 1) / NP;
    auto pf = [&](int K) { cols_load<Q, S0>(p, ws, u1.kp, u1.k2, true, t, v1, K * CH, (K + 1) * CH); };
    unit_run(u0, 0, v0, pf);
    unit_run(u1, 1, v1, [](int) {});   // its FFT's first barrier follows unit 0's post
}
template <int Q>
__global__ void __launch_bounds__(2 * ColRL<Q>::T * ColRL<Q>::C) ks_dct_cols_p(PlanSplit p, Io io) {
    ks_dct_cols_p_b<Q>(p, io_src<float2>(io), io_dst<float>(io));
}

// ---------------------------------------------------- fused spectral columns
// The middle of a spectral solve in split form (the Neumann Poisson solve, or
// the threshold compression): the forward q-point FFTs of a sequence pair
// (side by side, as ks_dct_cols), then for every row pair the four-element
// post, the pointwise step of PoissonTabs (the divide by the eigenvalues
// lam = l1(k1) + l2(k2) with U(0,0) = 0, or the threshold) and the four-read
// IDCT pre, written back to the same LDS slots, then the inverse q-point FFTs,
// in place in the workspace.  The spectrum F never reaches memory.
template <int Q, int MODE>
__device__ __forceinline__ void ks_poisson_cols_b(const PlanSplit &p, PoissonTabs pq, float2 *__restrict__ ws) {
    using CR = ColRL<Q>;
    using L_ = typename CR::type;
    constexpr int T = CR::T, C = CR::C, BUF = buf_len<L_>(Q);
    using S0 = StageK<L_, Q, T, 0, kCyclic, kCyclic>;
    using SL = StageK<L_, Q, T, L_::n - 1, kCyclic, kCyclic>;
    extern __shared__ float2 lds[];
    const int half = threadIdx.x / (C * T), ht = threadIdx.x % (C * T);
    const int c = ht % C, t = ht / C;
    const int M = p.m, N1 = p.n1, N2 = p.n2;
    const int ntiles = (M + C - 1) / C;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= 4 * ntiles) return;  // whole workgroup leaves together
    const int pg = unit / ntiles, tile = unit - pg * ntiles;
    const int kpA = pg == 0 ? 0 : pg, kpB = pg == 0 ? 4 : 8 - pg;
    const int kp = half == 0 ? kpA : kpB;
    const int k2 = tile * C + c;
    const bool act = k2 < M;
    float2 *buf = lds + half * C * BUF;
    {
        float2 v0[S0::NB][S0::R];
#pragma unroll
        for (int b = 0; b < S0::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < S0::R; ++rr) {
                const int qq = t + (b + rr * S0::NB) * T;
                v0[b][rr] = act ? *ws_at(ws, kp * Q + qq, M, k2) : make_float2(0.f, 0.f);
            }
        float2 v[SL::NB][SL::R];
        fft_run<L_, Q, T, kCyclic, kCyclic, false>(buf, C, c, t, v0, v, p.col);
        lds_sync();   // the last stage has read its inputs
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) buf[(t + (b + rr * SL::NB) * T) * C + c] = v[b][rr];
    }
    lds_sync();
    float2 *bA = lds, *bB = lds + C * BUF;
    const int ntask = (pg == 0) ? Q + 1 : Q;
    for (int i = threadIdx.x; i < ntask * C; i += blockDim.x) {
        const int cc = i % C, task = i / C;
        const int kk2 = tile * C + cc;
        if (kk2 >= M) continue;
        int k1;
        float2 *pa, *pb;
        if (pg != 0) {
            k1 = kpA + 8 * task;
            pa = bA + task * C + cc;
            pb = bB + (Q - 1 - task) * C + cc;
        } else if (task <= Q / 2) {
            k1 = 8 * task;
            pa = bA + task * C + cc;
            pb = bA + ((Q - task) & (Q - 1)) * C + cc;
        } else {
            const int kq = task - (Q / 2 + 1);
            k1 = 4 + 8 * kq;
            pa = bB + kq * C + cc;
            pb = bB + (Q - 1 - kq) * C + cc;
        }
        const int k1p = (k1 == 0) ? 0 : N1 - k1;
        const float2 A = *pa, B = *pb;
        const float2 a = p.ta[k1];
        const int k2r = (kk2 == 0) ? M : N2 - kk2;
        const float l1a = pq.l1[k1], l1b = pq.l1[k1p], l2a = pq.l2[kk2], l2b = pq.l2[k2r];
        float2 xa, xb;
        if (kk2 == 0) {
            const float2 v0a = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
            const float2 v0b = make_float2(0.5f * (B.x + A.x), 0.5f * (B.y - A.y));
            const float2 vma = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
            const float2 vmb = make_float2(0.5f * (B.y + A.y), -0.5f * (B.x - A.x));
            const float4 f0 = post4(a, p.tb[0], v0a, v0b);
            const float4 fm = post4(a, p.tb[M], vma, vmb);
            const float4 U = make_float4(spec_op<MODE>(pq, f0.x, l1a, l2a, k1 == 0), spec_op<MODE>(pq, fm.x, l1a, l2b, false),
                                         spec_op<MODE>(pq, f0.z, l1b, l2a, k1p == 0), spec_op<MODE>(pq, fm.z, l1b, l2b, false));
            const float2 P = make_float2(U.x, U.y), Qv = make_float2(U.z, U.w);
            const float2 Rv = (k1 == 0) ? make_float2(0.f, 0.f) : (k1p == k1 ? P : Qv);
            const float2 ai = pq.tai[k1], bi = pq.tbi[0], bim = pq.tbi[M];
            xa = pre1_dc(cmul(ai, bi), cmul(ai, bim), P, Rv);
            const float2 aip = pq.tai[k1p];
            xb = pre1_dc(cmul(aip, bi), cmul(aip, bim), Qv, P);
        } else {
            const float4 f = post4(a, p.tb[kk2], A, B);
            const float4 U = make_float4(spec_op<MODE>(pq, f.x, l1a, l2a, false), spec_op<MODE>(pq, f.y, l1a, l2b, false),
                                         spec_op<MODE>(pq, f.z, l1b, l2a, false), spec_op<MODE>(pq, f.w, l1b, l2b, false));
            const float2 P = make_float2(U.x, U.y), Qv = make_float2(U.z, U.w);
            const float2 Rv = (k1 == 0) ? make_float2(0.f, 0.f) : (k1p == k1 ? P : Qv);
            const float2 bi = pq.tbi[kk2];
            xa = pre1(cmul(pq.tai[k1], bi), P, Rv);
            xb = pre1(cmul(pq.tai[k1p], bi), Qv, P);
        }
        *pa = xa;
        if (k1p != k1) *pb = xb;
    }
    lds_sync();
    {
        float2 v0[S0::NB][S0::R];
#pragma unroll
        for (int b = 0; b < S0::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < S0::R; ++rr) v0[b][rr] = buf[(t + (b + rr * S0::NB) * T) * C + c];
        float2 v[SL::NB][SL::R];
        fft_run<L_, Q, T, kCyclic, kCyclic, true>(buf, C, c, t, v0, v, p.col);   // barrier before its first write
        if (!act) return;
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) {
                const int qq = t + (b + rr * SL::NB) * T;
                *ws_at(ws, kp * Q + qq, M, k2) = v[b][rr];
            }
    }
}
template <int Q, int MODE>
__global__ void __launch_bounds__(2 * ColRL<Q>::T * ColRL<Q>::C) ks_poisson_cols(PlanSplit p, PoissonTabs pq, Io io) {
    ks_poisson_cols_b<Q, MODE>(p, pq, io_dst<float2>(io));
}

// ---------------------------------------------------------- inverse columns
template <int Q, int MA, int MB, int XST, int W>
__device__ __forceinline__ void idct_cols_pair(const PlanSplit &p, const float *__restrict__ x,
                                               float2 *__restrict__ ws, float2 *lds, int c, int t, int k2, bool act,
                                               int kpA, int kpB) {
    using CR = ColRLInv<Q, W>;
    using L_ = typename CR::type;
    constexpr int T = CR::T, C = CR::C;
    using SA = StageK<L_, Q, T, 0, MA, kCyclic>;
    using SB = StageK<L_, Q, T, 0, MB, kCyclic>;
    using SL = StageK<L_, Q, T, L_::n - 1, MA, kCyclic>;
    constexpr int R = SA::R, Nb = SA::Nb;
    const int M = p.m;
    float2 va[SA::NB][SA::R], vb[SB::NB][SB::R];
#pragma unroll
    for (int b = 0; b < SA::NB; ++b)
#pragma unroll
        for (int rr = 0; rr < R; ++rr) va[b][rr] = vb[b][rr] = make_float2(0.f, 0.f);
    if (act) {
        if (MA == kMirror) {
            // sequence 0 (k1 = 8 kq with 8 (q - kq)), then sequence 4 (4 + 8 kq with 4 + 8 (q - 1 - kq))
            constexpr int H = SA::NB / 2;
#pragma unroll
            for (int b = 0; b < H; ++b) {
                const int jj = SA::j(t, b);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    const int kq = jj + rr * Nb;
                    float2 f, g;
                    if (b == 0 && t == 0) {
                        if (rr > R / 2) continue;
                        pre_rows<XST>(p, x, 8 * kq, k2, f, g);
                        va[0][rr] = f;
                        if (rr != 0 && rr != R / 2) va[0][(R - rr) % R] = g;
                    } else {
                        pre_rows<XST>(p, x, 8 * kq, k2, f, g);
                        va[b][rr] = f;
                        va[b + H][R - 1 - rr] = g;
                    }
                }
            }
            if (t == 0) {
#pragma unroll
                for (int rr = 0; rr < R / 2; ++rr) {
                    float2 f, g;
                    pre_rows<XST>(p, x, 8 * (Nb / 2 + rr * Nb), k2, f, g);
                    va[H][rr] = f;
                    va[H][R - 1 - rr] = g;
                }
            }
#pragma unroll
            for (int b = 0; b < H; ++b) {
                const int jj = SB::j(t, b);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    float2 f, g;
                    pre_rows<XST>(p, x, 4 + 8 * (jj + rr * Nb), k2, f, g);
                    vb[b][rr] = f;
                    vb[b + H][R - 1 - rr] = g;
                }
            }
        } else {
#pragma unroll
            for (int b = 0; b < SA::NB; ++b) {
                const int jj = SA::j(t, b);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) {
                    float2 f, g;
                    pre_rows<XST>(p, x, kpA + 8 * (jj + rr * Nb), k2, f, g);
                    va[b][rr] = f;
                    vb[b][R - 1 - rr] = g;
                }
            }
        }
    }
    auto store = [&](int kp, const float2(&v)[SL::NB][SL::R]) {
        if (!act) return;
#pragma unroll
        for (int b = 0; b < SL::NB; ++b)
#pragma unroll
            for (int rr = 0; rr < SL::R; ++rr) {
                const int q = t + (b + rr * SL::NB) * T;
                *ws_at(ws, kp * Q + q, M, k2) = v[b][rr];
            }
    };
    {
        float2 out[SL::NB][SL::R];
        fft_run<L_, Q, T, MA, kCyclic, true>(lds, C, c, t, va, out, p.col);
        store(kpA, out);
    }
    {
        float2 out[SL::NB][SL::R];
        fft_run<L_, Q, T, MB, kCyclic, true>(lds, C, c, t, vb, out, p.col);
        store(kpB, out);
    }
}

// XST: the IDXST axes of the plan (the p.xst bits), fixed at compile time.
template <int Q, int XST, int W>
__device__ __forceinline__ void ks_idct_cols_b(const PlanSplit &p, const float *__restrict__ x, float2 *__restrict__ ws) {
    constexpr int C = ColRLInv<Q, W>::C;
    extern __shared__ float2 lds[];
    const int c = threadIdx.x % C;
    const int t = threadIdx.x / C;
    const int ntiles = (p.m + C - 1) / C;
    const int unit = xcd_tile(blockIdx.x, gridDim.x);
    if (unit >= 4 * ntiles) return;
    const int pg = unit / ntiles, tile = unit - pg * ntiles;
    const int k2 = tile * C + c;
    const bool act = k2 < p.m;
    if (pg == 0)
        idct_cols_pair<Q, kMirror, kReverse, XST, W>(p, x, ws, lds, c, t, k2, act, 0, 4);
    else
        idct_cols_pair<Q, kCyclic, kRevCyclic, XST, W>(p, x, ws, lds, c, t, k2, act, pg, 8 - pg);
}
template <int Q, int XST, int W>
__global__ void __launch_bounds__((ColRLInv<Q, W>::T * ColRLInv<Q, W>::C)) ks_idct_cols(PlanSplit p, Io io) {
    ks_idct_cols_b<Q, XST, W>(p, io_src<float>(io), io_dst<float2>(io));
}

// ------------------------------------------------------------- inverse rows
// One workgroup per qq: the eight workspace rows kp q + qq are read with
// whole-row coalesced loads, conj-twiddled and inverse-DFT'd across kp into
// eight LDS buffers (row qq + q r in buffer r); then group g runs the inverse
// split and inverse FFT of its row from buffer g and stores output row
// p1(qq + q g) with the Eq. (2d_idct_post) reorder (16-byte stores).
template <int M>
struct RowInv {
    static constexpr int T = RowRL<M>::T;
    static constexpr int E = M / (16 * T);   // position pairs (k, k + 1) per thread in the 8-point stage
    static_assert(M % (16 * T) == 0, "whole position pairs per thread");
};

// The eight workspace rows kp q + qq at positions k, k + 1 (k = 2 tid + e 16T),
// one 16-byte load each; values [lo, hi) of the 8 E per thread (value e 8 + kp).
template <int M>
__device__ __forceinline__ void idct_rows_load(const PlanSplit &p, const float2 *__restrict__ ws, int qq,
                                               float4 (&v)[RowInv<M>::E][8], int lo = 0, int hi = 8 * RowInv<M>::E) {
    constexpr int T = RowInv<M>::T;
#pragma unroll
    for (int e = 0; e < RowInv<M>::E; ++e)
#pragma unroll
        for (int kp = 0; kp < 8; ++kp)
            if (e * 8 + kp >= lo && e * 8 + kp < hi)
                v[e][kp] = *reinterpret_cast<const float4 *>(ws + (size_t)(kp * p.q + qq) * M + 2 * threadIdx.x +
                                                             e * 16 * T);
}

template <int M, class TB, class HK>
__device__ __forceinline__ void idct_rows_body(const PlanSplit &p, const TB &tb, const HK &hook, float2 *lds, int qq,
                                               int g, int t, const float4 (&in)[RowInv<M>::E][8],
                                               float *__restrict__ y) {
    using L_ = typename RowRL<M>::type;
    constexpr int T = RowRL<M>::T;
    constexpr int BUF = buf_len<L_>(M);
    using S0 = StageK<L_, M, T, 0, kMirror, kReverse>;
    using SL = StageK<L_, M, T, L_::n - 1, kMirror, kReverse>;
    const int Q = p.q, N1 = p.n1;
    lds_sync();   // the previous call may still read the buffers
    {
        float2 w8[8];
#pragma unroll
        for (int kp = 0; kp < 8; ++kp) w8[kp] = tb.xtw(qq, kp);
#pragma unroll
        for (int e = 0; e < RowInv<M>::E; ++e) {
            const int k = 2 * threadIdx.x + e * 16 * T;
            float2 v[8], u[8];
#pragma unroll
            for (int kp = 0; kp < 8; ++kp) {
                const float4 f = in[e][kp];
                v[kp] = cmulc(make_float2(f.x, f.y), w8[kp]);
                u[kp] = cmulc(make_float2(f.z, f.w), w8[kp]);
            }
            Dft<8, true>::run(v);
            Dft<8, true>::run(u);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                lds[r * BUF + k] = v[r];
                lds[r * BUF + k + 1] = u[r];
            }
        }
    }
    hook(0);
    lds_sync();
    float2 *buf = lds + g * BUF;
    constexpr int H = S0::NB / 2, R = S0::R, Nb = S0::Nb;
    float2 v0[S0::NB][S0::R];
    // inverse split on the pairs (k, m - k), U(0) = Re P(0), U(m) = Im P(0)
    auto isp = [&](int k, float2 &zk, float2 &zm) {
        const float2 wk = tb.split(k);
        irsplit_pair(buf[k], buf[M - k], wk, make_float2(-wk.x, wk.y), zk, zm);
    };
#pragma unroll
    for (int b = 0; b < H; ++b) {
        const int jj = S0::j(t, b);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int k = jj + rr * Nb;
            if (b == 0 && t == 0) {
                if (rr > R / 2) continue;
                if (rr == 0) {
                    const float2 p0 = buf[0];
                    v0[0][0] = make_float2(p0.x + p0.y, p0.x - p0.y);
                    continue;
                }
                float2 f, gg;
                isp(k, f, gg);
                v0[0][rr] = f;
                if (rr != R / 2) v0[0][R - rr] = gg;
            } else {
                isp(k, v0[b][rr], v0[b + H][R - 1 - rr]);
            }
        }
    }
    if (t == 0) {
#pragma unroll
        for (int rr = 0; rr < R / 2; ++rr) isp(Nb / 2 + rr * Nb, v0[H][rr], v0[H][R - 1 - rr]);
    }
    float2 v2[SL::NB][SL::R];
    static_assert(64 % T == 0, "each row FFT lies inside one wavefront");
    fft_run<L_, M, T, kMirror, kReverse, true, true>(buf, 1, 0, t, v0, v2, p.row,
                                                     tb.tw([&hook](int K) { hook(K + 1); }));
    // Eq. (2d_idct_post): float4 q = j + r Nb of output row p1(n1) is
    // (z(q).x, z(m-1-q).y, z(q).y, z(m-1-q).x)
    const int orow = perm_fwd(qq + Q * g, N1);
    float4 *dst = reinterpret_cast<float4 *>(y + (size_t)orow * p.n2);
    constexpr int H2 = SL::NB / 2;
#pragma unroll
    for (int b = 0; b < SL::NB; ++b) {
        const int jj = SL::j(t, b);
        const int pb = b < H2 ? b + H2 : b - H2;
#pragma unroll
        for (int rr = 0; rr < SL::R / 2; ++rr) {
            const float2 a = v2[b][rr];
            const float2 m = v2[pb][SL::R - 1 - rr];
            nt_store4(dst + jj + rr * SL::Nb, xst_sign4(p.xst, orow, make_float4(a.x, m.y, a.y, m.x)));
        }
    }
}

template <int M>
__device__ __forceinline__ void ks_idct_rows_b(const PlanSplit &p, const float2 *__restrict__ ws, float *__restrict__ y) {
    extern __shared__ float2 lds[];
    constexpr int T = RowRL<M>::T;
    float4 v[RowInv<M>::E][8];
    idct_rows_load<M>(p, ws, blockIdx.x, v);
    idct_rows_body<M>(p, RowTabsG{&p}, [](int) {}, lds, blockIdx.x, threadIdx.x / T, threadIdx.x % T, v, y);
}
template <int M>
__global__ void __launch_bounds__(8 * RowRL<M>::T) ks_idct_rows(PlanSplit p, Io io) {
    ks_idct_rows_b<M>(p, io_src<float2>(io), io_dst<float>(io));
}

// Two qq per workgroup with the tables in LDS (see ks_dct_rows_p).
template <int M>
__device__ __forceinline__ void ks_idct_rows_p_b(const PlanSplit &p, const float2 *__restrict__ ws, float *__restrict__ y) {
    extern __shared__ float2 lds[];
    using LT = RowLdsTabs<M>;
    constexpr int T = RowRL<M>::T, E = RowInv<M>::E, NTH = 8 * T;
    constexpr int NTAB = (LT::F + NTH - 1) / NTH;
    float4 tv[NTAB];
#pragma unroll
    for (int i = 0; i < NTAB; ++i) tv[i] = LT::src(p, threadIdx.x + i * NTH);
    float4 v0[E][8], v1[E][8];
    idct_rows_load<M>(p, ws, blockIdx.x, v0);
    float4 *tab = reinterpret_cast<float4 *>(lds + 8 * buf_len<typename RowRL<M>::type>(M));
    // words past the tables land in row buffer 0, which is first written
    // after the body's opening barrier (an unconditional store keeps the
    // compiler from sinking the table loads behind the row loads)
#pragma unroll
    for (int i = 0; i < NTAB; ++i) {
        const int d = threadIdx.x + i * NTH;
        float4 *dst = d < LT::F ? tab + d : reinterpret_cast<float4 *>(lds) + (d - LT::F);
        *dst = tv[i];
    }
    const RowTabsL tb = LT::view(lds, p.n1);   // the body's first barrier publishes the tables
    // the second qq's workspace rows are loaded a part at a time over the
    // first's FFT (see ks_dct_rows_p)
    constexpr int NP = RowRL<M>::type::n + 1, CH = (8 * E + NP - 1) / NP;
    const int qq1 = blockIdx.x + gridDim.x;
    auto pf = [&](int K) { idct_rows_load<M>(p, ws, qq1, v1, K * CH, (K + 1) * CH); };
    idct_rows_body<M>(p, tb, pf, lds, blockIdx.x, threadIdx.x / T, threadIdx.x % T, v0, y);
    idct_rows_body<M>(p, tb, [](int) {}, lds, qq1, threadIdx.x / T, threadIdx.x % T, v1, y);
}
template <int M>
__global__ void __launch_bounds__(8 * RowRL<M>::T) ks_idct_rows_p(PlanSplit p, Io io) {
    ks_idct_rows_p_b<M>(p, io_src<float2>(io), io_dst<float>(io));
}

template <class K>
inline void set_lds(K kernel, size_t bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int M>
hipError_t rows_fwd(const PlanSplit &p, const Io &io, hipStream_t s) {
    const size_t lds = 8 * (size_t)buf_len<typename RowRL<M>::type>(M) * sizeof(float2);
    if constexpr (M == 2048) {
        if (p.persist && p.q % 2 == 0) {
            const size_t lp = RowLdsTabs<M>::bytes();
            set_lds(ks_dct_rows_p<M>, lp);
            hipLaunchKernelGGL(ks_dct_rows_p<M>, dim3(p.q / 2, io.n), dim3(8 * RowRL<M>::T), lp, s, p, io);
            return hipGetLastError();
        }
    }
    set_lds(ks_dct_rows<M>, lds);
    hipLaunchKernelGGL(ks_dct_rows<M>, dim3(p.q, io.n), dim3(8 * RowRL<M>::T), lds, s, p, io);
    return hipGetLastError();
}

template <int M>
hipError_t rows_inv(const PlanSplit &p, const Io &io, hipStream_t s) {
    const size_t lds = 8 * (size_t)buf_len<typename RowRL<M>::type>(M) * sizeof(float2);
    if constexpr (M == 2048) {
        if (p.persist && p.q % 2 == 0) {
            const size_t lp = RowLdsTabs<M>::bytes();
            set_lds(ks_idct_rows_p<M>, lp);
            hipLaunchKernelGGL(ks_idct_rows_p<M>, dim3(p.q / 2, io.n), dim3(8 * RowRL<M>::T), lp, s, p, io);
            return hipGetLastError();
        }
    }
    set_lds(ks_idct_rows<M>, lds);
    hipLaunchKernelGGL(ks_idct_rows<M>, dim3(p.q, io.n), dim3(8 * RowRL<M>::T), lds, s, p, io);
    return hipGetLastError();
}

template <int Q>
hipError_t cols_fwd(const PlanSplit &p, const Io &io, hipStream_t s) {
    constexpr int C = ColRL<Q>::C, T = ColRL<Q>::T;
    if constexpr (Q <= 512) {
        if (p.persist && p.m % C == 0 && (4 * (p.m / C)) % 16 == 0) {
            const size_t lp = ColLds<Q>::bytes();
            set_lds(ks_dct_cols_p<Q>, lp);
            hipLaunchKernelGGL(ks_dct_cols_p<Q>, dim3(2 * (p.m / C), io.n), dim3(2 * C * T), lp, s, p, io);
            return hipGetLastError();
        }
    }
    if constexpr (Q == 1024) {
        // one buffer, 16-column tiles once they give every CU a workgroup
        if (p.m >= 1024) {
            using CI = ColRLInv<Q, 1>;
            const size_t l1 = (size_t)CI::C * buf_len<typename CI::type>(Q) * sizeof(float2);
            set_lds(ks_dct_cols_seq<Q>, l1);
            const int u1 = 4 * ((p.m + CI::C - 1) / CI::C);
            hipLaunchKernelGGL(ks_dct_cols_seq<Q>, dim3((u1 + 7) & ~7, io.n), dim3(CI::C * CI::T), l1, s, p, io);
            return hipGetLastError();
        }
    }
    const size_t lds = (size_t)C * buf_len<typename ColRL<Q>::type>(Q) * sizeof(float2);
    set_lds(ks_dct_cols<Q>, 2 * lds);
    const int units = 4 * ((p.m + C - 1) / C);
    hipLaunchKernelGGL(ks_dct_cols<Q>, dim3((units + 7) & ~7, io.n), dim3(2 * C * T), 2 * lds, s, p, io);
    return hipGetLastError();
}

template <int Q, int MODE>
hipError_t cols_poisson_m(const PlanSplit &p, const PoissonTabs &q, const Io &io, hipStream_t s) {
    constexpr int C = ColRL<Q>::C, T = ColRL<Q>::T;
    const size_t lds = 2 * (size_t)C * buf_len<typename ColRL<Q>::type>(Q) * sizeof(float2);
    set_lds(ks_poisson_cols<Q, MODE>, lds);
    const int units = 4 * ((p.m + C - 1) / C);
    hipLaunchKernelGGL((ks_poisson_cols<Q, MODE>), dim3((units + 7) & ~7, io.n), dim3(2 * C * T), lds, s, p, q, io);
    return hipGetLastError();
}

template <int Q>
hipError_t cols_poisson(const PlanSplit &p, const PoissonTabs &q, const Io &io, hipStream_t s) {
    return q.mode == 1 ? cols_poisson_m<Q, 1>(p, q, io, s) : cols_poisson_m<Q, 0>(p, q, io, s);
}

template <int Q, int XST, int W>
hipError_t cols_inv_w(const PlanSplit &p, const Io &io, hipStream_t s) {
    constexpr int C = ColRLInv<Q, W>::C, T = ColRLInv<Q, W>::T;
    const size_t lds = (size_t)C * buf_len<typename ColRLInv<Q, W>::type>(Q) * sizeof(float2);
    set_lds(ks_idct_cols<Q, XST, W>, lds);
    const int units = 4 * ((p.m + C - 1) / C);
    hipLaunchKernelGGL((ks_idct_cols<Q, XST, W>), dim3((units + 7) & ~7, io.n), dim3(C * T), lds, s, p, io);
    return hipGetLastError();
}

// q = 1024: 16-column tiles once they make at least one workgroup per CU of
// the 256 (m >= 1024), else 8. Measured inverse column pass, 8 vs 16 columns:
// 8192^2 232 vs 202 us, 8192 x 2048 51 vs 45 us, 8192 x 1000 30 vs 35 us.
// Below q = 1024 both widths are 16.
template <int Q, int XST>
hipError_t cols_inv_x(const PlanSplit &p, const Io &io, hipStream_t s) {
    if constexpr (Q == 1024) {
        if (p.m < 1024) return cols_inv_w<Q, XST, 0>(p, io, s);
    }
    return cols_inv_w<Q, XST, 1>(p, io, s);
}

template <int Q>
hipError_t cols_inv(const PlanSplit &p, const Io &io, hipStream_t s) {
    switch (p.xst) {
        case 0: return cols_inv_x<Q, 0>(p, io, s);
        case 1: return cols_inv_x<Q, 1>(p, io, s);
        case 2: return cols_inv_x<Q, 2>(p, io, s);
        case 3: return cols_inv_x<Q, 3>(p, io, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------- separate radix-8 step
// Long columns (q = 1024): the first radix-8 step of the column FFTs as a pass
// of its own over the plain row pass's workspace,
//   forward: row kp q + qq <- W_n1^(qq kp) sum_r W_8^(r kp) Z(qq + q r),
//   inverse: row qq + q r  <- sum_kp W_8^(-r kp) conj(W_n1^(qq kp)) Z(kp q + qq).
// The eight rows read and written are the same rows qq + q j, so each thread
// works in place on its (qq, k2); 64 consecutive k2 make a wavefront's
// 512-byte row segments.
template <bool INV>
__global__ void __launch_bounds__(256) ks_step8(PlanSplit p, float2 *__restrict__ ws) {
    const int M = p.m, Q = p.q;
    const int k2 = blockIdx.x * 256 + threadIdx.x;
    const int qq = blockIdx.y;
    if (k2 >= M || qq >= Q) return;
    float2 v[8], w8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = ws[(size_t)(qq + Q * j) * M + k2];
#pragma unroll
    for (int kp = 0; kp < 8; ++kp) w8[kp] = p.xtw[qq * 8 + kp];
    if (!INV) {
        Dft<8, false>::run(v);
#pragma unroll
        for (int kp = 0; kp < 8; ++kp) v[kp] = cmul(v[kp], w8[kp]);
    } else {
#pragma unroll
        for (int kp = 0; kp < 8; ++kp) v[kp] = cmulc(v[kp], w8[kp]);
        Dft<8, true>::run(v);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) ws[(size_t)(qq + Q * j) * M + k2] = v[j];
}

template <class L_>
int copy_radices(int *rad) {
    for (int i = 0; i < L_::n; ++i) rad[i] = L_::r[i];
    return L_::n;
}

}  // namespace

bool split_supported(int n1, int m) {
    return (n1 == 2048 || n1 == 4096) && (m == 256 || m == 512 || m == 1024 || m == 2048);
}

bool split_long_supported(int n1, int m) { return n1 == 8 * 1024 && m >= 1; }

int split_row_radices(int m, int *rad) {
    switch (m) {
        case 2048: return copy_radices<RowRL<2048>::type>(rad);
        case 1024: return copy_radices<RowRL<1024>::type>(rad);
        case 512: return copy_radices<RowRL<512>::type>(rad);
        case 256: return copy_radices<RowRL<256>::type>(rad);
    }
    return 0;
}

int split_col_radices(int q, int *rad) {
    switch (q) {
        case 1024: return copy_radices<ColRL<1024>::type>(rad);
        case 512: return copy_radices<ColRL<512>::type>(rad);
        case 256: return copy_radices<ColRL<256>::type>(rad);
    }
    return 0;
}

#define DCTX_SPLIT_ROWS(FN, CALL)   \
    switch (p.m) {                  \
        case 2048: return FN<2048> CALL; \
        case 1024: return FN<1024> CALL; \
        case 512: return FN<512> CALL;   \
        case 256: return FN<256> CALL;   \
    }                               \
    return hipErrorInvalidValue

#define DCTX_SPLIT_COLS(FN, CALL)   \
    switch (p.q) {                  \
        case 512: return FN<512> CALL;   \
        case 256: return FN<256> CALL;   \
    }                               \
    return hipErrorInvalidValue

hipError_t launch_split_dct_rows(const PlanSplit &p, const Io &io, hipStream_t s) {
    DCTX_SPLIT_ROWS(rows_fwd, (p, io, s));
}
hipError_t launch_split_idct_rows(const PlanSplit &p, const Io &io, hipStream_t s) {
    DCTX_SPLIT_ROWS(rows_inv, (p, io, s));
}
hipError_t launch_split_dct_cols(const PlanSplit &p, const Io &io, hipStream_t s) {
    if (p.q == 1024) return cols_fwd<1024>(p, io, s);
    DCTX_SPLIT_COLS(cols_fwd, (p, io, s));
}
hipError_t launch_split_idct_cols(const PlanSplit &p, const Io &io, hipStream_t s) {
    if (p.q == 1024) return cols_inv<1024>(p, io, s);
    DCTX_SPLIT_COLS(cols_inv, (p, io, s));
}
hipError_t launch_split_step8(const PlanSplit &p, float2 *ws, bool inverse, hipStream_t s) {
    if (p.m < 1 || p.q < 1 || p.q > 65535 || 8 * p.q != p.n1) return hipErrorInvalidValue;
    const dim3 g((p.m + 255) / 256, p.q);
    if (inverse)
        hipLaunchKernelGGL(ks_step8<true>, g, dim3(256), 0, s, p, ws);
    else
        hipLaunchKernelGGL(ks_step8<false>, g, dim3(256), 0, s, p, ws);
    return hipGetLastError();
}
hipError_t launch_split_poisson_cols(const PlanSplit &p, const PoissonTabs &q, const Io &io, hipStream_t s) {
    DCTX_SPLIT_COLS(cols_poisson, (p, q, io, s));
}

}  // namespace dctx
