// Device-side FFT building blocks for gfx950: radix-2/3/4/5/8/16 butterflies in
// registers and mixed-radix Stockham stages over sequences held in LDS.
//
// The FFT here is written from the published mathematics (Cooley-Tukey mixed
// radix with Stockham autosort ordering); the paper itself calls a vendor FFT
// for this stage (Alg. alg:DCT, "2D_RFFT").
//
// Conventions
//  * forward transforms use W = exp(-2 pi j / L), inverse ones exp(+2 pi j / L);
//    nothing is normalised.
//  * A sequence of length L lives in LDS with element i at
//    base[lpad(i) * stride]; lpad() inserts one empty slot every 16 elements so
//    the strided Stockham writes spread over the 64 LDS banks.
//  * Stage s of a schedule has radix R_s and Ns = R_0 * ... * R_{s-1}.  Its
//    butterfly j (0 <= j < L/R_s) reads elements j + r * L/R_s, multiplies input
//    r by W_{Ns R}^{r (j mod Ns)}, applies the radix-R DFT and writes output r
//    to (j - j mod Ns) * R + (j mod Ns) + r * Ns.  The twiddles of butterfly j
//    form one contiguous record of a per-stage table (built in FP64 on the host
//    and rounded to FP32), read with 16-byte loads that coalesce across lanes.
#pragma once

#include <hip/hip_runtime.h>

#include "dctx_internal.h"
#include "lds_sync.h"

namespace dctx {

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
// LDS slot lpad(i) * stride.  Slot indices stay below 2^24, so a run-time
// stride takes the full-rate 24-bit multiply; a stride the compiler knows to be
// 1 (after inlining) takes none.
__device__ __forceinline__ int lslot(int i, int stride) {
    if (__builtin_constant_p(stride) && stride == 1) return lpad(i);
    return (int)__umul24((unsigned)lpad(i), (unsigned)stride);
}




// Element at byte offset off (below 4 GiB) from a base pointer that is the
// same for every lane: the compiler keeps the 64-bit base in scalar registers
// and adds each lane's 32-bit offset in the memory instruction, so no lane
// does 64-bit address arithmetic.  Offsets are formed with the full-rate
// 24-bit multiply (row < 2^24, row pitch in bytes < 2^24, product < 2^32).
template <class V>
__device__ __forceinline__ V *at_b(V *base, unsigned off) {
    return reinterpret_cast<V *>(reinterpret_cast<char *>(base) + off);
}
template <class V>
__device__ __forceinline__ const V *at_b(const V *base, unsigned off) {
    return reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + off);
}
__device__ __forceinline__ unsigned row_b(int row, unsigned pitch_b) {
    return __umul24((unsigned)row, pitch_b);
}

// ------------------------------------------------------------ output stores
// Every store of a transform's final output goes through out_store or
// nt_store4.  In the write-count build (-DDCTX_WRITE_COUNT, a test aid, not
// the product library) each of them also adds one to a device counter per
// 4-byte output word, so a test can check that every output is written
// exactly once (NaN-poisoned outputs only show the words never written).
// Each translation unit holds its own copy of the binding; the library sets
// all of them through dctx_debug_write_count.
#ifdef DCTX_WRITE_COUNT
static __device__ WriteCountBinding g_wc;
__device__ __forceinline__ void wc_add(const void *p, int nbytes) {
    const char *c = static_cast<const char *>(p);
    const WriteCountBinding w = g_wc;
    if (w.count && c >= w.base && c + nbytes <= w.base + w.bytes)
        for (int i = 0; i < nbytes / 4; ++i) atomicAdd(w.count + (c - w.base) / 4 + i, 1u);
}
namespace {
hipError_t wc_bind_unit(const WriteCountBinding &w) { return hipMemcpyToSymbol(HIP_SYMBOL(g_wc), &w, sizeof w); }
struct WcRegister {
    WcRegister() { wc_register(&wc_bind_unit); }
};
WcRegister wc_register_unit;
}  // namespace
#else
__device__ __forceinline__ void wc_add(const void *, int) {}
#endif
template <class V>
__device__ __forceinline__ void out_store(V *p, V v) {
    *p = v;
    wc_add(p, (int)sizeof(V));
}

// 16-byte loads and stores marked non-temporal (streamed data touched once;
// the stores write final outputs only).
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 nt_load4(const float4 *p) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store4(float4 *p, float4 v) {
    __builtin_nontemporal_store(nt_f4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_f4 *>(p));
    wc_add(p, 16);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * (sigma j), sigma = -1 for forward, +1 for inverse
template <bool INV>
__device__ __forceinline__ float2 mul_sj(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// a * w where w is given by (c, s) = (cos, sin) of the positive angle and the
// direction picks the sign of the imaginary part: w = c + sigma j s.
template <bool INV>
__device__ __forceinline__ float2 mul_cs(float2 a, float c, float s) {
    const float si = INV ? s : -s;
    return make_float2(a.x * c - a.y * si, a.x * si + a.y * c);
}

// ----------------------------------------------------------------- butterflies
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
    __device__ __forceinline__ static void run(float2 *a) {
        const float2 t = a[1];
        a[1] = csub(a[0], t);
        a[0] = cadd(a[0], t);
    }
};

template <bool INV> struct Dft<3, INV> {
    __device__ __forceinline__ static void run(float2 *a) {
        const float2 s = cadd(a[1], a[2]);
        const float2 d = mul_sj<INV>(cscale(csub(a[1], a[2]), kSin60));
        const float2 m = make_float2(a[0].x - 0.5f * s.x, a[0].y - 0.5f * s.y);
        a[0] = cadd(a[0], s);
        a[1] = cadd(m, d);
        a[2] = csub(m, d);
    }
};

template <bool INV> struct Dft<4, INV> {
    __device__ __forceinline__ static void run(float2 *a) {
        const float2 t0 = cadd(a[0], a[2]);
        const float2 t1 = csub(a[0], a[2]);
        const float2 t2 = cadd(a[1], a[3]);
        const float2 t3 = mul_sj<INV>(csub(a[1], a[3]));
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    }
};

template <bool INV> struct Dft<5, INV> {
    __device__ __forceinline__ static void run(float2 *a) {
        const float2 s1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
        const float2 s2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
        const float2 x0 = a[0];
        const float2 r1 = make_float2(x0.x + kCos72 * s1.x + kCos144 * s2.x,
                                      x0.y + kCos72 * s1.y + kCos144 * s2.y);
        const float2 r2 = make_float2(x0.x + kCos144 * s1.x + kCos72 * s2.x,
                                      x0.y + kCos144 * s1.y + kCos72 * s2.y);
        const float2 i1 = mul_sj<INV>(make_float2(kSin72 * d1.x + kSin144 * d2.x,
                                                  kSin72 * d1.y + kSin144 * d2.y));
        const float2 i2 = mul_sj<INV>(make_float2(kSin144 * d1.x - kSin72 * d2.x,
                                                  kSin144 * d1.y - kSin72 * d2.y));
        a[0] = make_float2(x0.x + s1.x + s2.x, x0.y + s1.y + s2.y);
        a[1] = cadd(r1, i1);
        a[4] = csub(r1, i1);
        a[2] = cadd(r2, i2);
        a[3] = csub(r2, i2);
    }
};

template <bool INV> struct Dft<8, INV> {
    __device__ __forceinline__ static void run(float2 *a) {
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, INV>::run(e);
        Dft<4, INV>::run(o);
        // o[k] *= W8^k
        o[1] = mul_cs<INV>(o[1], kSqrtHalf, kSqrtHalf);
        o[2] = mul_sj<INV>(o[2]);
        o[3] = mul_cs<INV>(o[3], -kSqrtHalf, kSqrtHalf);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = cadd(e[k], o[k]);
            a[k + 4] = csub(e[k], o[k]);
        }
    }
};

template <bool INV> struct Dft<16, INV> {
    // 4 x 4: X[k1 + 4 k2] = sum_n2 W4^{n2 k2} W16^{n2 k1} sum_n1 W4^{n1 k1} a[4 n1 + n2]
    __device__ __forceinline__ static void run(float2 *a) {
        float2 b[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            b[n2][0] = a[n2];
            b[n2][1] = a[n2 + 4];
            b[n2][2] = a[n2 + 8];
            b[n2][3] = a[n2 + 12];
            Dft<4, INV>::run(b[n2]);
        }
        // twiddles W16^{n2 k1}
        b[1][1] = mul_cs<INV>(b[1][1], kCos22_5, kSin22_5);
        b[1][2] = mul_cs<INV>(b[1][2], kSqrtHalf, kSqrtHalf);
        b[1][3] = mul_cs<INV>(b[1][3], kSin22_5, kCos22_5);
        b[2][1] = mul_cs<INV>(b[2][1], kSqrtHalf, kSqrtHalf);
        b[2][2] = mul_sj<INV>(b[2][2]);
        b[2][3] = mul_cs<INV>(b[2][3], -kSqrtHalf, kSqrtHalf);
        b[3][1] = mul_cs<INV>(b[3][1], kSin22_5, kCos22_5);
        b[3][2] = mul_cs<INV>(b[3][2], -kSqrtHalf, kSqrtHalf);
        b[3][3] = mul_cs<INV>(b[3][3], -kCos22_5, -kSin22_5);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 c[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
            Dft<4, INV>::run(c);
            a[k1] = c[0];
            a[k1 + 4] = c[1];
            a[k1 + 8] = c[2];
            a[k1 + 12] = c[3];
        }
    }
};

// ------------------------------------------------------------------ one stage
// Runs stage (R, Ns) of a length-L sequence held in LDS at base[lpad(i)*stride]
// (LDS slot indices are below 2^24, so the products use the full-rate 24-bit
// multiply).
// Threads t in [0, T) share the sequence; every thread of the block must call
// this (it contains block barriers); threads with t >= T only take part in the
// barriers.  MAXB = kEmax / R butterflies per thread at most (host-checked).
// twst: this stage's twiddle records (see FftDesc); magic = ceil(2^32 / Ns).
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(float2 *base, int stride, int t, int T, int L, int Ns,
                                          unsigned magic, const float2 *__restrict__ twst) {
    constexpr int MAXB = (kEmax / R) > 0 ? (kEmax / R) : 1;
    constexpr int REC = tw_record(R);
    const int Nb = L / R;
    float2 v[MAXB][R];
    // Every twiddle record of the thread's butterflies is fetched before the
    // LDS reads and the barrier, so the latency overlaps them.
    float4 w0[MAXB][REC / 2];
    if (Ns > 1) {
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int j = t + b * T;
            if (t < T && j < Nb) {
                const int q = (int)__umulhi((unsigned)j, magic);
                const float4 *rec = reinterpret_cast<const float4 *>(twst + (j - (int)__umul24(q, Ns)) * REC);
#pragma unroll
                for (int h = 0; h < REC / 2; ++h) w0[b][h] = rec[h];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int j = t + b * T;
        if (t < T && j < Nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = base[lslot(j + r * Nb, stride)];
        }
    }
    lds_sync();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int j = t + b * T;
        if (t < T && j < Nb) {
            // j / Ns (exact for j, Ns < 2^16; ceil(2^32 / 1) does not fit, so Ns = 1 is direct)
            const int q = (Ns == 1) ? j : (int)__umulhi((unsigned)j, magic);
            const int qn = (int)__umul24(q, Ns), k = j - qn;
            if (Ns > 1) {
                const float4(&w)[REC / 2] = w0[b];
#pragma unroll
                for (int h = 0; h < REC / 2; ++h) {
                    const int r0 = 2 * h, r1 = 2 * h + 1;
                    if (r0 >= 1 && r0 < R) {
                        const float2 tw = make_float2(w[h].x, w[h].y);
                        v[b][r0] = INV ? cmulc(v[b][r0], tw) : cmul(v[b][r0], tw);
                    }
                    if (r1 < R) {
                        const float2 tw = make_float2(w[h].z, w[h].w);
                        v[b][r1] = INV ? cmulc(v[b][r1], tw) : cmul(v[b][r1], tw);
                    }
                }
            }
            Dft<R, INV>::run(v[b]);
            const int o = qn * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) base[lslot(o + r * Ns, stride)] = v[b][r];
        }
    }
    lds_sync();
}

// Whole FFT of one sequence (all stages of the schedule `f`).  Block-uniform
// control flow: every thread of the block calls it with the same schedule.
template <bool INV>
__device__ __forceinline__ void fft_lds(float2 *base, int stride, int t, int T, const FftDesc &f) {
    for (int s = 0; s < f.nst; ++s) {
        const int R = f.rad[s];
        const int Ns = f.ns[s];
        const unsigned mg = f.nsmagic[s];
        const float2 *tw = f.tw + f.twoff[s];
        switch (R) {
            case 2: fft_stage<2, INV>(base, stride, t, T, f.L, Ns, mg, tw); break;
            case 3: fft_stage<3, INV>(base, stride, t, T, f.L, Ns, mg, tw); break;
            case 4: fft_stage<4, INV>(base, stride, t, T, f.L, Ns, mg, tw); break;
            case 5: fft_stage<5, INV>(base, stride, t, T, f.L, Ns, mg, tw); break;
            case 8: fft_stage<8, INV>(base, stride, t, T, f.L, Ns, mg, tw); break;
            default: fft_stage<16, INV>(base, stride, t, T, f.L, Ns, mg, tw); break;
        }
    }
}

// ------------------------------------------------------- real-FFT split steps
// Length-n real FFT from the length-m = n/2 complex FFT Z of z(q) = x(2q) + j x(2q+1):
//   X(k) = 1/2 (Z(k) + conj Z(m-k)) - 1/2 j W^k (Z(k) - conj Z(m-k)),  W = e^{-2 pi j / n}.
// Given Z(k), Z(m-k) and w_k = W^k, w_m = W^(m-k), returns X(k) and X(m-k).
__device__ __forceinline__ void rsplit_pair(float2 zk, float2 zm, float2 wk, float2 wm, float2 &xk,
                                            float2 &xm) {
    {
        const float2 A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        const float2 B = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
        const float2 wb = cmul(wk, B);
        xk = make_float2(A.x + wb.y, A.y - wb.x);
    }
    {
        const float2 A = make_float2(0.5f * (zm.x + zk.x), 0.5f * (zm.y - zk.y));
        const float2 B = make_float2(0.5f * (zm.x - zk.x), 0.5f * (zm.y + zk.y));
        const float2 wb = cmul(wm, B);
        xm = make_float2(A.x + wb.y, A.y - wb.x);
    }
}

// Inverse: the length-m complex sequence whose unnormalised inverse FFT is
// z(q) = x(2q) + j x(2q+1), x the unnormalised inverse real FFT of the
// Hermitian half spectrum U(0..m):
//   Z(k) = (U(k) + conj U(m-k)) + j e^{+2 pi j k/n} (U(k) - conj U(m-k)).
// w_k, w_m are the forward W^k, W^(m-k) (conjugated here).
__device__ __forceinline__ void irsplit_pair(float2 uk, float2 um, float2 wk, float2 wm, float2 &zk,
                                             float2 &zm) {
    {
        const float2 s = make_float2(uk.x + um.x, uk.y - um.y);
        const float2 d = make_float2(uk.x - um.x, uk.y + um.y);
        const float2 wd = cmulc(d, wk);
        zk = make_float2(s.x - wd.y, s.y + wd.x);
    }
    {
        const float2 s = make_float2(um.x + uk.x, um.y - uk.y);
        const float2 d = make_float2(um.x - uk.x, um.y + uk.y);
        const float2 wd = cmulc(d, wm);
        zm = make_float2(s.x - wd.y, s.y + wd.x);
    }
}

// Eq. (idxst): the IDXST along an axis is the IDCT of the sequence reversed on
// that axis, x'(n) = x(N - n) with x'(0) = x(N) = 0, followed by the sign
// (-1)^k on the output index.  The inverse pre of row k1, column k2 reads
// P = (x(k1, k2), x(k1, n2 - k2)) and Q = the same at row n1 - k1 (zero for
// k1 = 0); xst_reverse turns them into the reads of x' for the axes set in xst
// (bit 0: rows, bit 1: columns).  Column 0 packs columns 0 and m = n2 / 2:
// x'(., 0) = 0 and column m maps to itself.
__device__ __forceinline__ void xst_reverse(int xst, int k1, int k2, float2 &P, float2 &Q) {
    if (xst & 2) {
        if (k2 == 0) {
            P.x = 0.f;
            Q.x = 0.f;
        } else {
            P = make_float2(P.y, P.x);
            Q = make_float2(Q.y, Q.x);
        }
    }
    if (xst & 1) {
        if (k1 == 0) {
            P = make_float2(0.f, 0.f);   // row n1 (Q) is zero already
        } else {
            const float2 t = P;
            P = Q;
            Q = t;
        }
    }
}

// Output signs of the IDXST axes for output row r: (-1)^r (bit 0) and (-1)^col
// (bit 1) on four consecutive columns starting at an even one, and on two.
__device__ __forceinline__ float4 xst_sign4(int xst, int r, float4 v) {
    const float s = ((xst & 1) && (r & 1)) ? -1.f : 1.f;
    const float so = (xst & 2) ? -s : s;
    return make_float4(s * v.x, so * v.y, s * v.z, so * v.w);
}
__device__ __forceinline__ float2 xst_sign2(int xst, int r, float2 v) {
    const float s = ((xst & 1) && (r & 1)) ? -1.f : 1.f;
    const float so = (xst & 2) ? -s : s;
    return make_float2(s * v.x, so * v.y);
}

// p(n) of Eq. (2d_dct_pre) / (n_pre): 2n for n <= floor((N-1)/2), else 2N - 2n - 1.
__device__ __forceinline__ int perm_fwd(int n, int N) { return (n <= (N - 1) / 2) ? 2 * n : 2 * N - 2 * n - 1; }

// Source row of workspace row i for the row passes: Eq. (2d_dct_pre) along the
// row axis (2-D), or along both outer axes of a 3-D array when nsub > 0.
__device__ __forceinline__ int src_row(int i, int nrows, int nsub) {
    if (nsub == 0) return perm_fwd(i, nrows);
    const int a = i / nsub, b = i - a * nsub;
    return perm_fwd(a, nrows / nsub) * nsub + perm_fwd(b, nsub);
}

// Element n of a real row stored as complex pairs lives at float offset
// 2 * lpad(n / 2) + (n & 1) of the padded LDS sequence.
__device__ __forceinline__ int xq_off(int n) { return 2 * lpad(n >> 1) + (n & 1); }

// Tile index for a 1-D grid padded to a multiple of 8: consecutive tiles go to
// the same XCD (workgroup b is dispatched to XCD b % 8), so tiles that share
// cache lines of strided column accesses share one L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
    const int per = nblocks >> 3;
    return (b & 7) * per + (b >> 3);
}

}  // namespace dctx
