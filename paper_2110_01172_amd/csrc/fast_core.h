// Compile-time specialised FFT building blocks for power-of-two lengths on
// gfx950 (the fast path of the 2-D transforms; other 5-smooth lengths use the
// run-time schedules of fft_core.h).
//
// A length-L sequence is owned by T threads; thread t holds E = L / T values.
// Stage s (radix R, Ns = product of the earlier radices, Nb = L / R butterflies)
// is a Stockham decimation-in-time step: butterfly j reads elements j + r Nb,
// multiplies input r by W_{Ns R}^{r (j mod Ns)}, applies the radix-R DFT and
// produces output r at (j / Ns) Ns R + (j mod Ns) + r Ns.  Each thread runs its
// E / R butterflies in registers; between stages the values go through LDS once
// (write at the output positions, barrier, read the next stage's inputs).
//
// Butterfly-to-thread maps (compile-time per stage):
//   kCyclic  : butterflies t + b T.  Its inputs are the thread's cyclic values
//              t + e T, so a cyclic first stage reads global memory directly and
//              a cyclic last stage leaves its outputs cyclic.
//   kMirror  : butterflies j = t + b T (b < E/2R) and Nb - j (0 pairs with Nb/2).
//              Element k and L - k then sit in one thread, which is what the
//              real-FFT split, the four-element DCT post (Eqs. four-elements,
//              s-t) and the four-read IDCT pre (Eq. 2d_idct_pre) need.
//   kReverse : butterflies j = t + b T and Nb - 1 - j.  Element q and L - 1 - q
//              then sit in one thread; with the even/odd packing of a real row,
//              x[4q .. 4q+3] holds exactly z(q) and z(L-1-q), so the Eq.
//              (2d_dct_pre) reorder becomes one 16-byte load (or store).
//   kRevCyclic: butterflies Nb - 1 - (t + b T).  Run on a second sequence next
//              to a kCyclic one, element i of the first and L - 1 - i of the
//              second sit in one thread (slot (b, r) with slot (b, R - 1 - r)).
//
// LDS layout of the exchange after a stage with D = Ns R: element i lives at
// slot i + i / D, so both the writer's and the reader's addresses are a
// per-thread base plus compile-time offsets, and strided writes spread over the
// banks.
#pragma once

#include "fft_core.h"

namespace dctx {
namespace fast {

enum MapMode { kCyclic = 0, kMirror = 1, kReverse = 2, kRevCyclic = 3 };

template <int D>
__device__ __forceinline__ int pad(int i) {
    return i + i / D;
}

// Compile-time description of one stage of a length-L, T-thread FFT.
template <int L_, int T_, int R_, int NS_, int MODE_>
struct Stage {
    static constexpr int L = L_, T = T_, R = R_, NS = NS_, MODE = MODE_;
    static constexpr int E = L / T;
    static constexpr int NB = E / R;        // butterflies per thread
    static constexpr int Nb = L / R;        // butterflies per sequence
    static constexpr int D = NS * R;        // output block of this stage
    static constexpr int REC = tw_record(R);
    static_assert(L % T == 0 && E % R == 0, "radix must divide the values per thread");
    static_assert(MODE == kCyclic || MODE == kRevCyclic || NB % 2 == 0,
                  "paired maps need an even butterfly count");

    // butterfly index of slot b of thread t
    __device__ __forceinline__ static int j(int t, int b) {
        if (MODE == kCyclic) return t + b * T;
        if (MODE == kRevCyclic) return Nb - 1 - (t + b * T);
        constexpr int H = NB / 2;
        if (b < H) return t + b * T;
        const int jp = t + (b - H) * T;
        if (MODE == kMirror) return jp == 0 ? Nb / 2 : Nb - jp;
        return Nb - 1 - jp;
    }
};

// Twiddle and radix-R DFT of every butterfly of the thread, in place:
// v[b][r] = input r of slot b on entry, output r on exit.
// get(k, h) returns complex values 2h and 2h + 1 of twiddle record k.
template <class S, bool INV, class Get>
__device__ __forceinline__ void butterflies_with(float2 (&v)[S::NB][S::R], int t, const Get &get) {
#pragma unroll
    for (int b = 0; b < S::NB; ++b) {
        if (S::NS > 1) {
            const int k = S::j(t, b) & (S::NS - 1);
#pragma unroll
            for (int h = 0; h < S::REC / 2; ++h) {
                const float4 w = get(k, h);
                const int r0 = 2 * h, r1 = 2 * h + 1;
                if (r0 >= 1 && r0 < S::R) {
                    const float2 tw = make_float2(w.x, w.y);
                    v[b][r0] = INV ? cmulc(v[b][r0], tw) : cmul(v[b][r0], tw);
                }
                if (r1 < S::R) {
                    const float2 tw = make_float2(w.z, w.w);
                    v[b][r1] = INV ? cmulc(v[b][r1], tw) : cmul(v[b][r1], tw);
                }
            }
        }
        Dft<S::R, INV>::run(v[b]);
    }
}

// Twiddles from the stage's table in global memory (records of REC values).
template <class S, bool INV>
__device__ __forceinline__ void butterflies(float2 (&v)[S::NB][S::R], int t, const float2 *__restrict__ twst) {
    butterflies_with<S, INV>(v, t, [twst](int k, int h) {
        return reinterpret_cast<const float4 *>(twst + k * S::REC)[h];
    });
}

// LDS slot of output r of slot b (padding of this stage's exchange, D = NS R).
template <class S>
__device__ __forceinline__ int out_slot(int t, int b, int r) {
    if (S::MODE == kCyclic) {
        if (S::NS <= S::T) {
            // j = t + bT with NS | T: j / NS = t / NS + bT / NS, j mod NS = t mod NS
            const int base = (t / S::NS) * S::D + (t & (S::NS - 1)) + t / S::NS;
            return base + b * (S::T * S::R + S::T / S::NS) + r * S::NS;
        } else {
            // T | NS: j / NS = bT / NS, j mod NS = t + bT mod NS
            constexpr int unused = 0;
            (void)unused;
            const int q = (b * S::T) / S::NS;
            return t + q * S::D + ((b * S::T) & (S::NS - 1)) + r * S::NS + q;
        }
    }
    const int jj = S::j(t, b);
    const int o = (jj / S::NS) * S::D + (jj & (S::NS - 1)) + r * S::NS;
    return pad<S::D>(o);
}

// LDS slot of input r of slot b of stage S, reading the exchange written by a
// stage with output block DPREV.
template <class S, int DPREV>
__device__ __forceinline__ int in_slot(int t, int b, int r) {
    const int i = S::j(t, b) + r * S::Nb;
    if (S::MODE == kCyclic) {
        // i = t + e T with e = b + r NB
        const int e = b + r * S::NB;
        if (DPREV <= S::T) return t + t / DPREV + e * (S::T + S::T / DPREV);
        return t + e * S::T + (e * S::T) / DPREV;
    }
    return pad<DPREV>(i);
}

template <class S>
__device__ __forceinline__ void write_out(float2 *lds, int stride, int c, const float2 (&v)[S::NB][S::R], int t) {
#pragma unroll
    for (int b = 0; b < S::NB; ++b)
#pragma unroll
        for (int r = 0; r < S::R; ++r) lds[out_slot<S>(t, b, r) * stride + c] = v[b][r];
}

template <class S, int DPREV>
__device__ __forceinline__ void read_in(const float2 *lds, int stride, int c, float2 (&v)[S::NB][S::R], int t) {
#pragma unroll
    for (int b = 0; b < S::NB; ++b)
#pragma unroll
        for (int r = 0; r < S::R; ++r) v[b][r] = lds[in_slot<S, DPREV>(t, b, r) * stride + c];
}

// Partner of element (b, r) of a kMirror stage (its output index k = j + r Nb
// pairs with L - k): sets (pb, pr).  Slot b of thread t with j = 0 pairs within
// itself (r with R - r); its mirror slot (j = Nb/2) pairs r with R - 1 - r.
template <class S>
__device__ __forceinline__ void mirror_partner(int t, int b, int r, int &pb, int &pr) {
    constexpr int H = S::NB / 2;
    const int jj = S::j(t, b);
    if (jj == 0) {
        pb = b;
        pr = (S::R - r) & (S::R - 1);
    } else if (b >= H && t == 0 && b == H) {
        pb = b;
        pr = S::R - 1 - r;
    } else {
        pb = b < H ? b + H : b - H;
        pr = S::R - 1 - r;
    }
}

}  // namespace fast
}  // namespace dctx
