// Compile-time FFT chains for power-of-two lengths: a radix list, the stage
// types it implies (first and last stage maps chosen by the caller, middle
// stages kCyclic) and the LDS exchange between consecutive stages.
#pragma once

#include "fast_core.h"

namespace dctx {
namespace fast {

template <int... Rs>
struct RL {
    static constexpr int n = sizeof...(Rs);
    static constexpr int r[n] = {Rs...};
    static constexpr int ns(int k) {
        int v = 1;
        for (int i = 0; i < k; ++i) v *= r[i];
        return v;
    }
};

template <class L_, int LEN, int T, int K, int MF, int ML>
using StageK = Stage<LEN, T, L_::r[K], L_::ns(K), K == 0 ? MF : (K == L_::n - 1 ? ML : kCyclic)>;

// Barrier between the stages of one FFT: the whole workgroup, or (WAVE) only
// the wavefront when every FFT lies inside one wavefront.  LDS operations of
// a wavefront complete in issue order, so the fences that keep the compiler
// from moving LDS accesses across this point are all that is needed there.
template <bool WAVE>
__device__ __forceinline__ void stage_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        lds_sync();
    }
}

// Where the stage twiddles come from: the FftDesc tables in global memory, or
// an LDS copy whose records are stored transposed (float4 h of record k of
// stage K at tab[K][h NS + k]) so that neighbouring lanes read neighbouring
// 16-byte words.
struct GlobalTw {
    template <int K>
    __device__ __forceinline__ void after_stage() const {}
};
struct LdsTw {
    const float4 *tab[kMaxStages];
    template <int K>
    __device__ __forceinline__ void after_stage() const {}
};
// GlobalTw / LdsTw plus a call h(K) after the butterflies of every stage K,
// for work spread over the FFT (such as the loads of the next sequence).
template <class H>
struct GlobalTwHook : GlobalTw {
    H h;
    template <int K>
    __device__ __forceinline__ void after_stage() const {
        h(K);
    }
};
template <class H>
struct LdsTwHook : LdsTw {
    H h;
    template <int K>
    __device__ __forceinline__ void after_stage() const {
        h(K);
    }
};

// LDS copy of the stage twiddles of chain L_ for LdsTw: stage K >= 1 starts at
// float4 off(K); float4 h of its record k sits at off(K) + h NS + k.  A kernel
// copies words d < size (src(f, d) each) once, before the first FFT stage that
// reads them, so no twiddle fetch from global memory sits inside an FFT.
template <class L_>
struct TwTab {
    static constexpr int off(int K) {
        int o = 0;
        for (int i = 1; i < K; ++i) o += L_::ns(i) * tw_record(L_::r[i]) / 2;
        return o;
    }
    static constexpr int size = off(L_::n);   // float4
    // word d < size of the copy in the FftDesc tables (word 0 of them otherwise)
    __device__ __forceinline__ static const float4 *src(const FftDesc &f, int d) {
        const float4 *ptr = reinterpret_cast<const float4 *>(f.tw);
        int idx = 0;
#pragma unroll
        for (int K = 1; K < L_::n; ++K) {
            const int NS = L_::ns(K), H = tw_record(L_::r[K]) / 2;
            const bool in = d >= off(K) && d < off(K + 1);
            const int dd = d - off(K);
            ptr = in ? reinterpret_cast<const float4 *>(f.tw + f.twoff[K]) : ptr;
            idx = in ? (dd % NS) * H + dd / NS : idx;
        }
        return ptr + idx;
    }
    __device__ __forceinline__ static LdsTw view(const float4 *base) {
        LdsTw t;
#pragma unroll
        for (int K = 0; K < kMaxStages; ++K) t.tab[K] = base + (K >= 1 && K < L_::n ? off(K) : 0);
        return t;
    }
};

// A thread's share of copying TwTab<L_> to LDS in an NTH-thread workgroup:
// fetch() early (the loads overlap what follows), store() before the barrier
// that precedes the first FFT stage with twiddles.
template <class L_, int NTH>
struct TwCopy {
    static constexpr int size = TwTab<L_>::size, NTV = (size + NTH - 1) / NTH;
    float4 v[NTV > 0 ? NTV : 1];
    __device__ __forceinline__ void fetch(const FftDesc &f) {
#pragma unroll
        for (int i = 0; i < NTV; ++i) {
            const int d = threadIdx.x + i * NTH;
            v[i] = *TwTab<L_>::src(f, d < size ? d : 0);
        }
    }
    __device__ __forceinline__ void store(float4 *tab) const {
#pragma unroll
        for (int i = 0; i < NTV; ++i) {
            const int d = threadIdx.x + i * NTH;
            if (d < size) tab[d] = v[i];
        }
    }
};

template <class S, bool INV, int K>
__device__ __forceinline__ void stage_butterflies(float2 (&w)[S::NB][S::R], int t, const FftDesc &d, GlobalTw) {
    butterflies<S, INV>(w, t, d.tw + d.twoff[K]);
}

template <class S, bool INV, int K>
__device__ __forceinline__ void stage_butterflies(float2 (&w)[S::NB][S::R], int t, const FftDesc &, const LdsTw &tw) {
    const float4 *tab = tw.tab[K];
    butterflies_with<S, INV>(w, t, [tab](int k, int h) { return tab[h * S::NS + k]; });
}

template <class L_>
constexpr int buf_len(int len) {
    return len + len / L_::r[0] + 1;
}

// Stages K.. of an FFT whose stage K-1 outputs are in v (LDS exchange between
// consecutive stages; a barrier first, since the buffer may still be read).
template <class L_, int LEN, int T, int MF, int ML, bool INV, int K, bool WAVE = false, class TW = GlobalTw>
struct Run {
    using Prev = StageK<L_, LEN, T, K - 1, MF, ML>;
    using Cur = StageK<L_, LEN, T, K, MF, ML>;
    using Last = StageK<L_, LEN, T, L_::n - 1, MF, ML>;
    __device__ __forceinline__ static void go(float2 *buf, int stride, int c, int t,
                                              float2 (&v)[Prev::NB][Prev::R], float2 (&out)[Last::NB][Last::R],
                                              const FftDesc &d, const TW &tw = TW()) {
        stage_sync<WAVE>();
        fast::write_out<Prev>(buf, stride, c, v, t);
        stage_sync<WAVE>();
        float2 w[Cur::NB][Cur::R];
        fast::read_in<Cur, Prev::D>(buf, stride, c, w, t);
        stage_butterflies<Cur, INV, K>(w, t, d, tw);
        tw.template after_stage<K>();
        if constexpr (K + 1 < L_::n) {
            Run<L_, LEN, T, MF, ML, INV, K + 1, WAVE, TW>::go(buf, stride, c, t, w, out, d, tw);
        } else {
#pragma unroll
            for (int b = 0; b < Cur::NB; ++b)
#pragma unroll
                for (int r = 0; r < Cur::R; ++r) out[b][r] = w[b][r];
        }
    }
};

// Whole FFT from the stage-0 inputs in v0 (stage-0 slot layout).  WAVE: the
// T threads of each FFT lie in one wavefront (see stage_sync).
template <class L_, int LEN, int T, int MF, int ML, bool INV, bool WAVE = false, class TW = GlobalTw>
__device__ __forceinline__ void fft_run(float2 *buf, int stride, int c, int t,
                                        float2 (&v0)[StageK<L_, LEN, T, 0, MF, ML>::NB]
                                                    [StageK<L_, LEN, T, 0, MF, ML>::R],
                                        float2 (&out)[StageK<L_, LEN, T, L_::n - 1, MF, ML>::NB]
                                                     [StageK<L_, LEN, T, L_::n - 1, MF, ML>::R],
                                        const FftDesc &d, const TW &tw = TW()) {
    using S0 = StageK<L_, LEN, T, 0, MF, ML>;
    fast::butterflies<S0, INV>(v0, t, nullptr);
    tw.template after_stage<0>();
    Run<L_, LEN, T, MF, ML, INV, 1, WAVE, TW>::go(buf, stride, c, t, v0, out, d, tw);
}

}  // namespace fast
}  // namespace dctx
