// Batched 1-D DCT-II and DCT-III of length-n rows in one pass each: every row
// is one group of T threads of a workgroup, held in LDS.
//
// Forward: the Eq. (n_pre) reorder x'(i) = x(p(i)) fused into the loads, the
// length-n real FFT V of x' as a length-m = n / 2 complex FFT plus the
// even/odd split, and the Eq. (n_post_update) postprocess fused into the
// stores: with t(k) = exp(-j pi k / 2n) s(k) (s the norm's scale),
//   y(k) = Re(t(k) V(k)),  y(n - k) = -Im(t(k) V(k)),  k in [0, m]
// (the partner of k = m is itself; V(0) and V(m) are real).
// Inverse: U(k) = t'(k) (y(k) - j y(n - k)) with y(n) = 0 and t'(k) =
// exp(+j pi k / 2n) s'(k), the inverse split, the inverse length-m FFT, and the
// inverse reorder fused into the stores.
#include "dct1d.h"
#include "fft_core.h"

namespace dctx {

namespace {

constexpr int kSlots1 = kEmax;
constexpr int kHalf1 = kEmax / 2;
constexpr int kPairs1 = kEmax / 2 + 1;

__global__ void __launch_bounds__(kMaxBlock) k_dct1d(Plan1D p, int batch, int rpb, const float *__restrict__ x,
                                                      float *__restrict__ y) {
    extern __shared__ float2 lds[];
    const int T = p.row.T;
    const int r = threadIdx.x / T;
    const int t = threadIdx.x - r * T;
    const int row = blockIdx.x * rpb + r;
    const bool active = (r < rpb) && (row < batch);
    const int M = p.m, N = p.n;
    float2 *base = lds + (r < rpb ? r : 0) * lpad_len(M);
    float *bf = reinterpret_cast<float *>(base);
    if (active) {
        // source element i lands at x' index pinv(i): pinv(2q) = q, pinv(2q + 1) = n - 1 - q
        const float *src = x + (size_t)row * N;
        if ((N & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
            // x[4q .. 4q+3] gives z(q) = (x[4q], x[4q+2]) and z(m-1-q) = (x[4q+3], x[4q+1])
            const float4 *s4 = reinterpret_cast<const float4 *>(src);
            float4 v[kHalf1];
#pragma unroll
            for (int e = 0; e < kHalf1; ++e) {
                const int q = t + e * T;
                if (q < M / 2) v[e] = s4[q];
            }
#pragma unroll
            for (int e = 0; e < kHalf1; ++e) {
                const int q = t + e * T;
                if (q < M / 2) {
                    base[lpad(q)] = make_float2(v[e].x, v[e].z);
                    base[lpad(M - 1 - q)] = make_float2(v[e].w, v[e].y);
                }
            }
        } else {
            const float2 *s2 = reinterpret_cast<const float2 *>(src);
            float2 v[kSlots1];
#pragma unroll
            for (int e = 0; e < kSlots1; ++e) {
                const int q = t + e * T;
                if (q < M) v[e] = s2[q];
            }
#pragma unroll
            for (int e = 0; e < kSlots1; ++e) {
                const int q = t + e * T;
                if (q < M) {
                    bf[xq_off(q)] = v[e].x;
                    bf[xq_off(N - 1 - q)] = v[e].y;
                }
            }
        }
    }
    lds_sync();
    fft_lds<false>(base, 1, active ? t : T, T, p.row);
    if (!active) return;
    float *dst = y + (size_t)row * N;
    float2 wk[kPairs1], wm[kPairs1], tk[kPairs1], tm[kPairs1];
#pragma unroll
    for (int i = 0; i < kPairs1; ++i) {
        const int k = t + i * T;
        if (k <= M / 2) {
            wk[i] = p.split[k];
            wm[i] = p.split[M - k];
            tk[i] = p.tw[k];
            tm[i] = p.tw[M - k];
        }
    }
#pragma unroll
    for (int i = 0; i < kPairs1; ++i) {
        const int k = t + i * T;
        if (k > M / 2) continue;
        const float2 zk = base[lpad(k)];
        if (k == 0) {
            // V(0) = Re Z(0) + Im Z(0), V(m) = Re Z(0) - Im Z(0), both real
            out_store(&dst[0], tk[i].x * (zk.x + zk.y));
            out_store(&dst[M], tm[i].x * (zk.x - zk.y));
            continue;
        }
        const int km = M - k;
        float2 vk, vm;
        rsplit_pair(zk, base[lpad(km)], wk[i], wm[i], vk, vm);
        const float2 a = cmul(tk[i], vk);
        out_store(&dst[k], a.x);
        out_store(&dst[N - k], -a.y);
        if (km != k) {
            const float2 b = cmul(tm[i], vm);
            out_store(&dst[km], b.x);
            out_store(&dst[N - km], -b.y);
        }
    }
}

__global__ void __launch_bounds__(kMaxBlock) k_idct1d(Plan1D p, int batch, int rpb, const float *__restrict__ x,
                                                       float *__restrict__ y) {
    extern __shared__ float2 lds[];
    const int T = p.row.T;
    const int r = threadIdx.x / T;
    const int t = threadIdx.x - r * T;
    const int row = blockIdx.x * rpb + r;
    const bool active = (r < rpb) && (row < batch);
    const int M = p.m, N = p.n;
    float2 *base = lds + (r < rpb ? r : 0) * lpad_len(M);
    float *bf = reinterpret_cast<float *>(base);
    if (active) {
        const float *src = x + (size_t)row * N;
        // the four reads of pair (k, m - k): y(k), y(n - k), y(m - k), y(m + k)
        float ak[kPairs1], an[kPairs1], bk[kPairs1], bn[kPairs1];
#pragma unroll
        for (int i = 0; i < kPairs1; ++i) {
            const int k = t + i * T;
            if (k <= M / 2) {
                ak[i] = src[k];
                an[i] = (k == 0) ? 0.f : src[N - k];
                bk[i] = src[M - k];
                bn[i] = src[M + k];
            }
        }
        float2 zk[kPairs1], zm[kPairs1];
#pragma unroll
        for (int i = 0; i < kPairs1; ++i) {
            const int k = t + i * T;
            if (k > M / 2) continue;
            const float2 ua = cmul(p.tw[k], make_float2(ak[i], -an[i]));        // U(k)
            const float2 ub = cmul(p.tw[M - k], make_float2(bk[i], -bn[i]));    // U(m - k)
            if (k == 0) {
                // U(0) and U(m) are real
                zk[i] = make_float2(ua.x + ub.x, ua.x - ub.x);
            } else {
                const float2 w = p.split[k];
                irsplit_pair(ua, ub, w, p.split[M - k], zk[i], zm[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < kPairs1; ++i) {
            const int k = t + i * T;
            if (k <= M / 2) {
                base[lpad(k)] = zk[i];
                if (k != 0 && M - k != k) base[lpad(M - k)] = zm[i];
            }
        }
    }
    lds_sync();
    fft_lds<true>(base, 1, active ? t : T, T, p.row);
    if (!active) return;
    // Eq. (n_pre) inverted: output element i takes x' index pinv(i)
    float *drow = y + (size_t)row * N;
    if ((N & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
        float4 *d4 = reinterpret_cast<float4 *>(drow);
#pragma unroll
        for (int e = 0; e < kHalf1; ++e) {
            const int q = t + e * T;
            if (q < M / 2) {
                const float2 a = base[lpad(q)], b = base[lpad(M - 1 - q)];
                out_store(&d4[q], make_float4(a.x, b.y, a.y, b.x));
            }
        }
    } else {
        float2 *d2 = reinterpret_cast<float2 *>(drow);
#pragma unroll
        for (int e = 0; e < kSlots1; ++e) {
            const int q = t + e * T;
            if (q < M) out_store(&d2[q], make_float2(bf[xq_off(q)], bf[xq_off(N - 1 - q)]));
        }
    }
}

}  // namespace

hipError_t launch_dct1d(const Plan1D &p, int batch, int rpb, const float *x, float *y, hipStream_t s) {
    const size_t lds = (size_t)rpb * lpad_len(p.m) * sizeof(float2);
    hipLaunchKernelGGL(k_dct1d, dim3((batch + rpb - 1) / rpb), dim3(rpb * p.row.T), lds, s, p, batch, rpb, x, y);
    return hipGetLastError();
}

hipError_t launch_idct1d(const Plan1D &p, int batch, int rpb, const float *x, float *y, hipStream_t s) {
    const size_t lds = (size_t)rpb * lpad_len(p.m) * sizeof(float2);
    hipLaunchKernelGGL(k_idct1d, dim3((batch + rpb - 1) / rpb), dim3(rpb * p.row.T), lds, s, p, batch, rpb, x, y);
    return hipGetLastError();
}

}  // namespace dctx
