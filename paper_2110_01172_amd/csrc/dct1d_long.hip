// Batched 1-D DCT-II / DCT-III of long sequences (n / 2 beyond one
// workgroup's FFT) by the N-point algorithm (Section "Four Algorithms of 1D
// DCT", Eqs. n_pre and n_post_update) with the length-m = n / 2 complex FFT
// split four-step style, m = m1 m2, q = m2 n1 + n2, k = k1 + m1 k2:
//   Z(k1 + m1 k2) = sum_n2 W_m2^(n2 k2) [ W_m^(n2 k1) sum_n1 W_m1^(n1 k1) z(m2 n1 + n2) ].
// Forward: the column pass runs the bracket (length-m1 FFTs down the columns
// n2 of z, the reorder fused into their gathers, then the twiddle) into a
// workspace laid out [k1][n2]; the row pass runs the length-m2 FFTs of the
// rows k1 and m1 - k1 together, so that every pair (k, m - k) of the real-FFT
// split is in one workgroup, and applies the split and the postprocess:
//   y(k) = Re(t(k) V(k)),  y(n - k) = -Im(t(k) V(k)),  t(k) = exp(-j pi k / 2n) s(k).
// Inverse: the row pass forms U(k) = t'(k) (y(k) - j y(n - k)) for the pairs of
// its two rows, the inverse split, the inverse length-m2 FFTs and the conjugate
// twiddle; the column pass runs the inverse length-m1 FFTs and the inverse
// reorder fused into its scattered stores.  Tables and scale factors are
// those of the one-pass 1-D plan (FP64-built).
#include "dct1d.h"
#include "fft_core.h"

namespace dctx {

namespace {

constexpr int kSlotsL = kEmax;

// -------------------------------------------------------- column passes
// Workgroup: C consecutive columns n2 of sequence blockIdx.y; thread (c, t).
__global__ void __launch_bounds__(kMaxBlock) k_dct1dl_cols(Plan1D p, const float *__restrict__ x,
                                                            float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    const int C = p.cols_c, T = p.f1.T, M1 = p.m1, M2 = p.m2, M = p.m, N = p.n;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int n2 = blockIdx.x * C + c;
    const bool act = t < T && n2 < M2;
    const float *src = x + (size_t)blockIdx.y * N;
    {
        float2 v[kSlotsL];
#pragma unroll
        for (int e = 0; e < kSlotsL; ++e) {
            const int n1 = t + e * T;
            if (act && n1 < M1) {
                // z(q) = (x'(2q), x'(2q+1)), x'(i) = x(p(i)) (Eq. n_pre)
                const int q = M2 * n1 + n2;
                v[e] = make_float2(src[perm_fwd(2 * q, N)], src[perm_fwd(2 * q + 1, N)]);
            }
        }
#pragma unroll
        for (int e = 0; e < kSlotsL; ++e) {
            const int n1 = t + e * T;
            if (t < T && n1 < M1) lds[lpad(n1) * C + c] = act ? v[e] : make_float2(0.f, 0.f);
        }
    }
    lds_sync();
    fft_lds<false>(lds + c, C, t < T ? t : T, T, p.f1);
    if (!act) return;
    float2 *dst = ws + (size_t)blockIdx.y * M;
#pragma unroll
    for (int e = 0; e < kSlotsL; ++e) {
        const int k1 = t + e * T;
        if (k1 < M1) dst[(size_t)k1 * M2 + n2] = cmul(lds[lpad(k1) * C + c], p.roots[n2 * k1]);
    }
}

__global__ void __launch_bounds__(kMaxBlock) k_idct1dl_cols(Plan1D p, const float2 *__restrict__ ws,
                                                             float *__restrict__ y) {
    extern __shared__ float2 lds[];
    const int C = p.cols_c, T = p.f1.T, M1 = p.m1, M2 = p.m2, M = p.m, N = p.n;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int n2 = blockIdx.x * C + c;
    const bool act = t < T && n2 < M2;
    const float2 *src = ws + (size_t)blockIdx.y * M;
    {
        float2 v[kSlotsL];
#pragma unroll
        for (int e = 0; e < kSlotsL; ++e) {
            const int k1 = t + e * T;
            if (act && k1 < M1) v[e] = src[(size_t)k1 * M2 + n2];
        }
#pragma unroll
        for (int e = 0; e < kSlotsL; ++e) {
            const int k1 = t + e * T;
            if (t < T && k1 < M1) lds[lpad(k1) * C + c] = act ? v[e] : make_float2(0.f, 0.f);
        }
    }
    lds_sync();
    fft_lds<true>(lds + c, C, t < T ? t : T, T, p.f1);
    if (!act) return;
    float *dst = y + (size_t)blockIdx.y * N;
#pragma unroll
    for (int e = 0; e < kSlotsL; ++e) {
        const int n1 = t + e * T;
        if (n1 < M1) {
            // y(p(i)) = x'(i): z(q) holds x'(2q), x'(2q + 1)
            const int q = M2 * n1 + n2;
            const float2 z = lds[lpad(n1) * C + c];
            out_store(&dst[perm_fwd(2 * q, N)], z.x);
            out_store(&dst[perm_fwd(2 * q + 1, N)], z.y);
        }
    }
}

// ------------------------------------------------------------ row passes
// Workgroup: the row pair {k1, m1 - k1} (k1 = blockIdx.x <= m1 / 2) of sequence
// blockIdx.y; threads [0, T) hold row k1, [T, 2T) row m1 - k1 (idle when the
// row pairs with itself).  Position k2 of slot s holds Z(k1_s + m1 k2).
struct RowPair {
    int k1, k1p;
    bool two;
    int npairs;
    // k of pair i (rows by index) and its partner m - k, with their LDS slots.
    __device__ __forceinline__ void pair(int i, int M1, int M2, int RL, int &k, int &km, int &sk, int &skm) const {
        if (two) {
            // (k1 + m1 k2) with (k1p + m1 (m2 - 1 - k2)), k2 in [0, m2)
            k = k1 + M1 * i;
            km = k1p + M1 * (M2 - 1 - i);
            sk = lpad(i);
            skm = RL + lpad(M2 - 1 - i);
        } else if (k1 == 0) {
            // (m1 k2) with (m1 ((m2 - k2) mod m2)), k2 in [0, m2 / 2]
            const int i2 = (M2 - i) % M2;
            k = M1 * i;
            km = M1 * i2;
            sk = lpad(i);
            skm = lpad(i2);
        } else {
            // k1 = m1 / 2: (k1 + m1 k2) with (k1 + m1 (m2 - 1 - k2)), k2 in [0, (m2 - 1) / 2]
            k = k1 + M1 * i;
            km = k1 + M1 * (M2 - 1 - i);
            sk = lpad(i);
            skm = lpad(M2 - 1 - i);
        }
    }
};

__device__ __forceinline__ RowPair row_pair(int k1, int M1, int M2) {
    RowPair rp;
    rp.k1 = k1;
    rp.k1p = (M1 - k1) % M1;
    rp.two = rp.k1p != k1;
    rp.npairs = rp.two ? M2 : (k1 == 0 ? M2 / 2 + 1 : (M2 + 1) / 2);
    return rp;
}

__global__ void __launch_bounds__(kMaxBlock) k_dct1dl_rows(Plan1D p, const float2 *__restrict__ ws,
                                                            float *__restrict__ y) {
    extern __shared__ float2 lds[];
    const int T = p.f2.T, M1 = p.m1, M2 = p.m2, M = p.m, N = p.n, RL = lpad_len(M2);
    const RowPair rp = row_pair(blockIdx.x, M1, M2);
    const int r = threadIdx.x / T, t = threadIdx.x - r * T;
    const bool act = r == 0 || (r == 1 && rp.two);
    const int kr = r == 0 ? rp.k1 : rp.k1p;
    float2 *row = lds + (r == 1 ? RL : 0);
    const float2 *src = ws + (size_t)blockIdx.y * M;
    {
        float2 v[kSlotsL];
#pragma unroll
        for (int e = 0; e < kSlotsL; ++e) {
            const int n2 = t + e * T;
            if (act && n2 < M2) v[e] = src[(size_t)kr * M2 + n2];
        }
#pragma unroll
        for (int e = 0; e < kSlotsL; ++e) {
            const int n2 = t + e * T;
            if (act && n2 < M2) row[lpad(n2)] = v[e];
        }
    }
    lds_sync();
    fft_lds<false>(row, 1, act ? t : T, T, p.f2);
    float *dst = y + (size_t)blockIdx.y * N;
    for (int i = threadIdx.x; i < rp.npairs; i += blockDim.x) {
        int k, km, sk, skm;
        rp.pair(i, M1, M2, RL, k, km, sk, skm);
        const float2 zk = lds[sk];
        if (k == 0) {
            // V(0) = Re Z(0) + Im Z(0), V(m) = Re Z(0) - Im Z(0), both real
            out_store(&dst[0], p.tw[0].x * (zk.x + zk.y));
            out_store(&dst[M], p.tw[M].x * (zk.x - zk.y));
            continue;
        }
        float2 vk, vm;
        rsplit_pair(zk, lds[skm], p.split[k], p.split[km], vk, vm);
        const float2 a = cmul(p.tw[k], vk);
        out_store(&dst[k], a.x);
        out_store(&dst[N - k], -a.y);
        if (km != k) {
            const float2 b = cmul(p.tw[km], vm);
            out_store(&dst[km], b.x);
            out_store(&dst[N - km], -b.y);
        }
    }
}

__global__ void __launch_bounds__(kMaxBlock) k_idct1dl_rows(Plan1D p, const float *__restrict__ x,
                                                             float2 *__restrict__ ws) {
    extern __shared__ float2 lds[];
    const int T = p.f2.T, M1 = p.m1, M2 = p.m2, M = p.m, N = p.n, RL = lpad_len(M2);
    const RowPair rp = row_pair(blockIdx.x, M1, M2);
    const float *src = x + (size_t)blockIdx.y * N;
    // U(k) = t'(k) (y(k) - j y(n - k)) with y(n) = 0, for the pairs (k, m - k)
    // of the two rows, then the inverse split into the rows' slots
    for (int i = threadIdx.x; i < rp.npairs; i += blockDim.x) {
        int k, km, sk, skm;
        rp.pair(i, M1, M2, RL, k, km, sk, skm);
        // k = 0 pairs with m (U(0) and U(m) from y(0) and y(m) = y(n - m))
        const int kb = (k == 0) ? M : km;
        const float ak = src[k], an = (k == 0) ? 0.f : src[N - k];
        const float bk = src[kb], bn = src[N - kb];
        const float2 ua = cmul(p.tw[k], make_float2(ak, -an));
        const float2 ub = cmul(p.tw[kb], make_float2(bk, -bn));
        if (k == 0) {
            // U(0) and U(m) are real
            lds[sk] = make_float2(ua.x + ub.x, ua.x - ub.x);
            continue;
        }
        float2 zk, zm;
        irsplit_pair(ua, ub, p.split[k], p.split[km], zk, zm);
        lds[sk] = zk;
        if (km != k) lds[skm] = zm;
    }
    lds_sync();
    const int r = threadIdx.x / T, t = threadIdx.x - r * T;
    const bool act = r == 0 || (r == 1 && rp.two);
    const int kr = r == 0 ? rp.k1 : rp.k1p;
    float2 *row = lds + (r == 1 ? RL : 0);
    fft_lds<true>(row, 1, act ? t : T, T, p.f2);
    if (!act) return;
    float2 *dst = ws + (size_t)blockIdx.y * M;
#pragma unroll
    for (int e = 0; e < kSlotsL; ++e) {
        const int n2 = t + e * T;
        if (n2 < M2) dst[(size_t)kr * M2 + n2] = cmulc(row[lpad(n2)], p.roots[n2 * kr]);
    }
}

}  // namespace

hipError_t launch_dct1d_long(const Plan1D &p, int batch, const float *x, float2 *ws, float *y, hipStream_t s) {
    const int C = p.cols_c;
    const size_t lc = (size_t)lpad_len(p.m1) * C * sizeof(float2), lr = 2 * (size_t)lpad_len(p.m2) * sizeof(float2);
    hipLaunchKernelGGL(k_dct1dl_cols, dim3((p.m2 + C - 1) / C, batch), dim3(C * p.f1.T), lc, s, p, x, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dct1dl_rows, dim3(p.m1 / 2 + 1, batch), dim3(2 * p.f2.T), lr, s, p, ws, y);
    return hipGetLastError();
}

hipError_t launch_idct1d_long(const Plan1D &p, int batch, const float *x, float2 *ws, float *y, hipStream_t s) {
    const int C = p.cols_c;
    const size_t lc = (size_t)lpad_len(p.m1) * C * sizeof(float2), lr = 2 * (size_t)lpad_len(p.m2) * sizeof(float2);
    hipLaunchKernelGGL(k_idct1dl_rows, dim3(p.m1 / 2 + 1, batch), dim3(2 * p.f2.T), lr, s, p, x, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_idct1dl_cols, dim3((p.m2 + C - 1) / C, batch), dim3(C * p.f1.T), lc, s, p, ws, y);
    return hipGetLastError();
}

}  // namespace dctx
