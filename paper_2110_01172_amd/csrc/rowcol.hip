// Row-column baseline: the method the paper compares against (Section
// "Examples and Summary", Fig. operator-fusion).  A 2-D DCT is a 1-D N-point DCT
// along the rows (Alg. 1d-dct-via-fft, "DCT using N FFT"), a transpose, the same
// along the new rows, and a transpose back.  Each 1-D DCT is three separate
// kernels, each one full pass over HBM:
//   pre  : Eq. (n_pre) reorder, one thread per element;
//   rfft : batched length-n real FFT of every row (half spectrum, n/2 + 1 values);
//   post : Eq. (n_post_update), y(k) = 2 Re(e^{-j pi k/2n} X(k)) with conj X(n-k)
//          for k > n/2, one thread per output (scale folded into the table).
// The inverse runs the 1-D IDCT the same way: pre (e^{+j pi k/2n} (y(k) - j y(n-k)),
// y(n) = 0), inverse real FFT, inverse reorder.  3 x 2 + 2 = 8 memory stages.
#include "fft_core.h"

namespace dctx {

// ---------------------------------------------------------------- pre (fwd)
__global__ void __launch_bounds__(256) k_rc_pre(int n, const float *__restrict__ x, float *__restrict__ xr) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const size_t row = blockIdx.y;
    if (i < n) xr[row * n + i] = x[row * n + perm_fwd(i, n)];
}

// ------------------------------------------------------- batched real FFT
__global__ void __launch_bounds__(kMaxBlock) k_rc_rfft(PlanRC1D p, const float *__restrict__ xr,
                                                   float2 *__restrict__ spec) {
    extern __shared__ float2 lds[];
    const int T = p.fft.T;
    const int r = threadIdx.x / T;
    const int t = threadIdx.x - r * T;
    const int row = blockIdx.x * p.rows_per_block + r;
    const bool active = (r < p.rows_per_block) && (row < p.batch);
    const int M = p.m;
    if (p.odd) {
        // odd n: the length-n complex FFT of the real row, spectrum k = 0 .. m
        float2 *buf = lds + (r < p.rows_per_block ? r : 0) * lpad_len(p.n);
        if (active) {
            const float *src = xr + (size_t)row * p.n;
            for (int q = t; q < p.n; q += T) buf[lpad(q)] = make_float2(src[q], 0.f);
        }
        lds_sync();
        fft_lds<false>(buf, 1, active ? t : T, T, p.fft);
        if (active) {
            float2 *out = spec + (size_t)row * (M + 1);
            for (int k = t; k <= M; k += T) out[k] = buf[lpad(k)];
        }
        return;
    }
    float2 *base = lds + (r < p.rows_per_block ? r : 0) * lpad_len(M);
    if (active) {
        const float2 *src = reinterpret_cast<const float2 *>(xr + (size_t)row * p.n);
        for (int q = t; q < M; q += T) base[lpad(q)] = src[q];   // z(q) = x(2q) + j x(2q+1)
    }
    lds_sync();
    fft_lds<false>(base, 1, active ? t : T, T, p.fft);
    if (active) {
        float2 *out = spec + (size_t)row * (M + 1);
        for (int k = t; k <= M / 2; k += T) {
            const float2 zk = base[lpad(k)];
            if (k == 0) {
                out[0] = make_float2(zk.x + zk.y, 0.f);
                out[M] = make_float2(zk.x - zk.y, 0.f);
                continue;
            }
            const int km = M - k;
            float2 xk, xm;
            rsplit_pair(zk, base[lpad(km)], p.split[k], p.split[km], xk, xm);
            out[k] = xk;
            if (km != k) out[km] = xm;
        }
    }
}

// --------------------------------------------------------------- post (fwd)
__global__ void __launch_bounds__(256) k_rc_post(PlanRC1D p, const float2 *__restrict__ spec,
                                                  float *__restrict__ y) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const size_t row = blockIdx.y;
    const int n = p.n, M = p.m;
    if (k >= n) return;
    const float2 *X = spec + row * (M + 1);
    const float2 v = (k <= M) ? X[k] : conjf2(X[n - k]);
    const float2 w = p.tw[k];
    y[row * n + k] = w.x * v.x - w.y * v.y;   // Re(w X), w = 2 * scale * e^{-j pi k/2n} / 2
}

// ---------------------------------------------------------------- pre (inv)
__global__ void __launch_bounds__(256) k_rc_ipre(PlanRC1D p, const float *__restrict__ y,
                                                  float2 *__restrict__ spec) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const size_t row = blockIdx.y;
    const int n = p.n, M = p.m;
    if (k > M) return;
    const float *yr = y + row * n;
    const float a = yr[k];
    const float b = (k == 0) ? 0.f : yr[n - k];   // y(n) = 0
    spec[row * (M + 1) + k] = cmul(p.tw[k], make_float2(a, -b));
}

// -------------------------------------------------------- batched inverse FFT
__global__ void __launch_bounds__(kMaxBlock) k_rc_irfft(PlanRC1D p, const float2 *__restrict__ spec,
                                                    float *__restrict__ xr) {
    extern __shared__ float2 lds[];
    const int T = p.fft.T;
    const int r = threadIdx.x / T;
    const int t = threadIdx.x - r * T;
    const int row = blockIdx.x * p.rows_per_block + r;
    const bool active = (r < p.rows_per_block) && (row < p.batch);
    const int M = p.m;
    if (p.odd) {
        // odd n: the Hermitian length-n spectrum from k = 0 .. m, its inverse
        // FFT, the real part
        float2 *buf = lds + (r < p.rows_per_block ? r : 0) * lpad_len(p.n);
        if (active) {
            const float2 *U = spec + (size_t)row * (M + 1);
            for (int k = t; k <= M; k += T) {
                const float2 u = U[k];
                buf[lpad(k)] = u;
                if (k >= 1) buf[lpad(p.n - k)] = conjf2(u);
            }
        }
        lds_sync();
        fft_lds<true>(buf, 1, active ? t : T, T, p.fft);
        if (active) {
            float *dst = xr + (size_t)row * p.n;
            for (int q = t; q < p.n; q += T) dst[q] = buf[lpad(q)].x;
        }
        return;
    }
    float2 *base = lds + (r < p.rows_per_block ? r : 0) * lpad_len(M);
    constexpr int kPairs = kEmax / 2 + 1;
    float2 zk[kPairs], zm[kPairs];
    if (active) {
        const float2 *U = spec + (size_t)row * (M + 1);
#pragma unroll
        for (int i = 0; i < kPairs; ++i) {
            const int k = t + i * T;
            if (k <= M / 2) {
                if (k == 0) {
                    const float u0 = U[0].x, um = U[M].x;
                    zk[i] = make_float2(u0 + um, u0 - um);
                } else {
                    irsplit_pair(U[k], U[M - k], p.split[k], p.split[M - k], zk[i], zm[i]);
                }
            }
        }
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
    fft_lds<true>(base, 1, active ? t : T, T, p.fft);
    if (active) {
        float2 *dst = reinterpret_cast<float2 *>(xr + (size_t)row * p.n);
        for (int q = t; q < M; q += T) dst[q] = base[lpad(q)];
    }
}

// --------------------------------------------------------------- post (inv)
__global__ void __launch_bounds__(256) k_rc_ipost(int n, const float *__restrict__ xr, float *__restrict__ y) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const size_t row = blockIdx.y;
    if (i < n) y[row * n + perm_fwd(i, n)] = xr[row * n + i];
}

// ----------------------------------------------------------------- transpose
// out (cols x rows) = in (rows x cols)^T through a padded 64 x 64 LDS tile.
__global__ void __launch_bounds__(256) k_transpose(const float *__restrict__ in, float *__restrict__ out,
                                                    int rows, int cols) {
    __shared__ float tile[64][65];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int k = ty; k < 64; k += 4) {
        const int r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = in[(size_t)r * cols + c];
    }
    lds_sync();
    for (int k = ty; k < 64; k += 4) {
        const int c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) out_store(&out[(size_t)c * rows + r], tile[tx][k]);   // the final transpose writes y
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_rc_pre(const PlanRC1D &p, const float *x, float *xr, hipStream_t s) {
    hipLaunchKernelGGL(k_rc_pre, dim3((p.n + 255) / 256, p.batch), dim3(256), 0, s, p.n, x, xr);
    return hipGetLastError();
}

hipError_t launch_rc_rfft(const PlanRC1D &p, const float *xr, float2 *spec, hipStream_t s) {
    const int rpb = p.rows_per_block;
    const size_t lds = (size_t)rpb * lpad_len(p.odd ? p.n : p.m) * sizeof(float2);
    hipLaunchKernelGGL(k_rc_rfft, dim3((p.batch + rpb - 1) / rpb), dim3(rpb * p.fft.T), lds, s, p, xr, spec);
    return hipGetLastError();
}

hipError_t launch_rc_post(const PlanRC1D &p, const float2 *spec, float *y, hipStream_t s) {
    hipLaunchKernelGGL(k_rc_post, dim3((p.n + 255) / 256, p.batch), dim3(256), 0, s, p, spec, y);
    return hipGetLastError();
}

hipError_t launch_rc_ipre(const PlanRC1D &p, const float *x, float2 *spec, hipStream_t s) {
    hipLaunchKernelGGL(k_rc_ipre, dim3((p.m + 1 + 255) / 256, p.batch), dim3(256), 0, s, p, x, spec);
    return hipGetLastError();
}

hipError_t launch_rc_irfft(const PlanRC1D &p, const float2 *spec, float *xr, hipStream_t s) {
    const int rpb = p.rows_per_block;
    const size_t lds = (size_t)rpb * lpad_len(p.odd ? p.n : p.m) * sizeof(float2);
    hipLaunchKernelGGL(k_rc_irfft, dim3((p.batch + rpb - 1) / rpb), dim3(rpb * p.fft.T), lds, s, p, spec, xr);
    return hipGetLastError();
}

hipError_t launch_rc_ipost(const PlanRC1D &p, const float *xr, float *y, hipStream_t s) {
    hipLaunchKernelGGL(k_rc_ipost, dim3((p.n + 255) / 256, p.batch), dim3(256), 0, s, p.n, xr, y);
    return hipGetLastError();
}

hipError_t launch_transpose(const float *in, float *out, int rows, int cols, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose, dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, s, in, out, rows, cols);
    return hipGetLastError();
}

}  // namespace dctx
