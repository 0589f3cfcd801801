/*
 * FP64 CPU oracle for the multi-dimensional DCT-II / DCT-III.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * What it computes (paper, Section "Background: Discrete cosine transforms"):
 *   - DCT-II of a length-N sequence, Eq. (1d-definition a):
 *         out[k] = sum_{n=0}^{N-1} in[n] * cos(pi/N * (n + 1/2) * k)
 *   - DCT-III (the paper's IDCT), Eq. (1d-definition b):
 *         out[k] = in[0]/2 + sum_{n=1}^{N-1} in[n] * cos(pi/N * n * (k + 1/2))
 *   - multi-dimensional transforms as the composition of the 1-D transform
 *     along every axis, in any order (Eq. 2d-dct-definition and the 3-D text
 *     around Fig. 3d-dct).
 * No normalisation is applied here ("raw" sums); the Python wrapper applies the
 * backward / orthonormal scalings.
 *
 * The cosine is evaluated with exact integer argument reduction:
 *     cos(pi*(2n+1)*k / (2N)) = cos(pi * r / (2N)),  r = ((2n+1)*k) mod 4N,
 * so every coefficient is a correctly reduced FP64 cosine of an angle in
 * [0, 2*pi).  Sums are accumulated in FP64 in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* C[k][n] = cos(pi*(2n+1)*k/(2N)), one entry at a time (only the entries the
 * selected outputs use are ever evaluated, so long sequences need no N x N
 * table) */
static double cos_coef(int k, int n, int N)
{
    const int64_t fourN = 4 * (int64_t)N;
    const int64_t r = ((2 * (int64_t)n + 1) * (int64_t)k) % fourN;
    return cos(M_PI * (double)r / (2.0 * (double)N));
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Raw 1-D transform along axis `axis` of a C-ordered array of rank `nd`
 * (shape `dims`), keeping only the output indices listed in `sel` (nsel of
 * them, each in [0, dims[axis])); pass sel = NULL for all outputs in order.
 * The output array has the shape of the input with dims[axis] replaced by the
 * number of kept indices.  kind = 2: DCT-II, kind = 3: DCT-III.  `in` and
 * `out` must not overlap.  Returns 0 on success, -1 on bad arguments or
 * allocation failure.
 *
 *   out[o, p, i] = sum_m w(m) * in[o, m, i] * coef(q_p, m),   q_p = sel[p]
 *     DCT-II : coef(q, m) = C[q][m], w(m) = 1
 *     DCT-III: coef(q, m) = C[m][q], w(0) = 1/2, w(m > 0) = 1
 */
int oracle_dct_axis_sel(const double *in, double *out, int nd, const int *dims,
                        int axis, int kind, int nsel, const int *sel)
{
    if (!in || !out || !dims || nd < 1 || axis < 0 || axis >= nd) return -1;
    if (kind != 2 && kind != 3) return -1;
    int64_t outer = 1, inner = 1;
    for (int d = 0; d < nd; ++d) {
        if (dims[d] < 1) return -1;
        if (d < axis) outer *= dims[d];
        if (d > axis) inner *= dims[d];
    }
    const int N = dims[axis];
    if (!sel) nsel = N;
    if (nsel < 1) return -1;
    if (sel)
        for (int p = 0; p < nsel; ++p)
            if (sel[p] < 0 || sel[p] >= N) return -1;
    /* K[p][m] = w(m) * coef(q_p, m): one contiguous coefficient row per output */
    double *K = (double *)malloc(sizeof(double) * (size_t)nsel * (size_t)N);
    if (!K) return -1;
#pragma omp parallel for schedule(static)
    for (int p = 0; p < nsel; ++p) {
        const int q = sel ? sel[p] : p;
        for (int m = 0; m < N; ++m) {
            double c = (kind == 2) ? cos_coef(q, m, N) : cos_coef(m, q, N);
            if (kind == 3 && m == 0) c *= 0.5;
            K[(size_t)p * N + m] = c;
        }
    }

#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t o = 0; o < outer; ++o)
        for (int p = 0; p < nsel; ++p) {
            const double *restrict src = in + o * (int64_t)N * inner;
            double *restrict dst = out + o * (int64_t)nsel * inner + (int64_t)p * inner;
            const double *restrict krow = K + (size_t)p * N;
            if (inner == 1) {
                double s = 0.0;
                for (int m = 0; m < N; ++m) s += krow[m] * src[m];
                dst[0] = s;
            } else {
                for (int64_t i = 0; i < inner; ++i) dst[i] = 0.0;
                for (int m = 0; m < N; ++m) {
                    const double c = krow[m];
                    const double *restrict row = src + (int64_t)m * inner;
                    for (int64_t i = 0; i < inner; ++i) dst[i] += c * row[i];
                }
            }
        }
    free(K);
    return 0;
}
