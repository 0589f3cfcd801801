/*
 * dctx — multi-dimensional DCT-II / DCT-III (IDCT) on AMD MI355X (gfx950).
 *
 * Public C ABI.  Plain C types only: device buffers are passed as plain
 * pointers, streams as `void*` holding a `hipStream_t` (NULL = the null
 * stream).  Every entry point returns a dctx_status; on any error nothing has
 * been enqueued and the output buffer is untouched.  No C++ exception crosses
 * this boundary.
 *
 * Method (Jiang, Gu, Pan, "A New Acceleration Paradigm for Discrete Cosine
 * Transform and Other Fourier-Related Transforms"): an MD DCT is computed by
 * three stages — a reorder preprocess (Eq. 2d_dct_pre), a multi-dimensional
 * real-to-complex FFT, and a twiddle / symmetric-pair postprocess (Eqs.
 * 2d_dct_post, four-elements, s-t) — and the IDCT by the mirror image
 * (Eqs. 2d_idct_pre, 2d_idct_post).  Here the reorder is fused into the loads
 * of the first FFT pass and the postprocess into the stores of the last, so a
 * 2-D transform makes two passes over HBM.
 *
 * Conventions shared by all transforms:
 *  - Arrays are dense, row-major, FP32, the last dimension contiguous:
 *    a 2-D array is n1 x n2 (n2 contiguous), a 3-D array n1 x n2 x n3.
 *  - Input and output must not overlap (in-place is DCTX_ERR_INVALID).
 *  - Pointers must be device pointers, 8-byte aligned.  The caller owns them
 *    and keeps them alive until the work on `stream` has completed.
 *  - Execution is asynchronous on `stream`.
 *  - Supported sizes on the GPU: each dimension 2^a * 3^b * 5^c and >= 2.
 *    An even last (contiguous) dimension is packed into a half-length complex
 *    row FFT; an odd one runs full-length complex row FFTs of the real rows.
 *    Upper limits are given per call.  Anything else returns
 *    DCTX_ERR_UNSUPPORTED (there is no silent fallback of any kind).
 */
#ifndef DCTX_H
#define DCTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dctx_status {
    DCTX_OK = 0,
    DCTX_ERR_INVALID = 1,      /* null pointer, bad dimension, bad enum, aliasing */
    DCTX_ERR_UNSUPPORTED = 2,  /* valid arguments the GPU path does not implement */
    DCTX_ERR_NOMEM = 3,        /* device or host allocation failed */
    DCTX_ERR_DEVICE = 4,       /* a HIP runtime call failed */
    DCTX_ERR_BUSY = 5,         /* the request has not completed yet */
    DCTX_ERR_TOO_LARGE = 6,    /* the shape needs more scratch than dctx_dct2d_noalloc holds */
    DCTX_ERR_CANCELLED = 7     /* a served request cancelled before it was launched */
} dctx_status;

/*
 * Normalisation.  The paper states none (its three-stage output is 2^D times
 * the sum of Eq. 1d-definition a); both modes below are exact inverses.
 *  DCTX_NORM_BACKWARD: dct = the raw sums of Eq. (1d-definition a) along every
 *      axis; idct = prod_d (2 / N_d) * raw DCT-III (Eq. 1d-definition b), so
 *      idct(dct(x)) = x.
 *  DCTX_NORM_ORTHO: the orthonormal DCT-II (weights sqrt(1/N) at k = 0 and
 *      sqrt(2/N) otherwise, per axis) and its transpose; Parseval holds.
 */
typedef enum dctx_norm {
    DCTX_NORM_BACKWARD = 0,
    DCTX_NORM_ORTHO = 1
} dctx_norm;

/* Opaque library handle: device binding, plan cache (FP64-generated twiddle
 * tables rounded to FP32), and a workspace it grows on demand.  A handle is not
 * thread-safe and its plain calls must be issued on one stream at a time (they
 * share the workspace); use one handle per stream for concurrent work. */
typedef struct dctx_context *dctx_handle;

/* Static text for a status code (never NULL). */
const char *dctx_status_string(dctx_status s);

/* Library ABI version: (major << 16) | minor. */
int dctx_version(void);

/* Host-only check of the radix-butterfly constants compiled into the library
 * against FP64 cos/sin.  Returns DCTX_OK or DCTX_ERR_INVALID; *max_err (nullable)
 * receives the largest absolute difference.  Needs no GPU. */
dctx_status dctx_selfcheck(double *max_err);

/* Whether dctx_dct2d accepts length n along the contiguous dimension
 * (axis_last = 1, the other dimension 2) or along the first (axis_last = 0).
 * The other calls have their own limits: dctx_shape_supported answers for a
 * whole shape of each kind.  Needs no GPU. */
int dctx_length_supported(int n, int axis_last);

/* Create a handle bound to HIP device `device` (made current on every call). */
dctx_status dctx_create(int device, dctx_handle *out);

/* Destroy a handle: synchronises the device, frees tables and workspace. */
dctx_status dctx_destroy(dctx_handle h);

/* Bytes of device workspace one plain 2-D / 3-D call of this shape needs
 * (the packed half spectrum: n1 * (n2 / 2) complex64 in 2-D, n1 * n2 * (n3 / 2)
 * complex64 in 3-D; for a 2-D shape on the transposed route of dctx_dct2d,
 * also the two transposed arrays).  Needs no GPU. */
dctx_status dctx_workspace_bytes_2d(int n1, int n2, size_t *bytes);
dctx_status dctx_workspace_bytes_3d(int n1, int n2, int n3, size_t *bytes);

/*
 * 2-D DCT-II of an n1 x n2 array (three-stage method, Alg. alg:DCT "2D_DCT").
 *   x: device input, n1*n2 floats;  y: device output, n1*n2 floats.
 *   Two kernels on `stream`: (1) rows: Eq. (2d_dct_pre) reorder + length-n2
 *   real FFT of every row, written as the packed half spectrum; (2) columns:
 *   length-n1 complex FFT of every packed column + the four-element
 *   postprocess of Eqs. (four-elements)/(s-t), written to y.
 *   Limits: 2 <= n1 <= 8192, 3 <= n2 <= 16384 (n2 even >= 4, or odd and
 *   <= 7680: an odd n2 runs each row as one workgroup's full-length complex
 *   FFT of the real row, and the workspace holds columns 0 .. (n2-1)/2).
 *   An even n1 in (8192, 16384] with n2 <= 8192 takes the axis-order route
 *   (Section "Results on 2D DCTs": input and output can be transposed, the
 *   transposition folded into the pre- and postprocess): the same two passes
 *   on the n2 x n1 transpose, the row pass reading columns of x and the
 *   column pass writing rows of y (no transpose kernel, no extra pass).
 *   n1 = 8192 with even n2 runs three kernels: the row pass, the first
 *   radix-8 step of the column FFTs as an in-place pass over the workspace,
 *   and 1024-point column FFTs with the postprocess (same results).
 *   The first call for a new (n1, n2, norm) builds its tables (synchronous);
 *   a call that needs a larger workspace than the handle holds synchronises
 *   the device before replacing it.
 */
dctx_status dctx_dct2d(dctx_handle h, const float *x, float *y, int n1, int n2,
                       dctx_norm norm, void *stream);

/* 2-D IDCT (DCT-III, the inverse of dctx_dct2d under the same norm), Alg.
 * alg:DCT "2D_IDCT": (1) columns: Eq. (2d_idct_pre) (twiddle exponent +j; four
 * reads, two writes) + inverse column FFT; (2) rows: inverse real FFT of every
 * row + the Eq. (2d_idct_post) inverse reorder.  Same arguments and limits. */
dctx_status dctx_idct2d(dctx_handle h, const float *x, float *y, int n1, int n2,
                        dctx_norm norm, void *stream);

/*
 * Batched 1-D DCT-II of `batch` rows of length n (x, y: batch x n floats,
 * row-major), by the N-point algorithm (Section "Four Algorithms of 1D DCT",
 * Table 1ddct; Eqs. n_pre, n_post_update): one kernel, each row one group of
 * threads holding it in LDS, with the Eq. (n_pre) reorder fused into the
 * loads, the length-n real FFT (a length-n/2 complex FFT and the even/odd
 * split) and the Eq. (n_post_update) postprocess fused into the stores, so a
 * call reads and writes each element once.  norm as dctx_dct2d.
 * Longer rows (16384 < n <= 2^20) run the same algorithm with the length-n/2
 * FFT split four-step style, n/2 = m1 m2: a column pass (the reorder fused into
 * the gathers, length-m1 FFTs, twiddles) and a row pass (length-m2 FFTs of the
 * row pairs {k1, m1 - k1}, the split and the postprocess), through the
 * handle's workspace of batch x n/2 complex values (grown with a device
 * synchronisation as for the 2-D calls).
 * Limits: batch >= 1; n even, 2^a 3^b 5^c, 2 <= n <= 2^20; batch <= 65535 and
 * n * batch <= 2^30 for n > 16384; anything else is DCTX_ERR_UNSUPPORTED
 * (n < 1 or batch < 1: DCTX_ERR_INVALID).
 */
dctx_status dctx_dct1d(dctx_handle h, const float *x, float *y, int n, int batch,
                       dctx_norm norm, void *stream);

/* Batched 1-D DCT-III, the inverse of dctx_dct1d under the same norm: the
 * pre U(k) = exp(+j pi k / 2n) s(k) (y(k) - j y(n - k)), y(n) = 0, the inverse
 * split and inverse FFT, the inverse reorder fused into the stores.  Same
 * arguments and limits. */
dctx_status dctx_idct1d(dctx_handle h, const float *x, float *y, int n, int batch,
                        dctx_norm norm, void *stream);

/*
 * The mixed 2-D transforms of the DREAMPlace electric-field step (Section
 * "Other Transforms and Platforms", Eq. idxst), through the same two passes
 * as dctx_idct2d.  The 1-D IDXST of a length-N sequence is the IDCT of the
 * sequence reversed with a zero in front, x'(n) = x(N - n), x'(0) = x(N) = 0,
 * with the output multiplied by (-1)^k (so x(0) does not contribute).  A 1-D
 * transform of a matrix acts on its columns (as in MATLAB, which the paper
 * validates against), so, as the paper also states in words,
 *   dctx_idct_idxst2d: IDCT(IDXST(x)^T)^T = IDXST along n1, IDCT along n2;
 *   dctx_idxst_idct2d: IDXST(IDCT(x)^T)^T = IDCT along n1, IDXST along n2.
 * The reversal is folded into the four reads of the Eq. (2d_idct_pre)
 * preprocess and the sign into the row pass's stores.  IDCT and IDXST follow
 * `norm` as dctx_idct2d does.  Arguments and limits as dctx_idct2d.
 */
dctx_status dctx_idct_idxst2d(dctx_handle h, const float *x, float *y, int n1, int n2,
                              dctx_norm norm, void *stream);
dctx_status dctx_idxst_idct2d(dctx_handle h, const float *x, float *y, int n1, int n2,
                              dctx_norm norm, void *stream);

/* Same as dctx_dct2d / dctx_idct2d with a caller-provided device workspace of
 * at least dctx_workspace_bytes_2d(n1, n2) bytes (16-byte aligned); the handle's
 * own workspace is not used, so calls on different streams with different
 * workspaces may overlap. */
dctx_status dctx_dct2d_ws(dctx_handle h, const float *x, float *y, int n1, int n2,
                          dctx_norm norm, void *workspace, size_t ws_bytes, void *stream);
dctx_status dctx_idct2d_ws(dctx_handle h, const float *x, float *y, int n1, int n2,
                           dctx_norm norm, void *workspace, size_t ws_bytes, void *stream);

/*
 * Allocation-free form of dctx_dct2d_ws / dctx_idct2d_ws, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  inverse = 0: DCT-II as
 * dctx_dct2d; inverse = 1: DCT-III as dctx_idct2d; same kernels, same results
 * (bitwise), same arguments otherwise.
 *   The workspace and the FP32 tables live in one static device array of the
 *   library (DCTX_NOALLOC_WS_BYTES of workspace plus 4 MiB of tables), which
 *   every GPU the call runs on holds until the process ends.  The call makes
 *   no hipMalloc / hipFree and uses no allocating library routine; the first
 *   call for a new (n1, n2, norm, direction) copies its tables into the array
 *   with a synchronous hipMemcpy, and when the table part is full the call
 *   synchronises the device and starts it over.
 *   Limits as dctx_dct2d, and dctx_workspace_bytes_2d(n1, n2) must not exceed
 *   DCTX_NOALLOC_WS_BYTES (64 MiB: up to 4096 x 4096, and 8192 x 2048):
 *   otherwise DCTX_ERR_TOO_LARGE and nothing is enqueued.
 *   All calls on one GPU share that GPU's array and it keeps the last call's
 *   contents: calls that overlap on one GPU (other streams, other threads
 *   between enqueue and completion) race on the workspace.  Calls from
 *   several host threads are serialised while they enqueue.
 */
#define DCTX_NOALLOC_WS_BYTES ((size_t)64 << 20)
dctx_status dctx_dct2d_noalloc(dctx_handle h, const float *x, float *y, int n1, int n2,
                               dctx_norm norm, int inverse, void *stream);

/*
 * Row-column baseline (the paper's comparison method, Section "Examples and
 * Summary", Fig. operator-fusion): per axis a separate reorder kernel
 * (Eq. n_pre), a batched 1-D real FFT kernel, a separate postprocess kernel
 * (Eq. n_post_update) and a transpose — 8 full-array memory stages in all.
 * Same arguments and results as dctx_dct2d / dctx_idct2d; limits:
 * 2 <= n1, n2 <= 16384 (an odd length runs its 1-D real FFTs as full-length
 * complex FFTs).  The handle's workspace grows to 2 * n1 * n2 floats plus
 * max(n1 * (n2/2 + 1), n2 * (n1/2 + 1)) complex64.
 */
dctx_status dctx_rc_dct2d(dctx_handle h, const float *x, float *y, int n1, int n2,
                          dctx_norm norm, void *stream);
dctx_status dctx_rc_idct2d(dctx_handle h, const float *x, float *y, int n1, int n2,
                           dctx_norm norm, void *stream);

/*
 * 3-D DCT-II of an n1 x n2 x n3 array (n3 contiguous) by the three-stage method
 * extended to three dimensions (Section "Other Transforms and Platforms": 3-D
 * reorder, 3-D real FFT, a postprocess that reads four spectrum values and
 * writes eight outputs).
 *   x: device input, n1*n2*n3 floats;  y: device output, n1*n2*n3 floats.
 *   Three kernels on `stream`: (1) rows: reorder on all three axes + length-n3
 *   real FFT of every row into the packed half spectrum (workspace); (2) the
 *   length-n2 complex FFT inside every n1-plane, in place; (3) the length-n1
 *   complex FFT of the columns (k2, k3) and (n2 - k2, k3) together + the
 *   four-read / eight-write postprocess, written to y.
 *   Small n1-planes run two kernels instead, (1)+(2) as one plane pass (the
 *   n3 and n2 FFTs of a whole n1-plane in one workgroup, the packed
 *   half-spectrum plane in LDS) and then (3): by default for n1 a power of two
 *   in [64, 256], n2 in {64, 128}, n3 in {64, 128} and 16-byte aligned arrays
 *   (DCTX_FPLANE=0 in the environment when the plan is built keeps the three
 *   kernels); with DCTX_PLANE=1, a run-time-schedule plane pass for n1, n2
 *   powers of two in [64, 256], n3 even, n2 * n3 <= 128^2 (slower).  Same
 *   results on every route to FP32 rounding.
 *   Limits: 2 <= n1 <= 4096, 2 <= n2 <= 8192, 2 <= n3 <= 16384 (odd n3: the
 *   rows run full-length complex FFTs), all 2^a 3^b 5^c, n1 * n2 <= 2^26.
 *   Workspace: dctx_workspace_bytes_3d (the handle's).
 */
dctx_status dctx_dct3d(dctx_handle h, const float *x, float *y, int n1, int n2, int n3,
                       dctx_norm norm, void *stream);

/* 3-D IDCT (the inverse of dctx_dct3d under the same norm): (1) the separable
 * 3-D form of Eq. (2d_idct_pre) — per pair of columns eight reads of y at the
 * reflected indices (zero at index N_d), twiddle exp(+j pi k_d / 2N_d) per axis
 * — + the inverse length-n1 FFT; (2) the inverse n2 FFT; (3) the inverse real
 * FFT of every row + the inverse reorder on all three axes (Eq. 2d_idct_post
 * per axis); (2)+(3) as one plane pass where dctx_dct3d runs one (see
 * there).  Same arguments and limits. */
dctx_status dctx_idct3d(dctx_handle h, const float *x, float *y, int n1, int n2, int n3,
                        dctx_norm norm, void *stream);

/*
 * Spectral solve of the Neumann Poisson problem on a cell-centred n1 x n2 grid
 * (Section "Case studies", DREAMPlace: the potential from a DCT, a division by
 * the Laplacian eigenvalues and an inverse DCT):
 *   F = DCT-II(f);  U = F / lam with lam(k1,k2) = (2 cos(pi k1/n1) - 2)/h1^2 +
 *   (2 cos(pi k2/n2) - 2)/h2^2 and U(0,0) = 0;  u = DCT-III(U) (backward norm).
 * u solves the 5-point Neumann Laplacian equation Lap(u) = f - mean(f) and has
 * zero mean.  f: device input, u: device output, n1*n2 floats each.
 * h1, h2: grid spacings along n1, n2; a value <= 0 selects 1/n1 (1/n2), the
 * unit square; NaN or infinity is DCTX_ERR_INVALID.
 * Three kernels: the DCT row pass; one column pass that runs the forward
 * column FFT, the four-element post, the divide, the four-read IDCT pre and the
 * inverse column FFT without writing F to memory; the IDCT row pass.
 * Limits as dctx_dct2d without its axis-order route (n1 <= 8192); an odd n2
 * runs full-length row FFTs.
 */
dctx_status dctx_poisson2d(dctx_handle h, const float *f, float *u, int n1, int n2,
                           double h1, double h2, void *stream);

/*
 * Threshold compression of a 2-D array (Section "Case studies", image
 * compression, Alg. image-compression and Eq. image-compression):
 *   B = DCT-II(x) under `norm`;  C(i,j) = B(i,j) if |B(i,j)| >= eps, else 0;
 *   y = DCT-III(C) under `norm` (the inverse of the DCT).
 * The threshold runs inside the same fused column pass as dctx_poisson2d, in
 * place of the divide, so the call makes three passes over HBM and B never
 * reaches memory.  The decision |B| >= eps is taken on the FP32 coefficient.
 * eps: finite and >= 0 (eps = 0 keeps every coefficient); NaN, infinity or a
 * negative value is DCTX_ERR_INVALID.  Limits as dctx_poisson2d.
 */
dctx_status dctx_compress2d(dctx_handle h, const float *x, float *y, int n1, int n2,
                            dctx_norm norm, double eps, void *stream);

/*
 * Small-N batched 2-D DCT as the dense contraction Y = C X C^T on the matrix
 * cores (Section "Computation of DCTs": the DCT as a matrix product).
 *   x, y: device, batch matrices of n x n floats each, contiguous, 16-byte
 *   aligned; n in {16, 32, 64, 128}; 1 <= batch.
 *   inverse = 0: DCT-II (as dctx_dct2d), 1: DCT-III (as dctx_idct2d), under norm.
 *   prec: the arithmetic, chosen by the caller (there is no hidden fallback):
 *     DCTX_PREC_BF16X3      each operand split into two bf16 (hi + lo), three
 *                           MFMA products per product, FP32 accumulation;
 *                           relative L2 error about 1e-5 of the result.
 *     DCTX_PREC_FP16_SCALED per-matrix power-of-two scaling to fp16, FP32
 *                           accumulation; relative L2 error about 1e-3.
 *   One persistent launch on `stream`.
 */
typedef enum dctx_prec {
    DCTX_PREC_BF16X3 = 0,
    DCTX_PREC_FP16_SCALED = 1
} dctx_prec;

dctx_status dctx_dct2d_small(dctx_handle h, const float *x, float *y, int n, int batch, int inverse,
                             dctx_norm norm, dctx_prec prec, void *stream);

/*
 * Batched execution of many independent transforms of uneven sizes (the
 * transforms of a batch are independent, Section "Other Transforms and
 * Platforms"; each is computed exactly as by its plain call).
 */
typedef enum dctx_kind {
    DCTX_KIND_DCT2 = 0,      /* dctx_dct2d,  ndim 2 */
    DCTX_KIND_IDCT2 = 1,     /* dctx_idct2d, ndim 2 */
    DCTX_KIND_DCT3 = 2,      /* dctx_dct3d,  ndim 3 */
    DCTX_KIND_IDCT3 = 3,     /* dctx_idct3d, ndim 3 */
    DCTX_KIND_POISSON2 = 4   /* dctx_poisson2d, ndim 2 (norm ignored, h = spacings) */
} dctx_kind;

/* Whether the plain call of `kind` (dctx_dct2d, dctx_idct2d, dctx_dct3d,
 * dctx_idct3d, dctx_poisson2d) accepts an n1 x n2 (x n3) array: 1 exactly when
 * that call, given valid buffers and arguments, does not return
 * DCTX_ERR_UNSUPPORTED for the shape (the call's own size checks and plan
 * geometry, evaluated on the host for the gfx950 LDS size).  n3 is ignored for
 * the 2-D kinds.  Needs no GPU. */
int dctx_shape_supported(dctx_kind kind, int n1, int n2, int n3);

/* Host-only check of the batched passes' tile geometry for an n1 x n2 item
 * (no device needed): for every block size the autotuner tries and every pass
 * kind, the LDS slots the tile bodies touch lie within the LDS bytes the launch
 * passes (and within the device's 160 KB), every sequence of a tile has its
 * threads, and the tiles cover the rows / columns exactly.  Returns 1 when all
 * hold, else 0 with the first failing case in msg (nullable, msglen bytes). */
int dctx_batch_geometry_check(int n1, int n2, char *msg, int msglen);

typedef struct dctx_desc {
    dctx_kind kind;
    int ndim;                /* 2 or 3, as the kind requires */
    int dims[3];             /* n1, n2 (, n3); last dimension contiguous */
    const float *in;         /* device input, prod(dims) floats */
    float *out;              /* device output, prod(dims) floats */
    dctx_norm norm;
    double h[2];             /* Poisson grid spacings (<= 0: 1/n1, 1/n2) */
} dctx_desc;

/*
 * Enqueue `count` transforms on `stream` as one batch.  The 2-D items run as
 * at most five persistent launches, one per pass kind (forward rows, inverse
 * columns, forward columns + post, fused Poisson columns, inverse rows), each
 * covering the tiles of every item that needs it; 3-D items follow with their
 * plain kernels.  Launch geometry comes from dctx_autotune_batch for a batch
 * of the same shapes, else a default (one workgroup per tile, 256 threads for
 * the row passes, 512 for the column passes).
 *   Per-item rules are those of the plain calls; additionally no item's output
 *   may overlap any other item's input or output.  per_item (host, nullable,
 *   count entries) receives each item's check result.  If any item fails,
 *   nothing is enqueued and the first failure is returned.
 *   The item descriptors are copied through a pinned staging ring of 16
 *   slots (a 17th batch in flight waits for the first); the handle's batch
 *   workspace grows on demand (synchronising the device when it does).
 *   Descriptors and buffers must stay valid until the stream reaches the batch.
 */
dctx_status dctx_submit_batch(dctx_handle h, const dctx_desc *d, int count, void *stream,
                              dctx_status *per_item);

/* Result of dctx_autotune_batch, per pass kind (index: forward rows, forward
 * columns, inverse columns, inverse rows, Poisson columns). */
typedef struct dctx_tune_info {
    int block[5];            /* chosen threads per workgroup (0: pass unused) */
    int grid_factor[5];      /* chosen persistent workgroups per CU (0: one per tile) */
    int per_cap[5];          /* chosen cap on rows / packed columns per tile (0: none) */
    int tiles[5];            /* tiles of the pass */
    double pass_ms[5];       /* best measured time of the pass */
    double default_ms;       /* all passes with the default configuration */
    double tuned_ms;         /* all passes with the chosen configurations */
} dctx_tune_info;

/* Autotuner: runs the batch (synchronously, results written to the outputs)
 * under every candidate launch geometry (threads per workgroup 128/256/512 x
 * persistent workgroups per CU 2/4/8/16 or one per tile), then at the best one
 * under caps of 1/2/4/8 sequences per tile, times each pass with HIP events
 * (best of repeated runs) and keeps the fastest per pass in the handle's
 * tuning cache, keyed by the multiset of (kind, dims).  info is nullable. */
dctx_status dctx_autotune_batch(dctx_handle h, const dctx_desc *d, int count, void *stream,
                                dctx_tune_info *info);

/* The handle's tuning cache as a JSON file keyed by the device's gfx
 * architecture and the batch signature (a hash of the multiset of (kind,
 * dims)): dctx_tune_save writes (replaces) the file with the cache's entries
 * for this device's architecture, merged with the entries the file already
 * holds for other architectures; dctx_tune_load adds the file's entries for
 * this device's architecture to the cache (*loaded, nullable: how many).
 * DCTX_ERR_INVALID for a null handle or path, a file that cannot be opened
 * (load) or written (save), or a file not in this format (load). */
dctx_status dctx_tune_save(dctx_handle h, const char *path);
dctx_status dctx_tune_load(dctx_handle h, const char *path, int *loaded);

/* A batch captured once into a HIP graph (its own workspace and descriptor
 * buffers; the plans stay in the handle, which must outlive the graph) and
 * replayed by dctx_graph_launch on any stream.  The buffers named by the
 * descriptors are fixed at capture. */
typedef struct dctx_graph_s *dctx_graph;
dctx_status dctx_graph_create(dctx_handle h, const dctx_desc *d, int count, dctx_graph *out);
dctx_status dctx_graph_launch(dctx_graph g, void *stream);
/* Synchronises the device, then frees the graph and its buffers. */
dctx_status dctx_graph_destroy(dctx_graph g);

/*
 * Serving loop (continuous batching; the transforms of a batch are
 * independent, Section "Other Transforms and Platforms").  A scheduler thread
 * with a private handle, `nstreams` streams and a device pool of hbm_budget
 * bytes admits arrived requests in FIFO order while fewer than max_inflight
 * are on the GPU and their workspace fits in the pool, and launches them as
 * batches of at most max_batch requests on the streams in turn, so batches on
 * different streams overlap on the device.  While batches are on the GPU, a
 * new batch starts only once min_batch requests are waiting, the GPU has
 * gone idle, or the oldest waiting request has waited max_wait_us: requests
 * arriving during a busy period are gathered and join the next batch as slots
 * and memory free up, and at low load none waits longer than that bound.  The
 * default bound (1 us) launches what is ready at once: the requests that
 * arrive while a batch runs still form the next one.
 * Inside a batch, requests of one kind, shape, norm (and spacing) with at
 * least 2^16 elements on the compile-time kernels (power-of-two 2-D shapes of
 * any kind; 3-D shapes with n1, n2 in {64, 128, 256}; 16-byte aligned
 * buffers) run each pass as one launch over up to 16 of them, the launches of
 * their plain call with a grid layer per request; the others share the
 * persistent launches of dctx_submit_batch.  A result is therefore bitwise
 * the same alone and in any batch.
 * plain = 1 runs the per-request baseline instead: every request alone with
 * its plain entry point, in arrival order, on one stream.
 * Request buffers are the caller's (device memory, valid until the request is
 * done); results are those of the plain calls to FP32 rounding (bitwise where
 * the batch runs the plain call's kernels).
 */
typedef struct dctx_server_config {
    int device;
    size_t hbm_budget;       /* workspace pool bytes (batched mode) */
    int max_inflight;        /* requests on the GPU at once, >= 1 */
    int nstreams;            /* 1..16 */
    int max_batch;           /* requests per batch (0: 1024) */
    int plain;               /* 0: continuous batching, 1: per-request baseline */
    int min_batch;           /* waiting requests that start a batch while others run (0: 4) */
    int max_wait_us;         /* longest wait for min_batch while others run (0: 1 us; < 0: no bound) */
} dctx_server_config;

typedef struct dctx_server_s *dctx_server;

typedef struct dctx_req_stats {
    dctx_status status;      /* DCTX_OK or the failure */
    double arrival_s;        /* server clock (seconds since creation) */
    double launch_s;         /* batch enqueued */
    double done_s;           /* completion observed */
    double latency_ms;       /* done - arrival */
    int batch_size;          /* requests in its batch */
} dctx_req_stats;

typedef struct dctx_server_summary {
    int64_t completed;       /* successful requests with ticket >= first_ticket */
    double p50_ms, p99_ms, mean_ms, max_ms;   /* latency percentiles */
    double span_s;           /* first arrival to last completion */
    double req_per_s;        /* completed / span_s */
    int64_t batches;         /* batches launched since creation */
    double mean_batch;       /* mean requests per batch */
    size_t peak_pool_bytes;  /* peak workspace in use */
} dctx_server_summary;

dctx_status dctx_server_create(const dctx_server_config *cfg, dctx_server *out);
/* Seconds since the server was created (the clock of arrival times). */
dctx_status dctx_server_now(dctx_server s, double *t);
/* Queue one request arriving at arrival_s on the server clock (< 0: now).
 * The descriptor is checked like a batch item and copied; *ticket identifies
 * it.  DCTX_ERR_NOMEM if its workspace exceeds the whole pool. */
dctx_status dctx_server_submit(dctx_server s, const dctx_desc *d, double arrival_s, uint64_t *ticket);
/* DCTX_ERR_BUSY until the request is done; then fills *out (nullable). */
dctx_status dctx_server_poll(dctx_server s, uint64_t ticket, dctx_req_stats *out);
/* Blocks until every submitted request is done. */
dctx_status dctx_server_drain(dctx_server s);
/* Latency percentiles and throughput over the tickets >= first_ticket. */
dctx_status dctx_server_summary_get(dctx_server s, uint64_t first_ticket, dctx_server_summary *out);
/*
 * Write-count build only (libdctx_wc.so, the same sources built with
 * -DDCTX_WRITE_COUNT; a test aid): binds `count` (device memory, one unsigned
 * per 4-byte word of the output range [base, base + bytes), zeroed by the
 * caller) so that every later store of a transform's final output into that
 * range also adds one to that word's counter: a test then checks that each
 * output word is written exactly once.  count = base = NULL unbinds; exactly
 * one of them NULL is DCTX_ERR_INVALID.  Covered: every transform's final
 * output stores (1-D, 2-D, 3-D, IDXST, Poisson, compression, the small-N
 * matrix path and the row-column baseline; plain, batched and served).
 * The product library returns DCTX_ERR_UNSUPPORTED.  Binding is global to
 * the process's device, so it must not overlap calls on other handles.
 */
dctx_status dctx_debug_write_count(dctx_handle h, unsigned *count, const void *base, size_t bytes);

/* Cancels a request that has not been launched: one still before its arrival
 * time or waiting for admission.  It completes at once with status
 * DCTX_ERR_CANCELLED (poll reports batch_size 0) and its buffers are never
 * touched.  DCTX_ERR_BUSY if it is already on the GPU or done (it completes
 * normally), DCTX_ERR_INVALID for an unknown ticket. */
dctx_status dctx_server_cancel(dctx_server s, uint64_t ticket);
/* Failure injection, for tests of the error path: the next `count` batches
 * (plain mode: launches) that the scheduler forms fail as a device allocation
 * failure would, before anything of them is enqueued.  Their requests
 * complete with DCTX_ERR_NOMEM, their pool space and slots are released, and
 * serving goes on with the requests after them.  count >= 0 (0 clears). */
dctx_status dctx_server_inject_alloc_failures(dctx_server s, int count);
/* Drains, stops the scheduler and frees everything. */
dctx_status dctx_server_destroy(dctx_server s);

/*
 * Per-kernel timing (tracing).  While enabled, every kernel the handle launches
 * is bracketed by two HIP events on its stream (adding an event pair per
 * launch).  dctx_profile_read synchronises the device, aggregates the elapsed
 * times per kernel name into `stats` (capacity entries; *count receives how
 * many kernels were seen) and clears the records.
 */
typedef struct dctx_kernel_stat {
    char name[32];      /* kernel name, e.g. "dct2_cols" */
    int launches;
    double total_ms;
    double min_ms;
    double max_ms;
} dctx_kernel_stat;

dctx_status dctx_profile_enable(dctx_handle h, int enable);
dctx_status dctx_profile_read(dctx_handle h, dctx_kernel_stat *stats, int capacity, int *count);

#ifdef __cplusplus
}
#endif

#endif /* DCTX_H */
