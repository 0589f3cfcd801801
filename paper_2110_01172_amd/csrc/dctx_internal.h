// Internal declarations shared by the host runtime (plans, C ABI) and the HIP
// kernels of the dctx library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/dctx.h"

namespace dctx {

// Butterfly constants, written out to 20 significant digits and rounded to FP32
// by the compiler (dctx_selfcheck compares them with FP64 cos/sin on the host).
constexpr float kSqrtHalf = (float)0.70710678118654752440;   // cos(pi/4)
constexpr float kCos22_5 = (float)0.92387953251128675613;    // cos(pi/8)
constexpr float kSin22_5 = (float)0.38268343236508977173;    // sin(pi/8)
constexpr float kSin60 = (float)0.86602540378443864676;      // sin(pi/3)
constexpr float kCos72 = (float)0.30901699437494742410;      // cos(2pi/5)
constexpr float kSin72 = (float)0.95105651629515357212;      // sin(2pi/5)
constexpr float kCos144 = (float)-0.80901699437494742410;    // cos(4pi/5)
constexpr float kSin144 = (float)0.58778525229247312917;     // sin(4pi/5)

constexpr int kEmax = 16;       // complex values a thread holds in one FFT stage
constexpr int kMaxStages = 16;  // radix stages of one FFT
constexpr int kMaxLen = 16384;  // longest FFT / dimension handled on the GPU
constexpr int kMaxBlock = 512;  // threads per workgroup of the FFT kernels (256-VGPR budget)

// LDS slots a padded sequence of length n occupies (one empty slot every 16
// elements, see lpad() in fft_core.h).
__host__ __device__ constexpr int lpad_len(int n) { return n + (n >> 4) + 1; }

// Schedule of one complex FFT of length L (see fft_core.h).  Stage s (radix
// R = rad[s], Ns = ns[s]) reads its twiddles from a butterfly-major table at
// tw + twoff[s]: record k (k < Ns) holds W_{Ns R}^{r k} for r < R, padded to an
// even number of complex values so a record is read with 16-byte loads.
struct FftDesc {
    int L;
    int nst;
    int T;                        // threads that cooperate on one sequence
    int rad[kMaxStages];
    int ns[kMaxStages];           // product of the radices before stage s
    unsigned nsmagic[kMaxStages]; // ceil(2^32 / ns[s]): j / ns = umulhi(j, magic) for j < 2^16
    int twoff[kMaxStages];        // complex offset of the stage's twiddle records
    const float2 *tw;             // all stage tables, FP64-built, rounded to FP32
};

// Binding of the write-count build (see out_store in fft_core.h): one counter
// per 4-byte word of the output range [base, base + bytes).
struct WriteCountBinding {
    unsigned *count;
    const char *base;
    size_t bytes;
};
// Registers a translation unit's binding setter (write-count build).
void wc_register(hipError_t (*set)(const WriteCountBinding &));

// Complex values per twiddle record of a radix-R stage.
__host__ __device__ constexpr int tw_record(int R) { return R + (R & 1); }

// Compile-time schedule of the power-of-two fast path for length L: T threads
// per sequence, radices R0, R1, R2 (L = R0 R1 R2), and C sequences (columns)
// per workgroup in the column kernels.  L = 0 marks an unsupported length.
struct FastCfg {
    int T, R0, R1, R2, C;
};
__host__ __device__ constexpr FastCfg fast_cfg(int L) {
    return L == 4096 ? FastCfg{128, 16, 16, 16, 2}
         : L == 2048 ? FastCfg{64, 16, 16, 8, 4}
         : L == 1024 ? FastCfg{64, 8, 16, 8, 8}
         : L == 512  ? FastCfg{32, 8, 8, 8, 16}
         : L == 256  ? FastCfg{16, 8, 4, 8, 16}
         : L == 128  ? FastCfg{8, 8, 2, 8, 16}
         : L == 64   ? FastCfg{8, 4, 4, 4, 16}
         : L == 32   ? FastCfg{4, 4, 2, 4, 16}
                     : FastCfg{0, 0, 0, 0, 0};
}
// LDS complex slots of one sequence's exchange buffer on the fast path.
__host__ __device__ constexpr int fast_buf(int L) { return L + L / fast_cfg(L).R0 + 1; }

// Buffers of the transforms of one grouped launch: up to kGroupMax transforms
// of one shape and plan run as a single launch whose grid has one layer per
// transform (blockIdx.y selects it); a plain call is a group of one.  src is
// what the pass reads (input array or workspace), dst what it writes
// (workspace or output array; the same workspace for an in-place pass).
constexpr int kGroupMax = 16;
struct Io {
    const void *src[kGroupMax];
    void *dst[kGroupMax];
    int n;
};
inline Io io_one(const void *src, void *dst) {
    Io io{};
    io.src[0] = src;
    io.dst[0] = dst;
    io.n = 1;
    return io;
}
template <class T>
__device__ __forceinline__ const T *io_src(const Io &io) {
    return static_cast<const T *>(io.src[blockIdx.y]);
}
template <class T>
__device__ __forceinline__ T *io_dst(const Io &io) {
    return static_cast<T *>(io.dst[blockIdx.y]);
}

// Tables and launch geometry of a 2-D transform of an n1 x n2 array.
struct Plan2D {
    int n1, n2, m;            // m = n2 / 2 (packed half-spectrum width)
    dctx_norm norm;
    bool inverse;
    FftDesc row;              // length m complex FFT (rows)
    FftDesc col;              // length n1 complex FFT (columns)
    const float2 *split;      // exp(-2 pi j k / n2), k in [0, m]
    const float2 *ta;         // post/pre twiddle along n1 with scale folded, n1 entries
    const float2 *tb;         // post/pre twiddle along n2 with scale folded, m + 1 entries
    int rows_per_block;       // row pass: rows per workgroup
    int cols_per_block;       // column pass: packed columns per workgroup
    int fast;                 // 1: power-of-two fast path (row/col built from fast_cfg)
    int odd;                  // 1: n2 odd (generic path only): rows are length-n2 complex FFTs of the
                              //   real row, the workspace holds columns 0 .. m (m + 1 wide, m = (n2-1)/2)
    int nsub;                 // 0: 2-D; > 0: the n1 rows are the (a, b) rows of an
                              //   (n1/nsub) x nsub x n2 array (3-D, reordered on both axes)
    int xst;                  // inverse only: IDXST instead of IDCT along axis 0 (bit 0) / axis 1 (bit 1)
    int trans;                // 1 (generic kernels, even n2): the real input / output is stored transposed,
                              //   element (r, c) of the n1 x n2 array at c * n1 + r (the axis-order route)
    void *dev_mem;            // owning device allocation of all tables
};

// Width (complex columns) of the 2-D workspace: the packed half spectrum for
// even n2, columns 0 .. (n2-1)/2 for odd n2.
__host__ __device__ inline int ws_cols(const Plan2D &p) { return p.m + p.odd; }

// 3-D transform of an n1 x n2 x n3 array (n3 contiguous): the n3 pass runs the
// row kernels through a Plan2D with nsub = n2; the n2 and n1 passes use this.
struct Plan3D {
    int n1, n2, n3, m3;       // m3 = n3 / 2
    dctx_norm norm;
    bool inverse;
    FftDesc f2;               // length n2 complex FFT
    FftDesc f1;               // length n1 complex FFT
    const float2 *ta;         // axis-1 twiddle with scale folded, n1 entries
    const float2 *tb;         // axis-2 twiddle with scale folded, n2 entries
    const float2 *tc;         // axis-3 twiddle with scale folded, n3 entries
    int cols2;                // k3 columns per workgroup in the n2 pass
    int cols1;                // k3 columns per workgroup in the n1 pass (x2 sequences)
    int fast;                 // 1: n1, n2 powers of two in [64, 256], compile-time kernels
    FftDesc f2f;              // length n2, radices of fast3_radices(n2)
    FftDesc f1f;              // length n1, radices of fast3c_radices(n1)
    int odd;                  // 1: n3 odd (generic kernels): the workspace holds k3 = 0 .. m3,
                              //   m3 = (n3-1)/2, with column k3 = 0 alone (no packed n3/2 column)
    // Two-pass route (plane != 0): the n3 and n2 FFTs of an n1-plane run in one
    // workgroup (plane pass, run-time schedules), the n1 pass is the compile-time one.
    int plane;
    FftDesc f3;               // length m3 complex FFT of the n3 rows (run-time schedule)
    const float2 *split3;     // exp(-2 pi j k / n3), k in [0, m3]
    int plane_block;          // threads per workgroup of both plane kernels
    int plane_cw;             // forward plane pass: k3 columns per workgroup (divides m3)
    int plane_rw;             // inverse plane pass: n2 rows per workgroup (divides n2)
    // Compile-time two-pass route (fplane != 0, used when plane == 0): one
    // workgroup per n1-plane holds its packed half-spectrum plane in LDS
    // ((n2, m3) one of the shapes of fplane3_supported; 16-byte aligned arrays).
    int fplane;
    FftDesc f3f;              // length m3, radices of fplane3_radices(m3)
    FftDesc f2c;              // length n2, radices of fast3c_radices(n2) (the plane's n2 FFT)
    void *dev_mem;
};

// Width (complex columns along k3) of the 3-D workspace.
__host__ __device__ inline int ws3_cols(const Plan3D &p) { return p.m3 + p.odd; }

// Row-column baseline plan: 1-D N-point DCT along the last axis of a batch.
struct PlanRC1D {
    int n, m, batch;
    dctx_norm norm;
    bool inverse;
    int odd;                  // 1: n odd: a length-n complex FFT of the real row, spectrum k = 0 .. m,
                              //   m = (n-1)/2; 0: the length-m = n/2 complex FFT and the real-FFT split
    FftDesc fft;              // length m complex FFT (length n when odd)
    const float2 *split;      // exp(-2 pi j k / n), k in [0, m]
    const float2 *tw;         // exp(-j pi k / 2n) * scale (forward) or exp(+j pi k/2n) * scale (inverse), n entries
    int rows_per_block;
    void *dev_mem;
};

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error; they never synchronise.
hipError_t launch_dct2_rows(const Plan2D &p, const float *x, float2 *ws, hipStream_t s);
hipError_t launch_dct2_cols(const Plan2D &p, const float2 *ws, float *y, hipStream_t s);
hipError_t launch_idct2_cols(const Plan2D &p, const float *x, float2 *ws, hipStream_t s);
hipError_t launch_idct2_rows(const Plan2D &p, const float2 *ws, float *y, hipStream_t s);

hipError_t launch_dct3_mid(const Plan3D &p, float2 *ws, hipStream_t s);
hipError_t launch_dct3_cols(const Plan3D &p, const float2 *ws, float *y, hipStream_t s);
hipError_t launch_idct3_cols(const Plan3D &p, const float *x, float2 *ws, hipStream_t s);
// Plane passes of the two-pass 3-D route (forward: x -> spectrum after the n3
// and n2 FFTs; inverse: spectrum after the inverse n1 FFT -> y).
size_t plane_fwd_lds(const Plan3D &p);
size_t plane_inv_lds(const Plan3D &p);
hipError_t launch_plane3_fwd(const Plan3D &p, const Io &io, hipStream_t s);
hipError_t launch_plane3_inv(const Plan3D &p, const Io &io, hipStream_t s);
// Compile-time kernels of the 3-D n2 and n1 passes (power-of-two 64..256).
bool fplane3_supported(int n2, int m3);
size_t fplane3_lds(int n2, int m3);
int fplane3_radices(int m3, int *rad);
hipError_t launch_fplane3(const Plan3D &p, const Io &io, hipStream_t s);
bool fast3_supported(int n);
int fast3_radices(int n, int *rad);    // the n2 pass (and the plane pass's n2 FFT)
int fast3c_radices(int n, int *rad);   // the n1 pass
hipError_t launch_fast3_mid(const Plan3D &p, const Io &io, hipStream_t s);
hipError_t launch_fast3_cols(const Plan3D &p, const Io &io, hipStream_t s);
hipError_t launch_fast3_icols(const Plan3D &p, const Io &io, hipStream_t s);
inline hipError_t launch_fast3_mid(const Plan3D &p, float2 *ws, hipStream_t s) {
    return launch_fast3_mid(p, io_one(ws, ws), s);
}
inline hipError_t launch_fast3_cols(const Plan3D &p, const float2 *ws, float *y, hipStream_t s) {
    return launch_fast3_cols(p, io_one(ws, y), s);
}
inline hipError_t launch_fast3_icols(const Plan3D &p, const float *x, float2 *ws, hipStream_t s) {
    return launch_fast3_icols(p, io_one(x, ws), s);
}

// Fast path (power-of-two m and n1, 16-byte aligned real arrays).  The Io
// forms run a group of same-shape transforms as one launch.
bool fast_supported(int n1, int m);
bool fast_rows_supported(int m);
hipError_t launch_fast_dct2_rows(const Plan2D &p, const Io &io, hipStream_t s);
hipError_t launch_fast_dct2_cols(const Plan2D &p, const Io &io, hipStream_t s);
hipError_t launch_fast_idct2_cols(const Plan2D &p, const Io &io, hipStream_t s);
hipError_t launch_fast_idct2_rows(const Plan2D &p, const Io &io, hipStream_t s);
inline hipError_t launch_fast_dct2_rows(const Plan2D &p, const float *x, float2 *ws, hipStream_t s) {
    return launch_fast_dct2_rows(p, io_one(x, ws), s);
}
inline hipError_t launch_fast_dct2_cols(const Plan2D &p, const float2 *ws, float *y, hipStream_t s) {
    return launch_fast_dct2_cols(p, io_one(ws, y), s);
}
inline hipError_t launch_fast_idct2_cols(const Plan2D &p, const float *x, float2 *ws, hipStream_t s) {
    return launch_fast_idct2_cols(p, io_one(x, ws), s);
}
inline hipError_t launch_fast_idct2_rows(const Plan2D &p, const float2 *ws, float *y, hipStream_t s) {
    return launch_fast_idct2_rows(p, io_one(ws, y), s);
}

hipError_t launch_rc_pre(const PlanRC1D &p, const float *x, float *xr, hipStream_t s);
hipError_t launch_rc_rfft(const PlanRC1D &p, const float *xr, float2 *spec, hipStream_t s);
hipError_t launch_rc_post(const PlanRC1D &p, const float2 *spec, float *y, hipStream_t s);
hipError_t launch_rc_ipre(const PlanRC1D &p, const float *x, float2 *spec, hipStream_t s);
hipError_t launch_rc_irfft(const PlanRC1D &p, const float2 *spec, float *xr, hipStream_t s);
hipError_t launch_rc_ipost(const PlanRC1D &p, const float *xr, float *y, hipStream_t s);
hipError_t launch_transpose(const float *in, float *out, int rows, int cols, hipStream_t s);

// LDS bytes available to one workgroup on the current device.
size_t lds_budget_bytes();

}  // namespace dctx
