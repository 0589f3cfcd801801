// C ABI of the dctx library: argument checks, handle, plan cache, workspace,
// and the launch sequences of the plain transforms.  See include/dctx.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "dctx_internal.h"
#include "plan.h"

namespace dctx {
// Kernels the library launches, for the per-kernel timing records.
enum KernelId {
    K_DCT2_ROWS, K_DCT2_COLS, K_IDCT2_COLS, K_IDCT2_ROWS, K_RC_PRE, K_RC_RFFT, K_RC_POST,
    K_RC_IPRE, K_RC_IRFFT, K_RC_IPOST, K_TRANSPOSE, K_DCT3_ROWS, K_DCT3_MID, K_DCT3_COLS,
    K_IDCT3_COLS, K_IDCT3_MID, K_IDCT3_ROWS, K_COUNT
};
const char *const kKernelNames[K_COUNT] = {
    "dct2_rows", "dct2_cols", "idct2_cols", "idct2_rows", "rc_pre", "rc_rfft", "rc_post",
    "rc_ipre", "rc_irfft", "rc_ipost", "transpose", "dct3_rows", "dct3_mid", "dct3_cols",
    "idct3_cols", "idct3_mid", "idct3_rows"};
struct ProfRec {
    int kid;
    hipEvent_t a, b;
};
}  // namespace dctx

struct dctx_context {
    int device = 0;
    std::map<std::tuple<int, int, int, int, int>, dctx::Plan3D *> plans3d;
    std::map<std::tuple<int, int, int>, dctx::Plan2D *> plansrows;
    size_t lds_max = 65536;
    bool prof = false;
    std::vector<dctx::ProfRec> recs;
    std::vector<hipEvent_t> event_pool;
    std::map<std::tuple<int, int, int, int>, dctx::Plan2D *> plans2d;
    std::map<std::tuple<int, int, int, int>, dctx::PlanRC1D *> plansrc;
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

namespace dctx {

namespace {

thread_local size_t g_lds_budget = 65536;

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

dctx_status from_hip(hipError_t e) {
    if (e == hipSuccess) return DCTX_OK;
    if (e == hipErrorOutOfMemory) return DCTX_ERR_NOMEM;
    return DCTX_ERR_DEVICE;
}

// Upload a host table block into one device allocation.
dctx_status upload(const std::vector<float2> &host, void **dev) {
    *dev = nullptr;
    hipError_t e = hipMalloc(dev, host.size() * sizeof(float2));
    if (e != hipSuccess) return from_hip(e);
    e = hipMemcpy(*dev, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        return from_hip(e);
    }
    return DCTX_OK;
}

// Rows of one row-pass workgroup: LDS of `target` bytes, <= 1024 threads, and
// enough workgroups to cover the chip.
int pick_rows_per_block(int rows, int len, int T, size_t budget) {
    const size_t rowbytes = (size_t)lpad_len(len) * sizeof(float2);
    const size_t target = std::min<size_t>(budget, (size_t)env_int("DCTX_ROW_LDS", 64 * 1024));
    int r = (int)std::max<size_t>(1, target / rowbytes);
    r = std::min(r, std::max(1, kMaxBlock / T));
    r = std::min(r, std::max(1, rows / 512));
    if (len >= 1024) r = 1;
    const int forced = env_int("DCTX_ROWS_PER_BLOCK", 0);
    if (forced > 0) r = forced;
    return r;
}

int pick_cols_per_block(int cols, int len, int T, size_t budget) {
    const size_t colbytes = (size_t)lpad_len(len) * sizeof(float2);
    const size_t target = std::min<size_t>(budget, (size_t)env_int("DCTX_COL_LDS", 160 * 1024));
    int c = (int)std::max<size_t>(1, target / colbytes);
    c = std::min(c, std::max(1, kMaxBlock / T));
    c = std::min(c, 16);
    c = std::min(c, std::max(1, cols / 256));
    while (c & (c - 1)) c &= c - 1;   // power of two
    const int forced = env_int("DCTX_COLS_PER_BLOCK", 0);
    if (forced > 0) c = forced;
    return c;
}

bool fits_rows(int rpb, int len, int T, size_t budget) {
    return rpb * T <= kMaxBlock && (size_t)rpb * lpad_len(len) * sizeof(float2) <= budget;
}

bool fits_cols(int C, int len, int T, size_t budget) {
    return C * T <= kMaxBlock && (size_t)lpad_len(len) * C * sizeof(float2) <= budget;
}

dctx_status build_plan2d(dctx_context *h, int n1, int n2, dctx_norm norm, bool inverse, Plan2D **out) {
    auto key = std::make_tuple(n1, n2, (int)norm, (int)inverse);
    auto it = h->plans2d.find(key);
    if (it != h->plans2d.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<Plan2D> p(new Plan2D());
    std::memset(p.get(), 0, sizeof(Plan2D));
    p->n1 = n1;
    p->n2 = n2;
    p->m = n2 / 2;
    p->norm = norm;
    p->inverse = inverse;
    const int m = p->m;
    p->fast = fast_supported(n1, m) && env_int("DCTX_FAST", 1) != 0;
    if (p->fast) {
        if (!make_fast_schedule(m, p->row) || !make_fast_schedule(n1, p->col)) return DCTX_ERR_UNSUPPORTED;
    } else if (!make_schedule(m, p->row) || !make_schedule(n1, p->col)) {
        return DCTX_ERR_UNSUPPORTED;
    }
    p->rows_per_block = pick_rows_per_block(n1, m, p->row.T, h->lds_max);
    p->cols_per_block = pick_cols_per_block(m, n1, p->col.T, h->lds_max);
    if (!fits_rows(p->rows_per_block, m, p->row.T, h->lds_max) ||
        !fits_cols(p->cols_per_block, n1, p->col.T, h->lds_max))
        return DCTX_ERR_UNSUPPORTED;

    // table block: row twiddles | column twiddles | split | ta | tb (offsets kept even)
    auto even = [](size_t v) { return v + (v & 1); };
    const size_t o_row = 0, o_col = even(o_row + fft_twiddle_count(p->row)),
                 o_split = even(o_col + fft_twiddle_count(p->col)), o_ta = even(o_split + m + 1),
                 o_tb = even(o_ta + n1), total = even(o_tb + m + 1);
    std::vector<float2> host(total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p->row, &host[o_row]);
    fill_fft_twiddles(p->col, &host[o_col]);
    fill_split(n2, &host[o_split]);
    // forward: y = Re(b (a A + conj(a) B)) etc. with the post's factor 2 and the
    // 1/4 that turns 4 x raw into raw folded into b (extra = 2 / 4).
    fill_axis_twiddle(n1, n1, norm, inverse, 1.0, &host[o_ta]);
    fill_axis_twiddle(n2, m + 1, norm, inverse, inverse ? 1.0 : 0.5, &host[o_tb]);
    dctx_status st = upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    float2 *d = static_cast<float2 *>(p->dev_mem);
    p->row.tw = d + o_row;
    p->col.tw = d + o_col;
    p->split = d + o_split;
    p->ta = d + o_ta;
    p->tb = d + o_tb;
    *out = p.get();
    h->plans2d[key] = p.release();
    return DCTX_OK;
}

dctx_status ensure_ws(dctx_context *h, size_t bytes) {
    if (h->ws_bytes >= bytes) return DCTX_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return from_hip(e);
    if (h->ws) (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
    e = hipMalloc(&h->ws, bytes);
    if (e != hipSuccess) {
        h->ws = nullptr;
        return from_hip(e);
    }
    h->ws_bytes = bytes;
    return DCTX_OK;
}

hipEvent_t take_event(dctx_context *h) {
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch through `fn`, bracketed by an event pair when profiling is on.
template <class F>
hipError_t timed(dctx_context *h, int kid, hipStream_t s, F &&fn) {
    if (!h->prof) return fn();
    hipEvent_t a = take_event(h), b = take_event(h);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) {
        h->recs.push_back({kid, a, b});
    } else {
        h->event_pool.push_back(a);
        h->event_pool.push_back(b);
    }
    return e;
}

dctx_status check_2d(dctx_context *h, const float *x, float *y, int n1, int n2, dctx_norm norm) {
    if (!h || !x || !y) return DCTX_ERR_INVALID;
    if (n1 < 1 || n2 < 1) return DCTX_ERR_INVALID;
    if (norm != DCTX_NORM_BACKWARD && norm != DCTX_NORM_ORTHO) return DCTX_ERR_INVALID;
    const size_t bytes = (size_t)n1 * (size_t)n2 * sizeof(float);
    if (overlaps(x, bytes, y, bytes)) return DCTX_ERR_INVALID;
    if (!aligned8(x) || !aligned8(y)) return DCTX_ERR_INVALID;
    if (n1 < 2 || n2 < 4 || (n2 & 1) || !length_ok(n1) || !length_ok(n2)) return DCTX_ERR_UNSUPPORTED;
    return DCTX_OK;
}

size_t ws_bytes_2d(int n1, int n2) { return (size_t)n1 * (size_t)(n2 / 2) * sizeof(float2); }

dctx_status run_2d(dctx_context *h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                   bool inverse, void *ws, size_t ws_bytes, void *stream) {
    dctx_status st = check_2d(h, x, y, n1, n2, norm);
    if (st != DCTX_OK) return st;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    const size_t need = ws_bytes_2d(n1, n2);
    if (ws) {
        if (ws_bytes < need || !aligned8(ws)) return DCTX_ERR_INVALID;
        const size_t bytes = (size_t)n1 * n2 * sizeof(float);
        if (overlaps(ws, need, x, bytes) || overlaps(ws, need, y, bytes)) return DCTX_ERR_INVALID;
    }
    Plan2D *p = nullptr;
    st = build_plan2d(h, n1, n2, norm, inverse, &p);
    if (st != DCTX_OK) return st;
    if (!ws) {
        st = ensure_ws(h, need);
        if (st != DCTX_OK) return st;
        ws = h->ws;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    float2 *w = static_cast<float2 *>(ws);
    hipError_t e;
    // the fast kernels move the real arrays with 16-byte accesses
    const bool fast = p->fast && aligned16(x) && aligned16(y);
    if (!inverse) {
        e = timed(h, K_DCT2_ROWS, s, [&] {
            return fast ? launch_fast_dct2_rows(*p, x, w, s) : launch_dct2_rows(*p, x, w, s);
        });
        if (e == hipSuccess)
            e = timed(h, K_DCT2_COLS, s, [&] {
                return fast ? launch_fast_dct2_cols(*p, w, y, s) : launch_dct2_cols(*p, w, y, s);
            });
    } else {
        e = timed(h, K_IDCT2_COLS, s, [&] {
            return fast ? launch_fast_idct2_cols(*p, x, w, s) : launch_idct2_cols(*p, x, w, s);
        });
        if (e == hipSuccess)
            e = timed(h, K_IDCT2_ROWS, s, [&] {
                return fast ? launch_fast_idct2_rows(*p, w, y, s) : launch_idct2_rows(*p, w, y, s);
            });
    }
    return from_hip(e);
}

dctx_status build_planrc(dctx_context *h, int n, int batch, dctx_norm norm, bool inverse, PlanRC1D **out) {
    auto key = std::make_tuple(n, batch, (int)norm, (int)inverse);
    auto it = h->plansrc.find(key);
    if (it != h->plansrc.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<PlanRC1D> p(new PlanRC1D());
    std::memset(p.get(), 0, sizeof(PlanRC1D));
    p->n = n;
    p->m = n / 2;
    p->batch = batch;
    p->norm = norm;
    p->inverse = inverse;
    const int m = p->m;
    if (!make_schedule(m, p->fft)) return DCTX_ERR_UNSUPPORTED;
    p->rows_per_block = pick_rows_per_block(batch, m, p->fft.T, h->lds_max);
    if (!fits_rows(p->rows_per_block, m, p->fft.T, h->lds_max)) return DCTX_ERR_UNSUPPORTED;
    auto even = [](size_t v) { return v + (v & 1); };
    const size_t o_fft = 0, o_split = even(fft_twiddle_count(p->fft)), o_tw = even(o_split + m + 1),
                 total = even(o_tw + n);
    std::vector<float2> host(total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p->fft, &host[o_fft]);
    fill_split(n, &host[o_split]);
    // forward y(k) = 2 Re(e^{-j pi k/2n} X(k)) is 2 x raw: table = scale * e^{-j pi k/2n};
    // inverse: the unnormalised inverse real FFT returns 2 x raw DCT-III.
    fill_axis_twiddle(n, n, norm, inverse, 1.0, &host[o_tw]);
    dctx_status st = upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    float2 *d = static_cast<float2 *>(p->dev_mem);
    p->fft.tw = d + o_fft;
    p->split = d + o_split;
    p->tw = d + o_tw;
    *out = p.get();
    h->plansrc[key] = p.release();
    return DCTX_OK;
}

size_t ws_bytes_rc(int n1, int n2) {
    const size_t spec = std::max((size_t)n1 * (n2 / 2 + 1), (size_t)n2 * (n1 / 2 + 1));
    return 2 * (size_t)n1 * n2 * sizeof(float) + spec * sizeof(float2);
}

// Row-column 2-D transform: 1-D transform along rows, transpose, 1-D transform
// along the new rows, transpose back; every step a separate kernel.
dctx_status run_rc_2d(dctx_context *h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                      bool inverse, void *stream) {
    dctx_status st = check_2d(h, x, y, n1, n2, norm);
    if (st != DCTX_OK) return st;
    if ((n1 & 1) || n1 < 4) return DCTX_ERR_UNSUPPORTED;   // both axes run the real-FFT path
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    PlanRC1D *pa = nullptr, *pb = nullptr;
    st = build_planrc(h, n2, n1, norm, inverse, &pa);
    if (st != DCTX_OK) return st;
    st = build_planrc(h, n1, n2, norm, inverse, &pb);
    if (st != DCTX_OK) return st;
    st = ensure_ws(h, ws_bytes_rc(n1, n2));
    if (st != DCTX_OK) return st;
    float *A = static_cast<float *>(h->ws);
    float *B = A + (size_t)n1 * n2;
    float2 *S = reinterpret_cast<float2 *>(B + (size_t)n1 * n2);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
#define RC_STEP(KID, CALL) \
    if (e == hipSuccess) e = timed(h, KID, s, [&] { return CALL; })
    if (!inverse) {
        // x -pre-> A -rfft-> S -post-> B -T-> A -pre-> B -rfft-> S -post-> A -T-> y
        RC_STEP(K_RC_PRE, launch_rc_pre(*pa, x, A, s));
        RC_STEP(K_RC_RFFT, launch_rc_rfft(*pa, A, S, s));
        RC_STEP(K_RC_POST, launch_rc_post(*pa, S, B, s));
        RC_STEP(K_TRANSPOSE, launch_transpose(B, A, n1, n2, s));
        RC_STEP(K_RC_PRE, launch_rc_pre(*pb, A, B, s));
        RC_STEP(K_RC_RFFT, launch_rc_rfft(*pb, B, S, s));
        RC_STEP(K_RC_POST, launch_rc_post(*pb, S, A, s));
        RC_STEP(K_TRANSPOSE, launch_transpose(A, y, n2, n1, s));
    } else {
        // x -ipre-> S -irfft-> A -ipost-> B -T-> A -ipre-> S -irfft-> B -ipost-> A -T-> y
        RC_STEP(K_RC_IPRE, launch_rc_ipre(*pa, x, S, s));
        RC_STEP(K_RC_IRFFT, launch_rc_irfft(*pa, S, A, s));
        RC_STEP(K_RC_IPOST, launch_rc_ipost(*pa, A, B, s));
        RC_STEP(K_TRANSPOSE, launch_transpose(B, A, n1, n2, s));
        RC_STEP(K_RC_IPRE, launch_rc_ipre(*pb, A, S, s));
        RC_STEP(K_RC_IRFFT, launch_rc_irfft(*pb, S, B, s));
        RC_STEP(K_RC_IPOST, launch_rc_ipost(*pb, B, A, s));
        RC_STEP(K_TRANSPOSE, launch_transpose(A, y, n2, n1, s));
    }
#undef RC_STEP
    return from_hip(e);
}

// Row-pass plan for the n3 rows of a 3-D array: n1 * n2 rows of length n3,
// reordered on both outer axes (nsub = n2).  Only the row tables are built.
dctx_status build_rows_plan(dctx_context *h, int nrows, int nsub, int n3, Plan2D **out) {
    auto key = std::make_tuple(nrows, nsub, n3);
    auto it = h->plansrows.find(key);
    if (it != h->plansrows.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<Plan2D> p(new Plan2D());
    std::memset(p.get(), 0, sizeof(Plan2D));
    p->n1 = nrows;
    p->n2 = n3;
    p->m = n3 / 2;
    p->nsub = nsub;
    const int m = p->m;
    p->fast = fast_rows_supported(m) && env_int("DCTX_FAST", 1) != 0;
    if (p->fast ? !make_fast_schedule(m, p->row) : !make_schedule(m, p->row)) return DCTX_ERR_UNSUPPORTED;
    p->rows_per_block = pick_rows_per_block(nrows, m, p->row.T, h->lds_max);
    if (!fits_rows(p->rows_per_block, m, p->row.T, h->lds_max)) return DCTX_ERR_UNSUPPORTED;
    auto even = [](size_t v) { return v + (v & 1); };
    const size_t o_row = 0, o_split = even(fft_twiddle_count(p->row)), total = even(o_split + m + 1);
    std::vector<float2> host(total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p->row, &host[o_row]);
    fill_split(n3, &host[o_split]);
    dctx_status st = upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    float2 *d = static_cast<float2 *>(p->dev_mem);
    p->row.tw = d + o_row;
    p->split = d + o_split;
    *out = p.get();
    h->plansrows[key] = p.release();
    return DCTX_OK;
}

int pick_pow2_cols(int cols, int len, int threads_per_col, int seqs, size_t budget) {
    const size_t colbytes = (size_t)lpad_len(len) * sizeof(float2) * seqs;
    const size_t target = std::min<size_t>(budget, (size_t)env_int("DCTX_COL3_LDS", 80 * 1024));
    int c = (int)std::max<size_t>(1, target / colbytes);
    c = std::min(c, std::max(1, kMaxBlock / (threads_per_col * seqs)));
    c = std::min(c, std::max(1, cols));
    while (c & (c - 1)) c &= c - 1;
    return c;
}

dctx_status build_plan3d(dctx_context *h, int n1, int n2, int n3, dctx_norm norm, bool inverse, Plan3D **out) {
    auto key = std::make_tuple(n1, n2, n3, (int)norm, (int)inverse);
    auto it = h->plans3d.find(key);
    if (it != h->plans3d.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<Plan3D> p(new Plan3D());
    std::memset(p.get(), 0, sizeof(Plan3D));
    p->n1 = n1;
    p->n2 = n2;
    p->n3 = n3;
    p->m3 = n3 / 2;
    p->norm = norm;
    p->inverse = inverse;
    if (!make_schedule(n2, p->f2) || !make_schedule(n1, p->f1)) return DCTX_ERR_UNSUPPORTED;
    p->cols2 = pick_pow2_cols(p->m3, n2, p->f2.T, 1, h->lds_max);
    p->cols1 = pick_pow2_cols(p->m3, n1, p->f1.T, 2, h->lds_max);
    if (!fits_cols(p->cols2, n2, p->f2.T, h->lds_max) || !fits_cols(2 * p->cols1, n1, p->f1.T, h->lds_max))
        return DCTX_ERR_UNSUPPORTED;
    auto even = [](size_t v) { return v + (v & 1); };
    const size_t o_f2 = 0, o_f1 = even(fft_twiddle_count(p->f2)), o_ta = even(o_f1 + fft_twiddle_count(p->f1)),
                 o_tb = even(o_ta + n1), o_tc = even(o_tb + n2), total = even(o_tc + n3);
    std::vector<float2> host(total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p->f2, &host[o_f2]);
    fill_fft_twiddles(p->f1, &host[o_f1]);
    // forward: y = Re(tc S) is 1/8 of the three-stage 2 Re(...) (8 x raw): tc carries 2/8
    fill_axis_twiddle(n1, n1, norm, inverse, 1.0, &host[o_ta]);
    fill_axis_twiddle(n2, n2, norm, inverse, 1.0, &host[o_tb]);
    fill_axis_twiddle(n3, n3, norm, inverse, inverse ? 1.0 : 0.25, &host[o_tc]);
    dctx_status st = upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    float2 *d = static_cast<float2 *>(p->dev_mem);
    p->f2.tw = d + o_f2;
    p->f1.tw = d + o_f1;
    p->ta = d + o_ta;
    p->tb = d + o_tb;
    p->tc = d + o_tc;
    *out = p.get();
    h->plans3d[key] = p.release();
    return DCTX_OK;
}

size_t ws_bytes_3d(int n1, int n2, int n3) { return (size_t)n1 * n2 * (size_t)(n3 / 2) * sizeof(float2); }

dctx_status run_3d(dctx_context *h, const float *x, float *y, int n1, int n2, int n3, dctx_norm norm,
                   bool inverse, void *stream) {
    if (!h || !x || !y) return DCTX_ERR_INVALID;
    if (n1 < 1 || n2 < 1 || n3 < 1) return DCTX_ERR_INVALID;
    if (norm != DCTX_NORM_BACKWARD && norm != DCTX_NORM_ORTHO) return DCTX_ERR_INVALID;
    const size_t bytes = (size_t)n1 * n2 * (size_t)n3 * sizeof(float);
    if (overlaps(x, bytes, y, bytes)) return DCTX_ERR_INVALID;
    if (!aligned8(x) || !aligned8(y)) return DCTX_ERR_INVALID;
    if (n1 < 2 || n2 < 2 || n3 < 4 || (n3 & 1) || !length_ok(n1) || !length_ok(n2) || !length_ok(n3) ||
        n1 > 4096 || n2 > 8192 || (size_t)n1 * n2 > (size_t)1 << 26)
        return DCTX_ERR_UNSUPPORTED;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    Plan3D *p = nullptr;
    Plan2D *rp = nullptr;
    dctx_status st = build_plan3d(h, n1, n2, n3, norm, inverse, &p);
    if (st == DCTX_OK) st = build_rows_plan(h, n1 * n2, n2, n3, &rp);
    if (st == DCTX_OK) st = ensure_ws(h, ws_bytes_3d(n1, n2, n3));
    if (st != DCTX_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float2 *w = static_cast<float2 *>(h->ws);
    const bool fast = rp->fast && aligned16(x) && aligned16(y);
    hipError_t e;
    if (!inverse) {
        e = timed(h, K_DCT3_ROWS, s, [&] {
            return fast ? launch_fast_dct2_rows(*rp, x, w, s) : launch_dct2_rows(*rp, x, w, s);
        });
        if (e == hipSuccess) e = timed(h, K_DCT3_MID, s, [&] { return launch_dct3_mid(*p, w, s); });
        if (e == hipSuccess) e = timed(h, K_DCT3_COLS, s, [&] { return launch_dct3_cols(*p, w, y, s); });
    } else {
        e = timed(h, K_IDCT3_COLS, s, [&] { return launch_idct3_cols(*p, x, w, s); });
        if (e == hipSuccess) e = timed(h, K_IDCT3_MID, s, [&] { return launch_dct3_mid(*p, w, s); });
        if (e == hipSuccess)
            e = timed(h, K_IDCT3_ROWS, s, [&] {
                return fast ? launch_fast_idct2_rows(*rp, w, y, s) : launch_idct2_rows(*rp, w, y, s);
            });
    }
    return from_hip(e);
}

}  // namespace

size_t lds_budget_bytes() { return g_lds_budget; }

}  // namespace dctx

using namespace dctx;

extern "C" {

const char *dctx_status_string(dctx_status s) {
    switch (s) {
        case DCTX_OK: return "ok";
        case DCTX_ERR_INVALID: return "invalid argument";
        case DCTX_ERR_UNSUPPORTED: return "unsupported size or configuration";
        case DCTX_ERR_NOMEM: return "out of memory";
        case DCTX_ERR_DEVICE: return "HIP device error";
        case DCTX_ERR_BUSY: return "not complete";
    }
    return "unknown status";
}

int dctx_version(void) { return (0 << 16) | 1; }

dctx_status dctx_selfcheck(double *max_err) {
    const double pi = 3.14159265358979323846264338327950288;
    struct { float v; double ref; } checks[] = {
        {kSqrtHalf, std::cos(pi / 4)}, {kCos22_5, std::cos(pi / 8)}, {kSin22_5, std::sin(pi / 8)},
        {kSin60, std::sin(pi / 3)},    {kCos72, std::cos(2 * pi / 5)}, {kSin72, std::sin(2 * pi / 5)},
        {kCos144, std::cos(4 * pi / 5)}, {kSin144, std::sin(4 * pi / 5)},
    };
    double worst = 0.0;
    bool ok = true;
    for (auto &c : checks) {
        const double err = std::fabs((double)c.v - c.ref);
        worst = std::max(worst, err);
        // each constant must be the FP32 value nearest to the FP64 reference
        if ((float)c.ref != c.v) ok = false;
    }
    if (max_err) *max_err = worst;
    return ok ? DCTX_OK : DCTX_ERR_INVALID;
}

int dctx_length_supported(int n, int axis_last) {
    if (!length_ok(n)) return 0;
    if (axis_last) return (n >= 4 && (n % 2) == 0) ? 1 : 0;
    return n >= 2 ? 1 : 0;
}

dctx_status dctx_create(int device, dctx_handle *out) {
    if (!out) return DCTX_ERR_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return DCTX_ERR_DEVICE;
    if (device < 0 || device >= count) return DCTX_ERR_INVALID;
    if (hipSetDevice(device) != hipSuccess) return DCTX_ERR_DEVICE;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        return DCTX_ERR_DEVICE;
    dctx_context *h = new (std::nothrow) dctx_context();
    if (!h) return DCTX_ERR_NOMEM;
    h->device = device;
    h->lds_max = (size_t)lds;
    g_lds_budget = h->lds_max;
    *out = h;
    return DCTX_OK;
}

dctx_status dctx_destroy(dctx_handle h) {
    if (!h) return DCTX_ERR_INVALID;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : h->plans2d) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    for (auto &kv : h->plansrc) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    for (auto &kv : h->plans3d) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    for (auto &kv : h->plansrows) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    if (h->ws) (void)hipFree(h->ws);
    for (auto &r : h->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : h->event_pool) (void)hipEventDestroy(e);
    delete h;
    return DCTX_OK;
}

dctx_status dctx_workspace_bytes_2d(int n1, int n2, size_t *bytes) {
    if (!bytes || n1 < 1 || n2 < 1) return DCTX_ERR_INVALID;
    *bytes = ws_bytes_2d(n1, n2);
    return DCTX_OK;
}

dctx_status dctx_workspace_bytes_3d(int n1, int n2, int n3, size_t *bytes) {
    if (!bytes || n1 < 1 || n2 < 1 || n3 < 1) return DCTX_ERR_INVALID;
    *bytes = ws_bytes_3d(n1, n2, n3);
    return DCTX_OK;
}

dctx_status dctx_dct3d(dctx_handle h, const float *x, float *y, int n1, int n2, int n3, dctx_norm norm,
                       void *stream) {
    try {
        return run_3d(h, x, y, n1, n2, n3, norm, false, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_idct3d(dctx_handle h, const float *x, float *y, int n1, int n2, int n3, dctx_norm norm,
                        void *stream) {
    try {
        return run_3d(h, x, y, n1, n2, n3, norm, true, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_dct2d(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                       void *stream) {
    try {
        return run_2d(h, x, y, n1, n2, norm, false, nullptr, 0, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_idct2d(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                        void *stream) {
    try {
        return run_2d(h, x, y, n1, n2, norm, true, nullptr, 0, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_dct2d_ws(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                          void *workspace, size_t ws_bytes, void *stream) {
    if (!workspace) return DCTX_ERR_INVALID;
    try {
        return run_2d(h, x, y, n1, n2, norm, false, workspace, ws_bytes, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_idct2d_ws(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                           void *workspace, size_t ws_bytes, void *stream) {
    if (!workspace) return DCTX_ERR_INVALID;
    try {
        return run_2d(h, x, y, n1, n2, norm, true, workspace, ws_bytes, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_rc_dct2d(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                          void *stream) {
    try {
        return run_rc_2d(h, x, y, n1, n2, norm, false, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_rc_idct2d(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                           void *stream) {
    try {
        return run_rc_2d(h, x, y, n1, n2, norm, true, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_profile_enable(dctx_handle h, int enable) {
    if (!h) return DCTX_ERR_INVALID;
    h->prof = enable != 0;
    return DCTX_OK;
}

dctx_status dctx_profile_read(dctx_handle h, dctx_kernel_stat *stats, int capacity, int *count) {
    if (!h || !count || capacity < 0 || (capacity > 0 && !stats)) return DCTX_ERR_INVALID;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return DCTX_ERR_DEVICE;
    dctx_kernel_stat agg[K_COUNT];
    std::memset(agg, 0, sizeof(agg));
    dctx_status st = DCTX_OK;
    for (auto &r : h->recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) st = DCTX_ERR_DEVICE;
        dctx_kernel_stat &k = agg[r.kid];
        if (k.launches == 0 || ms < k.min_ms) k.min_ms = ms;
        if (ms > k.max_ms) k.max_ms = ms;
        k.launches += 1;
        k.total_ms += ms;
        h->event_pool.push_back(r.a);
        h->event_pool.push_back(r.b);
    }
    h->recs.clear();
    int n = 0;
    for (int i = 0; i < K_COUNT; ++i) {
        if (agg[i].launches == 0) continue;
        if (n < capacity) {
            stats[n] = agg[i];
            std::strncpy(stats[n].name, kKernelNames[i], sizeof(stats[n].name) - 1);
        }
        ++n;
    }
    *count = n;
    return st;
}

}  // extern "C"
