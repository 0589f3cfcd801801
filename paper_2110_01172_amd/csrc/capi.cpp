// C ABI of the dctx library: argument checks, handle, plan cache, workspace,
// and the launch sequences of the plain transforms.  See include/dctx.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "dctx_internal.h"
#include "batch.h"
#include "dct1d.h"
#include "poisson.h"
#include "small.h"
#include "split2d.h"
#include "plan.h"
#include "noalloc.h"

namespace dctx {
// Binding setters of the translation units (write-count build).
std::vector<hipError_t (*)(const WriteCountBinding &)> &wc_setters() {
    static std::vector<hipError_t (*)(const WriteCountBinding &)> v;
    return v;
}
void wc_register(hipError_t (*set)(const WriteCountBinding &)) { wc_setters().push_back(set); }
}  // namespace dctx

namespace dctx {
// Kernels the library launches, for the per-kernel timing records.
enum KernelId {
    K_DCT2_ROWS, K_DCT2_COLS, K_IDCT2_COLS, K_IDCT2_ROWS, K_RC_PRE, K_RC_RFFT, K_RC_POST,
    K_RC_IPRE, K_RC_IRFFT, K_RC_IPOST, K_TRANSPOSE, K_DCT3_ROWS, K_DCT3_MID, K_DCT3_COLS,
    K_IDCT3_COLS, K_IDCT3_MID, K_IDCT3_ROWS, K_POISSON_ROWS, K_POISSON_COLS, K_POISSON_IROWS,
    K_COMPRESS_ROWS, K_COMPRESS_COLS, K_COMPRESS_IROWS, K_DCT1D, K_IDCT1D,
    K_BATCH_DCT_ROWS, K_BATCH_DCT_COLS, K_BATCH_IDCT_COLS, K_BATCH_IDCT_ROWS, K_BATCH_POISSON_COLS, K_SMALL,
    K_DCT2_STEP8, K_IDCT2_STEP8, K_DCT3_PLANE, K_IDCT3_PLANE, K_COUNT
};
const char *const kKernelNames[K_COUNT] = {
    "dct2_rows", "dct2_cols", "idct2_cols", "idct2_rows", "rc_pre", "rc_rfft", "rc_post",
    "rc_ipre", "rc_irfft", "rc_ipost", "transpose", "dct3_rows", "dct3_mid", "dct3_cols",
    "idct3_cols", "idct3_mid", "idct3_rows", "poisson_rows", "poisson_cols", "poisson_irows",
    "compress_rows", "compress_cols", "compress_irows", "dct1d", "idct1d",
    "batch_dct_rows", "batch_dct_cols", "batch_idct_cols", "batch_idct_rows", "batch_poisson_cols", "small_mfma",
    "dct2_step8", "idct2_step8", "dct3_plane", "idct3_plane"};
struct ProfRec {
    int kid;
    hipEvent_t a, b;
};
}  // namespace dctx

struct dctx_context {
    int device = 0;
    std::map<std::tuple<int, int, int, int, int>, dctx::Plan3D *> plans3d;
    std::map<std::tuple<int, int, int>, dctx::Plan2D *> plansrows;
    std::map<std::tuple<int, int, double, double>, dctx::PlanPoisson *> planspoisson;
    std::map<std::tuple<int, int, int>, dctx::PlanPoisson *> planscompress;
    std::map<std::tuple<int, int, int>, dctx::Plan1D *> plans1d;
    // batched execution: device copies of plans, batch workspace, upload ring, tuning cache
    std::map<std::tuple<int, int, int>, std::pair<dctx::SmallTabs, void *>> planssmall;
    std::map<std::tuple<int, int, int, int>, dctx::PlanSplit *> planssplit;
    std::map<const void *, void *> dcopies;
    void *bws = nullptr;
    size_t bws_bytes = 0;
    struct Slot {
        void *host = nullptr;
        void *dev = nullptr;
        size_t bytes = 0;
        hipEvent_t done = nullptr;
        bool used = false;
    };
    Slot slots[16];
    int next_slot = 0;
    std::map<uint64_t, dctx::BatchTune> tune;
    int cus = 256;
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

// A caller may put any integer into an enum argument: read it as an int
// (loading an enum object whose value lies outside its enumeration is
// undefined behaviour).
template <class E>
int enum_value(const E &e) {
    static_assert(sizeof(E) == sizeof(int), "the C enums are int-sized");
    int v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}
bool norm_ok(dctx_norm n) {
    const int v = enum_value(n);
    return v == DCTX_NORM_BACKWARD || v == DCTX_NORM_ORTHO;
}

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

// Upload a host table block into the next free bytes of a table arena (no
// allocation).  kArenaFull when the arena has no room left: the caller
// synchronises the device, clears the arena and runs the call again.
dctx_status arena_upload(TableArena &a, const std::vector<float2> &host, void **dev) {
    *dev = nullptr;
    const size_t bytes = host.size() * sizeof(float2);
    const size_t span = (bytes + 255) & ~(size_t)255;
    if (a.used + span > a.cap) return kArenaFull;
    void *d = a.base + a.used;
    hipError_t e = hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return from_hip(e);
    a.used += span;
    *dev = d;
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

// Offsets (complex values) of a 2-D plan's tables in its FP32 image.
struct Tabs2D {
    size_t row, col, split, ta, tb, total;
};

void bind_plan2d(Plan2D &p, const Tabs2D &o, float2 *d) {
    p.row.tw = d + o.row;
    p.col.tw = d + o.col;
    p.split = d + o.split;
    p.ta = d + o.ta;
    p.tb = d + o.tb;
}

// Schedules, launch geometry and the FP64-built FP32 table image of a 2-D
// plan (table pointers left for bind_plan2d).
dctx_status image_plan2d(dctx_context *h, int n1, int n2, dctx_norm norm, bool inverse, Plan2D &p,
                         std::vector<float2> &host, Tabs2D &o) {
    std::memset(&p, 0, sizeof(Plan2D));
    p.n1 = n1;
    p.n2 = n2;
    p.m = n2 / 2;
    p.odd = n2 & 1;
    p.norm = norm;
    p.inverse = inverse;
    const int m = p.m;
    // odd n2: a full length-n2 complex row FFT on the generic path
    const int rowlen = p.odd ? n2 : m;
    p.fast = !p.odd && fast_supported(n1, m) && env_int("DCTX_FAST", 1) != 0;
    if (p.fast) {
        if (!make_fast_schedule(m, p.row) || !make_fast_schedule(n1, p.col)) return DCTX_ERR_UNSUPPORTED;
    } else if (!make_schedule(rowlen, p.row) || !make_schedule(n1, p.col)) {
        return DCTX_ERR_UNSUPPORTED;
    }
    p.rows_per_block = pick_rows_per_block(n1, rowlen, p.row.T, h->lds_max);
    p.cols_per_block = pick_cols_per_block(m + p.odd, n1, p.col.T, h->lds_max);
    if (!fits_rows(p.rows_per_block, rowlen, p.row.T, h->lds_max) ||
        !fits_cols(p.cols_per_block, n1, p.col.T, h->lds_max))
        return DCTX_ERR_UNSUPPORTED;

    // table block: row twiddles | column twiddles | split | ta | tb (offsets kept even)
    auto even = [](size_t v) { return v + (v & 1); };
    o.row = 0;
    o.col = even(o.row + fft_twiddle_count(p.row));
    o.split = even(o.col + fft_twiddle_count(p.col));
    o.ta = even(o.split + m + 1);
    o.tb = even(o.ta + n1);
    o.total = even(o.tb + m + 1);
    host.assign(o.total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p.row, &host[o.row]);
    fill_fft_twiddles(p.col, &host[o.col]);
    fill_split(n2, &host[o.split]);
    // forward: y = Re(b (a A + conj(a) B)) etc. with the post's factor 2 and the
    // 1/4 that turns 4 x raw into raw folded into b (extra = 2 / 4).
    fill_axis_twiddle(n1, n1, norm, inverse, 1.0, &host[o.ta]);
    fill_axis_twiddle(n2, m + 1, norm, inverse, inverse ? 1.0 : 0.5, &host[o.tb]);
    return DCTX_OK;
}

// ar (nullable): build the tables into a table arena and cache the plan there
// instead of in the handle.
dctx_status build_plan2d(dctx_context *h, int n1, int n2, dctx_norm norm, bool inverse, Plan2D **out,
                         TableArena *ar = nullptr) {
    auto key = std::make_tuple(n1, n2, (int)norm, (int)inverse);
    auto &cache = ar ? ar->p2d : h->plans2d;
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<Plan2D> p(new Plan2D());
    std::vector<float2> host;
    Tabs2D o{};
    dctx_status st = image_plan2d(h, n1, n2, norm, inverse, *p, host, o);
    if (st == DCTX_OK) st = ar ? arena_upload(*ar, host, &p->dev_mem) : upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    bind_plan2d(*p, o, static_cast<float2 *>(p->dev_mem));
    *out = p.get();
    cache[key] = p.release();
    return DCTX_OK;
}

// Offsets (complex values) of a split-column plan's tables in its image.
struct TabsSplit {
    size_t row, col, split, xtw, ta, tb, tl, total;
};

void bind_plan_split(PlanSplit &p, const TabsSplit &o, float2 *d) {
    p.row.tw = d + o.row;
    p.col.tw = d + o.col;
    p.split = d + o.split;
    p.xtw = d + o.xtw;
    p.ta = d + o.ta;
    p.tb = d + o.tb;
    p.tl = d + o.tl;
}

// Split-column plan (tall power-of-two arrays): row schedule with 8 values per
// thread, q-point column schedule, the cross twiddles W_n1^(qq kp), and the
// same split / post tables as the plain plan; image as image_plan2d.
dctx_status image_plan_split(int n1, int n2, dctx_norm norm, bool inverse, PlanSplit &p, std::vector<float2> &host,
                             TabsSplit &o) {
    const int m = n2 / 2;
    // long columns take the plain row kernels: no row schedule of this form
    const bool lng = !split_supported(n1, m) && split_long_supported(n1, m);
    if (!split_supported(n1, m) && !lng) return DCTX_ERR_UNSUPPORTED;
    std::memset(&p, 0, sizeof(PlanSplit));
    p.n1 = n1;
    p.n2 = n2;
    p.m = m;
    p.q = n1 / 8;
    p.norm = norm;
    p.inverse = inverse;
    // At m = 2048, q = 512 the row and column workgroups fill a CU's LDS
    // alone and every CU runs two of them: they become one workgroup that
    // loads the second's inputs while it computes the first.
    p.persist = (!lng && m == 2048 && p.q % 512 == 0 && env_int("DCTX_PERSIST", 1) != 0) ? 1 : 0;
    int rr[8], rc[8];
    const int nr = lng ? 0 : split_row_radices(m, rr), nc = split_col_radices(p.q, rc);
    if ((!lng && !make_schedule_radices(m, rr, nr, p.row)) || !make_schedule_radices(p.q, rc, nc, p.col))
        return DCTX_ERR_UNSUPPORTED;
    auto even = [](size_t v) { return v + (v & 1); };
    o.row = 0;
    o.col = even(o.row + fft_twiddle_count(p.row));
    o.split = even(o.col + fft_twiddle_count(p.col));
    o.xtw = even(o.split + m + 1);
    o.ta = even(o.xtw + n1);
    o.tb = even(o.ta + n1);
    o.tl = even(o.tb + m + 1);
    o.total = even(o.tl + 256);
    host.assign(o.total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p.row, &host[o.row]);
    fill_fft_twiddles(p.col, &host[o.col]);
    fill_split(n2, &host[o.split]);
    const double pi = 3.14159265358979323846264338327950288;
    // two-level tables: W_n^a and W_n^(64 b), a, b < 64, for n = n2 then n1
    for (int h2 = 0; h2 < 2; ++h2) {
        const int n = h2 == 0 ? n2 : n1;
        for (int a = 0; a < 64; ++a)
            for (int part = 0; part < 2; ++part) {
                const long long e = (part == 0 ? (long long)a : 64LL * a) % n;
                host[o.tl + (size_t)h2 * 128 + (size_t)part * 64 + a] =
                    make_float2((float)std::cos(2.0 * pi * e / n), (float)-std::sin(2.0 * pi * e / n));
            }
    }
    for (int qq = 0; qq < p.q; ++qq)
        for (int kp = 0; kp < 8; ++kp) {
            const long long r = (long long)qq * kp % n1;   // exp(-2 pi j qq kp / n1)
            host[o.xtw + (size_t)qq * 8 + kp] =
                make_float2((float)std::cos(2.0 * pi * r / n1), (float)-std::sin(2.0 * pi * r / n1));
        }
    fill_axis_twiddle(n1, n1, norm, inverse, 1.0, &host[o.ta]);
    fill_axis_twiddle(n2, m + 1, norm, inverse, inverse ? 1.0 : 0.5, &host[o.tb]);
    return DCTX_OK;
}

dctx_status build_plan_split(dctx_context *h, int n1, int n2, dctx_norm norm, bool inverse, PlanSplit **out,
                             TableArena *ar = nullptr) {
    auto key = std::make_tuple(n1, n2, (int)norm, (int)inverse);
    auto &cache = ar ? ar->ps : h->planssplit;
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<PlanSplit> p(new PlanSplit());
    std::vector<float2> host;
    TabsSplit o{};
    dctx_status st = image_plan_split(n1, n2, norm, inverse, *p, host, o);
    if (st == DCTX_OK) st = ar ? arena_upload(*ar, host, &p->dev_mem) : upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    bind_plan_split(*p, o, static_cast<float2 *>(p->dev_mem));
    *out = p.get();
    cache[key] = p.release();
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
    if (!norm_ok(norm)) return DCTX_ERR_INVALID;
    const size_t bytes = (size_t)n1 * (size_t)n2 * sizeof(float);
    if (overlaps(x, bytes, y, bytes)) return DCTX_ERR_INVALID;
    if (!aligned8(x) || !aligned8(y)) return DCTX_ERR_INVALID;
    // n2 even (packed half spectrum; n2 = 2 packs a length-1 row FFT) or odd
    // >= 3 (full-length row FFT)
    if (n1 < 2 || n2 < 2 || !length_ok(n1) || !length_ok(n2)) return DCTX_ERR_UNSUPPORTED;
    return DCTX_OK;
}

// Workspace columns: n2 / 2 (even n2, packed) or (n2 + 1) / 2 (odd n2).
size_t ws_bytes_plain_2d(int n1, int n2) { return (size_t)n1 * (size_t)((n2 + 1) / 2) * sizeof(float2); }

// Axis-order dispatch (Section "Results on 2D DCTs": the input and output of a
// 2-D transform can be transposed, folded into the pre- and postprocess).  A
// column longer than one workgroup holds (kEmax values x kMaxBlock threads) is
// run as a row: an n1 x n2 array with such an n1 (even) and n2 within the
// column limit is transformed as its n2 x n1 transpose, the transposes folded
// into the passes' loads and stores (Plan2D::trans): the row pass reads the
// columns of x, the column pass writes rows of y.
constexpr int kMaxCol = kEmax * kMaxBlock;
bool transposed_route(int n1, int n2) { return n1 > kMaxCol && !(n1 & 1) && n2 <= kMaxCol; }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of a plain 2-D call: the packed half spectrum (of the transposed
// problem on the axis-order route).
size_t ws_bytes_2d(int n1, int n2) {
    if (transposed_route(n1, n2)) return ws_bytes_plain_2d(n2, n1);
    return ws_bytes_plain_2d(n1, n2);
}

// Buffers of a group of same-shape transforms (see Io): input, output and
// workspace of each.
struct GroupBufs {
    const float *in[kGroupMax];
    float *out[kGroupMax];
    float2 *ws[kGroupMax];
    int n;
};

Io group_io(const GroupBufs &g, int pass) {
    Io io{};
    io.n = g.n;
    for (int i = 0; i < g.n; ++i) {
        // pass 0 reads the input and writes the workspace, pass 1 reads the
        // workspace and writes the output, pass 2 works in place on the workspace
        io.src[i] = pass == 0 ? static_cast<const void *>(g.in[i]) : g.ws[i];
        io.dst[i] = pass == 1 ? static_cast<void *>(g.out[i]) : g.ws[i];
    }
    return io;
}

// The two passes of a 2-D transform on the compile-time kernels (split form
// when ps is given, else the power-of-two fast form) for a group of same-shape
// transforms, one launch per pass.  A plain call is a group of one, so a
// transform gives bitwise the same result alone and in a group.
dctx_status enqueue_2d_group(dctx_context *h, const Plan2D &p, const PlanSplit *ps, bool inverse,
                             const GroupBufs &g, hipStream_t s) {
    const Io a = group_io(g, 0), b = group_io(g, 1);
    hipError_t e;
    if (!inverse) {
        e = timed(h, K_DCT2_ROWS, s, [&] {
            return ps ? launch_split_dct_rows(*ps, a, s) : launch_fast_dct2_rows(p, a, s);
        });
        if (e == hipSuccess)
            e = timed(h, K_DCT2_COLS, s, [&] {
                return ps ? launch_split_dct_cols(*ps, b, s) : launch_fast_dct2_cols(p, b, s);
            });
    } else {
        e = timed(h, K_IDCT2_COLS, s, [&] {
            return ps ? launch_split_idct_cols(*ps, a, s) : launch_fast_idct2_cols(p, a, s);
        });
        if (e == hipSuccess)
            e = timed(h, K_IDCT2_ROWS, s, [&] {
                return ps ? launch_split_idct_rows(*ps, b, s) : launch_fast_idct2_rows(p, b, s);
            });
    }
    return from_hip(e);
}

GroupBufs group_one(const float *x, float *y, float2 *w) {
    GroupBufs g{};
    g.in[0] = x;
    g.out[0] = y;
    g.ws[0] = w;
    g.n = 1;
    return g;
}

// xst (inverse only): IDXST instead of IDCT along axis 0 (bit 0) / axis 1 (bit 1).
// ar (nullable): plans come from this table arena (the allocation-free entry
// point; ws is then given).
dctx_status run_2d(dctx_context *h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                   bool inverse, void *ws, size_t ws_bytes, void *stream, int xst = 0,
                   TableArena *ar = nullptr) {
    dctx_status st = check_2d(h, x, y, n1, n2, norm);
    if (st != DCTX_OK) return st;
    if (xst && !inverse) return DCTX_ERR_INVALID;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    const size_t need = ws_bytes_2d(n1, n2);
    if (ws) {
        if (ws_bytes < need || !aligned16(ws)) return DCTX_ERR_INVALID;   // the kernels use 16-byte accesses
        const size_t bytes = (size_t)n1 * n2 * sizeof(float);
        if (overlaps(ws, need, x, bytes) || overlaps(ws, need, y, bytes)) return DCTX_ERR_INVALID;
    }
    if (transposed_route(n1, n2)) {
        // the n2 x n1 transpose on the run-time-schedule kernels (its rows are
        // longer than the compile-time kernels take), x and y read and written
        // transposed; the IDXST axes swap with the axes
        Plan2D *tp = nullptr;
        st = build_plan2d(h, n2, n1, norm, inverse, &tp, ar);
        if (st != DCTX_OK) return st;
        if (!ws) {
            st = ensure_ws(h, need);
            if (st != DCTX_OK) return st;
            ws = h->ws;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        float2 *w = static_cast<float2 *>(ws);
        Plan2D p = *tp;
        p.xst = ((xst & 1) << 1) | ((xst & 2) >> 1);
        p.trans = 1;
        hipError_t e;
        if (!inverse) {
            e = timed(h, K_DCT2_ROWS, s, [&] { return launch_dct2_rows(p, x, w, s); });
            if (e == hipSuccess) e = timed(h, K_DCT2_COLS, s, [&] { return launch_dct2_cols(p, w, y, s); });
        } else {
            e = timed(h, K_IDCT2_COLS, s, [&] { return launch_idct2_cols(p, x, w, s); });
            if (e == hipSuccess) e = timed(h, K_IDCT2_ROWS, s, [&] { return launch_idct2_rows(p, w, y, s); });
        }
        return from_hip(e);
    }
    Plan2D *pp = nullptr;
    st = build_plan2d(h, n1, n2, norm, inverse, &pp, ar);
    if (st != DCTX_OK) return st;
    if (!ws) {
        st = ensure_ws(h, need);
        if (st != DCTX_OK) return st;
        ws = h->ws;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    float2 *w = static_cast<float2 *>(ws);
    hipError_t e;
    // the kernels take their plan by value: the IDXST flags ride on a copy
    Plan2D p = *pp;
    p.xst = xst;
    // the fast kernels move the real arrays with 16-byte accesses
    const bool fast = p.fast && aligned16(x) && aligned16(y);
    PlanSplit *psp = nullptr;
    if (fast && !(n2 & 1) && split_supported(n1, n2 / 2) && env_int("DCTX_SPLIT", 1) != 0) {
        st = build_plan_split(h, n1, n2, norm, inverse, &psp, ar);
        if (st != DCTX_OK) return st;
    }
    if (psp) {
        PlanSplit ps = *psp;
        ps.xst = xst;
        return enqueue_2d_group(h, p, &ps, inverse, group_one(x, y, w), s);
    }
    // Long columns (n1 = 8192): the plain row pass, the radix-8 column step as
    // a pass of its own, and the split form's 1024-point column kernels, whose
    // tiles are 8 or 16 columns wide instead of the plain column kernel's 2.
    if (!(n2 & 1) && split_long_supported(n1, n2 / 2) && env_int("DCTX_SPLIT", 1) != 0) {
        st = build_plan_split(h, n1, n2, norm, inverse, &psp, ar);
        if (st != DCTX_OK) return st;
        PlanSplit ps = *psp;
        ps.xst = xst;
        if (!inverse) {
            e = timed(h, K_DCT2_ROWS, s, [&] {
                return fast ? launch_fast_dct2_rows(p, x, w, s) : launch_dct2_rows(p, x, w, s);
            });
            if (e == hipSuccess) e = timed(h, K_DCT2_STEP8, s, [&] { return launch_split_step8(ps, w, false, s); });
            if (e == hipSuccess) e = timed(h, K_DCT2_COLS, s, [&] { return launch_split_dct_cols(ps, w, y, s); });
        } else {
            e = timed(h, K_IDCT2_COLS, s, [&] { return launch_split_idct_cols(ps, x, w, s); });
            if (e == hipSuccess) e = timed(h, K_IDCT2_STEP8, s, [&] { return launch_split_step8(ps, w, true, s); });
            if (e == hipSuccess)
                e = timed(h, K_IDCT2_ROWS, s, [&] {
                    return fast ? launch_fast_idct2_rows(p, w, y, s) : launch_idct2_rows(p, w, y, s);
                });
        }
        return from_hip(e);
    }
    if (fast) return enqueue_2d_group(h, p, nullptr, inverse, group_one(x, y, w), s);
    if (!inverse) {
        e = timed(h, K_DCT2_ROWS, s, [&] { return launch_dct2_rows(p, x, w, s); });
        if (e == hipSuccess) e = timed(h, K_DCT2_COLS, s, [&] { return launch_dct2_cols(p, w, y, s); });
    } else {
        e = timed(h, K_IDCT2_COLS, s, [&] { return launch_idct2_cols(p, x, w, s); });
        if (e == hipSuccess) e = timed(h, K_IDCT2_ROWS, s, [&] { return launch_idct2_rows(p, w, y, s); });
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
    p->odd = n & 1;
    p->batch = batch;
    p->norm = norm;
    p->inverse = inverse;
    const int m = p->m;
    // odd n: a full length-n complex FFT of the real row (same unnormalised scale)
    const int len = p->odd ? n : m;
    if (!make_schedule(len, p->fft)) return DCTX_ERR_UNSUPPORTED;
    p->rows_per_block = pick_rows_per_block(batch, len, p->fft.T, h->lds_max);
    if (!fits_rows(p->rows_per_block, len, p->fft.T, h->lds_max)) return DCTX_ERR_UNSUPPORTED;
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
    if (n1 > 16384 || n2 > 16384) return DCTX_ERR_UNSUPPORTED;
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

// Schedule and launch geometry of the n3 row pass of a 3-D array (no tables).
dctx_status rows_plan_geometry(int nrows, int nsub, int n3, size_t lds_max, Plan2D &p) {
    std::memset(&p, 0, sizeof(Plan2D));
    p.n1 = nrows;
    p.n2 = n3;
    p.m = n3 / 2;
    p.odd = n3 & 1;
    p.nsub = nsub;
    const int m = p.m;
    // odd n3: a full length-n3 complex row FFT on the generic path
    const int rowlen = p.odd ? n3 : m;
    p.fast = !p.odd && fast_rows_supported(m) && env_int("DCTX_FAST", 1) != 0;
    if (p.fast ? !make_fast_schedule(m, p.row) : !make_schedule(rowlen, p.row)) return DCTX_ERR_UNSUPPORTED;
    p.rows_per_block = pick_rows_per_block(nrows, rowlen, p.row.T, lds_max);
    if (!fits_rows(p.rows_per_block, rowlen, p.row.T, lds_max)) return DCTX_ERR_UNSUPPORTED;
    return DCTX_OK;
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
    dctx_status st = rows_plan_geometry(nrows, nsub, n3, h->lds_max, *p);
    if (st != DCTX_OK) return st;
    const int m = p->m;
    auto even = [](size_t v) { return v + (v & 1); };
    const size_t o_row = 0, o_split = even(fft_twiddle_count(p->row)), total = even(o_split + m + 1);
    std::vector<float2> host(total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p->row, &host[o_row]);
    fill_split(n3, &host[o_split]);
    st = upload(host, &p->dev_mem);
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

// Schedules and launch geometry of the n2 and n1 passes of a 3-D transform
// (no tables).
dctx_status plan3d_geometry(int n1, int n2, int n3, dctx_norm norm, bool inverse, size_t lds_max, Plan3D &p) {
    std::memset(&p, 0, sizeof(Plan3D));
    p.n1 = n1;
    p.n2 = n2;
    p.n3 = n3;
    p.m3 = n3 / 2;
    p.odd = n3 & 1;
    p.norm = norm;
    p.inverse = inverse;
    if (!make_schedule(n2, p.f2) || !make_schedule(n1, p.f1)) return DCTX_ERR_UNSUPPORTED;
    p.cols2 = pick_pow2_cols(ws3_cols(p), n2, p.f2.T, 1, lds_max);
    p.cols1 = pick_pow2_cols(ws3_cols(p), n1, p.f1.T, 2, lds_max);
    if (!fits_cols(p.cols2, n2, p.f2.T, lds_max) || !fits_cols(2 * p.cols1, n1, p.f1.T, lds_max))
        return DCTX_ERR_UNSUPPORTED;
    // compile-time n2 / n1 kernels for powers of two in [64, 256] (packed k3 layout)
    p.fast = !p.odd && fast3_supported(n1) && fast3_supported(n2) && env_int("DCTX_FAST", 1) != 0;
    if (p.fast) {
        int r2[8], r1[8];
        const int c2 = fast3_radices(n2, r2), c1 = fast3c_radices(n1, r1);
        if (!make_schedule_radices(n2, r2, c2, p.f2f) || !make_schedule_radices(n1, r1, c1, p.f1f))
            return DCTX_ERR_UNSUPPORTED;
    }
    // Two-pass route (plane pass + compile-time n1 pass) for even n3 when an
    // n1-plane is at most 128 x 128 real values: the n3 and n2 FFTs of a plane
    // in one workgroup (16 B per element instead of 24).  Opt-in (DCTX_PLANE=1):
    // at 128^3 its plane pass (38-44 us) is slower than the row and n2 passes
    // it replaces (22 us), both being latency-bound at that size.
    // Compile-time two-pass route: one workgroup per n1-plane for the small
    // power-of-two planes (DCTX_FPLANE=0 selects the three-pass route).
    p.fplane = 0;
    if (p.fast && !p.odd && fplane3_supported(n2, p.m3) && fplane3_lds(n2, p.m3) <= lds_max &&
        env_int("DCTX_FPLANE", 1) != 0) {
        int r3[8], r2[8];
        const int c3 = fplane3_radices(p.m3, r3), c2 = fast3c_radices(n2, r2);
        if (!make_schedule_radices(p.m3, r3, c3, p.f3f) || !make_schedule_radices(n2, r2, c2, p.f2c))
            return DCTX_ERR_UNSUPPORTED;
        p.fplane = 1;
    }
    p.plane = 0;
    if (p.fast && !p.odd && (size_t)n2 * n3 <= (size_t)128 * 128 && env_int("DCTX_PLANE", 0) != 0 &&
        make_schedule(p.m3, p.f3)) {
        // tiles: the largest divisor of m3 up to 16 k3 columns, of n2 up to 32 rows
        auto divisor_upto = [](int n, int cap) {
            int d = std::min(n, cap);
            while (n % d) --d;
            return d;
        };
        p.plane_block = env_int("DCTX_PLANE_BLOCK", 256);
        p.plane_cw = env_int("DCTX_PLANE_CW", divisor_upto(p.m3, 16));
        p.plane_rw = env_int("DCTX_PLANE_RW", divisor_upto(n2, 32));
        const int B = p.plane_block, cw = p.plane_cw, rw = p.plane_rw;
        p.plane = B >= 64 && B <= kMaxBlock && B % 64 == 0 && cw >= 1 && p.m3 % cw == 0 && rw >= 1 &&
                  n2 % rw == 0 && cw * p.f2.T <= B && p.f3.T <= B && p.f2.T <= B && cw <= kEmax * p.f3.T &&
                  plane_fwd_lds(p) <= lds_max && plane_inv_lds(p) <= lds_max;
    }
    return DCTX_OK;
}

dctx_status build_plan3d(dctx_context *h, int n1, int n2, int n3, dctx_norm norm, bool inverse, Plan3D **out) {
    auto key = std::make_tuple(n1, n2, n3, (int)norm, (int)inverse);
    auto it = h->plans3d.find(key);
    if (it != h->plans3d.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<Plan3D> p(new Plan3D());
    dctx_status st = plan3d_geometry(n1, n2, n3, norm, inverse, h->lds_max, *p);
    if (st != DCTX_OK) return st;
    auto even = [](size_t v) { return v + (v & 1); };
    const size_t o_f2 = 0, o_f1 = even(fft_twiddle_count(p->f2)), o_ta = even(o_f1 + fft_twiddle_count(p->f1)),
                 o_tb = even(o_ta + n1), o_tc = even(o_tb + n2), o_f2f = even(o_tc + n3),
                 o_f1f = even(o_f2f + (p->fast ? fft_twiddle_count(p->f2f) : 0)),
                 o_f3 = even(o_f1f + (p->fast ? fft_twiddle_count(p->f1f) : 0)),
                 o_f3f = even(o_f3 + (p->plane ? fft_twiddle_count(p->f3) : 0)),
                 o_f2c = even(o_f3f + (p->fplane ? fft_twiddle_count(p->f3f) : 0)),
                 o_s3 = even(o_f2c + (p->fplane ? fft_twiddle_count(p->f2c) : 0)),
                 total = even(o_s3 + (p->plane || p->fplane ? p->m3 + 1 : 0));
    std::vector<float2> host(total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p->f2, &host[o_f2]);
    fill_fft_twiddles(p->f1, &host[o_f1]);
    if (p->fast) {
        fill_fft_twiddles(p->f2f, &host[o_f2f]);
        fill_fft_twiddles(p->f1f, &host[o_f1f]);
    }
    if (p->plane) fill_fft_twiddles(p->f3, &host[o_f3]);
    if (p->fplane) {
        fill_fft_twiddles(p->f3f, &host[o_f3f]);
        fill_fft_twiddles(p->f2c, &host[o_f2c]);
    }
    if (p->plane || p->fplane) fill_split(n3, &host[o_s3]);
    // forward: y = Re(tc S) is 1/8 of the three-stage 2 Re(...) (8 x raw): tc carries 2/8
    fill_axis_twiddle(n1, n1, norm, inverse, 1.0, &host[o_ta]);
    fill_axis_twiddle(n2, n2, norm, inverse, 1.0, &host[o_tb]);
    fill_axis_twiddle(n3, n3, norm, inverse, inverse ? 1.0 : 0.25, &host[o_tc]);
    st = upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    float2 *d = static_cast<float2 *>(p->dev_mem);
    p->f2.tw = d + o_f2;
    p->f1.tw = d + o_f1;
    p->ta = d + o_ta;
    p->tb = d + o_tb;
    p->tc = d + o_tc;
    if (p->fast) {
        p->f2f.tw = d + o_f2f;
        p->f1f.tw = d + o_f1f;
    }
    if (p->plane) p->f3.tw = d + o_f3;
    if (p->fplane) {
        p->f3f.tw = d + o_f3f;
        p->f2c.tw = d + o_f2c;
    }
    if (p->plane || p->fplane) p->split3 = d + o_s3;
    *out = p.get();
    h->plans3d[key] = p.release();
    return DCTX_OK;
}

// Workspace: k3 = 0 .. n3/2 - 1 (even n3, packed) or 0 .. (n3-1)/2 (odd n3).
size_t ws_bytes_3d(int n1, int n2, int n3) { return (size_t)n1 * n2 * (size_t)((n3 + 1) / 2) * sizeof(float2); }

dctx_status enqueue_3d(dctx_context *h, const Plan3D &P, const Plan2D &RP, const float *x, float *y, bool inverse,
                       float2 *w, hipStream_t s);

// Shape rules of the 3-D transforms (beyond null / alias / alignment checks).
dctx_status check_3d_shape(int n1, int n2, int n3) {
    if (n1 < 2 || n2 < 2 || n3 < 2 || !length_ok(n1) || !length_ok(n2) || !length_ok(n3) ||
        n1 > 4096 || n2 > 8192 || (size_t)n1 * n2 > (size_t)1 << 26)
        return DCTX_ERR_UNSUPPORTED;
    return DCTX_OK;
}

dctx_status run_3d(dctx_context *h, const float *x, float *y, int n1, int n2, int n3, dctx_norm norm,
                   bool inverse, void *stream, void *ws = nullptr) {
    if (!h || !x || !y) return DCTX_ERR_INVALID;
    if (n1 < 1 || n2 < 1 || n3 < 1) return DCTX_ERR_INVALID;
    if (!norm_ok(norm)) return DCTX_ERR_INVALID;
    const size_t bytes = (size_t)n1 * n2 * (size_t)n3 * sizeof(float);
    if (overlaps(x, bytes, y, bytes)) return DCTX_ERR_INVALID;
    if (!aligned8(x) || !aligned8(y)) return DCTX_ERR_INVALID;
    if (check_3d_shape(n1, n2, n3) != DCTX_OK) return DCTX_ERR_UNSUPPORTED;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    Plan3D *p = nullptr;
    Plan2D *rp = nullptr;
    dctx_status st = build_plan3d(h, n1, n2, n3, norm, inverse, &p);
    if (st == DCTX_OK) st = build_rows_plan(h, n1 * n2, n2, n3, &rp);
    if (st == DCTX_OK && !ws) st = ensure_ws(h, ws_bytes_3d(n1, n2, n3));
    if (st != DCTX_OK) return st;
    return enqueue_3d(h, *p, *rp, x, y, inverse, static_cast<float2 *>(ws ? ws : h->ws),
                      static_cast<hipStream_t>(stream));
}

// The three passes of a 3-D transform on the compile-time kernels (row
// kernels of the fast form, n2 / n1 kernels of the 3-D fast form) for a group
// of same-shape transforms, one launch per pass; the plain call on those
// kernels is a group of one.
dctx_status enqueue_3d_group(dctx_context *h, const Plan3D &P, const Plan2D &RP, bool inverse, const GroupBufs &g,
                             hipStream_t s) {
    const Io a = group_io(g, 0), b = group_io(g, 1), mid = group_io(g, 2);
    hipError_t e;
    if (P.plane) {
        // two passes: the plane pass (n3 and n2 FFTs) and the n1 pass
        if (!inverse) {
            e = timed(h, K_DCT3_PLANE, s, [&] { return launch_plane3_fwd(P, a, s); });
            if (e == hipSuccess) e = timed(h, K_DCT3_COLS, s, [&] { return launch_fast3_cols(P, b, s); });
        } else {
            e = timed(h, K_IDCT3_COLS, s, [&] { return launch_fast3_icols(P, a, s); });
            if (e == hipSuccess) e = timed(h, K_IDCT3_PLANE, s, [&] { return launch_plane3_inv(P, b, s); });
        }
        return from_hip(e);
    }
    if (P.fplane) {
        // two passes: the compile-time plane pass and the n1 pass
        if (!inverse) {
            e = timed(h, K_DCT3_PLANE, s, [&] { return launch_fplane3(P, a, s); });
            if (e == hipSuccess) e = timed(h, K_DCT3_COLS, s, [&] { return launch_fast3_cols(P, b, s); });
        } else {
            e = timed(h, K_IDCT3_COLS, s, [&] { return launch_fast3_icols(P, a, s); });
            if (e == hipSuccess) e = timed(h, K_IDCT3_PLANE, s, [&] { return launch_fplane3(P, b, s); });
        }
        return from_hip(e);
    }
    if (!inverse) {
        e = timed(h, K_DCT3_ROWS, s, [&] { return launch_fast_dct2_rows(RP, a, s); });
        if (e == hipSuccess) e = timed(h, K_DCT3_MID, s, [&] { return launch_fast3_mid(P, mid, s); });
        if (e == hipSuccess) e = timed(h, K_DCT3_COLS, s, [&] { return launch_fast3_cols(P, b, s); });
    } else {
        e = timed(h, K_IDCT3_COLS, s, [&] { return launch_fast3_icols(P, a, s); });
        if (e == hipSuccess) e = timed(h, K_IDCT3_MID, s, [&] { return launch_fast3_mid(P, mid, s); });
        if (e == hipSuccess) e = timed(h, K_IDCT3_ROWS, s, [&] { return launch_fast_idct2_rows(RP, b, s); });
    }
    return from_hip(e);
}

dctx_status enqueue_3d(dctx_context *h, const Plan3D &P, const Plan2D &RP, const float *x, float *y, bool inverse,
                       float2 *w, hipStream_t s) {
    const Plan3D *p = &P;
    const Plan2D *rp = &RP;
    const bool fast = rp->fast && aligned16(x) && aligned16(y);
    // the plane route (p->plane) and the n1-pass kernels need 8-byte alignment only
    if (p->plane || (fast && p->fast)) return enqueue_3d_group(h, P, RP, inverse, group_one(x, y, w), s);
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

// Plan of the fused spectral column pass: the forward and inverse 2-D plans of
// `norm` (and their split forms for tall power-of-two shapes), the inverse pre
// tables, and the per-axis terms lam (n1 then n2 entries, FP64-built, rounded
// once) on the device.
dctx_status build_plan_spectral(dctx_context *h, int n1, int n2, dctx_norm norm, const std::vector<double> &lam,
                                std::unique_ptr<PlanPoisson> &p) {
    p.reset(new PlanPoisson());
    std::memset(p.get(), 0, sizeof(PlanPoisson));
    dctx_status st = build_plan2d(h, n1, n2, norm, false, &p->fwd);
    if (st == DCTX_OK) st = build_plan2d(h, n1, n2, norm, true, &p->inv);
    if (st != DCTX_OK) return st;
    std::vector<float> lf(lam.size() + 1, 0.f);
    for (size_t i = 0; i < lam.size(); ++i) lf[i] = (float)lam[i];
    std::vector<float2> host((lf.size() + 1) / 2, make_float2(0.f, 0.f));
    std::memcpy(host.data(), lf.data(), lf.size() * sizeof(float));
    st = upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    const float *d = static_cast<const float *>(p->dev_mem);
    p->q.tai = p->inv->ta;
    p->q.tbi = p->inv->tb;
    p->q.l1 = d;
    p->q.l2 = d + n1;
    if (p->fwd->fast && split_supported(n1, n2 / 2) && env_int("DCTX_SPLIT", 1) != 0) {
        st = build_plan_split(h, n1, n2, norm, false, &p->fwds);
        if (st == DCTX_OK) st = build_plan_split(h, n1, n2, norm, true, &p->invs);
        if (st != DCTX_OK) return st;
        p->qs = p->q;
        p->qs.tai = p->invs->ta;
        p->qs.tbi = p->invs->tb;
    }
    return DCTX_OK;
}

// Poisson plan: backward norm, the Neumann eigenvalue terms
// (2 cos(pi k / n) - 2) / h^2 along each axis.
dctx_status build_plan_poisson(dctx_context *h, int n1, int n2, double h1, double h2, PlanPoisson **out) {
    auto key = std::make_tuple(n1, n2, h1, h2);
    auto it = h->planspoisson.find(key);
    if (it != h->planspoisson.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    const double pi = 3.14159265358979323846264338327950288;
    std::vector<double> lam((size_t)n1 + n2, 0.0);
    for (int k = 0; k < n1; ++k) lam[k] = (2.0 * std::cos(pi * k / n1) - 2.0) / (h1 * h1);
    for (int k = 0; k < n2; ++k) lam[(size_t)n1 + k] = (2.0 * std::cos(pi * k / n2) - 2.0) / (h2 * h2);
    std::unique_ptr<PlanPoisson> p;
    dctx_status st = build_plan_spectral(h, n1, n2, DCTX_NORM_BACKWARD, lam, p);
    if (st != DCTX_OK) return st;
    p->q.mode = p->qs.mode = 0;
    *out = p.get();
    h->planspoisson[key] = p.release();
    return DCTX_OK;
}

// Compression plan: the plans of the caller's norm; the per-axis terms are
// zeros (read, unused).
dctx_status build_plan_compress(dctx_context *h, int n1, int n2, dctx_norm norm, PlanPoisson **out) {
    auto key = std::make_tuple(n1, n2, (int)norm);
    auto it = h->planscompress.find(key);
    if (it != h->planscompress.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<PlanPoisson> p;
    dctx_status st = build_plan_spectral(h, n1, n2, norm, std::vector<double>((size_t)n1 + n2, 0.0), p);
    if (st != DCTX_OK) return st;
    p->q.mode = p->qs.mode = 1;
    *out = p.get();
    h->planscompress[key] = p.release();
    return DCTX_OK;
}

// The three passes of a fused spectral solve: the DCT row pass into the packed
// half spectrum, the fused column pass with the step of `q`, the IDCT row pass.
// The three passes of a group of same-shape fused spectral solves on the
// compile-time row kernels (split form where the plan has it), one launch per
// pass; the plain call on those kernels is a group of one.
dctx_status enqueue_spectral_group(dctx_context *h, const PlanPoisson &p, const PoissonTabs &q, const PoissonTabs &qs,
                                   const GroupBufs &g, hipStream_t s, const KernelId (&kid)[3]) {
    const Io a = group_io(g, 0), b = group_io(g, 1), mid = group_io(g, 2);
    hipError_t e;
    if (p.fwds) {
        e = timed(h, kid[0], s, [&] { return launch_split_dct_rows(*p.fwds, a, s); });
        if (e == hipSuccess) e = timed(h, kid[1], s, [&] { return launch_split_poisson_cols(*p.fwds, qs, mid, s); });
        if (e == hipSuccess) e = timed(h, kid[2], s, [&] { return launch_split_idct_rows(*p.invs, b, s); });
    } else {
        e = timed(h, kid[0], s, [&] { return launch_fast_dct2_rows(*p.fwd, a, s); });
        if (e == hipSuccess) e = timed(h, kid[1], s, [&] { return launch_poisson_cols(*p.fwd, q, mid, s); });
        if (e == hipSuccess) e = timed(h, kid[2], s, [&] { return launch_fast_idct2_rows(*p.inv, b, s); });
    }
    return from_hip(e);
}

dctx_status run_spectral(dctx_context *h, const PlanPoisson &p, PoissonTabs q, PoissonTabs qs, const float *f,
                         float *u, int n1, int n2, hipStream_t s, void *ws, const KernelId (&kid)[3]) {
    dctx_status st = ws ? DCTX_OK : ensure_ws(h, ws_bytes_2d(n1, n2));
    if (st != DCTX_OK) return st;
    float2 *w = static_cast<float2 *>(ws ? ws : h->ws);
    const bool fast = p.fwd->fast && aligned16(f) && aligned16(u);
    if (fast) return enqueue_spectral_group(h, p, q, qs, group_one(f, u, w), s, kid);
    hipError_t e = timed(h, kid[0], s, [&] { return launch_dct2_rows(*p.fwd, f, w, s); });
    if (e == hipSuccess) e = timed(h, kid[1], s, [&] { return launch_poisson_cols(*p.fwd, q, w, s); });
    if (e == hipSuccess) e = timed(h, kid[2], s, [&] { return launch_idct2_rows(*p.inv, w, u, s); });
    return from_hip(e);
}

dctx_status run_poisson(dctx_context *h, const float *f, float *u, int n1, int n2, double h1, double h2,
                        void *stream, void *ws = nullptr) {
    dctx_status st = check_2d(h, f, u, n1, n2, DCTX_NORM_BACKWARD);
    if (st != DCTX_OK) return st;
    if (!(h1 == h1) || !(h2 == h2) || std::isinf(h1) || std::isinf(h2)) return DCTX_ERR_INVALID;
    if (h1 <= 0.0) h1 = 1.0 / n1;
    if (h2 <= 0.0) h2 = 1.0 / n2;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    PlanPoisson *p = nullptr;
    st = build_plan_poisson(h, n1, n2, h1, h2, &p);
    if (st != DCTX_OK) return st;
    static const KernelId kid[3] = {K_POISSON_ROWS, K_POISSON_COLS, K_POISSON_IROWS};
    return run_spectral(h, *p, p->q, p->qs, f, u, n1, n2, static_cast<hipStream_t>(stream), ws, kid);
}

dctx_status run_compress(dctx_context *h, const float *x, float *y, int n1, int n2, dctx_norm norm, double eps,
                         void *stream) {
    dctx_status st = check_2d(h, x, y, n1, n2, norm);
    if (st != DCTX_OK) return st;
    if (!(eps == eps) || std::isinf(eps) || eps < 0.0) return DCTX_ERR_INVALID;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    PlanPoisson *p = nullptr;
    st = build_plan_compress(h, n1, n2, norm, &p);
    if (st != DCTX_OK) return st;
    PoissonTabs q = p->q, qs = p->qs;
    q.eps = qs.eps = (float)eps;
    static const KernelId kid[3] = {K_COMPRESS_ROWS, K_COMPRESS_COLS, K_COMPRESS_IROWS};
    return run_spectral(h, *p, q, qs, x, y, n1, n2, static_cast<hipStream_t>(stream), nullptr, kid);
}


// --------------------------------------------------------------- 1-D rows
// Plan of the batched 1-D transform of length n (even, 5-smooth, <= kMax1d):
// the length-m row schedule, the split twiddles and the post / pre twiddles
// with the norm's scale folded in (FP64-built).
dctx_status build_plan1d(dctx_context *h, int n, dctx_norm norm, bool inverse, Plan1D **out) {
    auto key = std::make_tuple(n, (int)norm, (int)inverse);
    auto it = h->plans1d.find(key);
    if (it != h->plans1d.end()) {
        *out = it->second;
        return DCTX_OK;
    }
    std::unique_ptr<Plan1D> p(new Plan1D());
    std::memset(p.get(), 0, sizeof(Plan1D));
    p->n = n;
    p->m = n / 2;
    p->norm = norm;
    p->inverse = inverse;
    const int m = p->m;
    if (n > kMax1d) {
        // four-step route: m = m1 m2 with m1 the smallest divisor >= sqrt(m)
        // (both factors within one workgroup's FFT)
        int m1 = 0;
        for (int d = (int)std::ceil(std::sqrt((double)m)); d <= m && !m1; ++d)
            if (m % d == 0 && m / d <= kEmax * kMaxBlock && d <= kEmax * kMaxBlock) m1 = d;
        if (!m1) return DCTX_ERR_UNSUPPORTED;
        p->m1 = m1;
        p->m2 = m / m1;
        if (!make_schedule(p->m1, p->f1) || !make_schedule(p->m2, p->f2) || p->f1.T > kMaxBlock ||
            2 * p->f2.T > kMaxBlock)
            return DCTX_ERR_UNSUPPORTED;
        // columns per workgroup: up to 16 (128-byte segments of the workspace
        // rows), within 512 threads and the LDS
        int C = 16;
        while (C > 1 && (C * p->f1.T > kMaxBlock || (size_t)lpad_len(p->m1) * C * sizeof(float2) > h->lds_max))
            C /= 2;
        p->cols_c = C;
        if ((size_t)lpad_len(p->m1) * C * sizeof(float2) > h->lds_max ||
            2 * (size_t)lpad_len(p->m2) * sizeof(float2) > h->lds_max)
            return DCTX_ERR_UNSUPPORTED;
        auto even = [](size_t v) { return v + (v & 1); };
        const size_t o_f1 = 0, o_f2 = even(fft_twiddle_count(p->f1)), o_split = even(o_f2 + fft_twiddle_count(p->f2)),
                     o_tw = even(o_split + m + 1), o_roots = even(o_tw + m + 1), total = even(o_roots + m);
        std::vector<float2> host(total, make_float2(0.f, 0.f));
        fill_fft_twiddles(p->f1, &host[o_f1]);
        fill_fft_twiddles(p->f2, &host[o_f2]);
        fill_split(n, &host[o_split]);
        fill_axis_twiddle(n, m + 1, norm, inverse, 1.0, &host[o_tw]);
        fill_roots(m, &host[o_roots]);
        dctx_status st = upload(host, &p->dev_mem);
        if (st != DCTX_OK) return st;
        float2 *d = static_cast<float2 *>(p->dev_mem);
        p->f1.tw = d + o_f1;
        p->f2.tw = d + o_f2;
        p->split = d + o_split;
        p->tw = d + o_tw;
        p->roots = d + o_roots;
        *out = p.get();
        h->plans1d[key] = p.release();
        return DCTX_OK;
    }
    p->fast = (m >= 32 && m <= 2048 && (m & (m - 1)) == 0 && env_int("DCTX_FAST", 1) != 0) ? 1 : 0;
    const bool sched = p->fast ? make_fast_schedule(m, p->row) : make_schedule(m, p->row);
    if (!sched || p->row.T > kMaxBlock) return DCTX_ERR_UNSUPPORTED;
    auto even = [](size_t v) { return v + (v & 1); };
    const size_t o_row = 0, o_split = even(fft_twiddle_count(p->row)), o_tw = even(o_split + p->m + 1),
                 total = even(o_tw + p->m + 1);
    std::vector<float2> host(total, make_float2(0.f, 0.f));
    fill_fft_twiddles(p->row, &host[o_row]);
    fill_split(n, &host[o_split]);
    fill_axis_twiddle(n, p->m + 1, norm, inverse, 1.0, &host[o_tw]);
    dctx_status st = upload(host, &p->dev_mem);
    if (st != DCTX_OK) return st;
    float2 *d = static_cast<float2 *>(p->dev_mem);
    p->row.tw = d + o_row;
    p->split = d + o_split;
    p->tw = d + o_tw;
    *out = p.get();
    h->plans1d[key] = p.release();
    return DCTX_OK;
}

dctx_status run_1d(dctx_context *h, const float *x, float *y, int n, int batch, dctx_norm norm, bool inverse,
                   void *stream) {
    if (!h || !x || !y || n < 1 || batch < 1) return DCTX_ERR_INVALID;
    if (!norm_ok(norm)) return DCTX_ERR_INVALID;
    const size_t bytes = (size_t)n * (size_t)batch * sizeof(float);
    if (overlaps(x, bytes, y, bytes) || !aligned8(x) || !aligned8(y)) return DCTX_ERR_INVALID;
    if ((n & 1) || n < 2 || n > kMax1dLong || !five_smooth(n) || (n <= kMax1d && !length_ok(n)))
        return DCTX_ERR_UNSUPPORTED;
    if ((long long)n * batch > (1LL << 31) / 2) return DCTX_ERR_UNSUPPORTED;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    Plan1D *p = nullptr;
    dctx_status st = build_plan1d(h, n, norm, inverse, &p);
    if (st != DCTX_OK) return st;
    if (p->m1) {
        // four-step route: two passes over a workspace of batch x m complex values
        if (batch > 65535) return DCTX_ERR_UNSUPPORTED;
        st = ensure_ws(h, (size_t)batch * p->m * sizeof(float2));
        if (st != DCTX_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        float2 *w = static_cast<float2 *>(h->ws);
        const hipError_t e =
            inverse ? timed(h, K_IDCT1D, s, [&] { return launch_idct1d_long(*p, batch, x, w, y, s); })
                    : timed(h, K_DCT1D, s, [&] { return launch_dct1d_long(*p, batch, x, w, y, s); });
        return from_hip(e);
    }
    const int rpb = pick_rows_per_block(batch, p->m, p->row.T, h->lds_max);
    if (!fits_rows(rpb, p->m, p->row.T, h->lds_max)) return DCTX_ERR_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the compile-time kernels move whole rows with 16-byte accesses
    const bool fast = p->fast && aligned16(x) && aligned16(y);
    const hipError_t e =
        inverse ? timed(h, K_IDCT1D, s, [&] {
            return fast ? launch_fast_idct1d(*p, batch, x, y, s) : launch_idct1d(*p, batch, rpb, x, y, s);
        })
                : timed(h, K_DCT1D, s, [&] {
                      return fast ? launch_fast_dct1d(*p, batch, x, y, s) : launch_dct1d(*p, batch, rpb, x, y, s);
                  });
    return from_hip(e);
}

// ------------------------------------------------------------------ batches
// Device copy of a host-side plan object (made once, kept by the handle).
template <class T>
dctx_status device_copy(dctx_context *h, const T *obj, const T **out) {
    auto it = h->dcopies.find(obj);
    if (it != h->dcopies.end()) {
        *out = static_cast<const T *>(it->second);
        return DCTX_OK;
    }
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(T));
    if (e == hipSuccess) e = hipMemcpy(d, obj, sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return from_hip(e);
    }
    h->dcopies[obj] = d;
    *out = static_cast<const T *>(d);
    return DCTX_OK;
}

bool is_2d_kind(int k) { return k == DCTX_KIND_DCT2 || k == DCTX_KIND_IDCT2 || k == DCTX_KIND_POISSON2; }

size_t desc_elems(const dctx_desc &d) {
    size_t n = 1;
    for (int i = 0; i < d.ndim; ++i) n *= (size_t)d.dims[i];
    return n;
}

// Argument checks of one descriptor (the same rules as the plain calls).
dctx_status check_desc(const dctx_desc &d) {
    if (enum_value(d.kind) < DCTX_KIND_DCT2 || enum_value(d.kind) > DCTX_KIND_POISSON2) return DCTX_ERR_INVALID;
    const int nd = is_2d_kind(d.kind) ? 2 : 3;
    if (d.ndim != nd) return DCTX_ERR_INVALID;
    for (int i = 0; i < nd; ++i)
        if (d.dims[i] < 1) return DCTX_ERR_INVALID;
    if (!d.in || !d.out || !aligned8(d.in) || !aligned8(d.out)) return DCTX_ERR_INVALID;
    if (d.kind != DCTX_KIND_POISSON2 && !norm_ok(d.norm)) return DCTX_ERR_INVALID;
    if (d.kind == DCTX_KIND_POISSON2)
        for (int i = 0; i < 2; ++i)
            if (!(d.h[i] == d.h[i]) || std::isinf(d.h[i])) return DCTX_ERR_INVALID;
    const size_t bytes = desc_elems(d) * sizeof(float);
    if (overlaps(d.in, bytes, d.out, bytes)) return DCTX_ERR_INVALID;
    if (nd == 2) {
        // the plain calls' shapes up to n1 = 8192 (a column of the batched
        // launches is one workgroup; longer ones take the plain call's
        // transposed route, which is not part of the batched launches)
        const int n1 = d.dims[0], n2 = d.dims[1];
        if (n1 < 2 || n2 < 2 || !length_ok(n1) || !length_ok(n2) || n1 > 8192) return DCTX_ERR_UNSUPPORTED;
        return DCTX_OK;
    }
    return check_3d_shape(d.dims[0], d.dims[1], d.dims[2]);
}

// No item's output may overlap any other item's input or output.
bool batch_overlaps(const dctx_desc *d, int count) {
    struct Iv {
        uintptr_t a, b;
        bool out;
        int item;
    };
    std::vector<Iv> iv;
    iv.reserve(2 * (size_t)count);
    for (int i = 0; i < count; ++i) {
        const size_t bytes = desc_elems(d[i]) * sizeof(float);
        iv.push_back({(uintptr_t)d[i].in, (uintptr_t)d[i].in + bytes, false, i});
        iv.push_back({(uintptr_t)d[i].out, (uintptr_t)d[i].out + bytes, true, i});
    }
    std::sort(iv.begin(), iv.end(), [](const Iv &x, const Iv &y) { return x.a < y.a; });
    uintptr_t end_any = 0, end_out = 0;
    for (const Iv &v : iv) {
        if (v.a < end_out) return true;
        if (v.out && v.a < end_any) return true;
        end_any = std::max(end_any, v.b);
        if (v.out) end_out = std::max(end_out, v.b);
    }
    return false;
}

uint64_t batch_signature(const dctx_desc *d, int count) {
    std::vector<std::array<int, 5>> k((size_t)count);
    for (int i = 0; i < count; ++i)
        k[i] = {(int)d[i].kind, d[i].ndim, d[i].dims[0], d[i].dims[1], d[i].ndim > 2 ? d[i].dims[2] : 0};
    std::sort(k.begin(), k.end());
    uint64_t hsh = 1469598103934665603ull;
    for (auto &e : k)
        for (int v : e) {
            hsh ^= (uint64_t)(uint32_t)v;
            hsh *= 1099511628211ull;
        }
    return hsh;
}

// Per-item plans and workspace offsets.
struct ItemPlan {
    int idx;
    int kind;
    Plan2D *fwd = nullptr, *inv = nullptr;
    PlanPoisson *pp = nullptr;
    Plan3D *p3 = nullptr;
    Plan2D *rp3 = nullptr;
    size_t ws_off = 0;
};

dctx_status plan_batch(dctx_context *h, const dctx_desc *d, int count, std::vector<ItemPlan> &items,
                       size_t &ws_total) {
    items.clear();
    items.reserve(count);
    ws_total = 0;
    for (int i = 0; i < count; ++i) {
        ItemPlan ip;
        ip.idx = i;
        ip.kind = d[i].kind;
        dctx_status st = DCTX_OK;
        size_t need = 0;
        if (is_2d_kind(d[i].kind)) {
            const int n1 = d[i].dims[0], n2 = d[i].dims[1];
            if (d[i].kind == DCTX_KIND_POISSON2) {
                const double h1 = d[i].h[0] > 0.0 ? d[i].h[0] : 1.0 / n1;
                const double h2 = d[i].h[1] > 0.0 ? d[i].h[1] : 1.0 / n2;
                st = build_plan_poisson(h, n1, n2, h1, h2, &ip.pp);
                if (st == DCTX_OK) {
                    ip.fwd = ip.pp->fwd;
                    ip.inv = ip.pp->inv;
                }
            } else if (d[i].kind == DCTX_KIND_DCT2) {
                st = build_plan2d(h, n1, n2, d[i].norm, false, &ip.fwd);
            } else {
                st = build_plan2d(h, n1, n2, d[i].norm, true, &ip.inv);
            }
            need = ws_bytes_2d(n1, n2);
        } else {
            const int n1 = d[i].dims[0], n2 = d[i].dims[1], n3 = d[i].dims[2];
            st = build_plan3d(h, n1, n2, n3, d[i].norm, d[i].kind == DCTX_KIND_IDCT3, &ip.p3);
            if (st == DCTX_OK) st = build_rows_plan(h, n1 * n2, n2, n3, &ip.rp3);
            need = ws_bytes_3d(n1, n2, n3);
        }
        if (st != DCTX_OK) return st;
        ip.ws_off = ws_total;
        ws_total += (need + 255) & ~(size_t)255;
        items.push_back(ip);
    }
    return DCTX_OK;
}

constexpr size_t kBatchTileLds = 64 * 1024;

// Tiles of one item in a batched pass: `per` sequences (rows of a row pass,
// packed columns of a column pass) of length len with T threads each per
// tile, the tile count, and the LDS bytes the tile body uses (per padded
// sequences; the workgroup of `block` threads runs per * T of them).
struct TileGeo {
    int per, tiles;
    size_t lds;
};
TileGeo tile_geometry(int len, int T, int n, int block, size_t lds_max, int cap = 0) {
    const size_t seqbytes = (size_t)lpad_len(len) * sizeof(float2);
    int per = std::max(1, block / T);
    per = std::min(per, (int)std::max<size_t>(1, std::min(kBatchTileLds, lds_max) / seqbytes));
    if (cap > 0) per = std::min(per, cap);
    per = std::min(per, n);
    return {per, (n + per - 1) / per, (size_t)per * seqbytes};
}

// Host image of one pass launch.
struct PassHost {
    std::vector<BatchItem> items;
    std::vector<int> tile_local, tile_item;
    size_t lds = 0;
    int block = 0, grid = 0;
    BatchLaunch L{};
};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Builds the five pass launches for the given per-pass block sizes and grid
// factors (0: one tile per workgroup, else factor x compute units).
dctx_status build_passes(dctx_context *h, const dctx_desc *d, const std::vector<ItemPlan> &items, float2 *ws_base,
                         const BatchTune &tn, PassHost (&ph)[kPassCount]) {
    struct Ent {
        int pass;
        const ItemPlan *ip;
        const Plan2D *plan;
        int len, T, n;   // sequence length, threads per sequence, sequences (rows or columns)
    };
    std::vector<Ent> ents;
    // row FFT length: m (packed half spectrum) or n2 (odd n2, full-length
    // complex FFT); workspace columns: ws_cols
    auto rlen = [](const Plan2D *p) { return p->odd ? p->n2 : p->m; };
    for (const ItemPlan &ip : items) {
        if (!ip.fwd && !ip.inv) continue;
        const int k = ip.kind;
        if (k == DCTX_KIND_DCT2 || k == DCTX_KIND_POISSON2)
            ents.push_back({kPassDctRows, &ip, ip.fwd, rlen(ip.fwd), ip.fwd->row.T, ip.fwd->n1});
        if (k == DCTX_KIND_DCT2)
            ents.push_back({kPassDctCols, &ip, ip.fwd, ip.fwd->n1, ip.fwd->col.T, ws_cols(*ip.fwd)});
        if (k == DCTX_KIND_POISSON2)
            ents.push_back({kPassPoissonCols, &ip, ip.fwd, ip.fwd->n1, ip.fwd->col.T, ws_cols(*ip.fwd)});
        if (k == DCTX_KIND_IDCT2)
            ents.push_back({kPassIdctCols, &ip, ip.inv, ip.inv->n1, ip.inv->col.T, ws_cols(*ip.inv)});
        if (k == DCTX_KIND_IDCT2 || k == DCTX_KIND_POISSON2)
            ents.push_back({kPassIdctRows, &ip, ip.inv, rlen(ip.inv), ip.inv->row.T, ip.inv->n1});
    }
    // larger sequences first: their tiles are the expensive ones
    std::stable_sort(ents.begin(), ents.end(), [](const Ent &a, const Ent &b) { return a.len > b.len; });
    int maxT[kPassCount] = {0, 0, 0, 0, 0};
    for (const Ent &e : ents) maxT[e.pass] = std::max(maxT[e.pass], e.T);
    for (int k = 0; k < kPassCount; ++k) {
        ph[k] = PassHost();
        if (maxT[k] == 0) continue;
        int B = tn.block[k] > 0 ? tn.block[k] : 256;
        B = std::min(kMaxBlock, std::max(B, round_up(maxT[k], 64)));
        ph[k].block = B;
    }
    for (const Ent &e : ents) {
        PassHost &P = ph[e.pass];
        const TileGeo tg = tile_geometry(e.len, e.T, e.n, P.block, h->lds_max, tn.per_cap[e.pass]);
        const int per = tg.per, tiles = tg.tiles;
        BatchItem it{};
        const dctx_desc &dd = d[e.ip->idx];
        dctx_status st = device_copy(h, e.plan, &it.plan);
        if (st != DCTX_OK) return st;
        if (e.pass == kPassPoissonCols) {
            st = device_copy(h, &e.ip->pp->q, &it.q);
            if (st != DCTX_OK) return st;
        }
        it.in = (e.pass == kPassDctRows || e.pass == kPassIdctCols) ? dd.in : nullptr;
        it.out = (e.pass == kPassDctCols || e.pass == kPassIdctRows) ? dd.out : nullptr;
        it.ws = reinterpret_cast<float2 *>(reinterpret_cast<char *>(ws_base) + e.ip->ws_off);
        it.per_tile = per;
        it.tiles = tiles;
        const int idx = (int)P.items.size();
        for (int t = 0; t < tiles; ++t) {
            P.tile_item.push_back(idx);
            P.tile_local.push_back(t);
        }
        P.items.push_back(it);
        P.lds = std::max(P.lds, tg.lds);
    }
    // Test aid: DCTX_BATCH_SHUFFLE=<seed> walks the tiles of every pass in a
    // seeded random order instead of largest sequences first (tiles are
    // independent, so results must not change).
    const int shuffle = env_int("DCTX_BATCH_SHUFFLE", 0);
    const bool xcd = env_int("DCTX_BATCH_XCD", 1) != 0;
    for (int k = 0; k < kPassCount; ++k) {
        PassHost &P = ph[k];
        const int total = (int)P.tile_item.size();
        if (total == 0) continue;
        if (P.lds > h->lds_max) return DCTX_ERR_UNSUPPORTED;
        if (xcd && !shuffle) {
            // XCD-aware order.  Workgroup b (and, in a persistent launch with a
            // grid that is a multiple of 8, every tile position b + i grid) runs
            // on XCD b % 8.  Each group of 128 consecutive tiles is cut into 8
            // blocks of 16; block x goes to positions x, x + 8, ..., x + 120 of
            // the group, so 16 neighbouring tiles (for a column pass: adjacent
            // column tiles, whose row segments share cache lines) run one after
            // another on one XCD and its L2, while consecutive blocks, of
            // similar cost, spread over the 8 XCDs.  A partial last group
            // keeps its order.
            std::vector<int> ti(P.tile_item), tl(P.tile_local);
            for (int g = 0; g + 128 <= total; g += 128)
                for (int x = 0; x < 8; ++x)
                    for (int i = 0; i < 16; ++i) {
                        ti[g + x + 8 * i] = P.tile_item[g + 16 * x + i];
                        tl[g + x + 8 * i] = P.tile_local[g + 16 * x + i];
                    }
            P.tile_item.swap(ti);
            P.tile_local.swap(tl);
        }
        if (shuffle) {
            uint64_t st = (uint64_t)shuffle * 0x9E3779B97F4A7C15ull + (uint64_t)k;
            for (int i = total - 1; i > 0; --i) {
                st ^= st << 13;
                st ^= st >> 7;
                st ^= st << 17;
                const int j = (int)(st % (uint64_t)(i + 1));
                std::swap(P.tile_item[i], P.tile_item[j]);
                std::swap(P.tile_local[i], P.tile_local[j]);
            }
        }
        const int f = tn.grid_factor[k];
        P.grid = f > 0 ? std::min(total, f * h->cus) : total;
        if (P.grid < total) P.grid &= ~7;   // persistent: keep positions b + i grid on XCD b % 8
        P.L.count = (int)P.items.size();
        P.L.total = total;
    }
    return DCTX_OK;
}

size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

size_t passes_bytes(const PassHost (&ph)[kPassCount]) {
    size_t n = 0;
    for (int k = 0; k < kPassCount; ++k) {
        n += align16(ph[k].items.size() * sizeof(BatchItem));
        n += align16(ph[k].tile_local.size() * sizeof(int));
        n += align16(ph[k].tile_item.size() * sizeof(int));
    }
    return n;
}

// Writes the pass arrays into `host` and points the launches at `dev`.
void pack_passes(PassHost (&ph)[kPassCount], char *host, char *dev) {
    size_t off = 0;
    for (int k = 0; k < kPassCount; ++k) {
        PassHost &P = ph[k];
        const size_t bi = P.items.size() * sizeof(BatchItem), bf = P.tile_local.size() * sizeof(int),
                     bt = P.tile_item.size() * sizeof(int);
        if (bi) std::memcpy(host + off, P.items.data(), bi);
        P.L.items = reinterpret_cast<const BatchItem *>(dev + off);
        off += align16(bi);
        if (bf) std::memcpy(host + off, P.tile_local.data(), bf);
        P.L.tile_local = reinterpret_cast<const int *>(dev + off);
        off += align16(bf);
        if (bt) std::memcpy(host + off, P.tile_item.data(), bt);
        P.L.tile_item = reinterpret_cast<const int *>(dev + off);
        off += align16(bt);
    }
}

const int kPassOrder[kPassCount] = {kPassDctRows, kPassIdctCols, kPassDctCols, kPassPoissonCols, kPassIdctRows};
const int kPassKernel[kPassCount] = {K_BATCH_DCT_ROWS, K_BATCH_DCT_COLS, K_BATCH_IDCT_COLS, K_BATCH_IDCT_ROWS,
                                     K_BATCH_POISSON_COLS};

// Enqueues the pass launches (in dependency order), then the 3-D items.
// pass_ev (nullable): an event pair per pass around its launch, for tuning.
dctx_status enqueue_passes(dctx_context *h, const dctx_desc *d, const std::vector<ItemPlan> &items,
                           const PassHost (&ph)[kPassCount], char *ws_base, hipStream_t s,
                           hipEvent_t (*pass_ev)[2]) {
    hipError_t e = hipSuccess;
    for (int o = 0; o < kPassCount && e == hipSuccess; ++o) {
        const int k = kPassOrder[o];
        const PassHost &P = ph[k];
        if (P.L.total == 0) continue;
        if (pass_ev) e = hipEventRecord(pass_ev[k][0], s);
        if (e == hipSuccess)
            e = timed(h, kPassKernel[k], s,
                      [&] { return launch_batch_pass((BatchPass)k, P.L, P.grid, P.block, P.lds, s); });
        if (e == hipSuccess && pass_ev) e = hipEventRecord(pass_ev[k][1], s);
    }
    if (e != hipSuccess) return from_hip(e);
    for (const ItemPlan &ip : items) {
        if (!ip.p3) continue;
        const dctx_desc &dd = d[ip.idx];
        dctx_status st = enqueue_3d(h, *ip.p3, *ip.rp3, dd.in, dd.out, ip.kind == DCTX_KIND_IDCT3,
                                    reinterpret_cast<float2 *>(ws_base + ip.ws_off), s);
        if (st != DCTX_OK) return st;
    }
    return DCTX_OK;
}

dctx_status ensure_bws(dctx_context *h, size_t bytes) {
    if (h->bws_bytes >= bytes) return DCTX_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return from_hip(e);
    if (h->bws) (void)hipFree(h->bws);
    h->bws = nullptr;
    h->bws_bytes = 0;
    e = hipMalloc(&h->bws, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        h->bws = nullptr;
        return from_hip(e);
    }
    h->bws_bytes = bytes;
    return DCTX_OK;
}

// Next upload slot with room for `bytes`: waits for its previous batch.
dctx_status take_slot(dctx_context *h, size_t bytes, dctx_context::Slot **out) {
    dctx_context::Slot &sl = h->slots[h->next_slot];
    h->next_slot = (h->next_slot + 1) % 16;
    hipError_t e = hipSuccess;
    if (!sl.done) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess && sl.used) e = hipEventSynchronize(sl.done);
    if (e != hipSuccess) return from_hip(e);
    sl.used = false;
    if (sl.bytes < bytes) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        sl.host = sl.dev = nullptr;
        sl.bytes = 0;
        const size_t cap = std::max<size_t>(bytes + bytes / 2, 64 * 1024);
        e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&sl.dev, cap);
        if (e != hipSuccess) {
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.dev) (void)hipFree(sl.dev);
            sl.host = sl.dev = nullptr;
            return from_hip(e);
        }
        sl.bytes = cap;
    }
    *out = &sl;
    return DCTX_OK;
}

dctx_status validate_batch(dctx_context *h, const dctx_desc *d, int count, dctx_status *per_item) {
    if (!h || count < 0 || (count > 0 && !d)) return DCTX_ERR_INVALID;
    dctx_status first = DCTX_OK;
    for (int i = 0; i < count; ++i) {
        const dctx_status st = check_desc(d[i]);
        if (per_item) per_item[i] = st;
        if (st != DCTX_OK && first == DCTX_OK) first = st;
    }
    if (first != DCTX_OK) return first;
    if (batch_overlaps(d, count)) {
        if (per_item)
            for (int i = 0; i < count; ++i) per_item[i] = DCTX_ERR_INVALID;
        return DCTX_ERR_INVALID;
    }
    return DCTX_OK;
}

// Untuned geometry: one workgroup per tile, 256 threads for the row passes and
// 512 for the column passes (the autotuner's choice on mixed batches of
// 5-smooth sides from 64 to 1024).
BatchTune default_tune() {
    BatchTune t;
    for (int k = 0; k < kPassCount; ++k) {
        const bool rows = k == kPassDctRows || k == kPassIdctRows;
        t.block[k] = rows ? 256 : 512;
        t.grid_factor[k] = 0;
        t.per_cap[k] = 0;
    }
    return t;
}

// One batch on `stream` with the given tuning (or the cached / default one).
// ws_base (nullable): a caller workspace of ws_cap bytes; else the handle's
// batch workspace.
dctx_status run_batch(dctx_context *h, const dctx_desc *d, int count, hipStream_t s, const BatchTune *force,
                      hipEvent_t (*pass_ev)[2], PassHost (*out_ph)[kPassCount], void *ws_base = nullptr,
                      size_t ws_cap = 0) {
    std::vector<ItemPlan> items;
    size_t ws_total = 0;
    dctx_status st = plan_batch(h, d, count, items, ws_total);
    if (st == DCTX_OK && !ws_base) st = ensure_bws(h, ws_total);
    if (st == DCTX_OK && ws_base && ws_cap < ws_total) st = DCTX_ERR_INVALID;
    if (st != DCTX_OK) return st;
    void *wsb = ws_base ? ws_base : h->bws;
    BatchTune tn = default_tune();
    if (force) {
        tn = *force;
    } else {
        auto it = h->tune.find(batch_signature(d, count));
        if (it != h->tune.end()) tn = it->second;
    }
    PassHost ph[kPassCount];
    st = build_passes(h, d, items, static_cast<float2 *>(wsb), tn, ph);
    if (st != DCTX_OK) return st;
    const size_t bytes = passes_bytes(ph);
    dctx_context::Slot *sl = nullptr;
    st = take_slot(h, bytes, &sl);
    if (st != DCTX_OK) return st;
    pack_passes(ph, static_cast<char *>(sl->host), static_cast<char *>(sl->dev));
    hipError_t e = bytes ? hipMemcpyAsync(sl->dev, sl->host, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    if (e != hipSuccess) return from_hip(e);
    st = enqueue_passes(h, d, items, ph, static_cast<char *>(wsb), s, pass_ev);
    e = hipEventRecord(sl->done, s);
    if (e == hipSuccess) sl->used = true;
    if (st == DCTX_OK && e != hipSuccess) st = from_hip(e);
    if (out_ph)
        for (int k = 0; k < kPassCount; ++k) (*out_ph)[k] = ph[k];
    return st;
}

// Smallest item (elements) that a grouped batch runs on its own compile-time
// launches; smaller ones are cheapest inside the persistent batch passes,
// which take every kind and shape in at most five launches.
constexpr size_t kGroupMinElems = (size_t)1 << 16;

// Whether an item of a grouped batch runs on grouped compile-time launches:
// power-of-two 2-D shapes of the fast or split form (any kind), power-of-two
// 3-D shapes with n1, n2 in [64, 256], 16-byte aligned buffers.
bool group_candidate(const dctx_desc &d) {
    if (!aligned16(d.in) || !aligned16(d.out) || desc_elems(d) < kGroupMinElems) return false;
    if (!is_2d_kind(d.kind))
        return fast3_supported(d.dims[0]) && fast3_supported(d.dims[1]) && !(d.dims[2] & 1) &&
               fast_rows_supported(d.dims[2] / 2);
    return !(d.dims[1] & 1) && fast_supported(d.dims[0], d.dims[1] / 2);
}

// One group (same kind, shape, norm and spacing; at most kGroupMax items):
// each pass of the transform as one launch over the group.  Items whose plan
// has no compile-time kernels (DCTX_FAST=0) run one by one.
dctx_status enqueue_group(dctx_context *h, const dctx_desc *d, const std::vector<int> &idx, char *ws,
                          const std::vector<size_t> &off, hipStream_t s) {
    const dctx_desc &d0 = d[idx[0]];
    GroupBufs g{};
    g.n = (int)idx.size();
    for (int i = 0; i < g.n; ++i) {
        g.in[i] = d[idx[i]].in;
        g.out[i] = d[idx[i]].out;
        g.ws[i] = reinterpret_cast<float2 *>(ws + off[i]);
    }
    const int n1 = d0.dims[0], n2 = d0.dims[1];
    dctx_status st = DCTX_OK;
    if (d0.kind == DCTX_KIND_DCT3 || d0.kind == DCTX_KIND_IDCT3) {
        const bool inv = d0.kind == DCTX_KIND_IDCT3;
        Plan3D *p = nullptr;
        Plan2D *rp = nullptr;
        st = build_plan3d(h, n1, n2, d0.dims[2], d0.norm, inv, &p);
        if (st == DCTX_OK) st = build_rows_plan(h, n1 * n2, n2, d0.dims[2], &rp);
        if (st != DCTX_OK) return st;
        if (p->plane || (p->fast && rp->fast)) return enqueue_3d_group(h, *p, *rp, inv, g, s);
        for (int i = 0; i < g.n && st == DCTX_OK; ++i) st = enqueue_3d(h, *p, *rp, g.in[i], g.out[i], inv, g.ws[i], s);
        return st;
    }
    if (d0.kind == DCTX_KIND_POISSON2) {
        const double h1 = d0.h[0] > 0.0 ? d0.h[0] : 1.0 / n1, h2 = d0.h[1] > 0.0 ? d0.h[1] : 1.0 / n2;
        PlanPoisson *pp = nullptr;
        st = build_plan_poisson(h, n1, n2, h1, h2, &pp);
        if (st != DCTX_OK) return st;
        static const KernelId kid[3] = {K_POISSON_ROWS, K_POISSON_COLS, K_POISSON_IROWS};
        if (pp->fwd->fast) return enqueue_spectral_group(h, *pp, pp->q, pp->qs, g, s, kid);
        for (int i = 0; i < g.n && st == DCTX_OK; ++i)
            st = run_spectral(h, *pp, pp->q, pp->qs, g.in[i], g.out[i], n1, n2, s, g.ws[i], kid);
        return st;
    }
    const bool inv = d0.kind == DCTX_KIND_IDCT2;
    Plan2D *pp = nullptr;
    st = build_plan2d(h, n1, n2, d0.norm, inv, &pp);
    if (st != DCTX_OK) return st;
    if (!pp->fast) {
        for (int i = 0; i < g.n && st == DCTX_OK; ++i)
            st = run_2d(h, g.in[i], g.out[i], n1, n2, d0.norm, inv, g.ws[i], ws_bytes_2d(n1, n2), s);
        return st;
    }
    PlanSplit *ps = nullptr;
    if (split_supported(n1, n2 / 2) && env_int("DCTX_SPLIT", 1) != 0) {
        st = build_plan_split(h, n1, n2, d0.norm, inv, &ps);
        if (st != DCTX_OK) return st;
    }
    return enqueue_2d_group(h, *pp, ps, inv, g, s);
}

// A batch with grouping (the serving loop's batches): items that
// group_candidate accepts are grouped by (kind, shape, norm, spacing) and each
// group of up to kGroupMax runs every pass as one launch of the compile-time
// kernels, exactly the launches of the plain call with one grid layer per
// item; the other items run through the persistent batch passes.  Workspace
// (ws, ws_cap bytes): the persistent passes' items first, then every grouped
// item's own footprint, in item order.
dctx_status run_batch_grouped(dctx_context *h, const dctx_desc *d, int count, hipStream_t s, void *ws,
                              size_t ws_cap) {
    std::vector<dctx_desc> rest;
    std::vector<int> grouped;
    size_t rest_bytes = 0;
    for (int i = 0; i < count; ++i) {
        const size_t need = is_2d_kind(d[i].kind) ? ws_bytes_2d(d[i].dims[0], d[i].dims[1])
                                                  : ws_bytes_3d(d[i].dims[0], d[i].dims[1], d[i].dims[2]);
        if (group_candidate(d[i])) {
            grouped.push_back(i);
        } else {
            rest.push_back(d[i]);
            rest_bytes += (need + 255) & ~(size_t)255;
        }
    }
    char *base = static_cast<char *>(ws);
    if (!rest.empty()) {
        dctx_status st = run_batch(h, rest.data(), (int)rest.size(), s, nullptr, nullptr, nullptr, base,
                                   std::min(rest_bytes, ws_cap));
        if (st != DCTX_OK) return st;
    }
    // workspace offsets of the grouped items, then groups in order of first appearance
    std::vector<size_t> off(count, 0);
    size_t o = rest_bytes;
    for (int i : grouped) {
        off[i] = o;
        const size_t need = is_2d_kind(d[i].kind) ? ws_bytes_2d(d[i].dims[0], d[i].dims[1])
                                                  : ws_bytes_3d(d[i].dims[0], d[i].dims[1], d[i].dims[2]);
        o += (need + 255) & ~(size_t)255;
    }
    if (o > ws_cap) return DCTX_ERR_INVALID;
    std::vector<bool> done(count, false);
    for (size_t a = 0; a < grouped.size(); ++a) {
        const int i = grouped[a];
        if (done[i]) continue;
        std::vector<int> idx;
        std::vector<size_t> offs;
        for (size_t b = a; b < grouped.size() && (int)idx.size() < kGroupMax; ++b) {
            const int j = grouped[b];
            const dctx_desc &x = d[i], &y = d[j];
            const bool same = !done[j] && x.kind == y.kind && x.ndim == y.ndim && x.dims[0] == y.dims[0] &&
                              x.dims[1] == y.dims[1] && (x.ndim < 3 || x.dims[2] == y.dims[2]) &&
                              (x.kind == DCTX_KIND_POISSON2 ? (x.h[0] == y.h[0] && x.h[1] == y.h[1])
                                                           : x.norm == y.norm);
            if (!same) continue;
            done[j] = true;
            idx.push_back(j);
            offs.push_back(off[j]);
        }
        dctx_status st = enqueue_group(h, d, idx, base, offs, s);
        if (st != DCTX_OK) return st;
    }
    return DCTX_OK;
}

dctx_status autotune_batch(dctx_context *h, const dctx_desc *d, int count, hipStream_t s, dctx_tune_info *info) {
    hipEvent_t ev[kPassCount][2];
    for (auto &p : ev)
        for (auto &q : p)
            if (hipEventCreate(&q) != hipSuccess) return DCTX_ERR_DEVICE;
    const bool prof = h->prof;
    h->prof = false;
    const int blocks[] = {128, 256, 512};
    const int grids[] = {2, 4, 8, 16, 0};
    BatchTune best = default_tune();
    double best_ms[kPassCount];
    for (double &v : best_ms) v = 1e30;
    double default_total = 0.0;
    dctx_status st = DCTX_OK;
    auto measure = [&](const BatchTune &tn, double (&ms)[kPassCount], PassHost (&ph)[kPassCount]) -> dctx_status {
        for (double &v : ms) v = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            dctx_status r = run_batch(h, d, count, s, &tn, ev, &ph);
            if (r != DCTX_OK) return r;
            if (hipStreamSynchronize(s) != hipSuccess) return DCTX_ERR_DEVICE;
            for (int k = 0; k < kPassCount; ++k) {
                if (ph[k].L.total == 0) continue;
                float t = 0.f;
                if (hipEventElapsedTime(&t, ev[k][0], ev[k][1]) != hipSuccess) return DCTX_ERR_DEVICE;
                if (rep > 0) ms[k] = std::min(ms[k], (double)t);
            }
        }
        return DCTX_OK;
    };
    PassHost ph[kPassCount];
    {
        double ms[kPassCount];
        st = measure(default_tune(), ms, ph);
        for (int k = 0; st == DCTX_OK && k < kPassCount; ++k)
            if (ph[k].L.total) default_total += ms[k];
    }
    for (int bi = 0; st == DCTX_OK && bi < 3; ++bi)
        for (int gi = 0; st == DCTX_OK && gi < 5; ++gi) {
            BatchTune tn = default_tune();
            for (int k = 0; k < kPassCount; ++k) {
                tn.block[k] = blocks[bi];
                tn.grid_factor[k] = grids[gi];
            }
            double ms[kPassCount];
            st = measure(tn, ms, ph);
            for (int k = 0; st == DCTX_OK && k < kPassCount; ++k)
                if (ph[k].L.total && ms[k] < best_ms[k]) {
                    best_ms[k] = ms[k];
                    best.block[k] = ph[k].block;
                    best.grid_factor[k] = grids[gi];
                }
        }
    // second stage: sequences per tile (narrower tiles give more workgroups
    // and fewer idle threads on short sequences), at each pass's best geometry
    const int caps[] = {1, 2, 4, 8};
    for (int ci = 0; st == DCTX_OK && ci < 4; ++ci) {
        BatchTune tn = best;
        for (int k = 0; k < kPassCount; ++k) tn.per_cap[k] = caps[ci];
        double ms[kPassCount];
        st = measure(tn, ms, ph);
        for (int k = 0; st == DCTX_OK && k < kPassCount; ++k)
            if (ph[k].L.total && ms[k] < best_ms[k]) {
                best_ms[k] = ms[k];
                best.per_cap[k] = caps[ci];
            }
    }
    h->prof = prof;
    for (auto &p : ev)
        for (auto &q : p) (void)hipEventDestroy(q);
    if (st != DCTX_OK) return st;
    h->tune[batch_signature(d, count)] = best;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        double tot = 0.0;
        for (int k = 0; k < kPassCount; ++k) {
            info->block[k] = best.block[k];
            info->grid_factor[k] = best.grid_factor[k];
            info->per_cap[k] = best.per_cap[k];
            info->tiles[k] = ph[k].L.total;
            info->pass_ms[k] = best_ms[k] < 1e29 ? best_ms[k] : 0.0;
            tot += info->pass_ms[k];
        }
        info->tuned_ms = tot;
        info->default_ms = default_total;
    }
    return DCTX_OK;
}


// ------------------------------------------------------------ small-N MFMA
uint16_t host_bf16_bits(double v) {
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
double host_bf16_val(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}
uint16_t host_f16_bits(double v) {
    const _Float16 h = (_Float16)(float)v;
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

// Transform matrix M (row = output index) of the n-point DCT-II (forward) or
// its inverse under `norm`, in FP64, as bf16 hi / lo and fp16 tables.
dctx_status build_plan_small(dctx_context *h, int n, bool inverse, dctx_norm norm, SmallTabs *out) {
    auto key = std::make_tuple(n, (int)inverse, (int)norm);
    auto it = h->planssmall.find(key);
    if (it != h->planssmall.end()) {
        *out = it->second.first;
        return DCTX_OK;
    }
    const double pi = 3.14159265358979323846264338327950288;
    const size_t nn = (size_t)n * n;
    std::vector<uint16_t> host(3 * nn);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            // forward: M[k][j] = g(k) cos(pi (2j+1) k / 2n); inverse: M[j][k] = w(k) cos(pi (2j+1) k / 2n)
            const int k = inverse ? c : r, j = inverse ? r : c;
            const long long num = (long long)(2 * j + 1) * k % (4LL * n);
            const double cs = std::cos(pi * (double)num / (2.0 * n));
            double w;
            if (norm == DCTX_NORM_ORTHO)
                w = k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
            else
                w = inverse ? (k == 0 ? 1.0 / n : 2.0 / n) : 1.0;
            const double v = w * cs;
            const uint16_t hi = host_bf16_bits(v);
            host[(size_t)r * n + c] = hi;
            host[nn + (size_t)r * n + c] = host_bf16_bits(v - host_bf16_val(hi));
            host[2 * nn + (size_t)r * n + c] = host_f16_bits(v);
        }
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, host.size() * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemcpy(d, host.data(), host.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return from_hip(e);
    }
    const uint16_t *b = static_cast<const uint16_t *>(d);
    SmallTabs tb{b, b + nn, b + 2 * nn};
    h->planssmall[key] = std::make_pair(tb, d);
    *out = tb;
    return DCTX_OK;
}

dctx_status run_small(dctx_context *h, const float *x, float *y, int n, int batch, int inverse, dctx_norm norm,
                      dctx_prec prec, void *stream) {
    if (!h || !x || !y || batch < 1 || n < 1) return DCTX_ERR_INVALID;
    if (!norm_ok(norm)) return DCTX_ERR_INVALID;
    if (enum_value(prec) != DCTX_PREC_BF16X3 && enum_value(prec) != DCTX_PREC_FP16_SCALED) return DCTX_ERR_INVALID;
    if (inverse != 0 && inverse != 1) return DCTX_ERR_INVALID;
    const size_t bytes = (size_t)batch * n * n * sizeof(float);
    if (overlaps(x, bytes, y, bytes) || !aligned16(x) || !aligned16(y)) return DCTX_ERR_INVALID;
    if (n != 16 && n != 32 && n != 64 && n != 128) return DCTX_ERR_UNSUPPORTED;
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    SmallTabs tb{};
    dctx_status st = build_plan_small(h, n, inverse != 0, norm, &tb);
    if (st != DCTX_OK) return st;
    const int groups = small_groups(n, batch);
    const int grid = std::max(1, std::min(groups, h->cus * env_int("DCTX_SMALL_WG_PER_CU", small_wg_per_cu(n, (int)prec))));
    hipStream_t s = static_cast<hipStream_t>(stream);
    return from_hip(timed(h, K_SMALL, s, [&] { return launch_small(tb, n, x, y, batch, (int)prec, grid, s); }));
}

}  // namespace

// ------------------------------------------------------ tuning cache file
// One JSON object per line inside "entries" (a format this file writes and
// reads back; not a general JSON parser).
std::string device_arch(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return std::string();
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

struct TuneEntry {
    std::string arch;
    uint64_t sig;
    BatchTune t;
};

std::string tune_entry_line(const TuneEntry &e) {
    std::ostringstream o;
    o << "{\"arch\": \"" << e.arch << "\", \"signature\": \"";
    char hex[17];
    std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)e.sig);
    o << hex << "\"";
    auto arr = [&](const char *name, const int *v) {
        o << ", \"" << name << "\": [";
        for (int k = 0; k < kPassCount; ++k) o << (k ? ", " : "") << v[k];
        o << "]";
    };
    arr("block", e.t.block);
    arr("grid_factor", e.t.grid_factor);
    arr("per_cap", e.t.per_cap);
    o << "}";
    return o.str();
}

// Parses one entry line; false if the line is not one.
bool parse_tune_line(const std::string &ln, TuneEntry &e) {
    auto str_field = [&](const char *name, std::string &out) {
        const std::string key = std::string("\"") + name + "\": \"";
        const size_t a = ln.find(key);
        if (a == std::string::npos) return false;
        const size_t b = ln.find('"', a + key.size());
        if (b == std::string::npos) return false;
        out = ln.substr(a + key.size(), b - a - key.size());
        return true;
    };
    auto arr_field = [&](const char *name, int *v) {
        const std::string key = std::string("\"") + name + "\": [";
        const size_t a = ln.find(key);
        if (a == std::string::npos) return false;
        const char *p = ln.c_str() + a + key.size();
        for (int k = 0; k < kPassCount; ++k) {
            char *end = nullptr;
            const long val = std::strtol(p, &end, 10);
            if (end == p || val < 0 || val > 4096) return false;
            v[k] = (int)val;
            p = end;
            while (*p == ',' || *p == ' ') ++p;
        }
        return *p == ']';
    };
    std::string sig;
    if (!str_field("arch", e.arch) || !str_field("signature", sig) || sig.size() != 16) return false;
    char *end = nullptr;
    e.sig = std::strtoull(sig.c_str(), &end, 16);
    if (!end || *end) return false;
    return arr_field("block", e.t.block) && arr_field("grid_factor", e.t.grid_factor) &&
           arr_field("per_cap", e.t.per_cap);
}

// Entries of a cache file (false if it cannot be read or is not one).
bool read_tune_file(const char *path, std::vector<TuneEntry> &out) {
    std::ifstream f(path);
    if (!f) return false;
    std::string ln;
    bool header = false;
    while (std::getline(f, ln)) {
        if (ln.find("\"format\": \"dctx-tune-1\"") != std::string::npos) header = true;
        TuneEntry e;
        if (ln.find("\"signature\"") != std::string::npos) {
            if (!parse_tune_line(ln, e)) return false;
            out.push_back(e);
        }
    }
    return header;
}

dctx_status tune_save(dctx_context *h, const char *path) {
    const std::string arch = device_arch(h->device);
    if (arch.empty()) return DCTX_ERR_DEVICE;
    std::vector<TuneEntry> keep, old;
    if (read_tune_file(path, old))
        for (const TuneEntry &e : old)
            if (e.arch != arch) keep.push_back(e);
    for (const auto &kv : h->tune) keep.push_back({arch, kv.first, kv.second});
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return DCTX_ERR_INVALID;
        f << "{\"format\": \"dctx-tune-1\", \"entries\": [\n";
        for (size_t i = 0; i < keep.size(); ++i) f << "  " << tune_entry_line(keep[i]) << (i + 1 < keep.size() ? "," : "") << "\n";
        f << "]}\n";
        if (!f) return DCTX_ERR_INVALID;
    }
    if (std::rename(tmp.c_str(), path) != 0) return DCTX_ERR_INVALID;
    return DCTX_OK;
}

dctx_status tune_load(dctx_context *h, const char *path, int *loaded) {
    std::vector<TuneEntry> ents;
    if (!read_tune_file(path, ents)) return DCTX_ERR_INVALID;
    const std::string arch = device_arch(h->device);
    int n = 0;
    for (const TuneEntry &e : ents)
        if (e.arch == arch) {
            h->tune[e.sig] = e.t;
            ++n;
        }
    if (loaded) *loaded = n;
    return DCTX_OK;
}

void arena_clear(TableArena &a) {
    for (auto &kv : a.p2d) delete kv.second;
    for (auto &kv : a.ps) delete kv.second;
    a.p2d.clear();
    a.ps.clear();
    a.used = 0;
}

size_t ws_bytes_2d_plain_call(int n1, int n2) { return ws_bytes_2d(n1, n2); }

dctx_status run_2d_in_arena(dctx_context *h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                            bool inverse, void *ws, size_t ws_bytes, void *stream, TableArena *ar) {
    return run_2d(h, x, y, n1, n2, norm, inverse, ws, ws_bytes, stream, 0, ar);
}

int handle_device(const dctx_context *h) { return h ? h->device : -1; }

// ------------------------------------------------ hooks for the serving loop
dctx_status rt_check_desc(const dctx_desc &d) { return check_desc(d); }

size_t rt_footprint(const dctx_desc &d) {
    const size_t ws = is_2d_kind(d.kind) ? ws_bytes_2d(d.dims[0], d.dims[1])
                                         : ws_bytes_3d(d.dims[0], d.dims[1], d.dims[2]);
    return (ws + 255) & ~(size_t)255;
}

dctx_status rt_run_batch(dctx_context *h, const dctx_desc *d, int count, hipStream_t s, void *ws, size_t ws_cap) {
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    return run_batch_grouped(h, d, count, s, ws, ws_cap);
}

// One request through its plain entry point; ws (nullable, at least
// rt_footprint bytes) replaces the handle's workspace.
dctx_status rt_run_plain(dctx_context *h, const dctx_desc &d, hipStream_t s, void *ws) {
    const size_t wb = ws ? rt_footprint(d) : 0;
    switch (d.kind) {
        case DCTX_KIND_DCT2: return run_2d(h, d.in, d.out, d.dims[0], d.dims[1], d.norm, false, ws, wb, s);
        case DCTX_KIND_IDCT2: return run_2d(h, d.in, d.out, d.dims[0], d.dims[1], d.norm, true, ws, wb, s);
        case DCTX_KIND_DCT3: return run_3d(h, d.in, d.out, d.dims[0], d.dims[1], d.dims[2], d.norm, false, s, ws);
        case DCTX_KIND_IDCT3: return run_3d(h, d.in, d.out, d.dims[0], d.dims[1], d.dims[2], d.norm, true, s, ws);
        case DCTX_KIND_POISSON2:
            return run_poisson(h, d.in, d.out, d.dims[0], d.dims[1], d.h[0], d.h[1], s, ws);
        default: return DCTX_ERR_INVALID;
    }
}

size_t lds_budget_bytes() { return g_lds_budget; }

// LDS per workgroup on gfx950 (what dctx_create reads from the device), for
// the host-only shape queries.
constexpr size_t kLdsPerWorkgroup = 160 * 1024;

// The size rules of the plain call of `kind`: the call's own shape checks and
// plan geometry (schedules, tile fits), evaluated on the host.  Returns 1 when
// the call with valid buffers does not refuse the shape.
int shape_supported(int kind, int n1, int n2, int n3) {
    try {
        dctx_context tmp;
        tmp.lds_max = kLdsPerWorkgroup;
        if (kind == DCTX_KIND_DCT3 || kind == DCTX_KIND_IDCT3) {
            if (check_3d_shape(n1, n2, n3) != DCTX_OK) return 0;
            Plan3D p3;
            Plan2D rp;
            return plan3d_geometry(n1, n2, n3, DCTX_NORM_BACKWARD, kind == DCTX_KIND_IDCT3, tmp.lds_max, p3) == DCTX_OK &&
                           rows_plan_geometry(n1 * n2, n2, n3, tmp.lds_max, rp) == DCTX_OK
                       ? 1
                       : 0;
        }
        if (kind != DCTX_KIND_DCT2 && kind != DCTX_KIND_IDCT2 && kind != DCTX_KIND_POISSON2) return 0;
        if (n1 < 2 || n2 < 2 || !length_ok(n1) || !length_ok(n2)) return 0;
        Plan2D p;
        Tabs2D o;
        std::vector<float2> img;
        // the transposed route of the plain DCT / IDCT runs the n2 x n1 transform
        if (kind != DCTX_KIND_POISSON2 && transposed_route(n1, n2))
            return image_plan2d(&tmp, n2, n1, DCTX_NORM_BACKWARD, false, p, img, o) == DCTX_OK ? 1 : 0;
        if (image_plan2d(&tmp, n1, n2, DCTX_NORM_BACKWARD, false, p, img, o) != DCTX_OK) return 0;
        if (!(n2 & 1) && (split_supported(n1, n2 / 2) || split_long_supported(n1, n2 / 2)) && p.fast) {
            PlanSplit ps;
            TabsSplit os;
            if (image_plan_split(n1, n2, DCTX_NORM_BACKWARD, false, ps, img, os) != DCTX_OK) return 0;
        }
        return 1;
    } catch (const std::bad_alloc &) {
        return 0;
    }
}

// Host-side check of the batched passes' tile geometry for one 2-D shape,
// over every block size the autotuner tries (128, 256, 512; the block is
// raised to a multiple of 64 holding one sequence) and every pass kind: the
// highest LDS slot each tile body touches (rows: `per` padded row buffers, the
// row FFT / split / reorder at slots lpad(0 .. len-1) of each; columns: the
// strided layout lpad(row) * C + c for rows < n1, c < C) lies below the LDS
// bytes the launch passes, that is within the device's LDS, and the tile's
// sequences have threads.  Returns 1 when every case holds, else 0 with the
// first failing case written to msg.
int batch_geometry_ok(int n1, int n2, char *msg, int msglen) {
    auto host_lpad = [](int i) { return i + (i >> 4); };   // lpad() of fft_core.h
    auto fail = [&](const char *what, int block, int pass) {
        if (msg && msglen > 0) std::snprintf(msg, (size_t)msglen, "%dx%d block %d pass %d: %s", n1, n2, block, pass, what);
        return 0;
    };
    dctx_context tmp;
    tmp.lds_max = kLdsPerWorkgroup;
    Plan2D p;
    Tabs2D o;
    std::vector<float2> img;
    if (image_plan2d(&tmp, n1, n2, DCTX_NORM_BACKWARD, false, p, img, o) != DCTX_OK) return fail("no plan", 0, -1);
    const int rlen = p.odd ? p.n2 : p.m;
    const int blocks[] = {128, 256, 512};
    for (int bi = 0; bi < 3; ++bi)
        for (int pass = 0; pass < kPassCount; ++pass) {
            const bool rows = pass == kPassDctRows || pass == kPassIdctRows;
            const int len = rows ? rlen : n1, T = rows ? p.row.T : p.col.T, n = rows ? n1 : ws_cols(p);
            const int block = std::min(kMaxBlock, std::max(blocks[bi], round_up(T, 64)));
            const TileGeo g = tile_geometry(len, T, n, block, tmp.lds_max);
            if (g.per < 1 || g.tiles * g.per < n || (g.tiles - 1) * g.per >= n) return fail("tiles", block, pass);
            if (g.per * T > block) return fail("threads", block, pass);
            if (T * kEmax < len) return fail("values per thread", block, pass);
            if (g.lds > tmp.lds_max) return fail("LDS above the device limit", block, pass);
            // highest float2 slot + 1 the body touches
            const size_t top = rows ? (size_t)(g.per - 1) * lpad_len(len) + (size_t)host_lpad(len - 1) + 1
                                    : (size_t)host_lpad(n1 - 1) * g.per + (size_t)g.per;
            if (top * sizeof(float2) > g.lds) return fail("LDS slot beyond the launch's bytes", block, pass);
        }
    return 1;
}


}  // namespace dctx


using namespace dctx;

extern "C" {

const char *dctx_status_string(dctx_status s) {
    // the caller may pass any integer: read it as one (loading an enum object
    // that holds a value outside the enumeration is undefined)
    int v = 0;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
        case DCTX_OK: return "ok";
        case DCTX_ERR_INVALID: return "invalid argument";
        case DCTX_ERR_UNSUPPORTED: return "unsupported size or configuration";
        case DCTX_ERR_NOMEM: return "out of memory";
        case DCTX_ERR_DEVICE: return "HIP device error";
        case DCTX_ERR_BUSY: return "not complete";
        case DCTX_ERR_TOO_LARGE: return "shape exceeds the static scratch of the allocation-free call";
        case DCTX_ERR_CANCELLED: return "request cancelled";
    }
    return "unknown status";
}

int dctx_version(void) { return (0 << 16) | 1; }

dctx_status dctx_debug_write_count(dctx_handle h, unsigned *count, const void *base, size_t bytes) {
    if (!h || (count == nullptr) != (base == nullptr)) return DCTX_ERR_INVALID;
#ifdef DCTX_WRITE_COUNT
    if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    const WriteCountBinding w{count, static_cast<const char *>(base), count ? bytes : 0};
    for (auto set : wc_setters())
        if (set(w) != hipSuccess) return DCTX_ERR_DEVICE;
    return DCTX_OK;
#else
    (void)bytes;
    return DCTX_ERR_UNSUPPORTED;
#endif
}

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
    if (n < 1) return 0;
    return axis_last ? shape_supported(DCTX_KIND_DCT2, 2, n, 0) : shape_supported(DCTX_KIND_DCT2, n, 2, 0);
}

int dctx_shape_supported(dctx_kind kind, int n1, int n2, int n3) {
    return shape_supported(enum_value(kind), n1, n2, n3);
}

int dctx_batch_geometry_check(int n1, int n2, char *msg, int msglen) {
    try {
        return batch_geometry_ok(n1, n2, msg, msglen);
    } catch (...) {
        return 0;
    }
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
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        h->cus = cus;
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
    for (auto &kv : h->planspoisson) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    for (auto &kv : h->planscompress) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    for (auto &kv : h->plans1d) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    for (auto &kv : h->dcopies) (void)hipFree(kv.second);
    for (auto &kv : h->planssmall) (void)hipFree(kv.second.second);
    for (auto &kv : h->planssplit) {
        (void)hipFree(kv.second->dev_mem);
        delete kv.second;
    }
    if (h->bws) (void)hipFree(h->bws);
    for (auto &sl : h->slots) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.done) (void)hipEventDestroy(sl.done);
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

dctx_status dctx_poisson2d(dctx_handle h, const float *f, float *u, int n1, int n2, double h1, double h2,
                           void *stream) {
    try {
        return run_poisson(h, f, u, n1, n2, h1, h2, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_dct1d(dctx_handle h, const float *x, float *y, int n, int batch, dctx_norm norm, void *stream) {
    try {
        return run_1d(h, x, y, n, batch, norm, false, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_idct1d(dctx_handle h, const float *x, float *y, int n, int batch, dctx_norm norm, void *stream) {
    try {
        return run_1d(h, x, y, n, batch, norm, true, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_compress2d(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm, double eps,
                            void *stream) {
    try {
        return run_compress(h, x, y, n1, n2, norm, eps, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_dct2d_small(dctx_handle h, const float *x, float *y, int n, int batch, int inverse, dctx_norm norm,
                             dctx_prec prec, void *stream) {
    try {
        return run_small(h, x, y, n, batch, inverse, norm, prec, stream);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_submit_batch(dctx_handle h, const dctx_desc *d, int count, void *stream, dctx_status *per_item) {
    try {
        dctx_status st = validate_batch(h, d, count, per_item);
        if (st != DCTX_OK || count == 0) return st;
        if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
        return run_batch(h, d, count, static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_autotune_batch(dctx_handle h, const dctx_desc *d, int count, void *stream, dctx_tune_info *info) {
    try {
        dctx_status st = validate_batch(h, d, count, nullptr);
        if (st != DCTX_OK) return st;
        if (count == 0) return DCTX_ERR_INVALID;
        if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
        return autotune_batch(h, d, count, static_cast<hipStream_t>(stream), info);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_tune_save(dctx_handle h, const char *path) {
    if (!h || !path) return DCTX_ERR_INVALID;
    try {
        return tune_save(h, path);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_tune_load(dctx_handle h, const char *path, int *loaded) {
    if (loaded) *loaded = 0;
    if (!h || !path) return DCTX_ERR_INVALID;
    try {
        return tune_load(h, path, loaded);
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

struct dctx_graph_s {
    dctx_context *h = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *dev = nullptr;
    void *ws = nullptr;
};

static void graph_free(dctx_graph_s *g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->dev) (void)hipFree(g->dev);
    if (g->ws) (void)hipFree(g->ws);
    delete g;
}

dctx_status dctx_graph_create(dctx_handle h, const dctx_desc *d, int count, dctx_graph *out) {
    if (!out) return DCTX_ERR_INVALID;
    *out = nullptr;
    dctx_graph_s *g = nullptr;
    try {
        dctx_status st = validate_batch(h, d, count, nullptr);
        if (st != DCTX_OK) return st;
        if (count == 0) return DCTX_ERR_INVALID;
        if (hipSetDevice(h->device) != hipSuccess) return DCTX_ERR_DEVICE;
        std::vector<ItemPlan> items;
        size_t ws_total = 0;
        st = plan_batch(h, d, count, items, ws_total);
        if (st != DCTX_OK) return st;
        g = new dctx_graph_s();
        g->h = h;
        hipError_t e = hipMalloc(&g->ws, std::max<size_t>(ws_total, 256));
        if (e != hipSuccess) {
            graph_free(g);
            return from_hip(e);
        }
        BatchTune tn = default_tune();
        auto it = h->tune.find(batch_signature(d, count));
        if (it != h->tune.end()) tn = it->second;
        PassHost ph[kPassCount];
        st = build_passes(h, d, items, static_cast<float2 *>(g->ws), tn, ph);
        if (st != DCTX_OK) {
            graph_free(g);
            return st;
        }
        const size_t bytes = passes_bytes(ph);
        std::vector<char> host(std::max<size_t>(bytes, 16));
        e = hipMalloc(&g->dev, std::max<size_t>(bytes, 16));
        if (e == hipSuccess) {
            pack_passes(ph, host.data(), static_cast<char *>(g->dev));
            if (bytes) e = hipMemcpy(g->dev, host.data(), bytes, hipMemcpyHostToDevice);
        }
        hipStream_t cs = nullptr;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) {
            graph_free(g);
            return from_hip(e);
        }
        const bool prof = h->prof;
        h->prof = false;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            st = enqueue_passes(h, d, items, ph, static_cast<char *>(g->ws), cs, nullptr);
            hipGraph_t graph = nullptr;
            const hipError_t e2 = hipStreamEndCapture(cs, &graph);
            g->graph = graph;
            if (e2 != hipSuccess && st == DCTX_OK) st = from_hip(e2);
        } else {
            st = from_hip(e);
        }
        h->prof = prof;
        (void)hipStreamDestroy(cs);
        if (st == DCTX_OK) st = from_hip(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        if (st != DCTX_OK) {
            graph_free(g);
            return st;
        }
        *out = g;
        return DCTX_OK;
    } catch (const std::bad_alloc &) {
        if (g) graph_free(g);
        return DCTX_ERR_NOMEM;
    } catch (...) {
        if (g) graph_free(g);
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_graph_launch(dctx_graph g, void *stream) {
    if (!g || !g->exec) return DCTX_ERR_INVALID;
    if (hipSetDevice(g->h->device) != hipSuccess) return DCTX_ERR_DEVICE;
    return from_hip(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
}

dctx_status dctx_graph_destroy(dctx_graph g) {
    if (!g) return DCTX_ERR_INVALID;
    (void)hipSetDevice(g->h->device);
    (void)hipDeviceSynchronize();
    graph_free(g);
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

dctx_status dctx_idct_idxst2d(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                              void *stream) {
    try {
        return run_2d(h, x, y, n1, n2, norm, true, nullptr, 0, stream, 1);   // IDXST along n1
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    } catch (...) {
        return DCTX_ERR_DEVICE;
    }
}

dctx_status dctx_idxst_idct2d(dctx_handle h, const float *x, float *y, int n1, int n2, dctx_norm norm,
                              void *stream) {
    try {
        return run_2d(h, x, y, n1, n2, norm, true, nullptr, 0, stream, 2);   // IDXST along n2
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
