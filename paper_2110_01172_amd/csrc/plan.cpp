// Plans: radix schedules and FP64-generated tables (rounded once to FP32),
// built once per shape and kept by the handle.  Building a plan is excluded
// from the transform itself, as the paper excludes its coefficient precompute
// (Section "Settings": the exp(-j pi n / 2N) sequence is computed in advance).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace dctx {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// exp(sign * j * pi * num / den) in FP64 with the integer part of the angle
// reduced exactly (num taken modulo 2 * den).
inline void expj(long long num, long long den, int sign, double &re, double &im) {
    long long r = num % (2 * den);
    if (r < 0) r += 2 * den;
    const double ang = kPi * (double)r / (double)den;
    re = std::cos(ang);
    im = sign * std::sin(ang);
}

inline float2 f2(double re, double im) { return make_float2((float)re, (float)im); }

}  // namespace

bool length_ok(int n) {
    if (n < 1 || n > kMaxLen) return false;
    for (int f : {2, 3, 5})
        while (n % f == 0) n /= f;
    return n == 1;
}

int max_butterflies(int R) { return std::max(1, kEmax / R); }

static bool fill_desc(int L, const std::vector<int> &rad, FftDesc &d);

bool make_fast_schedule(int L, FftDesc &d) {
    std::memset(&d, 0, sizeof(d));
    const FastCfg cf = fast_cfg(L);
    if (cf.T == 0) return false;
    return fill_desc(L, {cf.R0, cf.R1, cf.R2}, d);
}

bool make_schedule_radices(int L, const int *rad, int n, FftDesc &d) {
    std::memset(&d, 0, sizeof(d));
    int prod = 1;
    for (int i = 0; i < n; ++i) prod *= rad[i];
    if (n <= 0 || prod != L) return false;
    return fill_desc(L, std::vector<int>(rad, rad + n), d);
}

bool make_schedule(int L, FftDesc &d) {
    std::memset(&d, 0, sizeof(d));
    if (L == 1) {
        // the length-1 DFT is the identity: no stages (the half-length row FFT
        // of a length-2 real row)
        d.L = 1;
        d.nst = 0;
        d.T = 1;
        return true;
    }
    if (L < 2 || !length_ok(L)) return false;
    int rest = L;
    std::vector<int> rad;
    while (rest % 16 == 0) { rad.push_back(16); rest /= 16; }
    if (rest % 8 == 0) { rad.push_back(8); rest /= 8; }
    if (rest % 4 == 0) { rad.push_back(4); rest /= 4; }
    if (rest % 2 == 0) { rad.push_back(2); rest /= 2; }
    while (rest % 5 == 0) { rad.push_back(5); rest /= 5; }
    while (rest % 3 == 0) { rad.push_back(3); rest /= 3; }
    if (rest != 1 || rad.empty() || (int)rad.size() > kMaxStages) return false;
    return fill_desc(L, rad, d);
}

static bool fill_desc(int L, const std::vector<int> &rad, FftDesc &d) {
    if (rad.empty() || (int)rad.size() > kMaxStages) return false;
    d.L = L;
    d.nst = (int)rad.size();
    int ns = 1, T = 1, off = 0;
    for (int s = 0; s < d.nst; ++s) {
        d.rad[s] = rad[s];
        d.ns[s] = ns;
        d.nsmagic[s] = ns > 1 ? (unsigned)(((1ULL << 32) + (unsigned long long)ns - 1) / (unsigned long long)ns) : 0u;
        d.twoff[s] = off;
        if (ns > 1) off += ns * tw_record(rad[s]);
        const int nb = L / rad[s];
        const int mb = max_butterflies(rad[s]);
        T = std::max(T, (nb + mb - 1) / mb);
        ns *= rad[s];
    }
    d.T = T;
    return true;
}

size_t fft_twiddle_count(const FftDesc &d) {
    size_t n = 0;
    for (int s = 0; s < d.nst; ++s)
        if (d.ns[s] > 1) n += (size_t)d.ns[s] * tw_record(d.rad[s]);
    return n;
}

void fill_fft_twiddles(const FftDesc &d, float2 *tw) {
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.rad[s], Ns = d.ns[s], rec = tw_record(R);
        if (Ns == 1) continue;
        float2 *t = tw + d.twoff[s];
        for (int k = 0; k < Ns; ++k)
            for (int r = 0; r < rec; ++r) {
                double re = 0.0, im = 0.0;
                if (r < R) expj(2LL * r * k, (long long)Ns * R, -1, re, im);   // W_{Ns R}^{r k}
                t[(size_t)k * rec + r] = f2(re, im);
            }
    }
}

void fill_split(int n, float2 *split) {
    const int m = n / 2;
    for (int k = 0; k <= m; ++k) {
        double re, im;
        expj(2LL * k, n, -1, re, im);   // exp(-2 pi j k / n)
        split[k] = f2(re, im);
    }
}

void fill_roots(int m, float2 *out) {
    for (int e = 0; e < m; ++e) {
        double re, im;
        expj(2LL * e, m, -1, re, im);   // exp(-2 pi j e / m)
        out[e] = f2(re, im);
    }
}

bool five_smooth(long long n) {
    if (n < 1) return false;
    for (int f : {2, 3, 5})
        while (n % f == 0) n /= f;
    return n == 1;
}

// Per-axis scale of the forward post / inverse pre.  Forward: g(k) (ortho
// weights or 1); inverse: f(k) with the 1/2 per axis of the unnormalised
// inverse real FFT (which returns 2^D times the raw DCT-III) folded in.
double axis_scale(int n, int k, dctx_norm norm, bool inverse) {
    if (!inverse) {
        if (norm == DCTX_NORM_ORTHO) return k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
        return 1.0;
    }
    if (norm == DCTX_NORM_ORTHO) return k == 0 ? std::sqrt(1.0 / n) : 0.5 * std::sqrt(2.0 / n);
    return 1.0 / n;
}

// Twiddle along one axis for k in [0, count): forward exp(-j pi k / 2n),
// inverse exp(+j pi k / 2n), times the axis scale and an extra factor.
void fill_axis_twiddle(int n, int count, dctx_norm norm, bool inverse, double extra, float2 *out) {
    for (int k = 0; k < count; ++k) {
        double re, im;
        expj(k, 2LL * n, inverse ? +1 : -1, re, im);
        const double s = axis_scale(n, k, norm, inverse) * extra;
        out[k] = f2(re * s, im * s);
    }
}

}  // namespace dctx
