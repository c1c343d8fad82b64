// C ABI of libcwt: validation, planning (padded length, radix schedule,
// spectrum bands, band groups), device tables and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_internal.hpp"
#include "cwt_kernels.hpp"

using namespace cwtk;

// ------------------------------------------------------------ errors --

static thread_local std::string g_last_error;

namespace cwtrt {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(CWT_E_HIP, "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

// ----------------------------------------------------------- planning --

// Segmented plans: the longest padded length accepted, and the segment
// length used (7-smooth, at most CWT_MAX_LEN).
constexpr int64_t kMaxSegmentedLen = (int64_t)1 << 30;
constexpr int64_t kMaxSegmentLen = 20480;

static void set_chunks(cwt_plan &P);

static bool smooth7(int64_t m)
{
    if (m < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (m % p == 0) m /= p;
    return m == 1;
}

int64_t pad_length(int64_t n, int mode, int64_t explicit_len)
{
    switch (mode) {
    case CWT_PAD_SMOOTH7: {
        int64_t m = n;
        while (!smooth7(m)) ++m;
        return m;
    }
    case CWT_PAD_POW2: {
        int64_t m = 1;
        while (m < n) m <<= 1;
        return m;
    }
    case CWT_PAD_NONE: return n;
    case CWT_PAD_EXPLICIT: return explicit_len;
    default: return -1;
    }
}

// Composite radices the passes implement (small factors sharing one pass);
// 20, 21 and 24 only in plans of 24 values per thread.
static bool composite_radix(int r)
{
    return r == 6 || r == 9 || r == 10 || r == 12 || r == 14 || r == 15 || r == 20 || r == 21 ||
           r == 24;
}

// Fewest factors reachable from f by merging pairs into composite radices of
// at most maxv whose pass still fits the class's largest workgroup (L / R
// butterflies, maxv / R per thread); exhaustive over the few factors a
// length has.
static void merge_factors(std::vector<int> &f, int maxv, int L)
{
    std::vector<int> best = f;
    for (size_t i = 0; i < f.size(); ++i)
        for (size_t j = i + 1; j < f.size(); ++j) {
            const int pr = f[i] * f[j];
            if (!composite_radix(pr) || pr > maxv || L / pr > generic_max_threads(maxv) * (maxv / pr))
                continue;
            std::vector<int> g;
            for (size_t k = 0; k < f.size(); ++k)
                if (k != i && k != j) g.push_back(f[k]);
            g.push_back(pr);
            merge_factors(g, maxv, L);
            if (g.size() < best.size()) best = g;
        }
    f = best;
}

// Radix schedule: the largest radices first (16, 8, 4, 2, then 7, 5, 3),
// falling back to schedules without 16 (then without 8) when a thread of a
// 1024-wide workgroup would have to hold too many values; with `merge`, small
// factors are paired into composite radices (2x3, 3x3, 2x5, 4x3, 2x7, 3x5)
// wherever that saves passes, and the passes run largest radix first.  The
// workgroup size is the smallest multiple of 64 (at least L/16) for which no
// thread holds more than maxv values in any pass (maxv: the class asked for,
// 16, 24 or 32, with its own largest workgroup).
static bool try_radix_plan(int L, const int *order, int n_order, int maxv, bool merge,
                           RadixPlan &rp)
{
    rp = RadixPlan{};
    rp.L = L;
    int m = L;
    std::vector<int> f;
    for (int oi = 0; oi < n_order; ++oi) {
        const int r = order[oi];
        while (m % r == 0) {
            f.push_back(r);
            m /= r;
        }
    }
    if (m != 1) return false;
    if (merge && f.size() > 1) {
        merge_factors(f, maxv, L);
        std::stable_sort(f.begin(), f.end(), [](int a, int b) { return a > b; });
    }
    if ((int)f.size() > kMaxPasses) return false;
    int np = 0;
    for (int r : f) rp.radix[np++] = r;
    if (np == 0) rp.radix[np++] = 1;  // L == 1: a single identity pass
    rp.n_pass = np;
    const int tmax = generic_max_threads(maxv);
    for (int T = std::max(64, std::min(tmax, ((L / 16 + 63) / 64) * 64)); T <= tmax; T += 64) {
        bool ok = true;
        for (int i = 0; i < np && ok; ++i) {
            const int R = rp.radix[i];
            const int S = L / R;
            const int nb = (S + T - 1) / T;
            const int mb = std::max(1, maxv / R);
            if (nb > mb) ok = false;
        }
        if (ok) {
            rp.threads = T;
            rp.maxv = maxv;
            return true;
        }
    }
    return false;
}

static void ranked_plans(int L, std::vector<RadixPlan> &out);

void radix_candidates(int L, std::vector<RadixPlan> &out)
{
    static const int o1[] = {16, 8, 4, 2, 7, 5, 3};
    static const int o2[] = {8, 4, 2, 7, 5, 3};
    static const int o3[] = {4, 2, 7, 5, 3};
    const int *orders[] = {o1, o2, o3};
    const int lens[] = {7, 6, 5};
    out.clear();
    // the best-ranked schedules first (eight of them, at both workgroup sizes;
    // eight rather than four: the autotuned 256-recording batch 53.3 -> 52.9 ms)
    std::vector<RadixPlan> ranked;
    ranked_plans(L, ranked);
    for (size_t i = 0; i < ranked.size() && i < 8; ++i)
        for (int mul = 1; mul <= 2; ++mul) {
            RadixPlan c = ranked[i];
            c.threads = ranked[i].threads * mul;
            if (c.threads <= generic_max_threads(c.maxv)) out.push_back(c);
        }
    for (int maxv : {16, 24, 32})
        for (bool merge : {true, false})
            for (int o = 0; o < 3; ++o) {
                RadixPlan rp;
                if (!try_radix_plan(L, orders[o], lens[o], maxv, merge, rp)) continue;
                for (int mul = 1; mul <= 2; ++mul) {
                    RadixPlan c = rp;
                    c.threads = rp.threads * mul;
                    if (c.threads > generic_max_threads(maxv)) continue;
                    bool dup = false;
                    for (const RadixPlan &q : out)
                        if (q.threads == c.threads && q.maxv == c.maxv && q.n_pass == c.n_pass &&
                            std::equal(q.radix, q.radix + q.n_pass, c.radix))
                            dup = true;
                    if (!dup) out.push_back(c);
                }
            }
}

// Every radix the passes implement, largest first.
static const int kRadices[] = {24, 21, 20, 16, 15, 14, 12, 10, 9, 8, 7, 6, 5, 4, 3, 2};

// Workgroup size for a schedule at maxv values per thread: the smallest
// multiple of 64 (at least L/16) for which every pass's butterflies fit, or
// 0 when none up to the class's largest workgroup does.
static int schedule_threads(int L, const std::vector<int> &f, int maxv)
{
    const int tmax = generic_max_threads(maxv);
    int need = std::max(64, std::min(tmax, ((L / 16 + 63) / 64) * 64));
    for (int R : f) {
        if (R > maxv) return 0;
        const int mb = std::max(1, maxv / R);
        const int t = (L / R + mb - 1) / mb;
        need = std::max(need, ((t + 63) / 64) * 64);
    }
    return need <= tmax ? need : 0;
}

// All schedules (radix multisets, largest radix first) whose product is L.
static void enum_schedules(int rem, int maxr, std::vector<int> &cur,
                           std::vector<std::vector<int>> &out)
{
    if (rem == 1) {
        out.push_back(cur);
        return;
    }
    if ((int)cur.size() >= kMaxPasses) return;
    for (int r : kRadices)
        if (r <= maxr && rem % r == 0) {
            cur.push_back(r);
            enum_schedules(rem / r, r, cur, out);
            cur.pop_back();
        }
}

// Feasible plans of length L ordered best first: fewest passes (each pass is
// one LDS round trip and two barriers, and its twiddle products); then, above
// 16 384 points (where only the 24- and 32-value classes fit), the 32-value
// class first (at equal passes its schedules, radix-16 pairs without register
// spills, ran 17-35% faster: 64 ch x 100 freqs, power, L = 16 800 524 -> 339
// us, 18 432 475 -> 338, 19 200 492 -> 361, 20 160 533 -> 404), at or below
// it the 16- and 24-value classes before the 32-value one; then the least
// lane work Σ T ceil((L/R)/T) R (idle lanes of partly filled butterfly
// rounds count), then fewer values per thread.  Finally, among the plans
// tied with the first on passes, class and workgroup size, the one with the
// fewest passes of the three-factor composite radices 20, 21 and 24 goes
// first: those passes cost more per point than their lane work shows.
// Measured (64 ch, runtime-radix kernel; 61 freqs complex64 up to 14 000, 100
// freqs power above): 2400 [20, 15, 8] 40.1 -> [16, 15, 10] 35.3 us, 3072
// [24, 16, 8] 54.5 -> [16, 16, 12] 42.1, 14 000 [20, 14, 10, 5] 255 ->
// [14, 10, 10, 10] 219, 18 432 [24, 24, 8, 4] 406 -> [16, 12, 12, 8] 365, but
// 3528 [21, 21, 8] 57.7 -> [21, 14, 12] 62.6; where the alternative needs a
// larger workgroup it was no faster (1400: [14, 10, 10] at 192 threads 8%
// slower than [20, 14, 5] at 128, against 7% faster at 128).
static void ranked_plans(int L, std::vector<RadixPlan> &out)
{
    out.clear();
    std::vector<std::vector<int>> scheds;
    std::vector<int> cur;
    enum_schedules(L, 1 << 30, cur, scheds);
    struct Cand {
        RadixPlan rp;
        int64_t work;
    };
    std::vector<Cand> c;
    // 0 for the class taken first at equal passes: the 32-value class above
    // 16 384 points (where only it and the 24-value class fit), else the
    // 16- and 24-value classes
    auto class_rank = [L](int maxv) { return (maxv > 24) == (L > 16384) ? 0 : 1; };
    // passes of a composite radix with three prime factors (20, 21, 24)
    auto triple_radices = [](const RadixPlan &rp) {
        int n = 0;
        for (int i = 0; i < rp.n_pass; ++i)
            n += (rp.radix[i] == 20 || rp.radix[i] == 21 || rp.radix[i] == 24);
        return n;
    };
    for (const auto &f : scheds)
        for (int maxv : {16, 24, 32}) {
            const int T = schedule_threads(L, f, maxv);
            if (!T) continue;
            RadixPlan rp{};
            rp.L = L;
            rp.n_pass = (int)f.size();
            for (int i = 0; i < rp.n_pass; ++i) rp.radix[i] = f[i];
            rp.threads = T;
            rp.maxv = maxv;
            int64_t work = 0;
            for (int R : f) work += (int64_t)T * ((L / R + T - 1) / T) * R;
            c.push_back({rp, work});
        }
    std::stable_sort(c.begin(), c.end(), [&class_rank](const Cand &a, const Cand &b) {
        if (a.rp.n_pass != b.rp.n_pass) return a.rp.n_pass < b.rp.n_pass;
        if (class_rank(a.rp.maxv) != class_rank(b.rp.maxv))
            return class_rank(a.rp.maxv) < class_rank(b.rp.maxv);
        if (a.work != b.work) return a.work < b.work;
        return a.rp.maxv < b.rp.maxv;
    });
    // Among the plans tied with the first on passes, class and workgroup
    // size, the one with the fewest passes of the three-factor composites
    // goes first (the order is otherwise kept).
    if (!c.empty()) {
        const RadixPlan &h = c[0].rp;
        size_t best = 0;
        for (size_t i = 1; i < c.size(); ++i) {
            const RadixPlan &a = c[i].rp;
            if (a.n_pass != h.n_pass || class_rank(a.maxv) != class_rank(h.maxv) ||
                a.threads != h.threads)
                continue;
            if (triple_radices(a) < triple_radices(c[best].rp)) best = i;
        }
        std::rotate(c.begin(), c.begin() + (std::ptrdiff_t)best,
                    c.begin() + (std::ptrdiff_t)best + 1);
    }
    for (const Cand &x : c) out.push_back(x.rp);
}

bool make_radix_plan(int L, RadixPlan &rp)
{
    if (L == 1) {  // a single identity pass
        rp = RadixPlan{};
        rp.L = 1;
        rp.n_pass = 1;
        rp.radix[0] = 1;
        rp.threads = 64;
        rp.maxv = 16;
        return true;
    }
    std::vector<RadixPlan> ranked;
    ranked_plans(L, ranked);
    if (ranked.empty()) return false;
    rp = ranked.front();
    return true;
}

// Stored band of one frequency's spectrum: every signed bin whose value can
// reach 1e-12 of the spectrum's main Gaussian (and, for Morlet, of the
// kappa-weighted Gaussian at zero frequency), or of the GMW's peak.  For the
// GMW, sigma is the peak argument u_p, so s = sigma / (2 pi f) as for Morlet.
// GMW: the u > 0 where (u/u_p)^beta exp(u_p^gamma - u^gamma) = eps, one on
// each side of the peak u_p (the log ratio is concave with maximum 0 there),
// by bisection.
static void gmw_band(double beta, double gamma, double eps, double *ulo, double *uhi)
{
    const double up = std::pow(beta / gamma, 1.0 / gamma);
    const double target = std::log(eps);
    auto g = [&](double u) { return beta * std::log(u / up) - (std::pow(u, gamma) - std::pow(up, gamma)); };
    double a = up, b = up;
    while (g(a) > target && a > 1e-300) a *= 0.5;
    double lo = a, hi = up;
    for (int i = 0; i < 200; ++i) {
        const double m = 0.5 * (lo + hi);
        (g(m) > target ? hi : lo) = m;
    }
    *ulo = lo;
    while (g(b) > target) b *= 2.0;
    lo = up;
    hi = b;
    for (int i = 0; i < 200; ++i) {
        const double m = 0.5 * (lo + hi);
        (g(m) > target ? lo : hi) = m;
    }
    *uhi = hi;
}

BandDesc spectrum_band(int L, double sfreq, double f, double sigma, int wavelet, double beta,
                       double gamma)
{
    const double eps = 1e-12;
    const double xm = std::sqrt(2.0 * std::log(1.0 / eps));
    double ulo = sigma - xm, uhi = sigma + xm;
    if (wavelet == CWT_WAVELET_GMW) gmw_band(beta, gamma, eps, &ulo, &uhi);
    if (wavelet == CWT_WAVELET_MORLET) {
        const double kappa = std::exp(-0.5 * sigma * sigma);
        if (kappa > eps) {
            const double xk = std::sqrt(2.0 * std::log(kappa / eps));
            ulo = std::min(ulo, -xk);
        }
    }
    // u = s omega, omega = 2 pi sfreq b / L, s = sigma / (2 pi f)
    const double per_bin = sigma * sfreq / (f * (double)L);
    double blo = std::floor(ulo / per_bin) - 1.0;
    double bhi = std::ceil(uhi / per_bin) + 1.0;
    const double min_b = -(double)(L / 2);
    const double max_b = (double)((L + 1) / 2 - 1);
    blo = std::max(blo, min_b);
    bhi = std::min(bhi, max_b);
    BandDesc bd{};
    if (bhi < blo) {  // entirely outside the representable bins
        bd.lo = 0;
        bd.K = 0;
    } else {
        bd.lo = (int)blo;
        bd.K = (int)(bhi - blo) + 1;
    }
    return bd;
}

}  // namespace cwtrt

using namespace cwtrt;

// --------------------------------------------------------------- ABI --

static const double kDefaultBands[10] = {1.0, 4.0, 4.0, 8.0, 8.0, 13.0, 13.0, 30.0, 30.0, 100.0};

extern "C" int cwt_plan_opts_init(cwt_plan_opts *o)
{
    if (!o) return fail(CWT_E_INVALID, "cwt_plan_opts_init: opts is NULL");
    std::memset(o, 0, sizeof *o);
    o->wavelet = CWT_WAVELET_MORLET;
    o->gmw_beta = 17.5;
    o->gmw_gamma = 3.0;
    o->pad = CWT_PAD_SMOOTH7;
    o->out = CWT_OUT_COMPLEX64;
    o->precision = CWT_PREC_FP32;
    return CWT_OK;
}

extern "C" const char *cwt_last_error(void) { return g_last_error.c_str(); }

namespace cwtrt {

// Validation shared with other entry points: everything about the request
// that does not need the device.  Fills the host-side parts of the plan.
int validate_and_plan(cwt_plan &P, int64_t n, double sfreq, const double *freqs,
                      int32_t n_freqs, const double *n_cycles, double omega0,
                      const cwt_plan_opts *opts_in)
{
    cwt_plan_opts o;
    cwt_plan_opts_init(&o);
    if (opts_in) o = *opts_in;
    if (n < 1) return fail(CWT_E_INVALID, "n must be >= 1 (got %lld)", (long long)n);
    if (!std::isfinite(sfreq) || sfreq <= 0)
        return fail(CWT_E_INVALID, "sfreq must be finite and > 0");
    if (n_freqs < 1 || n_freqs > CWT_MAX_FREQS)
        return fail(CWT_E_INVALID, "n_freqs must be in [1, %d] (got %d)", CWT_MAX_FREQS, n_freqs);
    if (!freqs) return fail(CWT_E_INVALID, "freqs is NULL");
    if (o.wavelet != CWT_WAVELET_MORLET && o.wavelet != CWT_WAVELET_GABOR &&
        o.wavelet != CWT_WAVELET_GMW)
        return fail(CWT_E_INVALID, "unknown wavelet %d", o.wavelet);
    const bool gmw = o.wavelet == CWT_WAVELET_GMW;
    if (gmw && (!std::isfinite(o.gmw_beta) || o.gmw_beta <= 0 || !std::isfinite(o.gmw_gamma) ||
                o.gmw_gamma <= 0))
        return fail(CWT_E_INVALID, "GMW beta and gamma must be finite and > 0 (got %g, %g)",
                    o.gmw_beta, o.gmw_gamma);
    if (o.pad < CWT_PAD_SMOOTH7 || o.pad > CWT_PAD_LINEAR)
        return fail(CWT_E_INVALID, "unknown pad mode %d", o.pad);
    if (o.out < CWT_OUT_COMPLEX64 || o.out > CWT_OUT_BANDPOWER_F32)
        return fail(CWT_E_INVALID, "unknown output mode %d", o.out);
    if (o.precision < CWT_PREC_FP32 || o.precision > CWT_PREC_SPLIT_BF16)
        return fail(CWT_E_INVALID, "unknown precision %d", o.precision);
    if (o.max_channels < 0 || o.max_channels > ((int64_t)1 << 24))
        return fail(CWT_E_INVALID, "max_channels must be in [0, 2^24] (got %lld)",
                    (long long)o.max_channels);
    {
        const DevMem m{o.alloc, o.free, o.alloc_ctx};
        int rc = check_dev_mem(m);
        if (rc != CWT_OK) return rc;
        P.mem = m;
    }
    P.max_channels = o.max_channels;
    if (o.pad == CWT_PAD_EXPLICIT && o.explicit_len < n)
        return fail(CWT_E_INVALID, "explicit_len %lld < n %lld", (long long)o.explicit_len,
                    (long long)n);
    P.freqs.assign(freqs, freqs + n_freqs);
    P.sigmas.resize(n_freqs);
    for (int i = 0; i < n_freqs; ++i) {
        const double f = freqs[i];
        if (!std::isfinite(f) || f <= 0 || f >= 0.5 * sfreq)
            return fail(CWT_E_INVALID, "freqs[%d] = %g outside (0, sfreq/2 = %g)", i, f,
                        0.5 * sfreq);
        if (gmw) {
            P.sigmas[i] = std::pow(o.gmw_beta / o.gmw_gamma, 1.0 / o.gmw_gamma);
            continue;
        }
        const double s = n_cycles ? n_cycles[i] : omega0;
        if (!std::isfinite(s) || s <= 0)
            return fail(CWT_E_INVALID, "n_cycles/omega0 for freqs[%d] must be finite and > 0", i);
        P.sigmas[i] = s;
    }
    // bands
    P.band_of_freq.assign(n_freqs, -1);
    if (o.out == CWT_OUT_BANDPOWER_F32) {
        const double *edges = kDefaultBands;
        int nb = 5;
        if (o.n_bands != 0) {
            if (o.n_bands < 0 || o.n_bands > CWT_MAX_BANDS)
                return fail(CWT_E_INVALID, "n_bands must be in [1, %d]", CWT_MAX_BANDS);
            if (!o.band_edges) return fail(CWT_E_INVALID, "band_edges is NULL");
            edges = o.band_edges;
            nb = o.n_bands;
        }
        P.band_edges.assign(edges, edges + 2 * nb);
        P.grp_off.assign(1, 0);
        P.grp_freq.clear();
        for (int b = 0; b < nb; ++b) {
            const double lo = edges[2 * b], hi = edges[2 * b + 1];
            if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi))
                return fail(CWT_E_INVALID, "band %d has lo >= hi or non-finite edges", b);
            for (int i = 0; i < n_freqs; ++i) {
                const double f = freqs[i];
                const bool in = (f >= lo && f < hi) || (b == nb - 1 && f == hi);
                if (in) {
                    P.grp_freq.push_back(i);
                    if (P.band_of_freq[i] < 0) P.band_of_freq[i] = b;
                }
            }
            if ((int)P.grp_freq.size() == P.grp_off.back())
                return fail(CWT_E_INVALID, "band %d [%g, %g) owns no frequency", b, lo, hi);
            P.grp_off.push_back((int)P.grp_freq.size());
        }
        P.n_bands = nb;
    } else {
        P.n_bands = 0;
    }
    int64_t L;
    if (o.pad == CWT_PAD_LINEAR) {
        if (gmw)
            return fail(CWT_E_UNSUPPORTED,
                        "linear edge mode needs the Gaussian time support of Morlet / Gabor");
        // one-sided support of the widest wavelet: exp(-u^2/2) < 1e-12 beyond
        // u = sqrt(2 ln 1e12), u = t / s
        const double umax = std::sqrt(2.0 * std::log(1e12));
        double smax = 0;
        for (int i = 0; i < n_freqs; ++i)
            smax = std::max(smax, P.sigmas[i] / (2.0 * 3.14159265358979323846 * freqs[i]));
        const double S = std::ceil(umax * smax * sfreq) + 1.0;
        if (!(n + S <= (double)kMaxSegmentedLen))
            return fail(CWT_E_UNSUPPORTED, "linear edge mode needs L >= n + %.0f samples", S);
        L = pad_length(n + (int64_t)S, CWT_PAD_SMOOTH7, 0);
    } else {
        L = pad_length(n, o.pad, o.explicit_len);
    }
    P.L_full = L;
    P.n_seg = P.seg_B = P.seg_S = 0;
    if (L > CWT_MAX_LEN) {
        // Segmented: the wavelets' Gaussian time support bounds the samples
        // an output depends on (one side: envelope below 1e-8 of its peak
        // beyond u = sqrt(2 ln 1e8), u = t / s, s = sigma / (2 pi f)), so
        // segment transforms of length L reproduce the outputs that lie
        // further than that from their ends (overlap-save).
        if (gmw)
            return fail(CWT_E_UNSUPPORTED,
                        "padded length %lld above %d needs the Gaussian time support of "
                        "Morlet / Gabor", (long long)L, CWT_MAX_LEN);
        if (o.precision != CWT_PREC_FP32)
            return fail(CWT_E_UNSUPPORTED, "split precision is built for padded length 4096");
        if (L > kMaxSegmentedLen)
            return fail(CWT_E_UNSUPPORTED, "padded length %lld above %lld", (long long)L,
                        (long long)kMaxSegmentedLen);
        const double useg = std::sqrt(2.0 * std::log(1e8));
        double smax = 0;
        for (int i = 0; i < n_freqs; ++i)
            smax = std::max(smax, P.sigmas[i] / (2.0 * 3.14159265358979323846 * freqs[i]));
        const int64_t S = (int64_t)std::ceil(useg * smax * sfreq) + 1;
        const int64_t Lmax = kMaxSegmentLen;  // 7-smooth
        if (Lmax - 2 * S < Lmax / 8)
            return fail(CWT_E_UNSUPPORTED,
                        "padded length %lld above %d: the widest wavelet's support (2 x %lld "
                        "samples) leaves too little of a %lld-sample segment", (long long)L,
                        CWT_MAX_LEN, (long long)S, (long long)Lmax);
        const int64_t nseg = (n + (Lmax - 2 * S) - 1) / (Lmax - 2 * S);
        const int64_t B = (n + nseg - 1) / nseg;
        // The segment transform: the smallest 7-smooth length holding B + 2S,
        // or 16384 / 20480 when one of those holds it with at most 10% more
        // points: their schedules are radix-16 passes (16·16·16·4, 16·16·16·5),
        // which cost about 2.8 ns per output point at 64 channels x 100
        // frequencies against 3.3-4.8 for the other 7-smooth lengths from
        // 19 600 to 20 412 (20 160 = 24·21·20·2: 4.75).
        int64_t Ls = pad_length(B + 2 * S, CWT_PAD_SMOOTH7, 0);
        for (const int64_t fast : {(int64_t)16384, Lmax})
            if (fast >= B + 2 * S && 10 * fast <= 11 * Ls) {
                Ls = fast;
                break;
            }
        P.n_seg = (int)nseg;
        P.seg_B = (int)B;
        P.seg_S = (int)S;
        L = Ls;
    }
    if (!smooth7(L))
        return fail(CWT_E_UNSUPPORTED,
                    "padded length %lld has a prime factor above 7 (use SMOOTH7 or POW2)",
                    (long long)L);
    if (!make_radix_plan((int)L, P.rp))
        return fail(CWT_E_UNSUPPORTED, "no radix schedule fits length %lld in one workgroup",
                    (long long)L);
    P.n = n;
    P.sfreq = sfreq;
    P.L = (int)L;
    P.F = n_freqs;
    P.opts = o;
    P.opts.band_edges = nullptr;
    // spectrum bands
    P.bands.resize(n_freqs);
    int off = 0, maxK = 0;
    for (int i = 0; i < n_freqs; ++i) {
        BandDesc bd = spectrum_band(P.L, sfreq, freqs[i], P.sigmas[i], o.wavelet, o.gmw_beta,
                                    o.gmw_gamma);
        bd.off = off;
        off += bd.K;
        maxK = std::max(maxK, bd.K);
        P.bands[i] = bd;
    }
    P.total_bins = off;
    P.max_bins = maxK;
    // Register-resident kernels serve the lengths that have one, unless the
    // environment variable CWT_GENERIC_ONLY=1 asks for the generic kernel.
    const char *gen = std::getenv("CWT_GENERIC_ONLY");
    P.use_fixed = reg_main_available(P.L) && !(gen && gen[0] == '1') && P.n_seg == 0;
    set_chunks(P);
    const char *var = std::getenv("CWT_FIXED_VARIANT");
    P.variant = var ? std::atoi(var) : 1;
    apply_tuning_cache(P);
    return CWT_OK;
}

int check_device(int *dev_out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CWT_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", dev,
                    prop.gcnArchName);
    if (dev_out) *dev_out = dev;
    return CWT_OK;
}

template <class T>
static int dev_upload(cwt_plan &P, T **dst, const T *src, size_t count, hipStream_t s,
                      const char *what)
{
    *dst = nullptr;
    if (count == 0) return CWT_OK;
    int rc = plan_alloc(P, (void **)dst, count * sizeof(T), s, what);
    if (rc != CWT_OK) {
        *dst = nullptr;
        return rc;
    }
    if (src) {
        hipError_t e = hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        // src is owned by the plan and outlives the copy.
    }
    return CWT_OK;
}

// Band rows on the runtime-radix and split-precision kernels run a band's
// frequencies one after another in one workgroup; cut into chunks of at most
// a quarter of the largest band, the longest chain shrinks about 4-fold.
static void set_chunks(cwt_plan &P)
{
    P.n_chunks = 0;
    P.chunk_table.clear();
    if (P.opts.out != CWT_OUT_BANDPOWER_F32) return;
    if (P.use_fixed && P.opts.precision == CWT_PREC_FP32) return;  // sub-group rows instead
    int biggest = 0;
    for (int b = 0; b < P.n_bands; ++b)
        biggest = std::max(biggest, P.grp_off[b + 1] - P.grp_off[b]);
    const int g = std::max(1, (biggest + 3) / 4);
    std::vector<int> off{0}, first{0};
    for (int b = 0; b < P.n_bands; ++b) {
        const int lo = P.grp_off[b], hi = P.grp_off[b + 1];
        const int k = (hi - lo + g - 1) / g;  // chunks of this band, sizes differing by <= 1
        for (int j = 1; j <= k; ++j) off.push_back(lo + (int)((int64_t)(hi - lo) * j / k));
        first.push_back((int)off.size() - 1);
    }
    if ((int)off.size() - 1 == P.n_bands) return;  // one chunk per band: nothing gained
    P.n_chunks = (int)off.size() - 1;
    P.chunk_table = off;
    P.chunk_table.insert(P.chunk_table.end(), first.begin(), first.end());
}

// The band-power kernels take a band's frequencies one after another in one
// workgroup, so the band with the most frequencies is the longest job; its
// workgroups are launched first (longest-processing-time-first order), the
// order appended here after the offsets.  Ties keep the band order.
void set_group_table(cwt_plan &P)
{
    const int nb = (int)P.grp_off.size() - 1;
    P.grp_table = P.grp_off;
    std::vector<int> order(nb);
    for (int b = 0; b < nb; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&P](int a, int b) {
        return P.grp_off[a + 1] - P.grp_off[a] > P.grp_off[b + 1] - P.grp_off[b];
    });
    P.grp_table.insert(P.grp_table.end(), order.begin(), order.end());
}

void free_plan_device(cwt_plan &P, hipStream_t s)
{
    plan_free_all(P, s);
    if (P.ready) (void)hipEventDestroy(P.ready);
    P.ready = nullptr;
    P.own_ws = nullptr;
    P.own_ws_bytes = 0;
    P.d_freqs = P.d_sigmas = nullptr;
    P.d_band = nullptr;
    P.d_H = nullptr;
    P.d_Hc = nullptr;
    P.d_tw = nullptr;
    P.d_grp_freq = P.d_grp_off = nullptr;
    P.d_chunk = nullptr;
}

int upload_plan(cwt_plan &P, hipStream_t s)
{
    int rc;
    if ((rc = dev_upload(P, &P.d_freqs, P.freqs.data(), P.freqs.size(), s, "freqs"))) return rc;
    if ((rc = dev_upload(P, &P.d_sigmas, P.sigmas.data(), P.sigmas.size(), s, "sigmas")))
        return rc;
    if ((rc = dev_upload(P, &P.d_band, P.bands.data(), P.bands.size(), s, "bands"))) return rc;
    if ((rc = dev_upload<float>(P, &P.d_H, nullptr, std::max<int64_t>(P.total_bins, 1), s, "H")))
        return rc;
    if ((rc = dev_upload<float2>(P, &P.d_tw, nullptr, P.L, s, "twiddles"))) return rc;
    if (P.n_bands > 0) {
        if ((rc = dev_upload(P, &P.d_grp_freq, P.grp_freq.data(), P.grp_freq.size(), s,
                             "groups")))
            return rc;
        set_group_table(P);
        if ((rc = dev_upload(P, &P.d_grp_off, P.grp_table.data(), P.grp_table.size(), s,
                             "group offs")))
            return rc;
        if (P.n_chunks &&
            (rc = dev_upload(P, &P.d_chunk, P.chunk_table.data(), P.chunk_table.size(), s,
                             "band chunks")))
            return rc;
    }
    GenParams g{};
    g.sfreq = P.sfreq;
    g.L = P.L;
    g.F = P.F;
    g.wavelet = P.opts.wavelet;
    g.gmw_beta = P.opts.gmw_beta;
    g.gmw_gamma = P.opts.gmw_gamma;
    g.freqs = P.d_freqs;
    g.sigmas = P.d_sigmas;
    g.band = P.d_band;
    g.H = P.d_H;
    g.tw = P.d_tw;
    hipError_t e = launch_generate(g, P.max_bins, s);
    if (e != hipSuccess) return hip_fail(e, "generator launch");
    return CWT_OK;
}

int finish_plan(cwt_plan &P, hipStream_t s)
{
    if (P.max_channels > 0) {
        const size_t b = cwt_workspace_size(&P, P.max_channels);
        int rc = plan_alloc(P, &P.own_ws, b, s, "plan workspace");
        if (rc != CWT_OK) return rc;
        P.own_ws_bytes = b;
    }
    hipError_t e = hipEventCreateWithFlags(&P.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(P.ready, s);
    if (e != hipSuccess) return hip_fail(e, "plan ready event");
    return CWT_OK;
}

int wait_plan_ready(const cwt_plan &P, hipStream_t s)
{
    if (!P.ready) return CWT_OK;
    hipError_t e = hipEventQuery(P.ready);
    if (e == hipSuccess) return CWT_OK;  // tables already written
    if (e != hipErrorNotReady) return hip_fail(e, "hipEventQuery(plan ready)");
    e = hipStreamWaitEvent(s, P.ready, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(plan ready)");
    return CWT_OK;
}

size_t workspace_bytes(const cwt_plan &P, int64_t C)
{
    const int64_t Lh = P.L / 2 + 1;
    const int64_t rows = P.n_seg ? C * P.n_seg : C;
    size_t b = (size_t)rows * (size_t)Lh * sizeof(float2);
    b = (b + 255) & ~(size_t)255;
    // segmented plans: the gathered segment signals after the spectra
    if (P.n_seg) b += ((size_t)rows * (size_t)P.L * sizeof(float) + 255) & ~(size_t)255;
    // band chunks: their partial rows [C][n_chunks][n]
    if (P.n_chunks)
        b += ((size_t)C * (size_t)P.n_chunks * (size_t)P.n * sizeof(float) + 255) & ~(size_t)255;
    return b;
}

float *chunk_partials(const cwt_plan &P, int64_t C, void *ws)
{
    const int64_t rows = P.n_seg ? C * P.n_seg : C;
    size_t off = ((size_t)rows * (size_t)(P.L / 2 + 1) * sizeof(float2) + 255) & ~(size_t)255;
    if (P.n_seg) off += ((size_t)rows * (size_t)P.L * sizeof(float) + 255) & ~(size_t)255;
    return reinterpret_cast<float *>(static_cast<char *>(ws) + off);
}

int enqueue_chunk_reduce(const cwt_plan &P, int64_t C, const float *part, void *out,
                         hipStream_t s)
{
    ChunkReduceParams r{};
    r.part = part;
    r.out = static_cast<float *>(out);
    r.C = (int)C;
    r.n_chunks = P.n_chunks;
    r.n_bands = P.n_bands;
    r.N = (int)P.n;
    r.chunk_off = P.d_chunk;
    r.band_first = P.d_chunk + P.n_chunks + 1;
    hipError_t e = launch_chunk_reduce(r, s);
    if (e != hipSuccess) return hip_fail(e, "band chunk reduce launch");
    return CWT_OK;
}

int enqueue_forward(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride, void *ws,
                    hipStream_t s)
{
    if (C == 0) return CWT_OK;
    FwdParams fp{};
    fp.x = x;
    fp.C = (int)C;
    fp.N = (int)P.n;
    fp.x_stride = x_stride;
    if (P.n_seg) {
        // segmented: gather the segments (after the spectra in ws), then
        // transform them as C n_seg channels of L samples
        const int64_t rows = C * P.n_seg;
        const size_t spec = ((size_t)rows * (size_t)(P.L / 2 + 1) * sizeof(float2) + 255) &
                            ~(size_t)255;
        SegGatherParams g{};
        g.x = x;
        g.x_stride = x_stride;
        g.C = (int)C;
        g.N = (int)P.n;
        g.L_full = P.L_full;
        g.n_seg = P.n_seg;
        g.B = P.seg_B;
        g.S = P.seg_S;
        g.Ls = P.L;
        g.xs = reinterpret_cast<float *>(static_cast<char *>(ws) + spec);
        hipError_t e = launch_segment_gather(g, s);
        if (e != hipSuccess) return hip_fail(e, "segment gather launch");
        fp.x = g.xs;
        fp.C = (int)rows;
        fp.N = P.L;
        fp.x_stride = P.L;
    }
    fp.Xh = reinterpret_cast<float2 *>(ws);
    fp.Lh = P.L / 2 + 1;
    fp.tw = P.d_tw;
    fp.rp = P.rp;
    hipError_t e = P.use_fixed ? launch_forward_reg(fp, s) : launch_forward(fp, s);
    if (e != hipSuccess) return hip_fail(e, "forward FFT launch");
    return CWT_OK;
}

LaunchEvents next_launch_events(const cwt_plan &P)
{
    LaunchEvents ev;
    if (P.timing_used < P.timing_cap) {
        ev.start = P.timing_ev[2 * P.timing_used];
        ev.stop = P.timing_ev[2 * P.timing_used + 1];
        ++P.timing_used;
    }
    return ev;
}

int enqueue_transform(const cwt_plan &P, int64_t C, void *out, void *ws, hipStream_t s)
{
    if (C == 0) return CWT_OK;
    MainParams mp{};
    mp.Xh = reinterpret_cast<const float2 *>(ws);
    mp.Lh = P.L / 2 + 1;
    mp.H = P.d_H;
    mp.Hc = P.d_Hc;
    mp.band = P.d_band;
    mp.tw = P.d_tw;
    mp.out = out;
    mp.out_mode = P.opts.out;
    mp.N = (int)P.n;
    mp.F = P.F;
    mp.C = (int)C;
    mp.n_rows = (P.opts.out == CWT_OUT_BANDPOWER_F32) ? P.n_bands : P.F;
    mp.grp_freq = P.d_grp_freq;
    mp.grp_off = P.d_grp_off;
    mp.rp = P.rp;
    mp.variant = P.variant;
    if (P.n_seg) {
        mp.C = (int)(C * P.n_seg);
        mp.seg_n = P.n_seg;
        mp.seg_B = P.seg_B;
        mp.seg_S = P.seg_S;
    }
    float *part = nullptr;
    if (P.n_chunks) {  // chunk rows into the partial rows, then the band means
        part = chunk_partials(P, C, ws);
        mp.out = part;
        mp.n_rows = P.n_chunks;
        mp.grp_off = P.d_chunk;
    }
    const LaunchEvents ev = next_launch_events(P);
    hipError_t e = (P.use_fixed) ? launch_main_reg(mp, s, ev) : launch_main(mp, s, ev);
    if (e != hipSuccess) return hip_fail(e, "transform launch");
    if (part) return enqueue_chunk_reduce(P, C, part, out, s);
    return CWT_OK;
}

int enqueue_execute(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride, void *out,
                    void *ws, hipStream_t s)
{
    int rc = enqueue_forward(P, x, C, x_stride, ws, s);
    if (rc != CWT_OK) return rc;
    return enqueue_transform(P, C, out, ws, s);
}

}  // namespace cwtrt

extern "C" int cwt_plan_create(cwt_plan **out, int64_t n, double sfreq, const double *freqs,
                               int32_t n_freqs, const double *n_cycles, double omega0,
                               const cwt_plan_opts *opts, void *stream)
{
    clear_error();
    if (!out) return fail(CWT_E_INVALID, "cwt_plan_create: out is NULL");
    *out = nullptr;
    cwt_plan *P = new (std::nothrow) cwt_plan();
    if (!P) return fail(CWT_E_NOMEM, "host allocation of the plan failed");
    int rc = validate_and_plan(*P, n, sfreq, freqs, n_freqs, n_cycles, omega0, opts);
    if (rc == CWT_OK && P->opts.precision != CWT_PREC_FP32 && !split_precision_available())
        rc = fail(CWT_E_UNSUPPORTED, "split-precision MFMA path is not available in this build");
    if (rc == CWT_OK) rc = check_device(&P->device);
    if (rc == CWT_OK) rc = upload_plan(*P, (hipStream_t)stream);
    if (rc == CWT_OK && P->opts.precision != CWT_PREC_FP32)
        rc = prepare_split_precision(*P, (hipStream_t)stream);
    if (rc == CWT_OK) rc = finish_plan(*P, (hipStream_t)stream);
    if (rc != CWT_OK) {
        free_plan_device(*P, (hipStream_t)stream);
        delete P;
        return rc;
    }
    *out = P;
    return CWT_OK;
}

static void fill_desc(const cwt_plan *P, cwt_plan_desc *d)
{
    std::memset(d, 0, sizeof *d);
    d->n = P->n;
    d->L = P->n_seg ? P->L_full : P->L;
    d->n_segments = P->n_seg;
    d->segment_len = P->L;
    d->segment_outputs = P->n_seg ? P->seg_B : 0;
    d->segment_margin = P->n_seg ? P->seg_S : 0;
    d->band_chunks = P->n_chunks;
    d->n_freqs = P->F;
    d->n_bands = P->n_bands;
    d->out = P->opts.out;
    d->precision = P->opts.precision;
    d->wavelet = P->opts.wavelet;
    d->threads = P->rp.threads;
    d->n_passes = P->rp.n_pass;
    for (int i = 0; i < P->rp.n_pass && i < 16; ++i) d->radix[i] = P->rp.radix[i];
    if (P->use_fixed && P->opts.precision == CWT_PREC_FP32) {
        // the register-resident kernel's own schedule
        int r[16], th = 0;
        const int n = reg_schedule(P->L, P->opts.out == CWT_OUT_BANDPOWER_F32, r, &th);
        if (n > 0) {
            d->threads = th;
            d->n_passes = n;
            for (int i = 0; i < 16; ++i) d->radix[i] = (i < n) ? r[i] : 0;
        }
    }
    d->out_rows = (P->opts.out == CWT_OUT_BANDPOWER_F32) ? P->n_bands : P->F;
    d->out_elem_bytes = (P->opts.out == CWT_OUT_COMPLEX64) ? 8 : 4;
    d->spectrum_bins = P->total_bins;
    d->max_band_bins = P->max_bins;
    d->kernel = P->use_fixed ? 1 : 0;
    d->spectrum_complex = P->user ? 1 : 0;
    d->max_channels = P->max_channels;
    size_t bytes = 0;
    for (const auto &b : P->blocks) bytes += b.n;
    d->device_bytes = (int64_t)bytes;
}

extern "C" int cwt_plan_info(const cwt_plan *P, cwt_plan_desc *d)
{
    if (!P || !d) return fail(CWT_E_INVALID, "cwt_plan_info: NULL argument");
    fill_desc(P, d);
    return CWT_OK;
}

extern "C" int cwt_plan_describe(cwt_plan_desc *d, int64_t n, double sfreq, const double *freqs,
                                 int32_t n_freqs, const double *n_cycles, double omega0,
                                 const cwt_plan_opts *opts)
{
    clear_error();
    if (!d) return fail(CWT_E_INVALID, "cwt_plan_describe: desc is NULL");
    cwt_plan P;
    int rc = validate_and_plan(P, n, sfreq, freqs, n_freqs, n_cycles, omega0, opts);
    if (rc != CWT_OK) return rc;
    fill_desc(&P, d);
    return CWT_OK;
}

extern "C" int cwt_plan_band_of_freq(const cwt_plan *P, int32_t *bof)
{
    if (!P || !bof) return fail(CWT_E_INVALID, "cwt_plan_band_of_freq: NULL argument");
    for (int i = 0; i < P->F; ++i) bof[i] = P->band_of_freq[i];
    return CWT_OK;
}

extern "C" size_t cwt_workspace_size(const cwt_plan *P, int64_t C)
{
    if (!P || C < 0) return 0;
    return workspace_bytes(*P, C) + split_workspace_bytes(*P, C);
}

// Validation shared by cwt_execute and its two stages.  x_needed / out_needed
// say which device pointers the call uses.
int check_exec_args(const cwt_plan *P, const float *x, bool x_needed, int64_t C,
                           void *out, bool out_needed, void *ws, size_t ws_bytes)
{
    if (!P) return fail(CWT_E_INVALID, "plan is NULL");
    if (C < 0 || C > (int64_t)1 << 24) return fail(CWT_E_INVALID, "C out of range");
    if (C == 0) return CWT_OK;
    if (P->max_channels > 0 && C > P->max_channels)
        return fail(CWT_E_INVALID, "C = %lld exceeds the plan's max_channels %lld", (long long)C,
                    (long long)P->max_channels);
    if ((x_needed && !x) || (out_needed && !out))
        return fail(CWT_E_INVALID, "NULL device pointer");
    if (!ws)
        return fail(CWT_E_INVALID, "ws is NULL and the plan has no workspace of its own "
                                   "(create it with max_channels)");
    if (((uintptr_t)ws & 255) != 0) return fail(CWT_E_INVALID, "ws must be 256-byte aligned");
    if ((x_needed && ((uintptr_t)x & 3) != 0) || (out_needed && ((uintptr_t)out & 7) != 0))
        return fail(CWT_E_INVALID, "x must be 4-byte and out 8-byte aligned");
    const size_t need = cwt_workspace_size(P, C);
    if (ws_bytes < need)
        return fail(CWT_E_INVALID, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    const int64_t rows = ((P->opts.out == CWT_OUT_BANDPOWER_F32) ? P->n_bands : P->F) *
                         (P->n_seg ? P->n_seg : 1);
    if (C * rows > (int64_t)INT32_MAX)
        return fail(CWT_E_UNSUPPORTED, "C x rows exceeds the grid limit");
    // one workgroup per output row; a launch holds fewer than 2^32 work-items
    // (the forward-FFT workgroups of a pipelined launch included)
    const int64_t threads = (P->opts.precision != CWT_PREC_FP32) ? 256
                            : P->use_fixed                       ? reg_row_threads(P->L)
                                                                 : P->rp.threads;
    const int64_t fwd_blocks = (C * (P->n_seg ? P->n_seg : 1) + 1) / 2;
    if ((C * rows + fwd_blocks) * threads >= ((int64_t)1 << 32))
        return fail(CWT_E_UNSUPPORTED,
                    "%lld channels x %lld rows x %lld threads exceed one launch; split C",
                    (long long)C, (long long)rows, (long long)threads);
    return CWT_OK;
}

// A NULL workspace means the plan's own (plans created with max_channels).
static void resolve_ws(const cwt_plan *P, void *&ws, size_t &ws_bytes)
{
    if (P && !ws && ws_bytes == 0 && P->own_ws) {
        ws = P->own_ws;
        ws_bytes = P->own_ws_bytes;
    }
}

extern "C" int cwt_execute(const cwt_plan *P, const float *x, int64_t C, void *out, void *ws,
                           size_t ws_bytes, void *stream)
{
    clear_error();
    resolve_ws(P, ws, ws_bytes);
    int rc = check_exec_args(P, x, true, C, out, true, ws, ws_bytes);
    if (rc != CWT_OK || C == 0) return rc;
    if (P->opts.precision != CWT_PREC_FP32)
        return enqueue_execute_split(*P, x, C, P->n, out, ws, (hipStream_t)stream);
    return enqueue_execute(*P, x, C, P->n, out, ws, (hipStream_t)stream);
}

extern "C" int cwt_forward_spectra(const cwt_plan *P, const float *x, int64_t C, void *ws,
                                   size_t ws_bytes, void *stream)
{
    clear_error();
    resolve_ws(P, ws, ws_bytes);
    int rc = check_exec_args(P, x, true, C, nullptr, false, ws, ws_bytes);
    if (rc != CWT_OK || C == 0) return rc;
    if (P->opts.precision != CWT_PREC_FP32)
        return enqueue_forward_split(*P, x, C, P->n, ws, (hipStream_t)stream);
    return enqueue_forward(*P, x, C, P->n, ws, (hipStream_t)stream);
}

extern "C" int cwt_transform_spectra(const cwt_plan *P, int64_t C, void *out, void *ws,
                                     size_t ws_bytes, void *stream)
{
    clear_error();
    resolve_ws(P, ws, ws_bytes);
    int rc = check_exec_args(P, nullptr, false, C, out, true, ws, ws_bytes);
    if (rc != CWT_OK || C == 0) return rc;
    if (P->opts.precision != CWT_PREC_FP32)
        return enqueue_transform_split(*P, C, out, ws, (hipStream_t)stream);
    return enqueue_transform(*P, C, out, ws, (hipStream_t)stream);
}

extern "C" int cwt_plan_copy_tables(const cwt_plan *P, float *H_host, int32_t *band_host,
                                    float *tw_host, void *stream)
{
    if (!P) return fail(CWT_E_INVALID, "cwt_plan_copy_tables: plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (H_host && P->total_bins > 0) {
        e = P->user ? hipMemcpyAsync(H_host, P->d_Hc, P->total_bins * sizeof(float2),
                                     hipMemcpyDeviceToHost, s)
                    : hipMemcpyAsync(H_host, P->d_H, P->total_bins * sizeof(float),
                                     hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(e, "copy H");
    }
    if (tw_host) {
        e = hipMemcpyAsync(tw_host, P->d_tw, (size_t)P->L * sizeof(float2),
                           hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail(e, "copy twiddles");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (band_host)
        for (int i = 0; i < P->F; ++i) {
            band_host[3 * i] = P->bands[i].lo;
            band_host[3 * i + 1] = P->bands[i].K;
            band_host[3 * i + 2] = P->bands[i].off;
        }
    return CWT_OK;
}

extern "C" int cwt_plan_timing_start(cwt_plan *P, int32_t max_launches)
{
    clear_error();
    if (!P) return fail(CWT_E_INVALID, "cwt_plan_timing_start: plan is NULL");
    if (max_launches < 0 || max_launches > 65536)
        return fail(CWT_E_INVALID, "cwt_plan_timing_start: max_launches %d outside [0, 65536]",
                    (int)max_launches);
    P->timing_cap = 0;
    P->timing_used = 0;
    hipError_t e = hipSetDevice(P->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice in cwt_plan_timing_start");
    while ((int)P->timing_ev.size() < 2 * max_launches) {
        // Timing-only events: no system-scope fence when they complete, so
        // recording them adds no cache write-back to the timed stream.
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate in cwt_plan_timing_start");
        P->timing_ev.push_back(ev);
    }
    P->timing_cap = max_launches;
    return CWT_OK;
}

extern "C" int cwt_plan_timing_stop(cwt_plan *P, float *ms_host, int32_t max, int32_t *n_out)
{
    clear_error();
    if (!P) return fail(CWT_E_INVALID, "cwt_plan_timing_stop: plan is NULL");
    if (max < 0 || (max > 0 && !ms_host))
        return fail(CWT_E_INVALID, "cwt_plan_timing_stop: max %d with ms_host %p", (int)max,
                    (void *)ms_host);
    const int used = P->timing_used;
    P->timing_cap = 0;
    P->timing_used = 0;
    if (n_out) *n_out = used;
    for (int i = 0; i < used; ++i) {
        hipError_t e = hipEventSynchronize(P->timing_ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize in cwt_plan_timing_stop");
        if (i >= max) continue;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, P->timing_ev[2 * i], P->timing_ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime in cwt_plan_timing_stop");
        ms_host[i] = ms;
    }
    return CWT_OK;
}

extern "C" int cwt_plan_destroy(cwt_plan *P, void *stream)
{
    if (!P) return CWT_OK;
    clear_error();
    // Stream-ordered: the frees are enqueued on `stream` behind the work
    // already there; nothing here waits for the device.
    release_split_precision(*P);
    free_plan_device(*P, (hipStream_t)stream);
    for (hipEvent_t ev : P->timing_ev) (void)hipEventDestroy(ev);
    delete P;
    return CWT_OK;
}
