// cwt_plan_create_from_wavelets: plans whose wavelet spectra come from
// sampled time-domain wavelets (the two-FFT form) instead of a closed form.
//
// The spectra are computed on the GPU in FP64 (a direct DFT of each placed
// wavelet over an FP64 root table), rounded once, copied to the host, where
// each frequency's stored band — the shortest cyclic run of bins holding
// every bin of at least 1e-12 of its peak magnitude — is found and packed;
// the packed complex spectra and the band table go back to the device.  The
// transform kernels multiply by the complex spectrum when the plan has one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "cwt_internal.hpp"

using namespace cwtk;
using namespace cwtrt;

namespace {

// Shortest cyclic run of [0, L) covering every index with mag >= thr:
// the complement of the longest cyclic gap between such indices.
void cyclic_band(const std::vector<double> &mag, double thr, int &lo, int &K)
{
    const int L = (int)mag.size();
    std::vector<int> on;
    for (int b = 0; b < L; ++b)
        if (mag[b] >= thr) on.push_back(b);
    if (on.empty()) {
        lo = 0;
        K = 0;
        return;
    }
    const int k = (int)on.size();
    int best_gap = -1, best_i = 0;
    for (int i = 0; i < k; ++i) {
        const int nxt = (i + 1 < k) ? on[i + 1] : on[0] + L;
        const int gap = nxt - on[i] - 1;
        if (gap > best_gap) {
            best_gap = gap;
            best_i = i;
        }
    }
    lo = on[(best_i + 1) % k];
    K = L - best_gap;
}

// Device copy of count values of src (or uninitialised when src is NULL):
// a plan-owned block when `owned`, else a temporary the caller frees.
template <class T>
int upload(cwt_plan &P, bool owned, T **dst, const T *src, size_t count, hipStream_t s,
           const char *what)
{
    *dst = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void *p = nullptr;
    int rc = owned ? plan_alloc(P, &p, bytes, s, what) : dev_alloc(P.mem, &p, bytes, s, what);
    if (rc != CWT_OK) return rc;
    *dst = static_cast<T *>(p);
    if (src && count) {
        hipError_t e = hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    return CWT_OK;
}

int build_user_plan(cwt_plan &P, const float *wavelets, int64_t w_len, hipStream_t s)
{
    const int F = P.F, L = P.L, wl = (int)w_len, c = wl / 2;
    // device spectra, dense [F][L] (temporaries, freed in stream order below)
    float2 *d_w = nullptr, *d_Hd = nullptr;
    double2 *d_roots = nullptr;
    int rc = upload(P, false, &d_w, reinterpret_cast<const float2 *>(wavelets), (size_t)F * wl,
                    s, "wavelet upload");
    if (rc == CWT_OK) rc = upload<double2>(P, false, &d_roots, nullptr, (size_t)L, s, "root table");
    if (rc == CWT_OK)
        rc = upload<float2>(P, false, &d_Hd, nullptr, (size_t)F * L, s, "dense spectra");
    std::vector<float2> Hd((size_t)F * L);
    if (rc == CWT_OK) {
        hipError_t e = launch_user_spectra(d_w, F, wl, c, L, d_roots, d_Hd, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(Hd.data(), d_Hd, Hd.size() * sizeof(float2), hipMemcpyDeviceToHost,
                               s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "sampled-wavelet spectra");
    }
    dev_free(P.mem, d_w, std::max<size_t>((size_t)F * wl, 1) * sizeof(float2), s);
    dev_free(P.mem, d_roots, std::max<size_t>((size_t)L, 1) * sizeof(double2), s);
    dev_free(P.mem, d_Hd, std::max<size_t>((size_t)F * L, 1) * sizeof(float2), s);
    if (rc != CWT_OK) return rc;

    // bands and packing
    P.bands.assign(F, BandDesc{});
    std::vector<float2> packed;
    std::vector<double> mag(L);
    int maxK = 0;
    for (int f = 0; f < F; ++f) {
        double peak = 0;
        for (int b = 0; b < L; ++b) {
            const float2 h = Hd[(size_t)f * L + b];
            mag[b] = std::hypot((double)h.x, (double)h.y);
            peak = std::max(peak, mag[b]);
        }
        int lo = 0, K = 0;
        if (peak > 0) cyclic_band(mag, 1e-12 * peak, lo, K);
        BandDesc &bd = P.bands[f];
        bd.lo = lo;
        bd.K = K;
        bd.off = (int)packed.size();
        for (int k = 0; k < K; ++k) packed.push_back(Hd[(size_t)f * L + (lo + k) % L]);
        maxK = std::max(maxK, K);
    }
    P.total_bins = (int)packed.size();
    P.max_bins = maxK;

    // device tables: bands, packed complex spectra, twiddles, band groups
    rc = upload(P, true, &P.d_freqs, P.freqs.data(), P.freqs.size(), s, "freqs");
    if (rc == CWT_OK) rc = upload(P, true, &P.d_band, P.bands.data(), P.bands.size(), s, "bands");
    if (rc == CWT_OK)
        rc = upload(P, true, &P.d_Hc, packed.data(), packed.size(), s, "complex spectra");
    if (rc == CWT_OK) rc = upload<float2>(P, true, &P.d_tw, nullptr, (size_t)L, s, "twiddles");
    if (rc == CWT_OK && P.n_bands > 0) {
        rc = upload(P, true, &P.d_grp_freq, P.grp_freq.data(), P.grp_freq.size(), s, "groups");
        set_group_table(P);
        if (rc == CWT_OK)
            rc = upload(P, true, &P.d_grp_off, P.grp_table.data(), P.grp_table.size(), s,
                        "group offs");
        if (rc == CWT_OK && P.n_chunks)
            rc = upload(P, true, &P.d_chunk, P.chunk_table.data(), P.chunk_table.size(), s,
                        "band chunks");
    }
    if (rc != CWT_OK) return rc;
    GenParams g{};  // twiddles only (no closed-form spectra)
    g.sfreq = P.sfreq;
    g.L = L;
    g.F = 0;
    g.tw = P.d_tw;
    hipError_t e = launch_generate(g, 1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the packed host tables are freed next
    if (e != hipSuccess) return hip_fail(e, "twiddle generation");
    P.user = true;
    return CWT_OK;
}

}  // namespace

extern "C" int cwt_plan_create_from_wavelets(cwt_plan **out, int64_t n, double sfreq,
                                             const double *freqs, int32_t n_freqs,
                                             const float *wavelets, int64_t w_len,
                                             const cwt_plan_opts *opts, void *stream)
{
    clear_error();
    if (!out) return fail(CWT_E_INVALID, "cwt_plan_create_from_wavelets: out is NULL");
    *out = nullptr;
    if (!wavelets) return fail(CWT_E_INVALID, "wavelets is NULL");
    if (w_len < 1 || w_len > CWT_MAX_LEN)
        return fail(CWT_E_INVALID, "w_len %lld outside [1, %d]", (long long)w_len, CWT_MAX_LEN);
    if (n_freqs < 1 || n_freqs > CWT_MAX_FREQS)
        return fail(CWT_E_INVALID, "n_freqs must be in [1, %d] (got %d)", CWT_MAX_FREQS, n_freqs);
    for (int64_t i = 0; i < 2 * (int64_t)n_freqs * w_len; ++i)
        if (!std::isfinite(wavelets[i]))
            return fail(CWT_E_INVALID, "wavelet sample %lld is not finite", (long long)(i / 2));
    cwt_plan_opts o;
    cwt_plan_opts_init(&o);
    if (opts) o = *opts;
    o.wavelet = CWT_WAVELET_MORLET;  // not used; keeps the closed-form checks quiet
    if (o.precision != CWT_PREC_FP32)
        return fail(CWT_E_UNSUPPORTED, "plans from sampled wavelets run the FP32 path");
    const bool linear = o.pad == CWT_PAD_LINEAR;
    if (linear) {
        if (n < 1) return fail(CWT_E_INVALID, "n must be >= 1 (got %lld)", (long long)n);
        const int64_t c = w_len / 2;
        const int64_t S = std::max(c, w_len - 1 - c) + 1;
        if (n + S > CWT_MAX_LEN)
            return fail(CWT_E_UNSUPPORTED, "linear edge mode needs L >= n + %lld, above %d",
                        (long long)S, CWT_MAX_LEN);
        o.pad = CWT_PAD_EXPLICIT;
        o.explicit_len = pad_length(n + S, CWT_PAD_SMOOTH7, 0);
    }
    cwt_plan *P = new (std::nothrow) cwt_plan();
    if (!P) return fail(CWT_E_NOMEM, "host allocation of the plan failed");
    std::vector<double> ones((size_t)n_freqs, 1.0);
    int rc = validate_and_plan(*P, n, sfreq, freqs, n_freqs, ones.data(), 0.0, &o);
    if (rc == CWT_OK && w_len > P->L)
        rc = fail(CWT_E_INVALID, "w_len %lld exceeds the padded length %d", (long long)w_len,
                  P->L);
    if (linear) P->opts.pad = CWT_PAD_LINEAR;
    if (rc == CWT_OK) rc = check_device(&P->device);
    if (rc == CWT_OK) rc = build_user_plan(*P, wavelets, w_len, (hipStream_t)stream);
    if (rc == CWT_OK) rc = finish_plan(*P, (hipStream_t)stream);
    if (rc != CWT_OK) {
        free_plan_device(*P, (hipStream_t)stream);
        delete P;
        return rc;
    }
    *out = P;
    return CWT_OK;
}
