// HIP kernels of the plain FP32 CWT path for gfx950.
//
//   k_generate : FP64 wavelet spectra (Morlet / Gabor / generalized Morse
//                Fourier-domain equations, evaluated at s * omega_b) and the
//                FP64 twiddle table, each rounded once to FP32.
//   k_forward  : forward real FFT of two channels per workgroup (packed as
//                one complex transform), half spectra to the workspace.
//   k_main     : per (channel, frequency) or (channel, band): spectral
//                multiply over the stored band of the wavelet spectrum ->
//                LDS-resident inverse Stockham FFT -> crop to n samples ->
//                complex64 / |W|^2 / band-mean store, natural order.
#include <type_traits>

#include "cwt_kernels.hpp"
#include "fft_core.hpp"

namespace cwtk {

// ------------------------------------------------------------ generators --

__global__ void k_generate(GenParams p)
{
    const int f = blockIdx.y;
    if (f < p.F) {
        const BandDesc bd = p.band[f];
        const int k = blockIdx.x * blockDim.x + threadIdx.x;
        if (k >= bd.K) return;
        const double PI = 3.14159265358979323846;
        const double sigma = p.sigmas[f];
        const double s = sigma / (2.0 * PI * p.freqs[f]);
        double kappa = 0.0, c = 1.0;
        if (p.wavelet == 0) {
            kappa = exp(-0.5 * sigma * sigma);
            c = 1.0 / sqrt(1.0 + exp(-sigma * sigma) - 2.0 * exp(-0.75 * sigma * sigma));
        }
        const int bt = bd.lo + k;  // signed bin
        const double u = s * (2.0 * PI * p.sfreq * (double)bt / (double)p.L);
        double psi;
        if (p.wavelet == 2) {
            // generalized Morse: alpha u^beta exp(-u^gamma) for u > 0, zero
            // otherwise; alpha = 2 (e gamma / beta)^(beta / gamma), in logs
            const double be = p.gmw_beta, ga = p.gmw_gamma;
            const double log_alpha = log(2.0) + (be / ga) * (1.0 + log(ga / be));
            psi = (u > 0.0) ? exp(log_alpha + be * log(u) - pow(u, ga)) : 0.0;
        } else {
            const double du = sigma - u;
            psi = c * pow(PI, -0.25) * (exp(-0.5 * du * du) - kappa * exp(-0.5 * u * u));
        }
        const double h = sqrt(2.0 * PI * s * p.sfreq) * psi / (double)p.L;
        p.H[bd.off + k] = (float)h;
    } else {
        // twiddles exp(+2 pi i m / L)
        for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < p.L; m += gridDim.x * blockDim.x) {
            double sn, cs;
            sincospi(2.0 * (double)m / (double)p.L, &sn, &cs);
            p.tw[m] = make_float2((float)cs, (float)sn);
        }
    }
}

hipError_t launch_generate(const GenParams &p, int max_bins, hipStream_t s)
{
    int bx = (max_bins + 255) / 256;
    int bt = (p.L + 255) / 256;
    if (bt > bx) bx = bt;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL(k_generate, dim3(bx, p.F + 1), dim3(256), 0, s, p);
    return hipGetLastError();
}

// ------------------------------------------------ sampled-wavelet spectra --

__global__ void k_roots64(int L, double2 *roots)
{
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < L; m += gridDim.x * blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * (double)m / (double)L, &sn, &cs);
        roots[m] = make_double2(cs, sn);  // exp(-2 pi i m / L)
    }
}

// Bin b of frequency f: the root index b (j - c) mod L advances by b per
// sample, so only the first needs a division.
__global__ void k_user_spectra(const float2 *w, int wl, int c, int L, const double2 *roots,
                               float2 *Hd)
{
    const int f = blockIdx.y;
    const float2 *wf = w + (int64_t)f * wl;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < L; b += gridDim.x * blockDim.x) {
        int m = (int)(((int64_t)b * (int64_t)((L - c % L) % L)) % L);  // b (0 - c) mod L
        double re = 0.0, im = 0.0;
        for (int j = 0; j < wl; ++j) {
            const double2 r = roots[m];
            const double wr = wf[j].x, wi = wf[j].y;
            re += wr * r.x - wi * r.y;
            im += wr * r.y + wi * r.x;
            m += b;
            if (m >= L) m -= L;
        }
        Hd[(int64_t)f * L + b] = make_float2((float)(re / L), (float)(im / L));
    }
}

hipError_t launch_user_spectra(const float2 *w, int F, int wl, int c, int L, double2 *roots,
                               float2 *Hd, hipStream_t s)
{
    hipLaunchKernelGGL(k_roots64, dim3((L + 255) / 256), dim3(256), 0, s, L, roots);
    hipLaunchKernelGGL(k_user_spectra, dim3((L + 255) / 256, F), dim3(256), 0, s, w, wl, c, L,
                       roots, Hd);
    return hipGetLastError();
}

// --------------------------------------------------------- forward FFT --

// Most threads per workgroup of a runtime-radix kernel class, by the most
// values a thread holds in a pass: 1024 for the 16- and 24-value classes,
// 768 for the 32-value one, which at 12 waves per workgroup may use up to
// 168 registers per lane (the 24-value class, held to 128 by its 1024-thread
// bound, spills a few).
template <int MAXV>
struct GenThreads {
    static constexpr int value = MAXV > 24 ? 768 : 1024;
};

// Calls f with the compiled values-per-thread class of a plan (16, 24 or 32)
// as a compile-time constant.
template <class F>
static hipError_t with_maxv(int maxv, F &&f)
{
    if (maxv <= 16) return f(std::integral_constant<int, 16>{});
    if (maxv <= 24) return f(std::integral_constant<int, 24>{});
    return f(std::integral_constant<int, 32>{});
}

// Forward transform of channel pair `pair` (channels 2 pair, 2 pair + 1).
template <int MAXV, class P = FwdParams>
__device__ __forceinline__ void forward_task(const P &p, int pair)
{
    extern __shared__ cf lds[];
    const int L = p.rp.L, T = blockDim.x, tid = threadIdx.x;
    const int c0 = 2 * pair;
    const bool has1 = (c0 + 1) < p.C;
    const float *x0 = p.x + (int64_t)c0 * p.x_stride;
    const float *x1 = p.x + (int64_t)(c0 + 1) * p.x_stride;
    const gptr<cf> tw = as_global(reinterpret_cast<const cf *>(p.tw));
    const gptr<float> x0g = as_global(x0), x1g = as_global(x1);
    const int N = p.N;

    auto lds_load = [](int idx) -> cf { return lds[idx]; };
    auto lds_store = [](int, int idx, cf v) { lds[idx] = v; };
    auto lds_load_sw = [](int idx) -> cf { return lds[first_pass_slot(idx)]; };
    auto lds_store_sw = [](int, int idx, cf v) { lds[first_pass_slot(idx)] = v; };
    const bool swz = p.rp.n_pass >= 2 && (p.rp.radix[0] & 1) == 0;
    auto in_load = [=](int idx) -> cf {
        cf z = mk(0.f, 0.f);
        if (idx < N) {
            z.x = x0g[idx];
            if (has1) z.y = x1g[idx];
        }
        return z;
    };

    int Ns = 1;
    for (int i = 0; i < p.rp.n_pass; ++i) {
        const int R = p.rp.radix[i];
        if (i == 0 && swz)
            stockham_pass_rt<-1, MAXV, true>(R, L, Ns, T, tid, tw, in_load, lds_store_sw);
        else if (i == 0)
            stockham_pass_rt<-1, MAXV, true>(R, L, Ns, T, tid, tw, in_load, lds_store);
        else if (i == 1 && swz)
            stockham_pass_rt<-1, MAXV, true>(R, L, Ns, T, tid, tw, lds_load_sw, lds_store);
        else
            stockham_pass_rt<-1, MAXV, true>(R, L, Ns, T, tid, tw, lds_load, lds_store);
        __syncthreads();
        Ns *= R;
    }
    // Separate the two real channels: X0 = (Z[b] + conj Z[-b]) / 2,
    // X1 = (Z[b] - conj Z[-b]) / (2 i).
    float2 *X0 = p.Xh + (int64_t)c0 * p.Lh;
    float2 *X1 = X0 + p.Lh;
    for (int b = tid; b < p.Lh; b += T) {
        const cf z = lds[b];
        const int nb = (b == 0) ? 0 : L - b;
        const cf zc = mk(lds[nb].x, -lds[nb].y);
        const cf s = add(z, zc), d = sub(z, zc);
        X0[b] = make_float2(0.5f * s.x, 0.5f * s.y);
        if (has1) X1[b] = make_float2(0.5f * d.y, -0.5f * d.x);
    }
}

template <int MAXV>
__global__ void __launch_bounds__(GenThreads<MAXV>::value) k_forward(FwdParams p)
{
    forward_task<MAXV>(p, blockIdx.x);
}

static void set_lds_limit(const void *fn, size_t bytes)
{
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_forward(const FwdParams &p, hipStream_t s)
{
    const int blocks = (p.C + 1) / 2;
    const size_t lds = generic_lds_bytes(p.rp.L);
    return with_maxv(p.rp.maxv, [&](auto mv) {
        constexpr int M = decltype(mv)::value;
        // the kernels of a class are compiled for at most its workgroup size
        if (p.rp.threads > GenThreads<M>::value) return hipErrorInvalidConfiguration;
        set_lds_limit((const void *)k_forward<M>, lds);
        hipLaunchKernelGGL(k_forward<M>, dim3(blocks), dim3(p.rp.threads), lds, s, p);
        return hipGetLastError();
    });
}

// --------------------------------------------------------- main kernel --

// a / d for 0 <= a < 2^31 and d >= 1, from a double reciprocal inv = 1/d:
// the product is within one of the quotient, and one step corrects it.
__device__ __forceinline__ int idiv(int a, int d, double inv)
{
    int q = (int)((double)a * inv);
    const int r = a - q * d;
    if (r < 0)
        --q;
    else if (r >= d)
        ++q;
    return q;
}

// Leading passes made trivial by a narrow band.  After the passes of a
// Stockham prefix with radix product Ns0, element J Ns0 + k of the buffer
// (J < M = L / Ns0, k < Ns0) is the Ns0-point inverse DFT, over m, of the
// spectrum at bins J + m M.  When the stored band spans at most M cyclically
// consecutive bins, each such group holds at most one band bin b = J + m0 M,
// and the element is y_b exp(2 pi i m0 k / Ns0): one complex product in place
// of those passes.  Item g = J (Ns0 / R0) + c covers k = c R0 + kr (kr < R0),
// which sit at elements R0 g + kr, the first pass's own output positions, so
// the first-pass slot map keeps the writes conflict-free as there.  lo_u is
// the band's first bin in [0, L).
template <int R0, bool SW>
__device__ __attribute__((noinline)) void band_prologue(gptr<cf> X, gptr<float> Hf,
                                                        gptr<cf> Hcf, int lo_u, int K, int L,
                                                        int Lh, int Ns0, int T, int tid,
                                                        gptr<cf> tw)
{
    extern __shared__ cf lds[];
    const int M = L / Ns0, nc = Ns0 / R0, n_items = L / R0;
    const int lom = lo_u % M;
    const double inv_nc = 1.0 / nc, inv_M = 1.0 / M, inv_Ns = 1.0 / Ns0;
    for (int g = tid; g < n_items; g += T) {
        const int J = idiv(g, nc, inv_nc);
        const int c = g - J * nc;
        int o = J - lom;
        if (o < 0) o += M;
        const int base = R0 * g;
        if (o < K) {
            int b = lo_u + o;
            if (b >= L) b -= L;
            cf xv;
            if (b < Lh) {
                xv = load_cf(X + b);
            } else {
                xv = load_cf(X + (L - b));
                xv.y = -xv.y;
            }
            cf y = Hcf ? mul(xv, load_cf(Hcf + o)) : scale(xv, Hf[o]);
            const int m0 = idiv(b - J, M, inv_M);  // b - J = m0 M exactly
            const int a = m0 * c * R0;             // < Ns0^2 < 2^31
            const int e = a - idiv(a, Ns0, inv_Ns) * Ns0;
            y = mul(y, load_cf(tw + e * M));
            cf w[R0];
            twiddle_powers<R0>(load_cf(tw + m0 * M), w);
#pragma unroll
            for (int kr = 0; kr < R0; ++kr) {
                const int i = base + kr;
                lds[SW ? first_pass_slot(i) : i] = kr == 0 ? y : mul(y, w[kr]);
            }
        } else {
#pragma unroll
            for (int kr = 0; kr < R0; ++kr) {
                const int i = base + kr;
                lds[SW ? first_pass_slot(i) : i] = mk(0.f, 0.f);
            }
        }
    }
}

__device__ __forceinline__ void band_prologue_rt(int R0, bool sw, gptr<cf> X, gptr<float> Hf,
                                                 gptr<cf> Hcf, int lo_u, int K, int L, int Lh,
                                                 int Ns0, int T, int tid, gptr<cf> tw)
{
    switch (R0) {
    case 16:
        if (sw) band_prologue<16, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<16, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 8:
        if (sw) band_prologue<8, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<8, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 4:
        if (sw) band_prologue<4, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<4, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 2:
        if (sw) band_prologue<2, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<2, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 12:
        if (sw) band_prologue<12, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<12, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 14:
        if (sw) band_prologue<14, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<14, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 10:
        if (sw) band_prologue<10, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<10, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 6:
        if (sw) band_prologue<6, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<6, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 15: band_prologue<15, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw); break;
    case 20:
        if (sw) band_prologue<20, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<20, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 24:
        if (sw) band_prologue<24, true>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        else band_prologue<24, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw);
        break;
    case 21: band_prologue<21, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw); break;
    case 9: band_prologue<9, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw); break;
    case 7: band_prologue<7, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw); break;
    case 5: band_prologue<5, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw); break;
    case 3: band_prologue<3, false>(X, Hf, Hcf, lo_u, K, L, Lh, Ns0, T, tid, tw); break;
    default: break;
    }
}

// Output row `row` of channel c: one frequency (complex / power) or one
// band (band power, accumulated over the band's frequencies).
template <int MAXV, int MODE, class P = MainParams>
__device__ __forceinline__ void main_task(const P &p, int c, int row)
{
    extern __shared__ cf lds[];
    const int L = p.rp.L, T = blockDim.x, tid = threadIdx.x;
    const int N = p.N, Lh = p.Lh;
    const int n_pass = p.rp.n_pass;
    const gptr<cf> tw = as_global(reinterpret_cast<const cf *>(p.tw));
    int qb, qe;
    if (MODE == kOutBand) {
        qb = p.grp_off[row];
        qe = p.grp_off[row + 1];
    } else {
        qb = row;
        qe = row + 1;
    }
    const gptr<cf> X = as_global(reinterpret_cast<const cf *>(p.Xh) + (int64_t)c * Lh);

    // Output channel and the samples this row stores: [0, N), or for a
    // segment of a segmented plan its middle seg_B samples, shifted to the
    // segment's place in the output row.
    int oc = c, t_first = 0, t_count = N;
    int64_t shift = 0;
    if (p.seg_n > 0) {
        const int sg = c % p.seg_n;
        oc = c / p.seg_n;
        t_first = p.seg_S;
        t_count = max(0, min(p.seg_B, N - sg * p.seg_B));
        shift = (int64_t)sg * p.seg_B - p.seg_S;
    }
    float *orow_band =
        reinterpret_cast<float *>(p.out) + ((int64_t)oc * p.n_rows + row) * N + shift;
    const float inv_n = 1.0f / (float)(qe - qb);

    auto lds_load = [](int idx) -> cf { return lds[idx]; };
    auto lds_store = [](int, int idx, cf v) { lds[idx] = v; };
    auto lds_load_sw = [](int idx) -> cf { return lds[first_pass_slot(idx)]; };
    auto lds_store_sw = [](int, int idx, cf v) { lds[first_pass_slot(idx)] = v; };
    const bool swz = n_pass >= 2 && (p.rp.radix[0] & 1) == 0;

    for (int q = qb; q < qe; ++q) {
        const int f = (MODE == kOutBand) ? p.grp_freq[q] : q;
        const BandDesc bd = p.band[f];
        const gptr<float> Hf = as_global(p.H + bd.off);
        const gptr<cf> Hcf =
            p.Hc ? as_global(reinterpret_cast<const cf *>(p.Hc) + bd.off) : nullptr;
        const int lo = bd.lo, K = bd.K;
        auto spec_load = [=](int b) -> cf {
            int off = b - lo;
            if (off < 0) off += L;
            if (off >= L) off -= L;
            cf y = mk(0.f, 0.f);
            if (off < K) {
                cf xv;
                if (b < Lh) {
                    xv = load_cf(X + b);
                } else {
                    xv = load_cf(X + (L - b));
                    xv.y = -xv.y;
                }
                y = Hcf ? mul(xv, load_cf(Hcf + off)) : scale(xv, Hf[off]);
            }
            return y;
        };
        // Output row of this frequency (band mode: of the band, accumulated
        // over its frequencies; only this workgroup touches it, and every
        // thread revisits the same samples t for each frequency, so it reads
        // back its own earlier writes).  The store functor is kept to six
        // registers (row pointer, first sample, count, flags, 1/count).
        const gptr_mut<float> orow = as_global_mut(
            (MODE == kOutBand)
                ? orow_band
                : reinterpret_cast<float *>(p.out) +
                      (((int64_t)oc * p.n_rows + f) * N + shift) * (MODE == kOutComplex ? 2 : 1));
        const int eflags = (q == qb ? 1 : 0) | (q == qe - 1 ? 2 : 0);
        auto epi = [orow, t_first, t_count, eflags, inv_n](int, int t, cf v) {
            if ((unsigned)(t - t_first) < (unsigned)t_count) {
                const float pw = v.x * v.x + v.y * v.y;
                if (MODE == kOutComplex) {
                    reinterpret_cast<gptr_mut<f2_t>>(orow)[t] = f2_t{v.x, v.y};
                } else if (MODE == kOutPower) {
                    orow[t] = pw;
                } else {
                    const float a = (eflags & 1) ? pw : orow[t] + pw;
                    orow[t] = (eflags & 2) ? a * inv_n : a;
                }
            }
        };

        // Leading passes the band makes trivial: while the band fits in
        // L / (Ns R) consecutive bins (at least one pass stays, it stores).
        int p0 = 0, Ns = 1;
        while (p0 < n_pass - 1 && K * Ns * p.rp.radix[p0] <= L) Ns *= p.rp.radix[p0++];
        if (p0 > 0) {
            // a band's later frequencies reuse the buffer the previous one
            // read last (callers separate rows with a barrier)
            if (q != qb) __syncthreads();
            band_prologue_rt(p.rp.radix[0], swz, X, Hf, Hcf, lo < 0 ? lo + L : lo, K, L, Lh,
                             Ns, T, tid, tw);
            __syncthreads();
        }
        // the pass that reads the first buffer written (by pass 0 or by the
        // prologue, in the first-pass slot map when swz)
        const int first_read = p0 > 0 ? p0 : 1;
        for (int i = p0; i < n_pass; ++i) {
            const int R = p.rp.radix[i];
            const bool last = (i == n_pass - 1);
            const bool sw_in = swz && i == first_read;
            if (!last) {
                if (i == 0 && swz)
                    stockham_pass_rt<1, MAXV, true>(R, L, Ns, T, tid, tw, spec_load, lds_store_sw);
                else if (i == 0)
                    stockham_pass_rt<1, MAXV, true>(R, L, Ns, T, tid, tw, spec_load, lds_store);
                else if (sw_in)
                    stockham_pass_rt<1, MAXV, true>(R, L, Ns, T, tid, tw, lds_load_sw, lds_store);
                else
                    stockham_pass_rt<1, MAXV, true>(R, L, Ns, T, tid, tw, lds_load, lds_store);
                __syncthreads();
            } else {
                if (i == 0)
                    stockham_pass_rt<1, MAXV, false>(R, L, Ns, T, tid, tw, spec_load, epi);
                else if (sw_in)
                    stockham_pass_rt<1, MAXV, true>(R, L, Ns, T, tid, tw, lds_load_sw, epi);
                else
                    stockham_pass_rt<1, MAXV, true>(R, L, Ns, T, tid, tw, lds_load, epi);
            }
            Ns *= R;
        }
    }
}

template <int MAXV, int MODE>
__global__ void __launch_bounds__(GenThreads<MAXV>::value) k_main(MainParams p)
{
    const int c = blockIdx.x / p.n_rows;
    const int row = blockIdx.x - c * p.n_rows;
    main_task<MAXV, MODE>(p, c, row);
}

// ----------------------------------------------------- batched, persistent --
// Workgroups claim tasks from a counter until the list is exhausted; every
// wave leaves the loop once the counter passes n.  A barrier follows every
// task (the next one reuses LDS).

__device__ __forceinline__ int claim_task(int *counter)
{
    __shared__ int s_task;
    if (threadIdx.x == 0) s_task = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    return t;
}

template <int MAXV>
__global__ void __launch_bounds__(GenThreads<MAXV>::value)
    k_batch_forward(const FwdParams *items, const BatchTask *tasks, int n, int *counter)
{
    for (;;) {
        const int t = claim_task(counter);
        if (t >= n) break;
        const BatchTask tk = tasks[t];
        forward_task<MAXV>(items[tk.item], tk.a);
        __syncthreads();
    }
}

template <int MAXV>
__global__ void __launch_bounds__(GenThreads<MAXV>::value)
    k_batch_main(const MainParams *items, const BatchTask *tasks, int n, int *counter)
{
    for (;;) {
        const int t = claim_task(counter);
        if (t >= n) break;
        const BatchTask tk = tasks[t];
        const MainParams &p = items[tk.item];
        for (int r = tk.b; r < tk.b + tk.n; ++r) {
            switch (p.out_mode) {
            case kOutComplex: main_task<MAXV, kOutComplex>(p, tk.a, r); break;
            case kOutPower: main_task<MAXV, kOutPower>(p, tk.a, r); break;
            default: main_task<MAXV, kOutBand>(p, tk.a, r); break;
            }
            __syncthreads();  // the next row reuses LDS
        }
    }
}

// One output row per workgroup, for the batch classes whose persistent
// kernel would not fit in its registers (with a task loop around them the
// passes of a 1024-thread, 24-value workgroup spill): the hardware dispatcher
// hands out the rows, longest first in table order.  The parameter table is
// read through the constant address space, so that its fields may be loaded
// again after each out-of-line pass instead of being held in registers.
template <int MAXV, int MODE>
__global__ void __launch_bounds__(GenThreads<MAXV>::value)
    k_batch_rows(const MainParams *items, const BatchTask *rows)
{
    typedef const __attribute__((address_space(4))) MainParams CMP;
    typedef const __attribute__((address_space(4))) BatchTask CBT;
    CBT &tk = *(CBT *)(rows + blockIdx.x);
    CMP &p = *(CMP *)(items + tk.item);
    main_task<MAXV, MODE>(p, (int)tk.a, (int)tk.b);
}

// One item of a batch as its own launch (grid: the item's channel pairs or
// output rows), its parameters read from the batch's table through the
// constant address space: a captured graph of these launches stays valid for
// any later call with the same layout, as the table is uploaded per call.
template <int MAXV>
__global__ void __launch_bounds__(GenThreads<MAXV>::value) k_item_forward(const FwdParams *items, int item)
{
    typedef const __attribute__((address_space(4))) FwdParams CFP;
    CFP &p = *(CFP *)(items + item);
    forward_task<MAXV>(p, blockIdx.x);
}

template <int MAXV, int MODE>
__global__ void __launch_bounds__(GenThreads<MAXV>::value) k_item_main(const MainParams *items, int item)
{
    typedef const __attribute__((address_space(4))) MainParams CMP;
    CMP &p = *(CMP *)(items + item);
    const int n_rows = p.n_rows;
    const int c = blockIdx.x / n_rows;
    main_task<MAXV, MODE>(p, c, (int)blockIdx.x - c * n_rows);
}

__global__ void k_zero_counters(int *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

hipError_t launch_zero_counters(int *c, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, c, n);
    return hipGetLastError();
}

template <class K>
static int occupancy_grid(K kernel, int threads, size_t lds, int n_tasks)
{
    int dev = 0, cus = 256, per_cu = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int g = cus * per_cu;
    return n_tasks < g ? n_tasks : g;
}

hipError_t launch_batch_forward(const FwdParams *items, const BatchTask *tasks, int n,
                                int *counter, int threads, int maxv, size_t lds, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    return with_maxv(maxv, [&](auto mv) {
        constexpr int M = decltype(mv)::value;
        // the kernels of a class are compiled for at most its workgroup size
        if (threads > GenThreads<M>::value) return hipErrorInvalidConfiguration;
        set_lds_limit((const void *)k_batch_forward<M>, lds);
        const int g = occupancy_grid(k_batch_forward<M>, threads, lds, n);
        hipLaunchKernelGGL(k_batch_forward<M>, dim3(g), dim3(threads), lds, s, items, tasks, n,
                           counter);
        return hipGetLastError();
    });
}

hipError_t launch_batch_main(const MainParams *items, const BatchTask *tasks, int n,
                             int *counter, int threads, int maxv, size_t lds, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    return with_maxv(maxv, [&](auto mv) {
        constexpr int M = decltype(mv)::value;
        // the kernels of a class are compiled for at most its workgroup size
        if (threads > GenThreads<M>::value) return hipErrorInvalidConfiguration;
        set_lds_limit((const void *)k_batch_main<M>, lds);
        const int g = occupancy_grid(k_batch_main<M>, threads, lds, n);
        hipLaunchKernelGGL(k_batch_main<M>, dim3(g), dim3(threads), lds, s, items, tasks, n,
                           counter);
        return hipGetLastError();
    });
}

template <int MAXV, int MODE>
static hipError_t launch_batch_rows_t(const MainParams *items, const BatchTask *rows, int n,
                                      int threads, size_t lds, hipStream_t s)
{
    set_lds_limit((const void *)k_batch_rows<MAXV, MODE>, lds);
    // a launch holds fewer than 2^32 work-items: larger classes take several
    const int chunk = (int)((((int64_t)1 << 32) - 1) / threads);
    for (int off = 0; off < n; off += chunk) {
        const int m = n - off < chunk ? n - off : chunk;
        hipLaunchKernelGGL((k_batch_rows<MAXV, MODE>), dim3(m), dim3(threads), lds, s, items,
                           rows + off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_rows(const MainParams *items, const BatchTask *rows, int n, int threads,
                             int maxv, int mode, size_t lds, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    return with_maxv(maxv, [&](auto mv) {
        constexpr int M = decltype(mv)::value;
        // the kernels of a class are compiled for at most its workgroup size
        if (threads > GenThreads<M>::value) return hipErrorInvalidConfiguration;
        switch (mode) {
        case kOutComplex: return launch_batch_rows_t<M, kOutComplex>(items, rows, n, threads, lds, s);
        case kOutPower: return launch_batch_rows_t<M, kOutPower>(items, rows, n, threads, lds, s);
        default: return launch_batch_rows_t<M, kOutBand>(items, rows, n, threads, lds, s);
        }
    });
}

hipError_t launch_item_forward(const FwdParams *items, int item, int blocks, int threads,
                               int maxv, size_t lds, hipStream_t s)
{
    if (blocks == 0) return hipSuccess;
    return with_maxv(maxv, [&](auto mv) {
        constexpr int M = decltype(mv)::value;
        // the kernels of a class are compiled for at most its workgroup size
        if (threads > GenThreads<M>::value) return hipErrorInvalidConfiguration;
        set_lds_limit((const void *)k_item_forward<M>, lds);
        hipLaunchKernelGGL(k_item_forward<M>, dim3(blocks), dim3(threads), lds, s, items, item);
        return hipGetLastError();
    });
}

template <int MAXV, int MODE>
static hipError_t launch_item_main_t(const MainParams *items, int item, int blocks, int threads,
                                     size_t lds, hipStream_t s)
{
    set_lds_limit((const void *)k_item_main<MAXV, MODE>, lds);
    hipLaunchKernelGGL((k_item_main<MAXV, MODE>), dim3(blocks), dim3(threads), lds, s, items,
                       item);
    return hipGetLastError();
}

hipError_t launch_item_main(const MainParams *items, int item, int blocks, int threads, int maxv,
                            int mode, size_t lds, hipStream_t s)
{
    if (blocks == 0) return hipSuccess;
    return with_maxv(maxv, [&](auto mv) {
        constexpr int M = decltype(mv)::value;
        // the kernels of a class are compiled for at most its workgroup size
        if (threads > GenThreads<M>::value) return hipErrorInvalidConfiguration;
        switch (mode) {
        case kOutComplex: return launch_item_main_t<M, kOutComplex>(items, item, blocks, threads, lds, s);
        case kOutPower: return launch_item_main_t<M, kOutPower>(items, item, blocks, threads, lds, s);
        default: return launch_item_main_t<M, kOutBand>(items, item, blocks, threads, lds, s);
        }
    });
}

template <int MAXV, int MODE>
static hipError_t launch_main_t(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    const int blocks = p.C * p.n_rows;
    const size_t lds = generic_lds_bytes(p.rp.L);
    set_lds_limit((const void *)k_main<MAXV, MODE>, lds);
    hipExtLaunchKernelGGL((k_main<MAXV, MODE>), dim3(blocks), dim3(p.rp.threads), lds, s,
                          ev.start, ev.stop, 0, p);
    return hipGetLastError();
}

// Segment inputs of a segmented plan: row c n_seg + s of xs (length Ls) is
// the zero-padded signal's samples s B - S .. s B - S + Ls - 1, indices taken
// modulo the cyclic period L_full (samples at or beyond N are zero).
__global__ void k_segment_gather(SegGatherParams p)
{
    const int64_t total = (int64_t)p.C * p.n_seg * p.Ls;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / p.Ls;
        const int t = (int)(e - row * p.Ls);
        const int64_t c = row / p.n_seg;
        const int sg = (int)(row - c * p.n_seg);
        int64_t i = ((int64_t)sg * p.B - p.S + t) % p.L_full;
        if (i < 0) i += p.L_full;
        p.xs[e] = (i < p.N) ? p.x[c * p.x_stride + i] : 0.f;
    }
}

hipError_t launch_segment_gather(const SegGatherParams &p, hipStream_t s)
{
    const int64_t total = (int64_t)p.C * p.n_seg * p.Ls;
    if (total == 0) return hipSuccess;
    const int64_t want = (total + 255) / 256;
    const int blocks = (int)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(k_segment_gather, dim3(blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

__global__ void k_chunk_reduce(ChunkReduceParams p)
{
    const int64_t total = (int64_t)p.C * p.n_bands * p.N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / p.N;  // c n_bands + b
        const int t = (int)(e - row * p.N);
        const int c = (int)(row / p.n_bands), b = (int)(row - (int64_t)c * p.n_bands);
        const int k0 = p.band_first[b], k1 = p.band_first[b + 1];
        float acc = 0.f;
        for (int k = k0; k < k1; ++k)
            acc += p.part[((int64_t)c * p.n_chunks + k) * p.N + t] *
                   (float)(p.chunk_off[k + 1] - p.chunk_off[k]);
        p.out[e] = acc / (float)(p.chunk_off[k1] - p.chunk_off[k0]);
    }
}

hipError_t launch_chunk_reduce(const ChunkReduceParams &p, hipStream_t s)
{
    const int64_t total = (int64_t)p.C * p.n_bands * p.N;
    if (total == 0) return hipSuccess;
    const int64_t want = (total + 255) / 256;
    const int blocks = (int)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(k_chunk_reduce, dim3(blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_main(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    return with_maxv(p.rp.maxv, [&](auto mv) {
        constexpr int M = decltype(mv)::value;
        // the kernels of a class are compiled for at most its workgroup size
        if (p.rp.threads > GenThreads<M>::value) return hipErrorInvalidConfiguration;
        switch (p.out_mode) {
        case kOutComplex: return launch_main_t<M, kOutComplex>(p, s, ev);
        case kOutPower: return launch_main_t<M, kOutPower>(p, s, ev);
        default: return launch_main_t<M, kOutBand>(p, s, ev);
        }
    });
}

}  // namespace cwtk
