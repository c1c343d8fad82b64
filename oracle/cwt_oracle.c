/*
 * FP64 CPU oracle for the FFT-based Morlet continuous wavelet transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (Nakanishi, "Novel software for continuous wavelet
 * analysis ...", section "Fourier transformed formula"):
 *   The method takes the FFT of the (padded) signal, multiplies it by the
 *   wavelet's closed-form Fourier transform sampled on the DFT bins, and takes
 *   one inverse FFT.  By the cyclic convolution theorem that product equals
 *   the cyclic convolution of the padded signal with h = IDFT(H).  This file
 *   writes that plain definition out directly, with no FFT:
 *     1. L = pad(N)   (section "Fast Fourier transform": smallest length >= N
 *        whose only prime factors are 2, 3, 5, 7; or a power of two).
 *     2. Morlet constants kappa = exp(-sigma^2/2) (makes the transform vanish
 *        at zero frequency) and c = (1 + e^{-sigma^2} - 2 e^{-3 sigma^2/4})^{-1/2}
 *        (unit L2 energy); Gabor: kappa = 0, c = 1.  The paper says only that
 *        both follow from sigma (Morlet and Gabor equations).
 *     3. Scale s = sigma / (2 pi f); angular bin frequency
 *        omega_b = 2 pi sfreq btilde / L with btilde = b for 2b < L else b - L.
 *     4. H[b] = sqrt(2 pi s sfreq) * c pi^{-1/4} *
 *               (exp(-(sigma - s omega_b)^2 / 2) - kappa exp(-(s omega_b)^2 / 2))
 *        (Morlet Fourier-domain equation, evaluated at s*omega, with the
 *        prefactor that gives the sampled wavelet unit energy).
 *     5. h[j] = (1/L) sum_b H[b] exp(+2 pi i (b j mod L) / L)   (direct IDFT)
 *     6. W[t] = sum_{k<N} x[k] h[(t - k) mod L],  t in [0, N)   (direct cyclic
 *        convolution; O(N L) per channel and frequency).
 *
 * Generalized Morse wavelet (same section, the GMW equation): the paper
 * prints sign(omega) alpha omega^beta exp(-omega^gamma) with alpha "from
 * beta and gamma".  Read here, as in Lilly and Olhede's analytic GMW, with
 * the unit step U(omega) in place of sign(omega) (zero at omega <= 0) and
 * alpha = 2 (e gamma / beta)^(beta / gamma), which makes the peak value 2 at
 * u_p = (beta / gamma)^(1 / gamma).  The scale maps that peak to the analysis
 * frequency: s = u_p / (2 pi f), and H[b] = sqrt(2 pi s sfreq) Psi_hat(s
 * omega_b) as in step 4.
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
#ifndef M_E
#define M_E 2.71828182845904523536
#endif

/* ---- step 1: padded length ------------------------------------------- */

static int only_small_primes(int64_t m)
{
    static const int p[4] = {2, 3, 5, 7};
    for (int i = 0; i < 4; ++i)
        while (m % p[i] == 0) m /= p[i];
    return m == 1;
}

/* Smallest m >= n with no prime factor above 7 (plain trial division). */
int64_t orc_pad_smooth7(int64_t n)
{
    if (n < 1) return -1;
    int64_t m = n;
    while (!only_small_primes(m)) ++m;
    return m;
}

/* Smallest power of two >= n. */
int64_t orc_pad_pow2(int64_t n)
{
    if (n < 1) return -1;
    int64_t m = 1;
    while (m < n) m *= 2;
    return m;
}

/* ---- step 2: wavelet constants ---------------------------------------- */

/* kind 0 = Morlet, 1 = Gabor */
void orc_wavelet_constants(int kind, double sigma, double *c, double *kappa)
{
    if (kind == 1) {
        *kappa = 0.0;
        *c = 1.0;
        return;
    }
    *kappa = exp(-0.5 * sigma * sigma);
    *c = 1.0 / sqrt(1.0 + exp(-sigma * sigma) - 2.0 * exp(-0.75 * sigma * sigma));
}

/* Mother wavelet in the Fourier domain at angular argument u. */
double orc_mother_spectrum(int kind, double sigma, double u)
{
    double c, kappa;
    orc_wavelet_constants(kind, sigma, &c, &kappa);
    double a = sigma - u;
    return c * pow(M_PI, -0.25) * (exp(-0.5 * a * a) - kappa * exp(-0.5 * u * u));
}

/* Generalized Morse wavelet in the Fourier domain (reading above). */
double orc_gmw_peak(double beta, double gamma) { return pow(beta / gamma, 1.0 / gamma); }

double orc_gmw_spectrum(double beta, double gamma, double u)
{
    if (u <= 0.0) return 0.0;
    double alpha = 2.0 * pow(M_E * gamma / beta, beta / gamma);
    return alpha * pow(u, beta) * exp(-pow(u, gamma));
}

/* ---- steps 3-4: sampled wavelet spectrum ------------------------------ */

void orc_wavelet_spectrum(int64_t L, double sfreq, double f, double sigma, int kind,
                          double *H)
{
    double s = sigma / (2.0 * M_PI * f);
    double pref = sqrt(2.0 * M_PI * s * sfreq);
    for (int64_t b = 0; b < L; ++b) {
        int64_t bt = (2 * b < L) ? b : b - L;
        double omega = 2.0 * M_PI * sfreq * (double)bt / (double)L;
        H[b] = pref * orc_mother_spectrum(kind, sigma, s * omega);
    }
}

void orc_gmw_wavelet_spectrum(int64_t L, double sfreq, double f, double beta, double gamma,
                              double *H)
{
    double s = orc_gmw_peak(beta, gamma) / (2.0 * M_PI * f);
    double pref = sqrt(2.0 * M_PI * s * sfreq);
    for (int64_t b = 0; b < L; ++b) {
        int64_t bt = (2 * b < L) ? b : b - L;
        double omega = 2.0 * M_PI * sfreq * (double)bt / (double)L;
        H[b] = pref * orc_gmw_spectrum(beta, gamma, s * omega);
    }
}

/* ---- step 5: direct inverse DFT of a real spectrum --------------------- */

void orc_idft_real_spectrum(int64_t L, const double *H, double *h_re, double *h_im)
{
    double *cs = (double *)malloc(sizeof(double) * (size_t)L);
    double *sn = (double *)malloc(sizeof(double) * (size_t)L);
    for (int64_t m = 0; m < L; ++m) {
        double a = 2.0 * M_PI * (double)m / (double)L;
        cs[m] = cos(a);
        sn[m] = sin(a);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < L; ++j) {
        double re = 0.0, im = 0.0;
        int64_t m = 0; /* (b * j) mod L, advanced exactly in integers */
        for (int64_t b = 0; b < L; ++b) {
            re += H[b] * cs[m];
            im += H[b] * sn[m];
            m += j;
            if (m >= L) m -= L;
        }
        h_re[j] = re / (double)L;
        h_im[j] = im / (double)L;
    }
    free(cs);
    free(sn);
}

/* ---- step 6: direct cyclic convolution --------------------------------- */

/* One output row: W[t] for t in [t0, t0 + nt), t < N. */
void orc_cyclic_conv_row(const double *x, int64_t N, int64_t L, const double *h_re,
                         const double *h_im, int64_t t0, int64_t nt, double *w_re,
                         double *w_im)
{
    for (int64_t i = 0; i < nt; ++i) {
        int64_t t = t0 + i;
        double re = 0.0, im = 0.0;
        for (int64_t k = 0; k < N; ++k) {
            int64_t j = t - k;
            if (j < 0) j += L;
            re += x[k] * h_re[j];
            im += x[k] * h_im[j];
        }
        w_re[i] = re;
        w_im[i] = im;
    }
}

/*
 * Many rows at once.  x is [C][N] row-major; h_re/h_im are [F][L]; the
 * requested rows are (row_c[r], row_f[r]) for r < n_rows; each writes nt
 * outputs starting at t0 into w_re/w_im[r][nt].  Rows run in parallel.
 */
void orc_cwt_rows(const double *x, int64_t C, int64_t N, int64_t L, const double *h_re,
                  const double *h_im, int64_t F, const int64_t *row_c, const int64_t *row_f,
                  int64_t n_rows, int64_t t0, int64_t nt, double *w_re, double *w_im)
{
    (void)C;
    (void)F;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rows; ++r) {
        orc_cyclic_conv_row(x + row_c[r] * N, N, L, h_re + row_f[r] * L,
                            h_im + row_f[r] * L, t0, nt, w_re + r * nt, w_im + r * nt);
    }
}

/* Number of threads OpenMP will use (reported beside CPU timings). */
int orc_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
