/*
 * cwt.h — C ABI of the MI355X (gfx950) FFT-based Morlet continuous wavelet
 * transform library (libcwt.so).
 *
 * The method (Nakanishi, arXiv 2506.07793, section "Fourier transformed
 * formula"): one forward FFT per channel of the zero-padded signal, a
 * multiplication by the closed-form Fourier transform of the wavelet at every
 * analysis frequency (Morlet and Gabor equations of the same section), and one
 * inverse FFT per (channel, frequency); the result is complex, or its power
 * |W|^2 (section "Precision"), or the mean power of EEG bands (introduction).
 * Padding follows section "Fast Fourier transform": the smallest length >= n
 * whose prime factors are 2, 3, 5 and 7.
 *
 * Conventions shared by every call:
 *   - Every function returns CWT_OK (0) or a negative CWT_E_* code; a
 *     thread-local message is available from cwt_last_error().  No C++
 *     exception crosses this boundary.
 *   - Arguments are validated before any device memory is allocated, written
 *     or any kernel is launched; on error nothing has been enqueued.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued asynchronously on it; no call synchronises the
 *     host unless stated.
 *   - Device pointers are caller-owned unless stated; the library never
 *     frees them.
 *   - Distinct objects may be used from different threads concurrently; one
 *     object must not be used from two threads at once unless stated.
 *   - Only gfx950 devices are supported (CWT_E_UNSUPPORTED otherwise).
 */
#ifndef CWT_H
#define CWT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define CWT_OK 0
#define CWT_E_INVALID (-1)     /* bad argument; nothing was enqueued          */
#define CWT_E_UNSUPPORTED (-2) /* valid request beyond this build's limits     */
#define CWT_E_NOMEM (-3)       /* a device or host allocation failed           */
#define CWT_E_HIP (-4)         /* a HIP runtime call failed (name in message)  */
#define CWT_E_BUDGET (-5)      /* admission would exceed the HBM budget        */
#define CWT_E_AGAIN (-6)       /* nothing ready / queue full; retry later      */

/* ---- plan options ---------------------------------------------------- */
/* Morlet and Gabor: section "Fourier transformed formula"; GMW: the generalized
 * Morse wavelet equation of the same section, read with the unit step U(omega)
 * for sign(omega) and alpha = 2 (e gamma / beta)^(beta / gamma) (peak value 2). */
enum cwt_wavelet { CWT_WAVELET_MORLET = 0, CWT_WAVELET_GABOR = 1, CWT_WAVELET_GMW = 2 };
/* CWT_PAD_LINEAR: the smallest 7-smooth L >= n + S, S = ceil(sqrt(2 ln 1e12)
 * s_max sfreq) + 1 the one-sided time support of the widest wavelet (the
 * Morlet / Gabor Gaussian envelope falls below 1e-12 of its peak beyond it;
 * s_max = max sigma / (2 pi f)).  The cyclic wrap then never reaches an output
 * sample, and the result equals the linear convolution of the zero-extended
 * signal with the wavelet (no edge wrap-around; section "Fourier transformed
 * formula" notes the cyclic result differs near the edges).  Morlet and
 * Gabor only (the GMW gives CWT_E_UNSUPPORTED). */
enum cwt_pad {
    CWT_PAD_SMOOTH7 = 0,
    CWT_PAD_POW2 = 1,
    CWT_PAD_NONE = 2,
    CWT_PAD_EXPLICIT = 3,
    CWT_PAD_LINEAR = 4
};
enum cwt_out { CWT_OUT_COMPLEX64 = 0, CWT_OUT_POWER_F32 = 1, CWT_OUT_BANDPOWER_F32 = 2 };
/* Split precision (padded length 4096 only): the radix-16 stages of both the
 * forward transform of the channels (cwt_forward_spectra, cwt_execute) and
 * the inverse transforms (cwt_transform_spectra, cwt_execute) run as
 * DFT-as-GEMM on MFMA with each operand split into a high and a low
 * half-precision part, three products accumulated in FP32; twiddles and the
 * spectral multiply stay in FP32.  Other lengths: CWT_E_UNSUPPORTED at plan
 * creation. */
enum cwt_precision {
    CWT_PREC_FP32 = 0,       /* FP32 radix-2/3/4/5/7/8/16 FFT in LDS               */
    CWT_PREC_SPLIT_F16 = 1,  /* DFT-as-GEMM radix stages on FP16 MFMA, hi+lo split  */
    CWT_PREC_SPLIT_BF16 = 2  /* DFT-as-GEMM radix stages on BF16 MFMA, hi+lo split  */
};

/* ---- device memory --------------------------------------------------- */
/*
 * Device memory the library owns (plan tables, a plan's own workspace,
 * stream-session rings and batch buffers) comes from the caller's allocator
 * when one is given, e.g. a framework's caching allocator.
 *   alloc(bytes, stream, ctx): return device memory of at least `bytes`
 *     bytes, usable by work enqueued on `stream` after the call (stream-
 *     ordered allocation), or NULL on failure (the library then returns
 *     CWT_E_NOMEM).
 *   free(ptr, bytes, stream, ctx): give back a block alloc returned; the
 *     memory must not be reused by anything before the work already enqueued
 *     on `stream` has finished (stream-ordered free).
 * Without callbacks the library uses HIP's stream-ordered pool allocator
 * (hipMallocAsync / hipFreeAsync on the same streams).  Neither path
 * synchronises the host.
 */
typedef void *(*cwt_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*cwt_free_fn)(void *ptr, size_t bytes, void *stream, void *ctx);

/* Largest padded length one workgroup holds in LDS (complex64, 160 KB). */
#define CWT_MAX_LEN 20480
#define CWT_MAX_FREQS 4096
#define CWT_MAX_BANDS 16

typedef struct cwt_plan_opts {
    int32_t wavelet;          /* enum cwt_wavelet                                  */
    int32_t pad;              /* enum cwt_pad                                      */
    int64_t explicit_len;     /* padded length when pad == CWT_PAD_EXPLICIT (>= n) */
    int32_t out;              /* enum cwt_out                                      */
    int32_t precision;        /* enum cwt_precision                                */
    int32_t n_bands;          /* 0 = the five default EEG bands                    */
    const double *band_edges; /* 2*n_bands values (lo0, hi0, lo1, hi1, ...) in Hz.
                                 A frequency f belongs to band k when
                                 lo_k <= f < hi_k, or f == hi_k for the last band.
                                 Defaults: delta 1-4, theta 4-8, alpha 8-13,
                                 beta 13-30, gamma 30-100 Hz.  Copied at create. */
    double gmw_beta;          /* GMW beta (default 17.5, the paper's value)        */
    double gmw_gamma;         /* GMW gamma (default 3)                             */
    int64_t max_channels;     /* 0 (default): no limit.  > 0: execute calls take at
                                 most this many channels, and the plan owns a
                                 workspace for that many, used when ws is NULL   */
    cwt_alloc_fn alloc;       /* device allocator of the plan's memory, or NULL
                                 (HIP's stream-ordered pool); alloc and free are
                                 given together or not at all                    */
    cwt_free_fn free;
    void *alloc_ctx;          /* passed to alloc and free                        */
} cwt_plan_opts;

/* Fill *opts with the defaults: Morlet, SMOOTH7, complex64, FP32, default bands,
 * GMW beta = 17.5 and gamma = 3. */
int cwt_plan_opts_init(cwt_plan_opts *opts);

typedef struct cwt_plan cwt_plan;

/*
 * Create an immutable plan for signals of n samples at sfreq Hz, analysed at
 * n_freqs frequencies freqs[] (Hz).  The wavelet parameter sigma (the paper's
 * Morlet sigma, equal to the number of cycles and to omega0) is n_cycles[i]
 * per frequency, or omega0 for every frequency when n_cycles is NULL.  For
 * the GMW, n_cycles and omega0 are not used (n_cycles may be NULL); the
 * scale of frequency f is s = u_p / (2 pi f) with u_p = (beta/gamma)^(1/gamma)
 * the wavelet's peak, from opts->gmw_beta and opts->gmw_gamma.
 *
 * Validation (CWT_E_INVALID): out != NULL; n >= 1; sfreq finite and > 0;
 * 1 <= n_freqs <= CWT_MAX_FREQS; every frequency finite with
 * 0 < f < sfreq / 2; every sigma finite and > 0 (Morlet, Gabor), or
 * gmw_beta and gmw_gamma finite and > 0 (GMW); known enum values; for
 * CWT_PAD_EXPLICIT explicit_len >= n; for band output every band has
 * lo < hi and owns at least one frequency, and n_bands <= CWT_MAX_BANDS.
 * A padded length whose prime factors are not all in {2, 3, 5, 7} gives
 * CWT_E_UNSUPPORTED, unless it is above CWT_MAX_LEN.
 *
 * Padded lengths above CWT_MAX_LEN (long recordings) make a segmented plan
 * (Morlet / Gabor in FP32; otherwise CWT_E_UNSUPPORTED): the output is still
 * the cyclic transform of period L, computed segment by segment
 * (overlap-save).  Each segment is a transform of length segment_len <=
 * CWT_MAX_LEN of the zero-padded signal's samples, taken cyclically over L,
 * that reach segment_margin beyond its segment_outputs outputs on either
 * side.  The margin is the widest wavelet's time support (Gaussian envelope
 * above 1e-8 of its peak), so what a segment misses lies below that.  It
 * must leave at least 1/8 of a 20480-sample segment, and L is at most 2^30
 * (CWT_E_UNSUPPORTED otherwise).  Segmented plans run through cwt_execute,
 * cwt_forward_spectra and cwt_transform_spectra only; the other entry
 * points give CWT_E_UNSUPPORTED.
 *
 * On success the plan owns device memory for the wavelet spectra (FP64
 * evaluation on the GPU, rounded once to FP32, 1/L folded in, only the bins
 * whose magnitude is at least 1e-12 of the peak) and the twiddle table
 * exp(2 pi i m / L) (FP64 on the GPU, rounded once), and with max_channels a
 * workspace; all of it comes from opts->alloc on `stream` (or HIP's
 * stream-ordered pool), so the spectra and tables are made in GPU memory,
 * where the data they are applied to stays (section "Optimizing
 * performance").  Their generation is enqueued on `stream`; the plan may be
 * used on any stream once `stream` has reached that point (cwt_plan_create
 * does not synchronise; the stream server and cwt_execute_batch wait for it
 * themselves).  The spectra are the Fourier-domain wavelets of section
 * "Fourier transformed formula" (Morlet, Gabor, GMW equations), sampled on
 * the DFT bins.  Errors also include CWT_E_INVALID for max_channels < 0 or
 * only one of alloc / free, and CWT_E_NOMEM when an allocation fails.
 *
 * Environment, read when a plan is created: CWT_GENERIC_ONLY=1 makes
 * power-of-two lengths use the runtime-radix kernel instead of the
 * register-resident one; CWT_FIXED_VARIANT=0 makes the register-resident
 * kernel read every later-pass twiddle from the table (default 1: one table
 * value per butterfly, its powers by products); CWT_AUTOTUNE_CACHE names the
 * autotuner's cache file (see cwt_plan_autotune).  Each changes the rounding
 * of the results, not their tolerance.
 */
int cwt_plan_create(cwt_plan **out, int64_t n, double sfreq, const double *freqs,
                    int32_t n_freqs, const double *n_cycles, double omega0,
                    const cwt_plan_opts *opts, void *stream);

typedef struct cwt_plan_desc {
    int64_t n;               /* samples per channel                            */
    int64_t L;               /* padded FFT length                              */
    int64_t n_freqs;
    int64_t n_bands;         /* rows per channel in band mode                  */
    int32_t out;             /* enum cwt_out                                   */
    int32_t precision;       /* enum cwt_precision                             */
    int32_t wavelet;
    int32_t threads;         /* threads per workgroup of the transform kernel
                                (the register-resident kernel's when kernel = 1) */
    int32_t n_passes;        /* radix passes                                    */
    int32_t radix[16];       /* radix of each pass (of that kernel)             */
    int64_t out_rows;        /* rows per channel: n_freqs, or n_bands            */
    int64_t out_elem_bytes;  /* 8 (complex64) or 4 (float32)                     */
    int64_t spectrum_bins;   /* total stored wavelet-spectrum bins (all freqs)   */
    int64_t max_band_bins;   /* widest stored spectrum band                      */
    int32_t kernel;          /* 0 generic runtime-radix kernel, 1 register-resident
                                kernel specialised for this padded length          */
    int32_t spectrum_complex;/* 1: stored spectra are complex (sampled wavelets)  */
    int64_t max_channels;    /* opts->max_channels (0: no limit)                   */
    int64_t device_bytes;    /* device memory the plan owns (0 before creation)   */
    int64_t n_segments;      /* segmented plan (L above CWT_MAX_LEN): segments per
                                channel; 0 for plans transformed in one piece     */
    int64_t segment_len;     /* transform length of the kernels: L, or each
                                segment's length (the radix schedule's)           */
    int64_t segment_outputs; /* outputs each segment contributes                   */
    int64_t segment_margin;  /* input samples each segment reads on either side
                                of its outputs (the wavelets' time support)       */
    int64_t band_chunks;     /* band power on the runtime-radix or split kernels:
                                transform rows per channel, each band cut into
                                chunks of at most a quarter of the largest band
                                (combined by a second launch); 0: one row per
                                band                                                */
} cwt_plan_desc;

int cwt_plan_info(const cwt_plan *plan, cwt_plan_desc *desc);

/*
 * Validate a plan request and describe the plan cwt_plan_create would make
 * (padded length, radix schedule, stored spectrum bins) without touching
 * the device or allocating anything.  Same arguments and validation as
 * cwt_plan_create; needs no GPU.
 */
int cwt_plan_describe(cwt_plan_desc *desc, int64_t n, double sfreq, const double *freqs,
                      int32_t n_freqs, const double *n_cycles, double omega0,
                      const cwt_plan_opts *opts);

/*
 * Autotuner.  Times the candidate kernel configurations of this plan on the
 * current device (generic kernel: the planner's eight best-ranked schedules
 * and the radix orders 16-first / 8-first / 4-first, 16 or 24 values per
 * thread in workgroups of up to 1024 threads or 32 in workgroups of up to
 * 768, minimal or doubled workgroup; for the lengths with a
 * register-resident kernel (powers of two 1024-8192; 200, 400, 800, 1000,
 * 1600, 2000, 2500, 4000, 5000, 8000, 10000) also that
 * kernel with table or power twiddles) on min(C, 16) channels of zeros,
 * keeps the fastest in the
 * plan, and, when the environment variable CWT_AUTOTUNE_CACHE names a file,
 * appends the choice there.  cwt_plan_create applies a cached choice for the
 * same device, padded length, output mode and precision.  A tuned schedule
 * changes the rounding of the results, not their tolerance.  Synchronises
 * `stream`; allocates and frees temporary device buffers.  FP32 plans only
 * (other precisions return CWT_OK unchanged).
 */
typedef struct cwt_tune_result {
    int32_t n_candidates;
    int32_t kernel;        /* chosen: 0 generic, 1 register-resident            */
    int32_t variant;       /* register-resident twiddle method (0 table, 1 powers) */
    int32_t threads;       /* chosen workgroup size                              */
    int32_t n_passes;
    int32_t radix[16];
    float best_ms;         /* best time of one transform of the timed channels   */
    float default_ms;      /* time of the plan's original configuration          */
} cwt_tune_result;

int cwt_plan_autotune(cwt_plan *plan, int64_t C, void *stream, cwt_tune_result *result);

/* Lower and upper band-membership of each frequency: band_of_freq[i] is the
 * band index of frequency i, or -1 when it belongs to none (n_freqs ints). */
int cwt_plan_band_of_freq(const cwt_plan *plan, int32_t *band_of_freq);

/* Device workspace bytes cwt_execute needs for C channels (per-channel
 * half spectra, 256-byte aligned).  Returns 0 on invalid arguments. */
size_t cwt_workspace_size(const cwt_plan *plan, int64_t C);

/*
 * Transform C channels.  x: device float32 [C][n] row-major.  out: device
 * [C][n_freqs][n] complex64 (interleaved re, im) or float32 power, or
 * [C][n_bands][n] float32 band power, fully overwritten.  ws: device
 * workspace of at least cwt_workspace_size(plan, C) bytes, 256-byte aligned,
 * or NULL (with ws_bytes 0) to use the workspace of a plan created with
 * max_channels >= C; calls on one plan that share its own workspace must be
 * ordered on one stream.  x, out and ws must not overlap.  Asynchronous on
 * `stream`; the plan may be executed concurrently on several streams, each
 * with its own ws and out.  C == 0 is a no-op.  Errors: CWT_E_INVALID for
 * NULL or misaligned pointers (x 4-byte, out 8-byte, ws 256-byte aligned), C
 * outside [0, 2^24], C above the plan's max_channels, a NULL ws on a plan
 * without one, or a workspace too small; CWT_E_UNSUPPORTED when one launch would hold 2^32
 * work-items or more (one workgroup of cwt_plan_desc.threads per output row
 * of each channel, at most 1024 threads): split the channels over calls.
 */
int cwt_execute(const cwt_plan *plan, const float *x, int64_t C, void *out, void *ws,
                size_t ws_bytes, void *stream);

/*
 * cwt_execute without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The workspace (the
 * channels' half spectra, cwt_workspace_size(plan, C) bytes) is a static
 * device array of CWT_NOALLOC_SCRATCH_BYTES in the library, one copy per GPU,
 * held until the process ends.  x, C, out and stream as for cwt_execute (the
 * caller still owns x and out); results equal cwt_execute's bit for bit.
 * Every call on one GPU shares that GPU's array: calls whose work overlaps on
 * one GPU (on different streams, or from different threads without ordering)
 * race on it and give wrong results; calls ordered on one stream are safe.
 * The first call on a device looks up that device's array (the current
 * device).  Calls no hipMalloc, hipFree or allocating routine.  Errors: those
 * of cwt_execute, and CWT_E_UNSUPPORTED when cwt_workspace_size(plan, C)
 * exceeds CWT_NOALLOC_SCRATCH_BYTES (nothing is launched; split C or use
 * cwt_execute with a workspace).
 */
#define CWT_NOALLOC_SCRATCH_BYTES (16u << 20)
int cwt_execute_noalloc(const cwt_plan *plan, const float *x, int64_t C, void *out,
                        void *stream);

/*
 * The two stages of cwt_execute, for callers that reuse the channel spectra
 * or time the stages separately.  cwt_forward_spectra writes the half
 * spectra X[c][b] = sum_{k<n} x[c][k] exp(-2 pi i b k / L), b <= L/2, of the
 * zero-padded channels into ws (section "Fourier transformed formula": the
 * FFT of the signal).  cwt_transform_spectra reads them from ws and writes
 * out exactly as cwt_execute does (multiply by the wavelet spectra, inverse
 * FFT, crop, output mode).  Same arguments, validation and workspace as
 * cwt_execute; cwt_transform_spectra takes no x.
 */
int cwt_forward_spectra(const cwt_plan *plan, const float *x, int64_t C, void *ws,
                        size_t ws_bytes, void *stream);
int cwt_transform_spectra(const cwt_plan *plan, int64_t C, void *out, void *ws,
                          size_t ws_bytes, void *stream);

/*
 * Copy the plan's tables to host memory for inspection (synchronises
 * `stream`).  H_host receives spectrum_bins floats (the stored bins of every
 * frequency, frequency after frequency), or 2 * spectrum_bins floats
 * (complex, interleaved) when cwt_plan_desc.spectrum_complex is 1;
 * band_host receives 3 ints per frequency (first signed bin, number of bins,
 * offset into H_host); tw_host
 * receives 2*L floats (the twiddle table).  Any pointer may be NULL.
 */
int cwt_plan_copy_tables(const cwt_plan *plan, float *H_host, int32_t *band_host,
                         float *tw_host, void *stream);

/*
 * Per-launch timing of the transform kernel (the spectral multiply + inverse
 * FFT + store kernel), for measurements like those of section "Comparison
 * between devices and software" taken kernel by kernel.
 * cwt_plan_timing_start creates max_launches pairs of events (host call; not
 * while a stream is being captured into a graph) and binds one pair to each
 * of this plan's next max_launches transform dispatches (by cwt_execute or
 * cwt_transform_spectra, on any stream); each pair takes the start and end
 * timestamps of that dispatch (hipExtLaunchKernel; the events carry no
 * system-scope fence, so they add no cache write-back to the stream).
 * Later dispatches run untimed.  A second start discards earlier records.  cwt_plan_timing_stop waits for the timed
 * dispatches, writes min(recorded, max) durations in milliseconds, in launch
 * order, to ms_host (may be NULL when max == 0), the number recorded to
 * *n_out, and turns timing off.  Not thread-safe against concurrent enqueues
 * of the same plan.  Errors: CWT_E_INVALID for a NULL plan, max_launches
 * outside [0, 65536] or max < 0; CWT_E_HIP when an event call fails.
 */
int cwt_plan_timing_start(cwt_plan *plan, int32_t max_launches);
int cwt_plan_timing_stop(cwt_plan *plan, float *ms_host, int32_t max, int32_t *n_out);

/*
 * Throughput form of cwt_execute for n_batches batches of C channels with the
 * same plan, such as consecutive windows of a long recording or recordings
 * of equal shape (section "Comparison between devices and software" runs the
 * transform over and over).  Batch i reads x + i * x_batch_stride floats and
 * writes out + i * out_batch_stride bytes, with the layouts of cwt_execute; a
 * stride of 0 reuses one buffer (each batch then overwrites the previous
 * batch's output).  Everything runs on `stream`, in batch order.  With a
 * register-resident transform kernel (cwt_plan_desc.kernel == 1) each batch
 * is one launch that also computes the forward FFT of the next batch into
 * the other half of a double-buffered workspace; other plans run
 * cwt_execute's two stages per batch.  Results equal cwt_execute's bit for
 * bit.  ws: device, at least cwt_batches_workspace_size(plan, C) bytes,
 * 256-byte aligned.  The x of every batch, the out of every batch and ws must
 * not overlap; out_batch_stride must be a multiple of 8.  n_batches == 0 or
 * C == 0 is a no-op.  Errors: those of cwt_execute, CWT_E_INVALID for
 * n_batches < 0, a negative stride or a workspace under twice
 * cwt_workspace_size (on an error after the first launch, earlier batches
 * stay queued).
 */
size_t cwt_batches_workspace_size(const cwt_plan *plan, int64_t C);
int cwt_execute_batches(const cwt_plan *plan, const float *x, int64_t x_batch_stride,
                        int32_t n_batches, int64_t C, void *out, int64_t out_batch_stride,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * Plan from sampled time-domain wavelets: the two-FFT form of section
 * "Fourier transformed formula", where a wavelet's spectrum is the DFT of its
 * samples instead of a closed form.  wavelets: host, [n_freqs][w_len]
 * complex64 (interleaved re, im), read during the call; sample j of each sits
 * at time (j - w_len / 2) / sfreq, i.e. circularly at index
 * (j - w_len / 2) mod L, and is used as given (the samples carry their own
 * normalisation).  The transform is the cyclic convolution of the
 * zero-padded signal with each placed wavelet.  freqs: n_freqs labels in Hz,
 * 0 < f < sfreq / 2, used only to group frequencies into bands for
 * band-power output.  opts as for cwt_plan_create, except that `wavelet` is
 * not used, precision must be CWT_PREC_FP32, and CWT_PAD_LINEAR takes the
 * wavelets' longest one-sided extent, max(w_len/2, w_len - 1 - w_len/2) + 1
 * samples, as the support.  The spectra (1/L folded in) are computed in FP64
 * on the GPU and rounded once; each frequency stores the shortest cyclic run
 * of bins holding every bin of at least 1e-12 of its peak magnitude, found on
 * the host, so this call synchronises `stream`.  These plans run
 * cwt_execute, its two stages, cwt_execute_batches, cwt_execute_batch and
 * cwt_plan_autotune; stream sessions reject them (CWT_E_UNSUPPORTED).
 * Errors: those of cwt_plan_create, plus CWT_E_INVALID for wavelets == NULL,
 * w_len < 1, w_len above the padded length or a non-finite sample, and
 * CWT_E_UNSUPPORTED for a precision other than FP32.
 */
int cwt_plan_create_from_wavelets(cwt_plan **out, int64_t n, double sfreq, const double *freqs,
                                  int32_t n_freqs, const float *wavelets, int64_t w_len,
                                  const cwt_plan_opts *opts, void *stream);

/* ---- batches ---------------------------------------------------------- */
/*
 * Many recordings at once, each with its own plan (length, sampling rate,
 * frequency grid, output mode), channel count and device buffers, as in the
 * paper's use on EEG recordings of different lengths (section "Wavelength
 * and flexibility").  x and out have the same layouts as for cwt_execute.
 */
typedef struct cwt_batch_item {
    const cwt_plan *plan;  /* FP32 plan                                        */
    const float *x;        /* device [C][plan n]                               */
    int64_t C;             /* channels (0 = skip)                              */
    void *out;             /* device output, cwt_execute layout                */
} cwt_batch_item;

/* Device workspace bytes cwt_execute_batch needs for these items (tables,
 * task lists and per-item spectra).  Returns 0 on invalid items. */
size_t cwt_batch_workspace_size(const cwt_batch_item *items, int32_t n);

/*
 * Transform every item (recordings of uneven length, channel count and
 * frequency grid, the flexibility discussed in the paper's section
 * "Wavelength and flexibility") with one HIP graph launch.  Default form:
 * one forward and one transform launch per item inside the graph, each at
 * the item's own workgroup size and LDS, its parameters read from the table
 * uploaded into ws; items longest first, each on the least loaded of four
 * parallel graph branches.  With the environment variable
 * CWT_BATCH_KERNELS=persistent: one persistent forward and one transform
 * kernel per workgroup-size class instead, whose resident workgroups claim
 * tasks (channel pairs; runs of output rows) through atomic counters,
 * longest first.  The graph is captured the first time a (workspace, task
 * layout) pair is seen and replayed afterwards; the per-item tables are
 * uploaded into ws on `stream` before each launch.  Asynchronous; the items'
 * buffers must not overlap each other or ws.  Results equal cwt_execute's
 * for each item.  CWT_BATCH_GRAPH=0 launches the kernels directly instead of
 * through the graph.  Errors (nothing is launched): CWT_E_INVALID for a
 * null item, plan or device pointer, C outside [0, 2^24], a null or
 * misaligned ws or one smaller than cwt_batch_workspace_size;
 * CWT_E_UNSUPPORTED for a plan that is not FP32 or more than 2^31 - 1
 * (channel, row) tasks in one item.  CWT_E_HIP for a failed launch or
 * capture.
 */
int cwt_execute_batch(const cwt_batch_item *items, int32_t n, void *ws, size_t ws_bytes,
                      void *stream);

/* ---- streaming ------------------------------------------------------- */
/*
 * Real-time form (the paper's real-time EEG use, sections "Introduction" and
 * "Discussion"): sessions push samples, and for every completed hop the
 * server transforms the sliding window of the last n samples (the plan's n)
 * and reports, per channel and band, the band power averaged over the hop's
 * trailing samples of the window's transform.  A launcher thread batches the
 * hops of many sessions into one set of launches (up to max_batch hops,
 * launched when the oldest pending hop has waited deadline_us or the batch
 * is full; one session's hops in order, at most max_session_windows of its
 * window hops per launch), and a completion thread stamps the completion
 * time of each result; the next batch is enqueued while the previous one
 * completes (two batches of a session class in flight).
 */
typedef struct cwt_server cwt_server;
typedef struct cwt_session cwt_session;

typedef struct cwt_server_opts {
    int32_t max_batch;        /* hops per launch (default 256)                       */
    int32_t deadline_us;      /* longest wait of a pending hop before launch (500)   */
    int32_t max_pending;      /* queued window hops per session before CWT_E_AGAIN
                                 (64); hops before the first full window only fill
                                 the ring and are not counted                        */
    int32_t max_session_windows; /* K: window-producing hops of one session in one
                                 launch (default 4, at most 64); each ring holds
                                 n + (K - 1) hop samples per channel               */
    cwt_alloc_fn alloc;       /* device allocator of rings and batch buffers, or
                                 NULL (HIP's stream-ordered pool); with free       */
    cwt_free_fn free;
    void *alloc_ctx;
} cwt_server_opts;

typedef struct cwt_server_stats {
    uint64_t batches;         /* launches so far                                   */
    uint64_t hops;            /* hops processed (emitting or not)                  */
    uint64_t results;         /* band-power results delivered                      */
    uint64_t rejected;        /* pushes refused with CWT_E_AGAIN                   */
    uint64_t sessions_open;
    uint64_t hbm_bytes_used;  /* device bytes held by rings and batch workspaces   */
    uint64_t hbm_budget_bytes;
    uint64_t max_batch_hops;  /* most hops taken into one launch                   */
    uint64_t max_batch_ns;    /* longest time from a batch's formation to its
                                 completion (host clock, staging copy included)    */
    uint64_t slot_waits;      /* times the launcher waited for a free staging slot */
} cwt_server_stats;

int cwt_server_opts_init(cwt_server_opts *opts);

/* Create a server that may hold at most hbm_budget_bytes of device memory
 * for session rings and batch workspaces, allocated and freed through
 * opts->alloc / opts->free (or HIP's stream-ordered pool) on the server's
 * stream.  Every device operation of the server (allocation, ring clearing,
 * copies, launches, frees) is enqueued on `stream`, which the caller owns and
 * must keep alive until cwt_server_destroy returns; NULL makes the server
 * create (and later destroy) its own non-blocking stream of default priority.
 * The server runs a worker thread.  opts may be NULL (defaults).  Errors:
 * CWT_E_INVALID for bad options or only one of alloc / free. */
int cwt_server_create(cwt_server **out, size_t hbm_budget_bytes, const cwt_server_opts *opts,
                      void *stream);

/* Stop the worker (pending hops are processed first), free everything.
 * Sessions still open are closed. */
int cwt_server_destroy(cwt_server *srv);

/* Open a session of C channels on `plan` (which must use CWT_OUT_BANDPOWER_F32;
 * its n is the window length W) with hop samples per result, 1 <= hop <= W.
 * The session's device ring (W + (K - 1) hop samples per channel, K =
 * max_session_windows) is allocated and cleared in stream order on the
 * server's stream, and the server's stream waits for the plan's tables if
 * they are still being written; the call does not wait for the device.  No
 * result is produced before the first W samples have arrived.  Returns
 * CWT_E_BUDGET when the session's ring plus (for a new (plan, C, hop) class)
 * the class's batch buffers would exceed the server's budget.  The plan must
 * outlive the session. */
int cwt_stream_open(cwt_server *srv, const cwt_plan *plan, int64_t C, int64_t hop,
                    cwt_session **out);

/* Append m samples per channel (host, row-major [C][m], copied before
 * return).  Every completed hop is queued for the worker; t_arrival_ns
 * (CLOCK_MONOTONIC, 0 = now) is the time stamp reported with its result.
 * Returns CWT_E_AGAIN (nothing consumed) when the session already has
 * max_pending hops queued or the push would complete more than that. */
int cwt_stream_push(cwt_session *s, const float *samples, int64_t m, uint64_t t_arrival_ns);

/* Oldest completed result: bp receives [C][n_bands] floats (host), hop_idx
 * the hop's index since the session opened (0-based, counting every hop),
 * t_push_ns / t_done_ns the arrival and completion times.  Any output
 * pointer may be NULL.  Returns CWT_E_AGAIN when nothing is ready. */
int cwt_stream_poll(cwt_session *s, float *bp, uint64_t *hop_idx, uint64_t *t_push_ns,
                    uint64_t *t_done_ns);

/* Block until every hop queued so far on the server has been processed. */
int cwt_server_flush(cwt_server *srv);

/* Close a session: its queued hops are dropped, hops already launched are
 * waited for (their results are discarded), and its ring is freed in stream
 * order on the server's stream. */
int cwt_stream_close(cwt_session *s);

int cwt_server_get_stats(const cwt_server *srv, cwt_server_stats *stats);

/* CLOCK_MONOTONIC in nanoseconds (the clock of the stream time stamps). */
uint64_t cwt_now_ns(void);

/* Release the plan.  Its device memory is freed in stream order on `stream`
 * (opts->free, or hipFreeAsync): work already enqueued on `stream` that uses
 * the plan finishes before the memory can be reused, and the call does not
 * wait for it.  Work on other streams that uses the plan must be ordered
 * before `stream`'s current point (an event, or a synchronisation) first.
 * The host-side plan object is gone when the call returns. */
int cwt_plan_destroy(cwt_plan *plan, void *stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char *cwt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CWT_H */
