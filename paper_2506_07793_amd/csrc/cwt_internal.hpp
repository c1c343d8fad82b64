// Host-side plan object and internal entry points of libcwt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_kernels.hpp"

struct cwt_split_state;  // split-precision (MFMA) tables, when built

struct cwt_plan {
    int64_t n = 0;
    double sfreq = 0;
    int L = 0;
    int F = 0;
    int n_bands = 0;
    int device = 0;
    cwt_plan_opts opts{};
    cwtk::RadixPlan rp{};
    std::vector<double> freqs, sigmas, band_edges;
    std::vector<cwtk::BandDesc> bands;
    std::vector<int> grp_freq, grp_off, band_of_freq;
    int total_bins = 0;
    int max_bins = 0;
    bool use_fixed = false;  // register-resident kernel for this length
    int variant = 0;         // its twiddle method (0 table, 1 powers)
    // device tables
    double *d_freqs = nullptr;
    double *d_sigmas = nullptr;
    cwtk::BandDesc *d_band = nullptr;
    float *d_H = nullptr;
    float2 *d_Hc = nullptr;  // complex spectra of sampled wavelets (cwt_plan_create_from_wavelets)
    bool user = false;       // spectra from sampled wavelets
    float2 *d_tw = nullptr;
    int *d_grp_freq = nullptr;
    int *d_grp_off = nullptr;
    cwt_split_state *split = nullptr;
    // Per-launch timing of the transform kernel (cwt_plan_timing_start/stop):
    // event pairs bound to the next `timing_cap` transform dispatches.
    std::vector<hipEvent_t> timing_ev;  // 2 per slot: start, stop
    int timing_cap = 0;
    mutable int timing_used = 0;
};

namespace cwtrt {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();

int64_t pad_length(int64_t n, int mode, int64_t explicit_len);
bool make_radix_plan(int L, cwtk::RadixPlan &rp);
void radix_candidates(int L, std::vector<cwtk::RadixPlan> &out);
void apply_tuning_cache(cwt_plan &P);
cwtk::BandDesc spectrum_band(int L, double sfreq, double f, double sigma, int wavelet,
                             double gmw_beta, double gmw_gamma);
int validate_and_plan(cwt_plan &P, int64_t n, double sfreq, const double *freqs,
                      int32_t n_freqs, const double *n_cycles, double omega0,
                      const cwt_plan_opts *opts);
int check_device(int *dev_out);
int upload_plan(cwt_plan &P, hipStream_t s);
void free_plan_device(cwt_plan &P);
size_t workspace_bytes(const cwt_plan &P, int64_t C);
int enqueue_forward(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride, void *ws,
                    hipStream_t s);
int enqueue_transform(const cwt_plan &P, int64_t C, void *out, void *ws, hipStream_t s);
// Events for the next transform dispatch while timing is on, else a null pair.
cwtk::LaunchEvents next_launch_events(const cwt_plan &P);
int enqueue_execute(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride, void *out,
                    void *ws, hipStream_t s);

// split-precision MFMA path
bool split_precision_available();
int prepare_split_precision(cwt_plan &P, hipStream_t s);
void release_split_precision(cwt_plan &P);

size_t split_workspace_bytes(const cwt_plan &P, int64_t C);
int enqueue_execute_split(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride,
                          void *out, void *ws, hipStream_t s);
int enqueue_transform_split(const cwt_plan &P, int64_t C, void *out, void *ws, hipStream_t s);

}  // namespace cwtrt

// Argument checks shared by the execute entry points (sets the error message).
int check_exec_args(const cwt_plan *P, const float *x, bool x_needed, int64_t C, void *out,
                    bool out_needed, void *ws, size_t ws_bytes);
