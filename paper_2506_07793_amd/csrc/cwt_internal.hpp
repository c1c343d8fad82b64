// Host-side plan object and internal entry points of libcwt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_kernels.hpp"
#include "cwt_mixed.hpp"

namespace cwtk {
// Most threads per workgroup of a runtime-radix plan holding at most maxv
// values per thread in a pass (the kernels' launch bound of that class:
// 1024 for 16 and 24 values, 768 for 32).
inline int generic_max_threads(int maxv) { return maxv > 24 ? 768 : 1024; }
}  // namespace cwtk

struct cwt_split_state;  // split-precision (MFMA) tables, when built

namespace cwtrt {
// Allocator of a library object's device memory (both null: HIP's pool).
struct DevMem {
    cwt_alloc_fn alloc = nullptr;
    cwt_free_fn free = nullptr;
    void *ctx = nullptr;
};
}  // namespace cwtrt

struct cwt_plan {
    int64_t n = 0;
    double sfreq = 0;
    int L = 0;  // transform length of the kernels
    // Segmented plans (padded lengths above CWT_MAX_LEN): the cyclic
    // transform of period L_full computed segment by segment with transforms
    // of length L.  Segment s yields outputs [s seg_B, s seg_B + seg_B) from
    // the padded signal's samples s seg_B - seg_S .. s seg_B + seg_B + seg_S - 1
    // (mod L_full); n_seg = 0 for plans that are not segmented.
    int64_t L_full = 0;
    int seg_B = 0, seg_S = 0, n_seg = 0;
    int F = 0;
    int n_bands = 0;
    int device = 0;
    cwt_plan_opts opts{};
    cwtk::RadixPlan rp{};
    std::vector<double> freqs, sigmas, band_edges;
    std::vector<cwtk::BandDesc> bands;
    std::vector<int> grp_freq, grp_off, band_of_freq;
    // What d_grp_off holds: grp_off, then the band indices by frequency
    // count, largest first (set by set_group_table)
    std::vector<int> grp_table;
    // Band power on the runtime-radix and split-precision kernels: each band
    // is cut into chunks of at most chunk_max frequencies, one transform row
    // per chunk (its mean |W|^2 into a partial row of the workspace), then
    // the chunks of a band are combined.  n_chunks = 0: rows are whole bands.
    // chunk_table: [n_chunks + 1] offsets into grp_freq, then [n_bands + 1]
    // offsets of each band's first chunk.
    int n_chunks = 0;
    std::vector<int> chunk_table;
    int *d_chunk = nullptr;
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
    // Device memory the plan owns: every block came from mem (on the creation
    // stream) and goes back through it on the destroy stream.
    struct Block {
        void *p;
        size_t n;
    };
    cwtrt::DevMem mem{};
    std::vector<Block> blocks;
    // Recorded on the creation stream once the tables are written; the stream
    // server and the batch entry point wait for it on their own streams.
    hipEvent_t ready = nullptr;
    // With opts.max_channels > 0: the plan's own workspace for that many
    // channels (used when an execute call passes no workspace).
    int64_t max_channels = 0;
    void *own_ws = nullptr;
    size_t own_ws_bytes = 0;
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
// Fill P.grp_table from P.grp_off (band-power plans).
void set_group_table(cwt_plan &P);
// Frees the plan's device memory in stream order on s.
void free_plan_device(cwt_plan &P, hipStream_t s);
// Allocates the plan's own workspace (max_channels) and records P.ready on s.
int finish_plan(cwt_plan &P, hipStream_t s);
// Device memory (cwt_mem.cpp).
int check_dev_mem(const DevMem &m);
int dev_alloc(const DevMem &m, void **p, size_t bytes, hipStream_t s, const char *what);
void dev_free(const DevMem &m, void *p, size_t bytes, hipStream_t s);
int plan_alloc(cwt_plan &P, void **p, size_t bytes, hipStream_t s, const char *what);
void plan_free_all(cwt_plan &P, hipStream_t s);
// Make stream s wait until the plan's tables are written (no-op when they are).
int wait_plan_ready(const cwt_plan &P, hipStream_t s);
size_t workspace_bytes(const cwt_plan &P, int64_t C);
// Band-power chunk rows (P.n_chunks > 0): where the partial rows start in ws.
float *chunk_partials(const cwt_plan &P, int64_t C, void *ws);
// Combine the partial rows of each band into out (after a transform launch).
int enqueue_chunk_reduce(const cwt_plan &P, int64_t C, const float *part, void *out,
                         hipStream_t s);
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
int enqueue_forward_split(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride,
                          void *ws, hipStream_t s);
int enqueue_execute_split(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride,
                          void *out, void *ws, hipStream_t s);
int enqueue_transform_split(const cwt_plan &P, int64_t C, void *out, void *ws, hipStream_t s);

}  // namespace cwtrt

// Argument checks shared by the execute entry points (sets the error message).
int check_exec_args(const cwt_plan *P, const float *x, bool x_needed, int64_t C, void *out,
                    bool out_needed, void *ws, size_t ws_bytes);
