// Kernel launch interface shared by the host runtime of libcwt.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cwtk {

constexpr int kMaxPasses = 16;

// Radix schedule of one padded length: the passes of the Stockham FFT and
// the workgroup size that runs them.
struct RadixPlan {
    int L;
    int n_pass;
    int radix[kMaxPasses];
    int threads;
    int maxv;  // most complex values one thread holds in a pass (16 or 24)
};

// Per-frequency stored spectrum band: signed first bin, bin count, offset.
struct BandDesc {
    int lo;
    int K;
    int off;
    int pad_;
};

// Forward real FFT of C channels, two per workgroup: Xh[c][b], b <= L/2.
struct FwdParams {
    const float *x;   // [C][N]
    int C, N;
    int64_t x_stride; // elements between channels
    float2 *Xh;       // [C][Lh]
    int Lh;
    const float2 *tw; // [L]
    RadixPlan rp;
};

enum OutMode { kOutComplex = 0, kOutPower = 1, kOutBand = 2 };

// Fused spectral multiply -> inverse FFT -> crop -> epilogue.
struct MainParams {
    const float2 *Xh;      // [C][Lh] half spectra
    int Lh;
    const float *H;        // packed wavelet spectra (1/L folded in)
    const float2 *Hc;      // packed complex spectra of sampled wavelets, or null
    const BandDesc *band;  // [F]
    const float2 *tw;      // [L]
    void *out;
    int out_mode;
    int N, F, C;
    int n_rows;            // rows per channel in the output (F or n_bands)
    const int *grp_freq;   // band mode: frequency indices, band after band
    const int *grp_off;    // band mode: [n_bands + 1] offsets into grp_freq, then the
                           // [n_bands] band indices by frequency count, largest first
    RadixPlan rp;
    int variant;           // register-resident kernel: 0 table twiddles, 1 power twiddles
    // Segmented plans (runtime-radix kernel only): the C channels are
    // channel x segment rows, seg_n segments per channel; segment s stores its
    // samples [seg_S, seg_S + seg_B) at s seg_B .. of the output row (N long).
    // seg_n = 0: not segmented.
    int seg_n, seg_B, seg_S;
};

// ------------------------------------------------------------- batched --
// One task of a persistent batch kernel: item index and its channel pair
// (forward) or a run of consecutive output rows of one channel (transform).
struct BatchTask {
    int item;
    int a;  // channel pair (forward) or channel (transform)
    int b;  // first output row (transform)
    int n;  // number of consecutive output rows (transform)
};

hipError_t launch_zero_counters(int *c, int n, hipStream_t s);
hipError_t launch_batch_forward(const FwdParams *items, const BatchTask *tasks, int n,
                                int *counter, int threads, int maxv, size_t lds, hipStream_t s);
hipError_t launch_batch_main(const MainParams *items, const BatchTask *tasks, int n,
                             int *counter, int threads, int maxv, size_t lds, hipStream_t s);
// One workgroup per task of exactly one row (tasks[k].n == 1), all of one
// output mode; n workgroups.
hipError_t launch_batch_rows(const MainParams *items, const BatchTask *rows, int n, int threads,
                             int maxv, int mode, size_t lds, hipStream_t s);
// One batch item as its own launch, parameters read from the device table:
// `blocks` channel pairs (forward) or channels x rows (transform).
hipError_t launch_item_forward(const FwdParams *items, int item, int blocks, int threads,
                               int maxv, size_t lds, hipStream_t s);
hipError_t launch_item_main(const MainParams *items, int item, int blocks, int threads, int maxv,
                            int mode, size_t lds, hipStream_t s);

// ----------------------------------------------------------- streaming --
// One completed hop of one session.
struct StreamJob {
    float *ring;   // session ring [C][R]
    int pos;       // ring position of this hop's first sample
    int slab_off;  // offset of this hop's [C][hop] samples in the slab
    int emit_row;  // row block in the window batch (>= 0 when output is due)
    int pad_;
};

// Rings hold R >= W samples per channel: the hops of one session in one
// launch are all appended before any window is gathered, so a window must
// survive the appends of the session's later hops in that launch
// (R = W + (K - 1) hop for K windows of a session per launch).
struct StreamParams {
    const StreamJob *jobs;
    int n_jobs;
    const float *slab;  // [n_jobs][C][hop] new samples
    float *xb;          // [n_emit][C][W] unrolled windows (oldest sample first)
    int C, W, hop, R;
};

// Band power of the trailing hop of each window, by a direct partial
// inverse DFT over the stored spectrum bins (only hop outputs are needed).
struct StreamBPParams {
    const float2 *Xh;      // [rows][Lh]
    int Lh, L, W, hop, rows;
    const float *H;
    const BandDesc *band;
    const float2 *tw;
    const int *grp_freq;
    const int *grp_off;
    int n_bands;
    int n_grouped;         // frequencies in some band (grp_off[n_bands])
    float *part;           // [rows][n_grouped] workspace: sum over the hop of |W_f[t]|^2
    float *out;            // [rows][n_bands]
};

// Largest dynamic LDS of the stream band-power kernel (spectrum band bins x 8 B).
constexpr int kStreamMaxLds = 159 * 1024;
hipError_t launch_stream_append(const StreamParams &p, hipStream_t s);
hipError_t launch_stream_gather(const StreamParams &p, hipStream_t s);
hipError_t launch_stream_bandpower(const StreamBPParams &p, int max_bins, hipStream_t s);

// FP64 generators (run once per plan).
struct GenParams {
    double sfreq;
    int L;
    int F;
    int wavelet;           // 0 Morlet, 1 Gabor, 2 generalized Morse
    double gmw_beta, gmw_gamma;
    const double *freqs;   // [F] device
    const double *sigmas;  // [F] device
    const BandDesc *band;  // [F] device
    float *H;              // packed output
    float2 *tw;            // [L]
};

// Optional pair of events bound to one kernel dispatch (hipExtLaunchKernel):
// they take the dispatch's own start and end timestamps.  Null: untimed.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// LDS bytes of the runtime-radix kernels for padded length L: the buffer
// holds L rounded up to 16 elements (the first-pass slot map stays inside
// aligned blocks of 16).
inline size_t generic_lds_bytes(int L) { return (size_t)((L + 15) & ~15) * 8; }

hipError_t launch_generate(const GenParams &p, int total_bins, hipStream_t s);
// Spectra of sampled wavelets: Hd[f][b] = (1/L) sum_j w[f][j] exp(-2 pi i b
// ((j - c) mod L) / L) in FP64, rounded once; roots: [L] FP64 scratch.
hipError_t launch_user_spectra(const float2 *w, int F, int wl, int c, int L, double2 *roots,
                               float2 *Hd, hipStream_t s);
// Segment inputs of a segmented plan (see MainParams::seg_n).
struct SegGatherParams {
    const float *x;    // [C][N] signal, x_stride elements between channels
    int64_t x_stride;
    int C, N;
    int64_t L_full;    // cyclic period
    int n_seg, B, S, Ls;
    float *xs;         // [C n_seg][Ls]
};
hipError_t launch_segment_gather(const SegGatherParams &p, hipStream_t s);
// Band power from chunk rows: out[c][b][t] = sum over the chunks k of band b
// of part[c][k][t] (the chunk's mean) times its frequency count, over the
// band's count.
struct ChunkReduceParams {
    const float *part;       // [C][n_chunks][N]
    float *out;              // [C][n_bands][N]
    int C, n_chunks, n_bands, N;
    const int *chunk_off;    // [n_chunks + 1] frequency offsets of the chunks
    const int *band_first;   // [n_bands + 1] first chunk of each band
};
hipError_t launch_chunk_reduce(const ChunkReduceParams &p, hipStream_t s);
hipError_t launch_forward(const FwdParams &p, hipStream_t s);
hipError_t launch_main(const MainParams &p, hipStream_t s, LaunchEvents ev = {});
// Register-resident kernels for the padded lengths that have one.
bool fixed_main_available(int L);
hipError_t launch_main_fixed(const MainParams &p, hipStream_t s, LaunchEvents ev = {});
hipError_t launch_forward_fixed(const FwdParams &p, hipStream_t s);
// Transform of p's spectra and forward FFT f of the next batch in one launch.
hipError_t launch_fused_fixed(const MainParams &p, const FwdParams &f, hipStream_t s,
                              LaunchEvents ev = {});

}  // namespace cwtk
