// HIP kernels of the streaming form: ring append, window gather and the
// trailing-hop band power of each window.
//
// A session keeps the last R >= W samples of each channel in a device ring.
// Each completed hop appends its samples; once W samples have arrived, the
// window of the W samples ending with the hop (oldest first) is transformed:
// the forward FFT of the window uses
// the plain path's kernel, and this file's k_stream_freqpower evaluates the
// inverse transform only at the hop's trailing samples t = W - hop .. W - 1,
//   W_f[t] = sum over stored bins b of X~[b] H_f[b] exp(2 pi i b t / L),
// one workgroup per (window-channel row, frequency), and k_stream_bandreduce
// averages |W_f[t]|^2 over the band's frequencies and over those t.
#include "cwt_kernels.hpp"
#include "fft_core.hpp"

namespace cwtk {

__global__ void k_stream_append(StreamParams p)
{
    const StreamJob jb = p.jobs[blockIdx.x];
    const int c = blockIdx.y;
    const float *src = p.slab + jb.slab_off + (int64_t)c * p.hop;
    float *ring = jb.ring + (int64_t)c * p.R;
    for (int k = threadIdx.x; k < p.hop; k += blockDim.x) {
        int q = jb.pos + k;
        if (q >= p.R) q -= p.R;
        ring[q] = src[k];
    }
}

__global__ void k_stream_gather(StreamParams p)
{
    const StreamJob jb = p.jobs[blockIdx.x];
    if (jb.emit_row < 0) return;
    const int c = blockIdx.y;
    const float *ring = jb.ring + (int64_t)c * p.R;
    float *dst = p.xb + ((int64_t)jb.emit_row * p.C + c) * p.W;
    // the window ends with this job's hop: its oldest sample is W - hop
    // slots before the hop's first one (pos, hop <= W <= R)
    int start = jb.pos + p.hop - p.W;
    if (start < 0) start += p.R;
    for (int k = threadIdx.x; k < p.W; k += blockDim.x) {
        int q = start + k;
        if (q >= p.R) q -= p.R;
        dst[k] = ring[q];
    }
}

hipError_t launch_stream_append(const StreamParams &p, hipStream_t s)
{
    if (p.n_jobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stream_append, dim3(p.n_jobs, p.C), dim3(128), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_stream_gather(const StreamParams &p, hipStream_t s)
{
    if (p.n_jobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stream_gather, dim3(p.n_jobs, p.C), dim3(256), 0, s, p);
    return hipGetLastError();
}

// One workgroup per (window-channel row, grouped frequency): the band
// products X~[b] H_f[b] of the frequency are staged in LDS and read by every
// lane; lane t handles trailing samples t, t + T, ... < hop, with the
// twiddles exp(2 pi i b t / L) read from the table, the index advanced
// exactly in integers.  The lanes' sums of |W_f[t]|^2 are reduced in a fixed
// order and written to part[row][q].
__global__ void __launch_bounds__(128) k_stream_freqpower(StreamBPParams p)
{
    extern __shared__ cf ys[];
    __shared__ float red[128];
    const int row = blockIdx.x, q = blockIdx.y;
    const int tid = threadIdx.x, T = blockDim.x;
    const int L = p.L, Lh = p.Lh;
    const cf *X = reinterpret_cast<const cf *>(p.Xh) + (int64_t)row * Lh;
    const cf *tw = reinterpret_cast<const cf *>(p.tw);
    const int t0 = p.W - p.hop;
    const BandDesc bd = p.band[p.grp_freq[q]];
    const float *Hf = p.H + bd.off;
    const int K = bd.K;
    const int lo_u = bd.lo < 0 ? bd.lo + L : bd.lo;
    for (int k = tid; k < K; k += T) {
        int b = lo_u + k;
        if (b >= L) b -= L;
        const bool upper = 2 * b > L;
        cf xv = X[upper ? L - b : b];
        if (upper) xv.y = -xv.y;
        ys[k] = scale(xv, Hf[k]);
    }
    __syncthreads();
    float psum = 0.f;
    for (int t = tid; t < p.hop; t += T) {
        const int ta = t0 + t;
        int idx = (int)(((int64_t)lo_u * ta) % L);
        float ar = 0.f, ai = 0.f;
        for (int k = 0; k < K; ++k) {
            const cf y = ys[k];
            const cf w = tw[idx];
            ar += y.x * w.x - y.y * w.y;
            ai += y.x * w.y + y.y * w.x;
            idx += ta;
            if (idx >= L) idx -= L;
        }
        psum += ar * ar + ai * ai;
    }
    red[tid] = psum;
    __syncthreads();
    for (int s = T / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) p.part[(int64_t)row * p.n_grouped + q] = red[0];
}

// out[row][band] = mean over the band's frequencies and the hop's samples,
// the frequencies summed in band order.
__global__ void __launch_bounds__(256) k_stream_bandreduce(StreamBPParams p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)p.rows * p.n_bands) return;
    const int row = (int)(i / p.n_bands), bnd = (int)(i - (int64_t)row * p.n_bands);
    const int qb = p.grp_off[bnd], qe = p.grp_off[bnd + 1];
    const float *pr = p.part + (int64_t)row * p.n_grouped;
    float s = 0.f;
    for (int q = qb; q < qe; ++q) s += pr[q];
    p.out[i] = s / ((float)(qe - qb) * (float)p.hop);
}

hipError_t launch_stream_bandpower(const StreamBPParams &p, int max_bins, hipStream_t s)
{
    if (p.rows == 0) return hipSuccess;
    if (p.n_grouped > 0) {
        const size_t lds = (size_t)(max_bins > 0 ? max_bins : 1) * sizeof(cf);
        // once per process, for the largest dynamic LDS any plan may ask for
        // (stream sessions accept spectrum bands up to this size)
        static const bool attr_set = [] {
            (void)hipFuncSetAttribute((const void *)k_stream_freqpower,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)kStreamMaxLds);
            return true;
        }();
        (void)attr_set;
        // one wave covers hops up to 64 samples; longer hops use two
        const int threads = p.hop <= 64 ? 64 : 128;
        hipLaunchKernelGGL(k_stream_freqpower, dim3(p.rows, p.n_grouped), dim3(threads), lds, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t n = (int64_t)p.rows * p.n_bands;
    hipLaunchKernelGGL(k_stream_bandreduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace cwtk
