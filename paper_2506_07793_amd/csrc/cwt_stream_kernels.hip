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
// products y[k] = X~[b] H_f[b], b = lo + k, of the frequency are staged in
// LDS and read by every lane; lane t handles trailing samples t, t + T, ...
// < hop.  With s = exp(2 pi i t_a / L) (t_a the sample's index in the
// window), W_f[t_a] = sum over chunks of G bins of
//   exp(2 pi i (lo + k0) t_a / L) * sum_{j < G} y[k0 + j] s^j,
// the inner sum by Horner's rule (one complex multiply-add per bin, no
// table read) and the chunk's root read from the table at an index advanced
// exactly in integers; the rounding of the at most G - 1 products by s stays
// within a few units of the last place of each chunk sum.  (Reading every
// root from the table, one gather per bin, made the kernel bound by those
// gathers: 4.5x slower at L = 5600.)  The lanes' sums of |W_f[t]|^2 are
// reduced in a fixed order and written to part[row][q].
constexpr int kHornerChunk = 8;

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
        const int ta = t0 + t;  // < W <= L
        const cf sr = tw[ta];   // exp(2 pi i t_a / L)
        const int step = (int)(((int64_t)kHornerChunk * ta) % L);
        int idx = (int)(((int64_t)lo_u * ta) % L);  // root index of the chunk's first bin
        float ar = 0.f, ai = 0.f;
        int k0 = 0;
        for (; k0 + kHornerChunk <= K; k0 += kHornerChunk) {
            cf c = ys[k0 + kHornerChunk - 1];
#pragma unroll
            for (int j = kHornerChunk - 2; j >= 0; --j) c = add(mul(c, sr), ys[k0 + j]);
            const cf w = tw[idx];
            ar += c.x * w.x - c.y * w.y;
            ai += c.x * w.y + c.y * w.x;
            idx += step;
            if (idx >= L) idx -= L;
        }
        if (k0 < K) {  // the last, partial chunk
            cf c = ys[K - 1];
            for (int j = K - 2; j >= k0; --j) c = add(mul(c, sr), ys[j]);
            const cf w = tw[idx];
            ar += c.x * w.x - c.y * w.y;
            ai += c.x * w.y + c.y * w.x;
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
