// Split-precision DFT-as-GEMM path on MFMA (gfx950), padded length 4096.
//
// The inverse transform runs as three radix-16 Stockham stages.  Each stage's
// 16-point complex DFTs are one real GEMM per 16 butterflies:
//   [Yr; Yi] = [[Fr, -Fi], [Fi, Fr]] [Xr; Xi],  F[k][r] = exp(+2 pi i k r / 16),
// on v_mfma_f32_16x16x32_{f16,bf16} (M = 16 outputs, K = 32 = re and im of
// the 16 inputs, N = 16 butterflies).  Operands are split into a high and a
// low half-precision part (x = hi + lo) and the product is formed from three
// MFMAs, hi*hi + hi*lo + lo*hi, accumulated in FP32.  For FP16 every
// butterfly's inputs are scaled by a power of two that puts their largest
// magnitude in [2^14, 2^15) (FP16 range; undone exactly after the MFMA); BF16
// keeps FP32's exponent range and is not scaled.  Twiddles are applied in
// FP32 on the VALU when a stage stores its outputs; the DFT constants and
// twiddles are FP64 values rounded once (the plan's twiddle table).  The
// forward transform of the channels (two real channels per complex
// transform) runs as the same three stages with the conjugate matrices.
#include "cwt_internal.hpp"
#include "fft_core.hpp"

using namespace cwtk;

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kL = 4096;
constexpr int kT = 256;

template <int PREC>
struct SplitOps;

template <>
struct SplitOps<CWT_PREC_SPLIT_F16> {
    typedef h8 vec;
    typedef _Float16 scalar;
    static __device__ __forceinline__ void split(float v, _Float16 &hi, _Float16 &lo)
    {
        hi = (_Float16)v;
        lo = (_Float16)(v - (float)hi);
    }
    static __device__ __forceinline__ f4 mfma(vec a, vec b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    static constexpr bool kScale = true;
};

template <>
struct SplitOps<CWT_PREC_SPLIT_BF16> {
    typedef b8 vec;
    typedef __bf16 scalar;
    static __device__ __forceinline__ void split(float v, __bf16 &hi, __bf16 &lo)
    {
        hi = (__bf16)v;
        lo = (__bf16)(v - (float)hi);
    }
    static __device__ __forceinline__ f4 mfma(vec a, vec b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static constexpr bool kScale = false;
};

// Largest power-of-two exponent e with max * 2^e < 2^15 (0 when max is 0).
__device__ __forceinline__ int fp16_exponent(float m)
{
    if (!(m > 0.f)) return 0;
    // m = f 2^e with f in [0.5, 1), so floor(log2 m) = e - 1
    return 15 - __builtin_amdgcn_frexp_expf(m);
}

// DFT-16 operands of lane (n, q): row m = n, columns k = 8 q + i of
// [[Fr, -Fi], [Fi, Fr]] with F[m][r] = exp(SIGN 2 pi i m r / 16), from the
// 16th roots of unity of the twiddle table (FP64 values rounded once), split
// into high and low parts.
template <int SIGN, class Ops>
__device__ __forceinline__ void dft16_operands(const cf *root16, int n, int q,
                                               typename Ops::vec &ar_hi, typename Ops::vec &ar_lo,
                                               typename Ops::vec &ai_hi, typename Ops::vec &ai_lo)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 8 * q + i;
        const int r = k & 15;
        const cf w = root16[(n * r) & 15];
        const float wy = SIGN > 0 ? w.y : -w.y;
        // columns 0..15 multiply Xr, 16..31 multiply Xi
        const float fr = (k < 16) ? w.x : -wy;
        const float fi = (k < 16) ? wy : w.x;
        typename Ops::scalar h, l;
        Ops::split(fr, h, l);
        ar_hi[i] = h;
        ar_lo[i] = l;
        Ops::split(fi, h, l);
        ai_hi[i] = h;
        ai_lo[i] = l;
    }
}

// The 16-point DFTs of 16 butterflies as split-precision MFMAs: v holds this
// lane's 8 inputs (lane (n, q): butterfly n, real parts of inputs 8 q .. 8 q + 7
// for q < 2, imaginary parts of inputs 8 (q - 2) .. for q >= 2).  On return
// zr / zi hold outputs 4 q .. 4 q + 3 of butterfly n, scaled by 2^e (FP16:
// the butterfly's largest input magnitude scaled into [2^14, 2^15)).
template <class Ops>
__device__ __forceinline__ void dft16_mfma(const float *v, typename Ops::vec ar_hi,
                                           typename Ops::vec ar_lo, typename Ops::vec ai_hi,
                                           typename Ops::vec ai_lo, f4 &zr, f4 &zi, int &e)
{
    e = 0;
    if (Ops::kScale) {
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[i]));
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        e = fp16_exponent(m);
    }
    typename Ops::vec bh, bl;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        typename Ops::scalar h, l;
        Ops::split(ldexpf(v[i], e), h, l);
        bh[i] = h;
        bl[i] = l;
    }
    zr = f4{0.f, 0.f, 0.f, 0.f};
    zi = f4{0.f, 0.f, 0.f, 0.f};
    zr = Ops::mfma(ar_hi, bh, zr);
    zr = Ops::mfma(ar_hi, bl, zr);
    zr = Ops::mfma(ar_lo, bh, zr);
    zi = Ops::mfma(ai_hi, bh, zi);
    zi = Ops::mfma(ai_hi, bl, zi);
    zi = Ops::mfma(ai_lo, bh, zi);
}

}  // namespace

// Four workgroups (four waves per SIMD) per CU: the register budget this
// leaves (128) holds the kernel without spills, and it runs about 10% faster
// than at three.
template <int MODE, int PREC>
__global__ void __launch_bounds__(kT, 4) k_split_main(MainParams p)
{
    typedef SplitOps<PREC> Ops;
    typedef typename Ops::vec vec;
    __shared__ cf lds[kL];
    __shared__ cf root16[16];  // exp(2 pi i e / 16), from the twiddle table
    float *ldsf = reinterpret_cast<float *>(lds);
    const int tid = threadIdx.x;
    const int N = p.N;
    const cf *tw = reinterpret_cast<const cf *>(p.tw);

    if (tid < 16) root16[tid] = tw[tid * (kL / 16)];
    __syncthreads();

    vec ar_hi, ar_lo, ai_hi, ai_lo;
    dft16_operands<1, Ops>(root16, tid & 15, (tid & 63) >> 4, ar_hi, ar_lo, ai_hi, ai_lo);

    const int c = blockIdx.x / p.n_rows;
    const int row = blockIdx.x - c * p.n_rows;
    int qb, qe;
    if (MODE == kOutBand) {
        qb = p.grp_off[row];
        qe = p.grp_off[row + 1];
    } else {
        qb = row;
        qe = row + 1;
    }
    const cf *X = reinterpret_cast<const cf *>(p.Xh) + (int64_t)c * p.Lh;
    float *orow_band = reinterpret_cast<float *>(p.out) + ((int64_t)c * p.n_rows + row) * N;
    const float inv_n = 1.0f / (float)(qe - qb);
    // Band power: each lane owns the same 16 output samples of every
    // frequency's transform (slot j + 256 k of the last stage), so the sum
    // over the band's frequencies stays in registers and the row is stored
    // once.
    float acc[4][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[g][i] = 0.f;

    for (int qq = qb; qq < qe; ++qq) {
        const int f = (MODE == kOutBand) ? p.grp_freq[qq] : qq;
        const BandDesc bd = p.band[f];
        const float *Hf = p.H + bd.off;
        const int K = bd.K;
        const int lo_u = bd.lo < 0 ? bd.lo + kL : bd.lo;
        float2 *ocx = reinterpret_cast<float2 *>(p.out) + ((int64_t)c * p.n_rows + f) * N;
        float *opw = reinterpret_cast<float *>(p.out) + ((int64_t)c * p.n_rows + f) * N;
        if (qq != qb) __syncthreads();
        // Over a band's frequencies this body repeats with the same lane, input
        // row and twiddle table.  The compiler would hoist every address and
        // index that depends only on those out of the loop, holding far more
        // registers than the budget of four workgroups per CU leaves, and
        // spill.  Here they are made opaque, so they are recomputed per
        // frequency; the other modes run the body once and are unaffected.
        const cf *Xq = X;
        const cf *twq = tw;
        int tq = tid;
        if (MODE == kOutBand) asm volatile("" : "+s"(Xq), "+s"(twq), "+v"(tq));
        const int wave = tq >> 6, n = (tq & 63) & 15, q = (tq & 63) >> 4;

        // A band of at most L/16 bins leaves one nonzero input in each
        // first-stage butterfly (the 16 inputs j + 256 r lie 256 bins apart):
        // its outputs are that input times exp(2 pi i r0 k / 16), written here
        // in FP32 with the second stage's twiddle folded in, and the MFMA
        // stages start at the second.
        const bool band = K <= kL / 16;
        if (band) {
#pragma unroll 1
            for (int m = 0; m < kL / kT; ++m) {
                const int d = tq + kT * m;  // first-stage output slot 16 j + k
                const int j = d >> 4, k = d & 15;
                const int o = (j - lo_u) & 255;  // band offset of the bin = j mod 256
                cf val = mk(0.f, 0.f);
                if (o < K) {
                    const int b = (lo_u + o) & (kL - 1);
                    const bool upper = b > kL / 2;
                    cf xv = Xq[upper ? kL - b : b];
                    if (upper) xv.y = -xv.y;
                    // exp(2 pi i r0 k / 16) of input r0 = b div 256, then the
                    // second stage's twiddle of slot d (d div 256 = m)
                    const cf y = mul(scale(xv, Hf[o]), root16[((b >> 8) * k) & 15]);
                    val = mul(y, twq[(16 * k * m) & (kL - 1)]);
                }
                lds[d] = val;
            }
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int Ns = 1 << (4 * s);
            if (s == 0 && band) continue;
            f4 dr[4], di[4];
            int ex[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int j = 64 * wave + 16 * g + n;
                float v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int r = 8 * (q & 1) + i;
                    const int idx = j + 256 * r;  // Stockham input element (j, r)
                    if (s == 0) {
                        const int o = (idx - lo_u) & (kL - 1);
                        float val = 0.f;
                        if (o < K) {
                            const bool upper = idx > kL / 2;
                            const cf xv = Xq[upper ? kL - idx : idx];
                            const float part = (q >> 1) ? (upper ? -xv.y : xv.y) : xv.x;
                            val = part * Hf[o];
                        }
                        v[i] = val;
                    } else {
                        v[i] = ldsf[2 * idx + (q >> 1)];
                    }
                }
                dft16_mfma<Ops>(v, ar_hi, ar_lo, ai_hi, ai_lo, dr[g], di[g], ex[g]);
            }
            __syncthreads();  // every wave has read this stage's inputs
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int j = 64 * wave + 16 * g + n;
                const int jm = j & (Ns - 1);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = 4 * q + i;
                    cf y = mk(ldexpf(dr[g][i], -ex[g]), ldexpf(di[g][i], -ex[g]));
                    const int d = (j - jm) * 16 + jm + k * Ns;  // Stockham output slot
                    if (s < 2) {
                        // next stage's twiddle on its input element (d mod 256, d / 256)
                        const int Nn = Ns * 16;
                        const int jn = d & 255, rn = d >> 8;
                        y = mul(y, twq[(jn & (Nn - 1)) * rn * (kL / (Nn * 16))]);
                        lds[d] = y;
                    } else if (MODE == kOutBand) {
                        acc[g][i] += y.x * y.x + y.y * y.y;
                    } else if (d < N) {
                        if (MODE == kOutComplex)
                            ocx[d] = make_float2(y.x, y.y);
                        else
                            opw[d] = y.x * y.x + y.y * y.y;
                    }
                }
            }
            if (s < 2) __syncthreads();
        }
    }
    if (MODE == kOutBand) {
        // last-stage slot of (g, i): j + 256 k with j = 64 wave + 16 g + n < 256
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int d = 64 * (tid >> 6) + 16 * g + (tid & 15) + 256 * (4 * ((tid & 63) >> 4) + i);
                if (d < N) orow_band[d] = acc[g][i] * inv_n;
            }
    }
}

// Forward transform of two real channels packed as z = x0 + i x1 (zero
// beyond N), as the same three radix-16 stages with F[k][r] =
// exp(-2 pi i k r / 16) and conjugated twiddles, then the separation
// X0 = (Z[b] + conj Z[-b]) / 2, X1 = (Z[b] - conj Z[-b]) / (2i) into the half
// spectra.
template <int PREC>
__global__ void __launch_bounds__(kT, 4) k_split_forward(FwdParams p)
{
    typedef SplitOps<PREC> Ops;
    typedef typename Ops::vec vec;
    __shared__ cf lds[kL];
    __shared__ cf root16[16];
    float *ldsf = reinterpret_cast<float *>(lds);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, q = lane >> 4;
    const int N = p.N;
    const cf *tw = reinterpret_cast<const cf *>(p.tw);

    if (tid < 16) root16[tid] = tw[tid * (kL / 16)];
    __syncthreads();

    vec ar_hi, ar_lo, ai_hi, ai_lo;
    dft16_operands<-1, Ops>(root16, n, q, ar_hi, ar_lo, ai_hi, ai_lo);

    const int c0 = 2 * blockIdx.x;
    const bool has1 = (c0 + 1) < p.C;
    // lanes q < 2 read the real parts (channel c0), q >= 2 the imaginary
    // parts (channel c0 + 1, zero when there is none)
    const float *xq = p.x + (int64_t)(c0 + ((q >> 1) & (int)has1)) * p.x_stride;
    const bool live = (q >> 1) == 0 || has1;

#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int Ns = 1 << (4 * s);
        f4 dr[4], di[4];
        int ex[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int j = 64 * wave + 16 * g + n;
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int r = 8 * (q & 1) + i;
                const int idx = j + 256 * r;  // Stockham input element (j, r)
                if (s == 0)
                    v[i] = (live && idx < N) ? xq[idx] : 0.f;
                else
                    v[i] = ldsf[2 * idx + (q >> 1)];
            }
            dft16_mfma<Ops>(v, ar_hi, ar_lo, ai_hi, ai_lo, dr[g], di[g], ex[g]);
        }
        __syncthreads();  // every wave has read this stage's inputs
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int j = 64 * wave + 16 * g + n;
            const int jm = j & (Ns - 1);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = 4 * q + i;
                cf y = mk(ldexpf(dr[g][i], -ex[g]), ldexpf(di[g][i], -ex[g]));
                const int d = (j - jm) * 16 + jm + k * Ns;  // Stockham output slot
                if (s < 2) {
                    // next stage's twiddle, conjugated, on its input element
                    const int Nn = Ns * 16;
                    const int jn = d & 255, rn = d >> 8;
                    const cf w = tw[(jn & (Nn - 1)) * rn * (kL / (Nn * 16))];
                    y = mul(y, mk(w.x, -w.y));
                }
                lds[d] = y;  // the last stage leaves Z in natural order
            }
        }
        __syncthreads();
    }
    float2 *X0 = p.Xh + (int64_t)c0 * p.Lh;
    float2 *X1 = X0 + p.Lh;
    for (int b = tid; b < p.Lh; b += kT) {
        const cf z = lds[b];
        const cf zn = lds[(kL - b) & (kL - 1)];
        const cf zc = mk(zn.x, -zn.y);
        const cf sm = add(z, zc), df = sub(z, zc);
        X0[b] = make_float2(0.5f * sm.x, 0.5f * sm.y);
        if (has1) X1[b] = make_float2(0.5f * df.y, -0.5f * df.x);
    }
}

namespace cwtrt {

bool split_precision_available() { return true; }

int prepare_split_precision(cwt_plan &P, hipStream_t)
{
    if (P.L != kL)
        return fail(CWT_E_UNSUPPORTED,
                    "split-precision MFMA path is built for padded length %d (plan has %d)", kL,
                    P.L);
    return CWT_OK;
}

void release_split_precision(cwt_plan &) {}

size_t split_workspace_bytes(const cwt_plan &, int64_t) { return 0; }

template <int MODE, int PREC>
static hipError_t launch_split_t(const MainParams &mp, hipStream_t s, LaunchEvents ev)
{
    hipExtLaunchKernelGGL((k_split_main<MODE, PREC>), dim3(mp.C * mp.n_rows), dim3(kT), 0, s,
                          ev.start, ev.stop, 0, mp);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_split_modes(const MainParams &mp, hipStream_t s, LaunchEvents ev)
{
    switch (mp.out_mode) {
    case kOutComplex: return launch_split_t<kOutComplex, PREC>(mp, s, ev);
    case kOutPower: return launch_split_t<kOutPower, PREC>(mp, s, ev);
    default: return launch_split_t<kOutBand, PREC>(mp, s, ev);
    }
}

int enqueue_transform_split(const cwt_plan &P, int64_t C, void *out, void *ws, hipStream_t s)
{
    if (C == 0) return CWT_OK;
    MainParams mp{};
    mp.Xh = reinterpret_cast<const float2 *>(ws);
    mp.Lh = P.L / 2 + 1;
    mp.H = P.d_H;
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
    float *part = nullptr;
    if (P.n_chunks) {  // chunk rows into the partial rows, then the band means
        part = chunk_partials(P, C, ws);
        mp.out = part;
        mp.n_rows = P.n_chunks;
        mp.grp_off = P.d_chunk;
    }
    const LaunchEvents ev = next_launch_events(P);
    hipError_t e = (P.opts.precision == CWT_PREC_SPLIT_F16)
                       ? launch_split_modes<CWT_PREC_SPLIT_F16>(mp, s, ev)
                       : launch_split_modes<CWT_PREC_SPLIT_BF16>(mp, s, ev);
    if (e != hipSuccess) return hip_fail(e, "split-precision transform launch");
    if (part) return enqueue_chunk_reduce(P, C, part, out, s);
    return CWT_OK;
}

int enqueue_forward_split(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride,
                          void *ws, hipStream_t s)
{
    if (C == 0) return CWT_OK;
    FwdParams fp{};
    fp.x = x;
    fp.C = (int)C;
    fp.N = (int)P.n;
    fp.x_stride = x_stride;
    fp.Xh = reinterpret_cast<float2 *>(ws);
    fp.Lh = P.L / 2 + 1;
    fp.tw = P.d_tw;
    fp.rp = P.rp;
    const dim3 grid((unsigned)((C + 1) / 2));
    if (P.opts.precision == CWT_PREC_SPLIT_F16)
        hipLaunchKernelGGL(k_split_forward<CWT_PREC_SPLIT_F16>, grid, dim3(kT), 0, s, fp);
    else
        hipLaunchKernelGGL(k_split_forward<CWT_PREC_SPLIT_BF16>, grid, dim3(kT), 0, s, fp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "split-precision forward launch");
    return CWT_OK;
}

int enqueue_execute_split(const cwt_plan &P, const float *x, int64_t C, int64_t x_stride,
                          void *out, void *ws, hipStream_t s)
{
    int rc = enqueue_forward_split(P, x, C, x_stride, ws, s);
    if (rc != CWT_OK) return rc;
    return enqueue_transform_split(P, C, out, ws, s);
}

}  // namespace cwtrt
