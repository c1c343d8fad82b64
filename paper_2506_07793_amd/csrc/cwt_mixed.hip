// Register-resident FFT kernels for padded lengths that are not powers of two
// (gfx950): L = 200 = 10 x 20, 400 = 20 x 20, 800 = 4 x 10 x 20,
// 1000 = 5 x 20 x 10, 1600 = 4 x 20 x 20, 2000 = 5 x 20 x 20, 2500 =
// 5 x 5 x 20 x 5, 4000 = 10 x 20 x 20, 5000 = 5 x 20 x 10 x 5, 8000 =
// 20 x 20 x 20 and 10000 = 5 x 20 x 20 x 5.
//
// The scheme of the power-of-two kernels, generalised.  Every thread holds
// V = 20 complex values in registers and every radix of the compile-time list
// divides V, so a pass is V / R whole butterflies per thread: thread t of a
// transform's T = L / V threads owns butterflies j = t + kb T, element r of
// butterfly kb in v[kb + r V / R], and the strides and twiddle indexes of every
// pass are compile-time constants.  Before a pass, v[m] is element t + T m of
// its input; after the last, sample t + T m of the output (natural order).
// Since T (10, 20, 40, 50, 80, 100, 125, 200, 250, 400 or 500) is not a
// multiple of the 64-lane wave, a workgroup runs SUB transforms side by side,
// one per group of T threads with its own LDS slab: 32 x 10 threads at
// L = 200, 16 x 20 at 400, 8 x 40 at 800, 5 x 50 at 1000, 4 x 80 at 1600 and
// 3 x 100 at 2000 (5 waves, 4 at L = 1000); 2 x 125 at 2500 and 2 x 200 at
// 4000 (4 and 7 waves); one transform of 250, 400 or 500 threads at 5000,
// 8000 and 10000 (4, 7 and 8 waves).
//
// Inverse kernel.  The wavelet spectrum of one frequency is non-zero only on
// a band of K cyclically consecutive bins.  The first pass (radix R0, no
// twiddles) combines the bins j + r S, r < R0, S = L / R0, in butterfly j;
// when K <= S at most one of them is in the band, at b = j + r* S, so the
// pass reduces to one product per output: element k of butterfly j is
// Z[b] exp(2 pi i r* k / R0), Z[b] = X~[b] H[b].  Those rows skip the first
// pass's transform and the staging of the band through LDS.  Wider bands
// stage their K products in LDS and run every pass.  Complex and power rows
// are one transform each, SUB rows per workgroup; a band-power row is one
// (band, channel) pair per workgroup whose SUB sub-groups take the band's
// frequencies in turn and keep the sum of |W|^2 in registers.
#include "cwt_kernels.hpp"
#include "cwt_mixed.hpp"
#include "fft_core.hpp"

namespace cwtk {

namespace {

constexpr int kMV = 20;  // complex values per thread

template <int... Rs>
struct MList;
template <int R0, int... Rest>
struct MList<R0, Rest...> {
    static constexpr int first = R0;
    static constexpr int product = R0 * MList<Rest...>::product;
    static constexpr bool divides = (kMV % R0 == 0) && MList<Rest...>::divides;
};
template <>
struct MList<> {
    static constexpr int product = 1;
    static constexpr bool divides = true;
};

// Transforms per workgroup.
template <int L>
struct MSub {
    static constexpr int value = (L == 200)    ? 32
                                 : (L == 400)  ? 16
                                 : (L == 800)  ? 8
                                 : (L == 1000) ? 5
                                 : (L == 1600) ? 4
                                 : (L == 2000) ? 3
                                 : (L == 2500 || L == 4000) ? 2
                                                            : 1;
};

// LDS slots.  The buffer after pass p holds element i at slot
// i + C (i div P), (C, P) = MPad<L, p>: a gap of C slots after every P
// elements, which spreads the passes' strided scatters over the banks
// (64-bit writes are conflict-free when the slots of each 16-lane group
// differ modulo 16, reads when those of each 32-lane group differ modulo 32).
// P is a multiple of the storing pass's Ns R and of T, so the gap index is
// one division per butterfly on the store side and a constant on the load
// side.  The gaps and the radix order were chosen by a model of that bank
// rule over every access of these kernels (SUB transforms per workgroup
// included): 2.5 and 2.2 conflict cycles per access summed over the two
// buffers (ideal 2.0), against 3.7 and 2.9 for plain slots with radices
// [5, 10, 20] and [5, 20, 20]; each slab stays within the LDS that keeps 4
// (L = 1000, 2500, 5000), 3 (the other lengths up to 2000) or 2 (L = 4000,
// 8000, 10000) workgroups on a CU.  At L = 800 and 1600 the first radix is 4
// (its first pass is the one a band of at most L / 4 bins skips, which covers
// the EEG bands there), whose stride-4 scatter no gap with P a multiple of T
// spreads: 4.0 and 4.3 in the model against 4.8 and 6.1 for plain slots.
template <int L, int PASS>
struct MPad {  // plain slots: the buffers the model left unpadded
    static constexpr int C = 0, P = L;
};
template <>
struct MPad<2500, 2> {
    static constexpr int C = 5, P = 500;
};
template <>
struct MPad<5000, 2> {
    static constexpr int C = 12, P = 1000;
};
template <>
struct MPad<10000, 2> {
    static constexpr int C = 4, P = 2000;
};
template <>
struct MPad<1000, 0> {
    static constexpr int C = 6, P = 250;
};
template <>
struct MPad<1000, 1> {
    static constexpr int C = 1, P = 100;
};
template <>
struct MPad<200, 0> {
    static constexpr int C = 1, P = 30;
};
template <>
struct MPad<200, 1> {  // two passes: one buffer
    static constexpr int C = 1, P = 30;
};
template <>
struct MPad<400, 0> {
    static constexpr int C = 1, P = 80;
};
template <>
struct MPad<400, 1> {  // two passes: one buffer
    static constexpr int C = 1, P = 80;
};
template <>
struct MPad<800, 0> {
    static constexpr int C = 1, P = 40;
};
template <>
struct MPad<800, 1> {
    static constexpr int C = 4, P = 160;
};
template <>
struct MPad<1600, 0> {
    static constexpr int C = 1, P = 80;
};
template <>
struct MPad<1600, 1> {
    static constexpr int C = 2, P = 80;
};
template <>
struct MPad<4000, 0> {
    static constexpr int C = 1, P = 200;
};
template <>
struct MPad<4000, 1> {
    static constexpr int C = 2, P = 200;
};
template <>
struct MPad<8000, 0> {
    static constexpr int C = 1, P = 400;
};
template <>
struct MPad<8000, 1> {
    static constexpr int C = 4, P = 400;
};
template <>
struct MPad<2000, 0> {
    static constexpr int C = 12, P = 500;
};
template <>
struct MPad<2000, 1> {
    static constexpr int C = 1, P = 100;
};

template <int L, int PASS>
constexpr int pad_span()
{
    return L + MPad<L, PASS>::C * ((L - 1) / MPad<L, PASS>::P);
}

// Complex slots of one transform's LDS slab (the buffers after passes 0, 1
// and, in four-pass lists, 2).
template <int L>
struct MSlab {
    static constexpr int a = pad_span<L, 0>() > pad_span<L, 1>() ? pad_span<L, 0>()
                                                                  : pad_span<L, 1>();
    static constexpr int value = a > pad_span<L, 2>() ? a : pad_span<L, 2>();
};

// exp(2 pi i m / 20), m < 20: the internal roots of the composite radices 10
// and 20 (W_R^m = exp(2 pi i m 20 / R / 20)), as constants rather than table
// loads, so that they take no vector registers.
struct Root20 {
    static constexpr float c[20] = {
        1.0f, 0.95105651629515357212f, 0.80901699437494742410f, 0.58778525229247312917f,
        0.30901699437494742410f, 0.0f, -0.30901699437494742410f, -0.58778525229247312917f,
        -0.80901699437494742410f, -0.95105651629515357212f, -1.0f, -0.95105651629515357212f,
        -0.80901699437494742410f, -0.58778525229247312917f, -0.30901699437494742410f, 0.0f,
        0.30901699437494742410f, 0.58778525229247312917f, 0.80901699437494742410f,
        0.95105651629515357212f};
    static constexpr float s[20] = {
        0.0f, 0.30901699437494742410f, 0.58778525229247312917f, 0.80901699437494742410f,
        0.95105651629515357212f, 1.0f, 0.95105651629515357212f, 0.80901699437494742410f,
        0.58778525229247312917f, 0.30901699437494742410f, 0.0f, -0.30901699437494742410f,
        -0.58778525229247312917f, -0.80901699437494742410f, -0.95105651629515357212f, -1.0f,
        -0.95105651629515357212f, -0.80901699437494742410f, -0.58778525229247312917f,
        -0.30901699437494742410f};
};

// Twiddle methods, as for the power-of-two kernels: every twiddle from the
// table, or w = exp(i theta) from the table and its powers by products.
constexpr int kMTwTable = 0;
constexpr int kMTwPowers = 1;

template <int R, int SIGN, int L, int NS, int TWM>
__device__ __forceinline__ void mpass_compute(cf *v, int t, const cf *__restrict__ tw)
{
    constexpr int T = L / kMV;
    constexpr int NB = kMV / R;
    static_assert(20 % R == 0, "radices of the mixed-radix kernels divide 20");
    // internal twiddles of a composite radix: W_R^m, SIGN's direction
    cf wn[CompSplit<R>::r1 > 0 ? R : 1];
    if constexpr (CompSplit<R>::r1 > 0) {
#pragma unroll
        for (int m = 0; m < R; ++m)
            wn[m] = mk(Root20::c[m * (20 / R)], (float)SIGN * Root20::s[m * (20 / R)]);
    }
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        cf e[R];
#pragma unroll
        for (int r = 0; r < R; ++r) e[r] = v[kb + r * NB];
        if constexpr (NS > 1) {
            const int j = t + kb * T;
            const int jm = j % NS;
            constexpr int step = L / (NS * R);
            cf w[R];
            if (TWM == kMTwTable) {
#pragma unroll
                for (int r = 1; r < R; ++r) w[r] = conj_if<SIGN>(tw[jm * step * r]);
            } else {
                twiddle_powers<R>(conj_if<SIGN>(tw[jm * step]), w);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) e[r] = mul(e[r], w[r]);
        }
        codelet<R, SIGN>(e, wn);
#pragma unroll
        for (int r = 0; r < R; ++r) v[kb + r * NB] = e[r];
    }
}

template <int R, int L, int NS, int PASS>
__device__ __forceinline__ void mpass_store(const cf *v, int t, cf *lds)
{
    constexpr int T = L / kMV;
    constexpr int NB = kMV / R;
    constexpr int C = MPad<L, PASS>::C, P = MPad<L, PASS>::P;
    static_assert(P % (NS * R) == 0 && P % T == 0, "gap period fits the pass and the loads");
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        const int j = t + kb * T;
        const int jm = j % NS;
        // element (j - jm) R + jm + r Ns; its gap index, (j div Ns) div
        // (P / (Ns R)), is j div (P / R)
        const int base = (j - jm) * R + jm + C * (j / (P / R));
#pragma unroll
        for (int r = 0; r < R; ++r) lds[base + r * NS] = v[kb + r * NB];
    }
}

template <int L, int PASS>
__device__ __forceinline__ void mload_columns(cf *v, int t, const cf *lds)
{
    constexpr int T = L / kMV;
    constexpr int C = MPad<L, PASS>::C, P = MPad<L, PASS>::P;
    // t < T and T divides P, so (t + T m) div P = T m div P
#pragma unroll
    for (int m = 0; m < kMV; ++m) v[m] = lds[t + T * m + C * ((T * m) / P)];
}

// Passes PASS, PASS + 1, ... of the list (Ns = NS before the first), data in
// v; every pass but the last goes through LDS, the last leaves the
// natural-order values in v.
template <int SIGN, int L, int NS, int TWM, int PASS, int R, int... Rest>
__device__ __forceinline__ void mrun_passes(cf *v, int t, const cf *__restrict__ tw, cf *lds,
                                            MList<R, Rest...>)
{
    mpass_compute<R, SIGN, L, NS, TWM>(v, t, tw);
    if constexpr (sizeof...(Rest) > 0) {
        __syncthreads();  // everyone has read the previous contents of lds
        mpass_store<R, L, NS, PASS>(v, t, lds);
        __syncthreads();
        mload_columns<L, PASS>(v, t, lds);
        mrun_passes<SIGN, L, NS * R, TWM, PASS + 1>(v, t, tw, lds, MList<Rest...>{});
    }
}

// First inverse pass of a band of K <= S = L / R0 bins starting at bin lo:
// butterfly j's one in-band bin is b = lo + d (mod L), d = (j - lo) mod S,
// when d < K; its outputs Z[b] w^k, w = exp(2 pi i r* / R0), r* = b div S,
// go to LDS in the first pass's output layout (element k at j R0 + k).
template <int L, int R0>
__device__ __forceinline__ void mnarrow_first(const cf *__restrict__ X,
                                              const float *__restrict__ Hf,
                                              const cf *__restrict__ Hcf, int lo, int K,
                                              const cf *__restrict__ tw, cf *lds, int t)
{
    constexpr int T = L / kMV;
    constexpr int S = L / R0;
    constexpr int NB = kMV / R0;  // S / T butterflies per thread
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        const int j = t + kb * T;
        int d = (j - lo) % S;
        if (d < 0) d += S;
        const bool in = d < K;
        const int dc = in ? d : 0;
        int b = lo + dc;
        if (b >= L) b -= L;
        cf z = mk(0.f, 0.f);
        if (K > 0) {  // uniform per transform; loads issued before the select
            const bool upper = b > L / 2;
            cf xv = X[upper ? L - b : b];
            if (upper) xv.y = -xv.y;
            const cf y = Hcf ? mul(xv, Hcf[dc]) : scale(xv, Hf[dc]);
            if (in) z = y;
        }
        cf w[R0];
        twiddle_powers<R0>(tw[(b / S) * S], w);
        // element j R0 + k of the first pass's output buffer
        constexpr int C = MPad<L, 0>::C, P = MPad<L, 0>::P;
        static_assert(P % R0 == 0 && P % T == 0, "gap period fits the first pass");
        const int base = j * R0 + C * (j / (P / R0));
        lds[base] = z;
#pragma unroll
        for (int k = 1; k < R0; ++k) lds[base + k] = mul(z, w[k]);
    }
}

// One workgroup of the inverse kernel: SUB complex / power rows (row item
// blk SUB + g for sub-group g; sub-groups past the last item repeat it and
// store nothing), or one band-power row (band by rank, channel fastest).
template <int MODE, int TWM, int R0, int... Rest>
__device__ __forceinline__ void mixed_main_block(const MainParams &p, int blk)
{
    using RL = MList<R0, Rest...>;
    constexpr int L = RL::product;
    constexpr int T = L / kMV;
    constexpr int SUB = MSub<L>::value;
    constexpr int SL = MSlab<L>::value;
    constexpr int S = L / R0;
    static_assert(RL::divides && L % kMV == 0, "every radix divides the values per thread");
    extern __shared__ cf lds_all[];
    const int N = p.N;
    const int n_items = p.C * p.n_rows;

    int c, row, qb = 0, nq = 1;
    {
        const int g0 = (int)threadIdx.x / T;
        if (MODE == kOutBand) {
            const int rank = blk / p.C;
            c = blk - rank * p.C;
            row = p.grp_off[p.n_rows + 1 + rank];
            qb = p.grp_off[row];
            nq = p.grp_off[row + 1] - qb;
        } else {
            const int it = min(blk * SUB + g0, n_items - 1);
            c = it / p.n_rows;
            row = it - c * p.n_rows;
        }
    }
    // frequency of sub-group j in round r
    auto freq_of = [&](int r, int j) -> int {
        if (MODE == kOutBand) return p.grp_freq[qb + min(r * SUB + j, nq - 1)];
        return min(blk * SUB + j, n_items - 1) % p.n_rows;
    };
    const cf *X0 = reinterpret_cast<const cf *>(p.Xh) + (int64_t)c * p.Lh;
    const cf *tw0 = reinterpret_cast<const cf *>(p.tw);
    float acc[kMV];
#pragma unroll
    for (int m = 0; m < kMV; ++m) acc[m] = 0.f;

    const int rounds = (MODE == kOutBand) ? (nq + SUB - 1) / SUB : 1;
    for (int r = 0; r < rounds; ++r) {
        // the lane, input row and twiddle table are the same in every round;
        // opaque here, so that what derives from them is recomputed per round
        // rather than held (and spilled) across the loop
        int tid = threadIdx.x;
        const cf *X = X0;
        const cf *tw = tw0;
        if (MODE == kOutBand) asm volatile("" : "+v"(tid), "+s"(X), "+s"(tw));
        const int g = tid / T;
        const int t = tid - g * T;
        cf *lds = lds_all + g * SL;
        const bool live = (MODE == kOutBand) ? (r * SUB + g < nq) : (blk * SUB + g < n_items);
        const int f = freq_of(r, g);
        const BandDesc bd = p.band[f];
        const float *Hf = p.H + bd.off;
        const cf *Hcf = p.Hc ? reinterpret_cast<const cf *>(p.Hc) + bd.off : nullptr;
        const int K = bd.K;
        const int lo = bd.lo < 0 ? bd.lo + L : bd.lo;
        // one path for the whole workgroup (the paths differ in their barriers)
        bool narrow = true;
#pragma unroll
        for (int j = 0; j < SUB; ++j) narrow = narrow && p.band[freq_of(r, j)].K <= S;
        if (r > 0) __syncthreads();  // the previous round is done with lds
        cf v[kMV];
        if (narrow) {
            mnarrow_first<L, R0>(X, Hf, Hcf, lo, K, tw, lds, t);
            __syncthreads();
            mload_columns<L, 0>(v, t, lds);
            mrun_passes<1, L, R0, TWM, 1>(v, t, tw, lds, MList<Rest...>{});
        } else {
            // band products y[k] = X~[b] H[k], b = lo + k (mod L), into lds[0, K)
            const int nit = (K + T - 1) / T;
            for (int i = 0; i < nit; ++i) {
                const int k = t + i * T;
                const int kc = k < K ? k : K - 1;
                int b = lo + kc;
                if (b >= L) b -= L;
                const bool upper = b > L / 2;
                cf xv = X[upper ? L - b : b];
                if (upper) xv.y = -xv.y;
                if (k < K) lds[k] = Hcf ? mul(xv, Hcf[kc]) : scale(xv, Hf[kc]);
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kMV; ++m) {
                int o = t + T * m - lo;
                if (o < 0) o += L;
                const cf y = lds[o];
                v[m] = (o < K) ? y : mk(0.f, 0.f);
            }
            mrun_passes<1, L, 1, TWM, 0>(v, t, tw, lds, RL{});
        }
        // v[m] is sample t + T m
        if (MODE == kOutBand) {
            if (live) {
#pragma unroll
                for (int m = 0; m < kMV; ++m) acc[m] += v[m].x * v[m].x + v[m].y * v[m].y;
            }
            continue;
        }
        if (!live) continue;
        const int64_t orow = ((int64_t)c * p.n_rows + row) * N;
#pragma unroll
        for (int m = 0; m < kMV; ++m) {
            const int ts = t + T * m;
            if (N == L || ts < N) {
                const cf w = v[m];
                if (MODE == kOutComplex)
                    reinterpret_cast<float2 *>(p.out)[orow + ts] = make_float2(w.x, w.y);
                else
                    reinterpret_cast<float *>(p.out)[orow + ts] = w.x * w.x + w.y * w.y;
            }
        }
    }
    if (MODE == kOutBand) {
        // sub-group sums through LDS (sub-group g's L floats at g L), added in
        // sub-group order and stored once
        float *orow = reinterpret_cast<float *>(p.out) + ((int64_t)c * p.n_rows + row) * N;
        const float inv_n = 1.0f / (float)nq;
        float *ldsf = reinterpret_cast<float *>(lds_all);
        const int tid = threadIdx.x;
        const int g = tid / T, t = tid - g * T;
        __syncthreads();  // every sub-group is done with its slab
#pragma unroll
        for (int m = 0; m < kMV; ++m) ldsf[g * L + t + T * m] = acc[m];
        __syncthreads();
        for (int o = tid; o < L; o += SUB * T) {
            float a = ldsf[o];
#pragma unroll
            for (int j = 1; j < SUB; ++j) a += ldsf[j * L + o];
            if (N == L || o < N) orow[o] = a * inv_n;
        }
    }
}

// Forward real FFT of channel pair `pair` by thread t of its group (two real
// channels as one complex sequence, then the separation
// X0 = (Z[b] + conj Z[-b]) / 2, X1 = (Z[b] - conj Z[-b]) / (2i) through LDS).
// Pairs past the last channel compute on zeros and store nothing, so every
// group of a workgroup meets the same barriers.
template <int... Rs>
__device__ __forceinline__ void mixed_forward_pair(const FwdParams &p, int pair, int t, cf *lds)
{
    using RL = MList<Rs...>;
    constexpr int L = RL::product;
    constexpr int T = L / kMV;
    const int c0 = 2 * pair;
    const bool has0 = c0 < p.C;
    const bool has1 = (c0 + 1) < p.C;
    const cf *tw = reinterpret_cast<const cf *>(p.tw);
    const int N = p.N;
    cf v[kMV];
    {
        const float *x0 = p.x + (int64_t)(has0 ? c0 : 0) * p.x_stride;
        const float *x1 = p.x + (int64_t)(has1 ? c0 + 1 : 0) * p.x_stride;
#pragma unroll
        for (int m = 0; m < kMV; ++m) {
            const int idx = t + T * m;
            cf z = mk(0.f, 0.f);
            if (has0 && idx < N) {
                z.x = x0[idx];
                if (has1) z.y = x1[idx];
            }
            v[m] = z;
        }
    }
    mrun_passes<-1, L, 1, kMTwPowers, 0>(v, t, tw, lds, RL{});
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kMV; ++m) lds[t + T * m] = v[m];
    __syncthreads();
    if (!has0) return;  // no barrier follows
    float2 *Xa = p.Xh + (int64_t)c0 * p.Lh;
    float2 *Xb = Xa + p.Lh;
    for (int b = t; b < p.Lh; b += T) {
        const cf z = lds[b];
        const cf zn = lds[b == 0 ? 0 : L - b];
        const cf zc = mk(zn.x, -zn.y);
        const cf s = add(z, zc), d = sub(z, zc);
        Xa[b] = make_float2(0.5f * s.x, 0.5f * s.y);
        if (has1) Xb[b] = make_float2(0.5f * d.y, -0.5f * d.x);
    }
}

template <int... Rs>
struct MShape {
    static constexpr int L = MList<Rs...>::product;
    static constexpr int T = L / kMV;
    static constexpr int SUB = MSub<L>::value;
    static constexpr int threads = SUB * T;
    static constexpr size_t lds_bytes = (size_t)SUB * MSlab<L>::value * sizeof(cf);
};

// Waves per SIMD the register budget allows: four (at most 128 registers)
// for complex and power rows with power twiddles, which with a workgroup's
// LDS is 4 workgroups per CU at L = 1000 (16 waves), 3 at L = 200 to 2000
// (15), 2 of 7 waves at 4000 and 8000, 4 of 4 at 2500 and 5000 and 2 of 8 at
// 10000;
// three for band rows (20 running sums) and for table twiddles (their loads
// are issued early), which would otherwise spill.
template <int MODE, int TWM>
struct MWaves {
    static constexpr int value = (MODE == kOutBand || TWM == kMTwTable) ? 3 : 4;
};

template <int MODE, int TWM, int... Rs>
__global__ void __launch_bounds__(MShape<Rs...>::threads)
    __attribute__((amdgpu_waves_per_eu(MWaves<MODE, TWM>::value))) k_mixed_main(MainParams p)
{
    mixed_main_block<MODE, TWM, Rs...>(p, blockIdx.x);
}

template <int... Rs>
__global__ void __launch_bounds__(MShape<Rs...>::threads) k_mixed_forward(FwdParams p)
{
    using SH = MShape<Rs...>;
    extern __shared__ cf lds[];
    const int g = (int)threadIdx.x / SH::T;
    mixed_forward_pair<Rs...>(p, (int)blockIdx.x * SH::SUB + g, (int)threadIdx.x - g * SH::T,
                              lds + g * MSlab<SH::L>::value);
}

// Transform of one batch and forward FFT of the next in one launch: blocks
// [0, n_fwd) take channel pairs of the next batch (SUB per block), the rest
// the transform rows of this batch.
template <int MODE, int TWM, int... Rs>
__global__ void __launch_bounds__(MShape<Rs...>::threads)
    __attribute__((amdgpu_waves_per_eu(MWaves<MODE, TWM>::value)))
    k_mixed_fused(MainParams p, FwdParams f, int n_fwd)
{
    using SH = MShape<Rs...>;
    if ((int)blockIdx.x < n_fwd) {
        extern __shared__ cf lds[];
        const int g = (int)threadIdx.x / SH::T;
        mixed_forward_pair<Rs...>(f, (int)blockIdx.x * SH::SUB + g,
                                  (int)threadIdx.x - g * SH::T, lds + g * MSlab<SH::L>::value);
    } else {
        mixed_main_block<MODE, TWM, Rs...>(p, blockIdx.x - n_fwd);
    }
}

// Workgroups of the inverse kernel: SUB rows each, or one band row each.
template <int... Rs>
int main_blocks(const MainParams &p)
{
    const int64_t items = (int64_t)p.C * p.n_rows;
    return (int)((p.out_mode == kOutBand) ? items
                                          : (items + MShape<Rs...>::SUB - 1) / MShape<Rs...>::SUB);
}

template <int... Rs>
int forward_blocks(const FwdParams &f)
{
    return ((f.C + 1) / 2 + MShape<Rs...>::SUB - 1) / MShape<Rs...>::SUB;
}

template <int MODE, int TWM, int... Rs>
hipError_t launch_mixed_t(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    using SH = MShape<Rs...>;
    hipExtLaunchKernelGGL((k_mixed_main<MODE, TWM, Rs...>), dim3(main_blocks<Rs...>(p)),
                          dim3(SH::threads), SH::lds_bytes, s, ev.start, ev.stop, 0, p);
    return hipGetLastError();
}

template <int MODE, int TWM, int... Rs>
hipError_t launch_mixed_fused_t(const MainParams &p, const FwdParams &f, hipStream_t s,
                                LaunchEvents ev)
{
    using SH = MShape<Rs...>;
    const int n_fwd = forward_blocks<Rs...>(f);
    hipExtLaunchKernelGGL((k_mixed_fused<MODE, TWM, Rs...>),
                          dim3(n_fwd + main_blocks<Rs...>(p)), dim3(SH::threads), SH::lds_bytes,
                          s, ev.start, ev.stop, 0, p, f, n_fwd);
    return hipGetLastError();
}

template <int TWM, int... Rs>
hipError_t launch_mixed_modes(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    switch (p.out_mode) {
    case kOutComplex: return launch_mixed_t<kOutComplex, TWM, Rs...>(p, s, ev);
    case kOutPower: return launch_mixed_t<kOutPower, TWM, Rs...>(p, s, ev);
    default: return launch_mixed_t<kOutBand, TWM, Rs...>(p, s, ev);
    }
}

template <int TWM, int... Rs>
hipError_t launch_mixed_fused_modes(const MainParams &p, const FwdParams &f, hipStream_t s,
                                    LaunchEvents ev)
{
    switch (p.out_mode) {
    case kOutComplex: return launch_mixed_fused_t<kOutComplex, TWM, Rs...>(p, f, s, ev);
    case kOutPower: return launch_mixed_fused_t<kOutPower, TWM, Rs...>(p, f, s, ev);
    default: return launch_mixed_fused_t<kOutBand, TWM, Rs...>(p, f, s, ev);
    }
}

template <int... Rs>
hipError_t launch_mixed_main_v(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    return p.variant == 1 ? launch_mixed_modes<kMTwPowers, Rs...>(p, s, ev)
                          : launch_mixed_modes<kMTwTable, Rs...>(p, s, ev);
}

template <int... Rs>
hipError_t launch_mixed_fused_v(const MainParams &p, const FwdParams &f, hipStream_t s,
                                LaunchEvents ev)
{
    return p.variant == 1 ? launch_mixed_fused_modes<kMTwPowers, Rs...>(p, f, s, ev)
                          : launch_mixed_fused_modes<kMTwTable, Rs...>(p, f, s, ev);
}

template <int... Rs>
hipError_t launch_mixed_forward_t(const FwdParams &f, hipStream_t s)
{
    using SH = MShape<Rs...>;
    hipLaunchKernelGGL((k_mixed_forward<Rs...>), dim3(forward_blocks<Rs...>(f)),
                       dim3(SH::threads), SH::lds_bytes, s, f);
    return hipGetLastError();
}

}  // namespace

bool mixed_main_available(int L)
{
    return L == 200 || L == 400 || L == 800 || L == 1000 || L == 1600 || L == 2000 ||
           L == 2500 || L == 4000 || L == 5000 || L == 8000 || L == 10000;
}

int mixed_block_threads(int L)
{
    switch (L) {
    case 200: return MShape<10, 20>::threads;
    case 400: return MShape<20, 20>::threads;
    case 800: return MShape<4, 10, 20>::threads;
    case 1000: return MShape<5, 20, 10>::threads;
    case 1600: return MShape<4, 20, 20>::threads;
    case 2000: return MShape<5, 20, 20>::threads;
    case 4000: return MShape<10, 20, 20>::threads;
    case 2500: return MShape<5, 5, 20, 5>::threads;
    case 5000: return MShape<5, 20, 10, 5>::threads;
    case 8000: return MShape<20, 20, 20>::threads;
    case 10000: return MShape<5, 20, 20, 5>::threads;
    default: return 0;
    }
}

int reg_schedule(int L, bool band, int *radix, int *threads)
{
    // power-of-two kernels: radix 16 first, L / 16 threads per transform, 4
    // (L <= 4096) or 2 transforms per workgroup in band-power mode
    static const int p1024[] = {16, 16, 4}, p2048[] = {16, 16, 8}, p4096[] = {16, 16, 16},
                     p8192[] = {16, 16, 16, 2}, m200[] = {10, 20}, m400[] = {20, 20},
                     m800[] = {4, 10, 20}, m1000[] = {5, 20, 10},
                     m1600[] = {4, 20, 20}, m2000[] = {5, 20, 20}, m4000[] = {10, 20, 20},
                     m2500[] = {5, 5, 20, 5}, m5000[] = {5, 20, 10, 5}, m8000[] = {20, 20, 20},
                     m10000[] = {5, 20, 20, 5};
    const int *r = nullptr;
    int n = 0;
    switch (L) {
    case 1024: r = p1024, n = 3, *threads = (band ? 4 : 1) * (L / 16); break;
    case 2048: r = p2048, n = 3, *threads = (band ? 4 : 1) * (L / 16); break;
    case 4096: r = p4096, n = 3, *threads = (band ? 4 : 1) * (L / 16); break;
    case 8192: r = p8192, n = 4, *threads = (band ? 2 : 1) * (L / 16); break;
    case 200: r = m200, n = 2, *threads = MShape<10, 20>::threads; break;
    case 400: r = m400, n = 2, *threads = MShape<20, 20>::threads; break;
    case 800: r = m800, n = 3, *threads = MShape<4, 10, 20>::threads; break;
    case 1000: r = m1000, n = 3, *threads = MShape<5, 20, 10>::threads; break;
    case 1600: r = m1600, n = 3, *threads = MShape<4, 20, 20>::threads; break;
    case 2000: r = m2000, n = 3, *threads = MShape<5, 20, 20>::threads; break;
    case 4000: r = m4000, n = 3, *threads = MShape<10, 20, 20>::threads; break;
    case 2500: r = m2500, n = 4, *threads = MShape<5, 5, 20, 5>::threads; break;
    case 5000: r = m5000, n = 4, *threads = MShape<5, 20, 10, 5>::threads; break;
    case 8000: r = m8000, n = 3, *threads = MShape<20, 20, 20>::threads; break;
    case 10000: r = m10000, n = 4, *threads = MShape<5, 20, 20, 5>::threads; break;
    default: return 0;
    }
    for (int i = 0; i < n; ++i) radix[i] = r[i];
    return n;
}

hipError_t launch_main_mixed(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    if (p.C <= 0 || p.n_rows <= 0) return hipSuccess;
    switch (p.rp.L) {
    case 200: return launch_mixed_main_v<10, 20>(p, s, ev);
    case 400: return launch_mixed_main_v<20, 20>(p, s, ev);
    case 800: return launch_mixed_main_v<4, 10, 20>(p, s, ev);
    case 1000: return launch_mixed_main_v<5, 20, 10>(p, s, ev);
    case 1600: return launch_mixed_main_v<4, 20, 20>(p, s, ev);
    case 2000: return launch_mixed_main_v<5, 20, 20>(p, s, ev);
    case 4000: return launch_mixed_main_v<10, 20, 20>(p, s, ev);
    case 2500: return launch_mixed_main_v<5, 5, 20, 5>(p, s, ev);
    case 5000: return launch_mixed_main_v<5, 20, 10, 5>(p, s, ev);
    case 8000: return launch_mixed_main_v<20, 20, 20>(p, s, ev);
    case 10000: return launch_mixed_main_v<5, 20, 20, 5>(p, s, ev);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_forward_mixed(const FwdParams &f, hipStream_t s)
{
    if (f.C <= 0) return hipSuccess;
    switch (f.rp.L) {
    case 200: return launch_mixed_forward_t<10, 20>(f, s);
    case 400: return launch_mixed_forward_t<20, 20>(f, s);
    case 800: return launch_mixed_forward_t<4, 10, 20>(f, s);
    case 1000: return launch_mixed_forward_t<5, 20, 10>(f, s);
    case 1600: return launch_mixed_forward_t<4, 20, 20>(f, s);
    case 2000: return launch_mixed_forward_t<5, 20, 20>(f, s);
    case 4000: return launch_mixed_forward_t<10, 20, 20>(f, s);
    case 2500: return launch_mixed_forward_t<5, 5, 20, 5>(f, s);
    case 5000: return launch_mixed_forward_t<5, 20, 10, 5>(f, s);
    case 8000: return launch_mixed_forward_t<20, 20, 20>(f, s);
    case 10000: return launch_mixed_forward_t<5, 20, 20, 5>(f, s);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_fused_mixed(const MainParams &p, const FwdParams &f, hipStream_t s,
                              LaunchEvents ev)
{
    // both roles have work (a launch of the pipelined batches)
    if (p.C <= 0 || p.n_rows <= 0 || f.C <= 0) return hipErrorInvalidValue;
    switch (p.rp.L) {
    case 200: return launch_mixed_fused_v<10, 20>(p, f, s, ev);
    case 400: return launch_mixed_fused_v<20, 20>(p, f, s, ev);
    case 800: return launch_mixed_fused_v<4, 10, 20>(p, f, s, ev);
    case 1000: return launch_mixed_fused_v<5, 20, 10>(p, f, s, ev);
    case 1600: return launch_mixed_fused_v<4, 20, 20>(p, f, s, ev);
    case 2000: return launch_mixed_fused_v<5, 20, 20>(p, f, s, ev);
    case 4000: return launch_mixed_fused_v<10, 20, 20>(p, f, s, ev);
    case 2500: return launch_mixed_fused_v<5, 5, 20, 5>(p, f, s, ev);
    case 5000: return launch_mixed_fused_v<5, 20, 10, 5>(p, f, s, ev);
    case 8000: return launch_mixed_fused_v<20, 20, 20>(p, f, s, ev);
    case 10000: return launch_mixed_fused_v<5, 20, 20, 5>(p, f, s, ev);
    default: return hipErrorNotSupported;
    }
}

}  // namespace cwtk
