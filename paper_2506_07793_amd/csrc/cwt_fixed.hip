// Register-resident FFT kernels for power-of-two padded lengths (gfx950).
//
// Each workgroup of T = L/16 threads transforms one length-L sequence; every
// thread holds 16 complex values in registers and the radix passes exchange
// data through LDS.  LDS slots are XOR-swizzled (the low four index bits
// XORed with higher bits) so that neither the strided writes of the first
// passes nor the unit-stride reads meet bank conflicts (see sw() below for
// the gfx950 rule).  Twiddles come from the plan's exp(2 pi i m / L) table.  The
// radix schedule is a compile-time list whose first entry is 16, so every
// pass is fully unrolled with constant strides.
//
// Inverse kernel (k_fixed_main): the wavelet spectrum of one frequency is
// non-zero only on a band of K consecutive bins (cyclically).  Bands of at
// most 256 bins take the band path below: the bins, pre-multiplied by the
// phase of each output residue, fill the L LDS slots, and two radix-16
// passes finish the transform (about two thirds of the full transform's
// work, and no carrier multiply).  Wider bands stage their K products
// X~[b] H[b] in LDS and run the full set of passes.  Both leave thread t
// with the natural-order samples t + T m, which it stores straight to
// global memory.
#include "cwt_kernels.hpp"
#include "fft_core.hpp"

namespace cwtk {

namespace {

constexpr int kV = 16;  // values per thread
typedef float f2v __attribute__((ext_vector_type(2)));

// Slot of element i: the low four bits are XORed with bits 4-7 and 8-11.  On
// gfx950 a 64-bit LDS read is conflict-free when the slots of each 32-lane
// group differ modulo 32, a 64-bit write when those of each 16-lane group
// differ modulo 16; with this map the unit-stride column reads t + T m, the
// radix-16 scatter 16 t + r and both second-pass scatters satisfy that.
__device__ __forceinline__ int sw(int i) { return i ^ (((i >> 4) ^ (i >> 8)) & 15); }

// w[r] = exp(SIGN 2 pi i base r / L) for 0 < r < R, from the table.
template <int R, int SIGN>
__device__ __forceinline__ void table_twiddles(const cf *__restrict__ tw, int base, cf *w)
{
#pragma unroll
    for (int r = 1; r < R; ++r) w[r] = conj_if<SIGN>(tw[base * r]);
}

template <int... Rs>
struct RList;

template <int R0, int... Rest>
struct RList<R0, Rest...> {
    static constexpr int first = R0;
    static constexpr int count = 1 + sizeof...(Rest);
    static constexpr int product = R0 * RList<Rest...>::product;
};
template <>
struct RList<> {
    static constexpr int count = 0;
    static constexpr int product = 1;
};

// One register-resident Stockham pass of radix R on v[16] (thread t holds
// butterflies j = t + kb T, element r of butterfly kb in v[kb + r 16/R]).
// Input is already in v; the result stays in v.
// Twiddle methods: kTwTable reads every twiddle from the table; kTwPowers
// reads w = exp(i theta) once per butterfly and forms w^r by balanced products.
constexpr int kTwTable = 0;
constexpr int kTwPowers = 1;

template <int R, int SIGN, int L, int NS, int TWM>
__device__ __forceinline__ void reg_pass_compute(cf *v, int t, const cf *__restrict__ tw)
{
    constexpr int T = L / kV;
    constexpr int NB = kV / R;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        cf e[R];
#pragma unroll
        for (int r = 0; r < R; ++r) e[r] = v[kb + r * NB];
        if (NS > 1) {
            const int j = t + kb * T;
            const int jm = j & (NS - 1);
            cf w[R];
            if (TWM == kTwTable)
                table_twiddles<R, SIGN>(tw, jm * (L / (NS * R)), w);
            else
                twiddle_powers<R>(conj_if<SIGN>(tw[jm * (L / (NS * R))]), w);
#pragma unroll
            for (int r = 1; r < R; ++r) e[r] = mul(e[r], w[r]);
        }
        Dft<R, SIGN>::run(e);
#pragma unroll
        for (int r = 0; r < R; ++r) v[kb + r * NB] = e[r];
    }
}

template <int R, int L, int NS>
__device__ __forceinline__ void reg_pass_store_lds(const cf *v, int t, cf *lds)
{
    constexpr int T = L / kV;
    constexpr int NB = kV / R;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
        const int j = t + kb * T;
        const int jm = j & (NS - 1);
        const int base = (j - jm) * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[sw(base + r * NS)] = v[kb + r * NB];
    }
}

template <int L>
__device__ __forceinline__ void load_lds_columns(cf *v, int t, const cf *lds)
{
    constexpr int T = L / kV;
#pragma unroll
    for (int m = 0; m < kV; ++m) v[m] = lds[sw(t + T * m)];
}

// Passes [P, end) of the radix list, data in v (already loaded for pass P).
// Every pass but the last writes LDS and reloads; the last leaves the
// natural-order values in v.
template <int SIGN, int L, int NS, int TWM, int R, int... Rest>
__device__ __forceinline__ void run_passes(cf *v, int t, const cf *__restrict__ tw, cf *lds,
                                           RList<R, Rest...>)
{
    reg_pass_compute<R, SIGN, L, NS, TWM>(v, t, tw);
    if constexpr (sizeof...(Rest) > 0) {
        __syncthreads();  // everyone has read the previous contents of lds
        reg_pass_store_lds<R, L, NS>(v, t, lds);
        __syncthreads();
        load_lds_columns<L>(v, t, lds);
        run_passes<SIGN, L, NS * R, TWM>(v, t, tw, lds, RList<Rest...>{});
    }
}

// ---------------------------------------------------------- band path --
// Inverse transform of a spectrum that is non-zero on at most 256 consecutive
// bins (cyclically), for L = 256 NV.  With n = NV u + v (v < NV, u < 256) and
// every in-band bin written b = s + 256 a (s = b mod 256),
//   y[NV u + v] = sum_s P_v[s] exp(2 pi i s u / 256),
//   P_v[s]      = Z[b] exp(2 pi i b v / L),
// because exp(2 pi i b n / L) = exp(2 pi i s u / 256) exp(2 pi i b v / L)
// (the factor exp(2 pi i a u) is 1).  So the band's own position (its
// carrier) is absorbed exactly: NV transforms of length 256, each one radix-16
// pass without twiddles (over s = k1 + 16 k2, k2 first) and one with the
// twiddle exp(2 pi i k1 u1 / 256), u = u1 + 16 u2.  The last pass leaves
// thread t = NV u1 + v with samples t + T u2, the same natural order as the
// full transform.
constexpr int kBandMax = 256;

// LDS slot of P_v[s]: rows of 256, bit 4 flipped on odd rows so that the two
// rows a 32-lane group reads fall in different bank halves.
__device__ __forceinline__ int band_p_slot(int v, int s) { return v * 256 + (s ^ ((v & 1) << 4)); }

template <int L, int TWM>
__device__ __forceinline__ void band_transform(const cf *__restrict__ X,
                                               const float *__restrict__ Hf,
                                               const cf *__restrict__ Hcf, int lo_u, int K,
                                               const cf *__restrict__ tw, cf *lds, int t, cf *v_out)
{
    constexpr int NV = L / 256;
    constexpr int T = L / kV;
    constexpr int VB = NV < 16 ? NV : 16;  // residues per prologue item
    constexpr int NIT = 256 * (NV / VB);    // prologue items (bin, residue block)
    constexpr int LOG_VB = __builtin_ctz(VB);
    static_assert(NV >= 4 && NV <= 32, "band path covers L = 1024 .. 8192");
    static_assert(NIT % T == 0, "whole prologue rounds");

    // 1) P_v[s] for every slot: item k < 256 of residue block vb takes bin
    //    b = lo + k; items k >= K are the empty slots and write zeros.
#pragma unroll
    for (int it0 = 0; it0 < NIT; it0 += T) {
        const int it = it0 + t;
        const int k = it & 255, vb = it >> 8;
        const int b = (lo_u + k) & (L - 1);
        const int s = b & 255;
        cf zz[VB];
#pragma unroll
        for (int i = 0; i < VB; ++i) zz[i] = mk(0.f, 0.f);
        if (k < K) {
            const bool upper = b > L / 2;
            cf xv = X[upper ? L - b : b];
            if (upper) xv.y = -xv.y;
            cf z = Hcf ? mul(xv, Hcf[k]) : scale(xv, Hf[k]);
            // exp(2 pi i b 2^j / L) straight from the table (each rounded once)
            cf pw[LOG_VB + 1];
#pragma unroll
            for (int j = 0; j <= LOG_VB; ++j) pw[j] = tw[(b << j) & (L - 1)];
            if (NV > VB && vb) z = mul(z, pw[LOG_VB]);  // residues 16 .. 31
            zz[0] = z;
#pragma unroll
            for (int j = 0; j < LOG_VB; ++j)
#pragma unroll
                for (int i = 0; i < (1 << j); ++i) zz[(1 << j) + i] = mul(zz[i], pw[j]);
        }
#pragma unroll
        for (int i = 0; i < VB; ++i) lds[band_p_slot(vb * VB + i, s)] = zz[i];
    }
    __syncthreads();

    // 2) radix 16 over k2 for thread (k1, v) = (t mod 16, t / 16); slot
    //    k1 + 16 k2 of row v is base + 16 (k2 xor odd).
    cf e[16];
    {
        const int k1 = t & 15, v = t >> 4;
        const int odd = v & 1;
        const cf *pe = lds + v * 256 + k1 + 16 * odd;
        const cf *po = lds + v * 256 + k1 - 16 * odd;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) e[k2] = (k2 & 1) ? po[16 * k2] : pe[16 * k2];
        Dft<16, 1>::run(e);
        __syncthreads();  // every thread has read P
        // element (v, u1, k1) of the exchange goes to
        //   v 256 + 16 (u1 ^ g) + ((k1 ^ f)),  f = tB mod 16, g = bit 4 of tB,
        // tB = NV u1 + v the reading thread (g unused when NV = 16), which keeps
        // both the writes (16 lanes of one v) and the reads (32 lanes of
        // consecutive tB) on distinct banks.
        const int xl = k1 ^ (v & 15);
        const int gofs = (NV == 32) ? ((v >> 4) & 1) << 4 : 0;
#pragma unroll
        for (int u1 = 0; u1 < 16; ++u1) {
            const int c = (NV * u1) & 15;
            const int g16 = (NV < 16) ? (((NV * u1) >> 4) & 1) << 4 : 0;
            lds[v * 256 + (((16 * u1) ^ g16) ^ gofs) + (xl ^ c)] = e[u1];
        }
    }
    __syncthreads();

    // 3) twiddle exp(2 pi i k1 u1 / 256) and radix 16 over k1 for thread
    //    t = NV u1 + v; output u2 is sample t + T u2.
    {
        const int u1 = t / NV, v = t & (NV - 1);
        const int f = t & 15;
        const int g16 = (NV == 16) ? 0 : ((t >> 4) & 1) << 4;
        const int row = v * 256 + ((16 * u1) ^ g16);
        const int rf = row | f;
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) e[k1] = lds[rf ^ k1];
        cf w[16];
        if (TWM == kTwTable)
            table_twiddles<16, 1>(tw, u1 * NV, w);
        else
            twiddle_powers<16>(tw[u1 * NV], w);
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) e[k1] = mul(e[k1], w[k1]);
        Dft<16, 1>::run(e);
#pragma unroll
        for (int u2 = 0; u2 < 16; ++u2) v_out[u2] = e[u2];
    }
}

}  // namespace

// ------------------------------------------------------------ inverse --

// Band-power workgroups run RowSub transforms side by side: sub-group g of
// T threads owns LDS slab g and takes frequencies g, g + RowSub, ... of the
// band, so a band of n frequencies is a chain of n / RowSub transform rounds
// rather than n.  Complex and power rows are one transform per workgroup.
template <int MODE, int L>
struct RowSub {
    static constexpr int value = (MODE != kOutBand) ? 1 : (L <= 4096 ? 4 : 2);
};

// One output row (channel, frequency or band) item of the transform.
template <int MODE, int TWM, int... Rs>
__device__ __forceinline__ void fixed_main_row(const MainParams &p, int item)
{
    using RL = RList<Rs...>;
    constexpr int L = RL::product;
    constexpr int T = L / kV;
    constexpr int SUB = RowSub<MODE, L>::value;
    static_assert(RL::first == kV, "the first pass must be radix 16");
    extern __shared__ cf lds_all[];
    const int N = p.N;

    int c, row;
    if (MODE == kOutBand) {
        // bands largest first, channel fastest
        const int rank = item / p.C;
        c = item - rank * p.C;
        row = p.grp_off[p.n_rows + 1 + rank];
    } else {
        c = item / p.n_rows;
        row = item - c * p.n_rows;
    }
    int qb, qe;
    if (MODE == kOutBand) {
        qb = p.grp_off[row];
        qe = p.grp_off[row + 1];
    } else {
        qb = row;
        qe = row + 1;
    }
    const cf *X0 = reinterpret_cast<const cf *>(p.Xh) + (int64_t)c * p.Lh;
    const cf *tw0 = reinterpret_cast<const cf *>(p.tw);
    // Band power: thread t of a sub-group owns samples t + T m of each of its
    // frequencies' transforms, so its share of the band sum stays in
    // registers; the sub-groups' sums meet in LDS at the end.
    float acc[kV];
#pragma unroll
    for (int m = 0; m < kV; ++m) acc[m] = 0.f;

    // Complex and power rows are one transform: a trip count the compiler
    // sees as 1.
    const int nq = (MODE == kOutBand) ? qe - qb : 1;
    const int rounds = (nq + SUB - 1) / SUB;
    for (int r = 0; r < rounds; ++r) {
        // Over a band's rounds the lane, input row and twiddle table stay the
        // same; hoisted out of the loop, every address derived from them would
        // be held in registers across it (and spilled).  Made opaque here they
        // are recomputed per round.
        int tid = threadIdx.x;
        const cf *X = X0;
        const cf *tw = tw0;
        if (MODE == kOutBand) asm volatile("" : "+v"(tid), "+s"(X), "+s"(tw));
        const int g = (SUB == 1) ? 0 : tid / T;
        const int t = (SUB == 1) ? tid : tid - g * T;
        cf *lds = lds_all + g * L;
        const int qi = r * SUB + g;
        const bool live = qi < nq;  // a short last round repeats the band's last frequency
        const int q = qb + (live ? qi : nq - 1);
        const int f = (MODE == kOutBand) ? p.grp_freq[q] : q;
        const BandDesc bd = p.band[f];
        const float *Hf = p.H + bd.off;
        const cf *Hcf = p.Hc ? reinterpret_cast<const cf *>(p.Hc) + bd.off : nullptr;
        const int K = bd.K;
        const int lo_u = bd.lo < 0 ? bd.lo + L : bd.lo;
        // One path for the whole workgroup (the paths differ in their
        // barriers): the band path only when every transform of the round fits.
        bool narrow = K <= kBandMax;
        if (SUB > 1) {
#pragma unroll
            for (int j = 0; j < SUB; ++j) {
                const int qj = qb + min(r * SUB + j, nq - 1);
                narrow = narrow && p.band[p.grp_freq[qj]].K <= kBandMax;
            }
        }
        if (r > 0) __syncthreads();  // previous transforms finished with lds
        cf v[kV];
        if (narrow) {
            band_transform<L, TWM>(X, Hf, Hcf, lo_u, K, tw, lds, t, v);
        } else {
            // Band products y[k] = X~[b] H[k], b = lo + k (mod L), into lds[0, K).
            // Loads are issued unconditionally (clamped index) so that they do not
            // serialise behind branches.
            {
                const int nit = (K + T - 1) / T;
#pragma unroll 2
                for (int i = 0; i < nit; ++i) {
                    const int k = t + i * T;
                    const int kc = k < K ? k : K - 1;
                    const int b = (lo_u + kc) & (L - 1);
                    const bool upper = b > L / 2;
                    cf xv = X[upper ? L - b : b];
                    if (upper) xv.y = -xv.y;
                    if (k < K) lds[k] = Hcf ? mul(xv, Hcf[kc]) : scale(xv, Hf[kc]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < kV; ++m) {
                const int o = (t + T * m - lo_u) & (L - 1);
                const cf y = lds[o];
                v[m] = (o < K) ? y : mk(0.f, 0.f);
            }
            run_passes<1, L, 1, TWM>(v, t, tw, lds, RL{});
        }
        // epilogue: v[m] is sample t + T m
        if (MODE == kOutBand) {
            if (live) {
#pragma unroll
                for (int m = 0; m < kV; ++m) acc[m] += v[m].x * v[m].x + v[m].y * v[m].y;
            }
            continue;
        }
        float2 *ocx = reinterpret_cast<float2 *>(p.out) + ((int64_t)c * p.n_rows + f) * N;
        float *opw = reinterpret_cast<float *>(p.out) + ((int64_t)c * p.n_rows + f) * N;
        auto store = [&](int m) {
            const int ts = t + T * m;
            const cf w = v[m];
            if (MODE == kOutComplex)
                *reinterpret_cast<f2v *>(ocx + ts) = f2v{w.x, w.y};
            else
                opw[ts] = w.x * w.x + w.y * w.y;
        };
        if (N == L) {
            // whole rows (uniform branch): no per-sample bounds test
#pragma unroll
            for (int m = 0; m < kV; ++m) store(m);
        } else {
#pragma unroll
            for (int m = 0; m < kV; ++m)
                if (t + T * m < N) store(m);
        }
    }
    if (MODE == kOutBand) {
        float *orow = reinterpret_cast<float *>(p.out) + ((int64_t)c * p.n_rows + row) * N;
        const float inv_n = 1.0f / (float)nq;
        const int tid = threadIdx.x;
        if (SUB == 1) {
#pragma unroll
            for (int m = 0; m < kV; ++m)
                if (N == L || tid + T * m < N) orow[tid + T * m] = acc[m] * inv_n;
        } else {
            // sub-group sums through LDS (slab g holds L floats of sub-group
            // g), added in sub-group order and stored once
            float *ldsf = reinterpret_cast<float *>(lds_all);
            const int g = tid / T, t = tid - g * T;
            __syncthreads();  // every sub-group is done with its slab
#pragma unroll
            for (int m = 0; m < kV; ++m) ldsf[g * L + t + T * m] = acc[m];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < L / (SUB * T); ++i) {
                const int o = tid + SUB * T * i;
                float a = ldsf[o];
#pragma unroll
                for (int j = 1; j < SUB; ++j) a += ldsf[j * L + o];
                if (N == L || o < N) orow[o] = a * inv_n;
            }
        }
    }
}

// Occupancy of the transform kernels: 5 waves per SIMD for complex and power
// rows at L = 4096 (the LDS of 5 workgroups fills the CU), 4 for the
// band-power workgroups of several sub-groups, no constraint otherwise.
template <int MODE, int L>
struct FixedWaves {
    static constexpr int value =
        (MODE != kOutBand && L == 4096) ? 5 : (RowSub<MODE, L>::value > 1 ? 4 : 1);
};

template <int MODE, int TWM, int... Rs>
__global__ void __launch_bounds__((RList<Rs...>::product / kV *
                                   RowSub<MODE, RList<Rs...>::product>::value))
    __attribute__((amdgpu_waves_per_eu(FixedWaves<MODE, RList<Rs...>::product>::value)))
    k_fixed_main(MainParams p)
{
    fixed_main_row<MODE, TWM, Rs...>(p, blockIdx.x);
}

// ------------------------------------------------------------ forward --
// Two real channels packed as one complex sequence, forward transform in
// registers, then the separation X0 = (Z[b] + conj Z[-b]) / 2,
// X1 = (Z[b] - conj Z[-b]) / (2i) through LDS.

// Thread t of a group of T threads with its own LDS slab transforms channel
// pair `pair`.  With MAYBE_PAST_END, pairs past the last channel compute on
// zeros and store nothing, so every group of a workgroup meets the same
// barriers; without it every pair exists (one group per workgroup).
template <bool MAYBE_PAST_END, int... Rs>
__device__ __forceinline__ void fixed_forward_pair(const FwdParams &p, int pair, int t, cf *lds)
{
    using RL = RList<Rs...>;
    constexpr int L = RL::product;
    constexpr int T = L / kV;
    const int c0 = 2 * pair;
    const bool has0 = !MAYBE_PAST_END || c0 < p.C;
    const bool has1 = (c0 + 1) < p.C;
    const cf *tw = reinterpret_cast<const cf *>(p.tw);
    const int N = p.N;
    cf v[kV];
    {
        const float *x0 = p.x + (int64_t)(has0 ? c0 : 0) * p.x_stride;
        const float *x1 = p.x + (int64_t)(has1 ? c0 + 1 : 0) * p.x_stride;
#pragma unroll
        for (int m = 0; m < kV; ++m) {
            const int idx = t + T * m;
            cf z = mk(0.f, 0.f);
            if (has0 && idx < N) {
                z.x = x0[idx];
                if (has1) z.y = x1[idx];
            }
            v[m] = z;
        }
    }
    run_passes<-1, L, 1, kTwPowers>(v, t, tw, lds, RL{});
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kV; ++m) lds[sw(t + T * m)] = v[m];
    __syncthreads();
    if (!has0) return;  // no barrier follows
    float2 *X0 = p.Xh + (int64_t)c0 * p.Lh;
    float2 *X1 = X0 + p.Lh;
    for (int b = t; b < p.Lh; b += T) {
        const cf z = lds[sw(b)];
        const cf zn = lds[sw((L - b) & (L - 1))];
        const cf zc = mk(zn.x, -zn.y);
        const cf s = add(z, zc), d = sub(z, zc);
        X0[b] = make_float2(0.5f * s.x, 0.5f * s.y);
        if (has1) X1[b] = make_float2(0.5f * d.y, -0.5f * d.x);
    }
}

template <int... Rs>
__global__ void __launch_bounds__(RList<Rs...>::product / kV) k_fixed_forward(FwdParams p)
{
    extern __shared__ cf lds[];
    fixed_forward_pair<false, Rs...>(p, blockIdx.x, threadIdx.x, lds);
}

// Transform of one batch and forward FFT of the next in one launch: blocks
// [0, n_fwd) take the forward role (channel pairs of the next batch, into the
// other half of the workspace; RowSub pairs per block, one per group of T
// threads) and start first, the rest the transform rows, so the short
// forward work runs beside the transform instead of between two launches.
template <int MODE, int TWM, int... Rs>
__global__ void __launch_bounds__((RList<Rs...>::product / kV *
                                   RowSub<MODE, RList<Rs...>::product>::value))
    __attribute__((amdgpu_waves_per_eu(FixedWaves<MODE, RList<Rs...>::product>::value)))
    k_fixed_fused(MainParams p, FwdParams f, int n_fwd)
{
    constexpr int L = RList<Rs...>::product;
    constexpr int T = L / kV;
    constexpr int SUB = RowSub<MODE, L>::value;
    if ((int)blockIdx.x < n_fwd) {
        extern __shared__ cf lds[];
        const int g = (SUB == 1) ? 0 : (int)threadIdx.x / T;
        fixed_forward_pair<(SUB > 1), Rs...>(f, (int)blockIdx.x * SUB + g,
                                             (int)threadIdx.x - g * T, lds + g * L);
    } else {
        fixed_main_row<MODE, TWM, Rs...>(p, blockIdx.x - n_fwd);
    }
}

template <int... Rs>
static hipError_t launch_fixed_forward_t(const FwdParams &p, hipStream_t s)
{
    constexpr int L = RList<Rs...>::product;
    const size_t lds = (size_t)L * sizeof(cf);
    // once per process (thread-safe static initialisation)
    static const bool attr_set = [lds] {
        (void)hipFuncSetAttribute((const void *)k_fixed_forward<Rs...>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((k_fixed_forward<Rs...>), dim3((p.C + 1) / 2), dim3(L / kV), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_forward_fixed(const FwdParams &p, hipStream_t s)
{
    switch (p.rp.L) {
    case 1024: return launch_fixed_forward_t<16, 16, 4>(p, s);
    case 2048: return launch_fixed_forward_t<16, 16, 8>(p, s);
    case 4096: return launch_fixed_forward_t<16, 16, 16>(p, s);
    case 8192: return launch_fixed_forward_t<16, 16, 16, 2>(p, s);
    default: return hipErrorNotSupported;
    }
}

template <int MODE, int TWM, int... Rs>
static hipError_t launch_fixed_t(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    constexpr int L = RList<Rs...>::product;
    constexpr int SUB = RowSub<MODE, L>::value;
    const size_t lds = (size_t)SUB * L * sizeof(cf);
    // once per process (thread-safe static initialisation)
    static const bool attr_set = [lds] {
        (void)hipFuncSetAttribute((const void *)k_fixed_main<MODE, TWM, Rs...>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        return true;
    }();
    (void)attr_set;
    hipExtLaunchKernelGGL((k_fixed_main<MODE, TWM, Rs...>), dim3(p.C * p.n_rows),
                          dim3(SUB * L / kV), lds, s, ev.start, ev.stop, 0, p);
    return hipGetLastError();
}

template <int TWM, int... Rs>
static hipError_t launch_fixed_modes_t(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    switch (p.out_mode) {
    case kOutComplex: return launch_fixed_t<kOutComplex, TWM, Rs...>(p, s, ev);
    case kOutPower: return launch_fixed_t<kOutPower, TWM, Rs...>(p, s, ev);
    default: return launch_fixed_t<kOutBand, TWM, Rs...>(p, s, ev);
    }
}

template <int... Rs>
static hipError_t launch_fixed_modes(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    return p.variant == 1 ? launch_fixed_modes_t<kTwPowers, Rs...>(p, s, ev)
                          : launch_fixed_modes_t<kTwTable, Rs...>(p, s, ev);
}

template <int MODE, int TWM, int... Rs>
static hipError_t launch_fused_t(const MainParams &p, const FwdParams &f, hipStream_t s,
                                 LaunchEvents ev)
{
    constexpr int L = RList<Rs...>::product;
    constexpr int SUB = RowSub<MODE, L>::value;
    const size_t lds = (size_t)SUB * L * sizeof(cf);
    // once per process (thread-safe static initialisation)
    static const bool attr_set = [lds] {
        (void)hipFuncSetAttribute((const void *)k_fixed_fused<MODE, TWM, Rs...>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        return true;
    }();
    (void)attr_set;
    const int n_fwd = ((f.C + 1) / 2 + SUB - 1) / SUB;
    hipExtLaunchKernelGGL((k_fixed_fused<MODE, TWM, Rs...>), dim3(n_fwd + p.C * p.n_rows),
                          dim3(SUB * L / kV), lds, s, ev.start, ev.stop, 0, p, f, n_fwd);
    return hipGetLastError();
}

template <int TWM, int... Rs>
static hipError_t launch_fused_modes_t(const MainParams &p, const FwdParams &f, hipStream_t s,
                                       LaunchEvents ev)
{
    switch (p.out_mode) {
    case kOutComplex: return launch_fused_t<kOutComplex, TWM, Rs...>(p, f, s, ev);
    case kOutPower: return launch_fused_t<kOutPower, TWM, Rs...>(p, f, s, ev);
    default: return launch_fused_t<kOutBand, TWM, Rs...>(p, f, s, ev);
    }
}

template <int... Rs>
static hipError_t launch_fused_modes(const MainParams &p, const FwdParams &f, hipStream_t s,
                                     LaunchEvents ev)
{
    return p.variant == 1 ? launch_fused_modes_t<kTwPowers, Rs...>(p, f, s, ev)
                          : launch_fused_modes_t<kTwTable, Rs...>(p, f, s, ev);
}

hipError_t launch_fused_fixed(const MainParams &p, const FwdParams &f, hipStream_t s,
                              LaunchEvents ev)
{
    switch (p.rp.L) {
    case 1024: return launch_fused_modes<16, 16, 4>(p, f, s, ev);
    case 2048: return launch_fused_modes<16, 16, 8>(p, f, s, ev);
    case 4096: return launch_fused_modes<16, 16, 16>(p, f, s, ev);
    case 8192: return launch_fused_modes<16, 16, 16, 2>(p, f, s, ev);
    default: return hipErrorNotSupported;
    }
}

bool fixed_main_available(int L)
{
    return L == 1024 || L == 2048 || L == 4096 || L == 8192;
}

hipError_t launch_main_fixed(const MainParams &p, hipStream_t s, LaunchEvents ev)
{
    switch (p.rp.L) {
    case 1024: return launch_fixed_modes<16, 16, 4>(p, s, ev);
    case 2048: return launch_fixed_modes<16, 16, 8>(p, s, ev);
    case 4096: return launch_fixed_modes<16, 16, 16>(p, s, ev);
    case 8192: return launch_fixed_modes<16, 16, 16, 2>(p, s, ev);
    default: return hipErrorNotSupported;
    }
}

}  // namespace cwtk
