// Register-resident FFT kernels for power-of-two padded lengths (gfx950).
//
// Each workgroup of T = L/16 threads transforms one length-L sequence; every
// thread holds 16 complex values in registers and the radix passes exchange
// data through LDS.  LDS slots are XOR-swizzled (low five index bits XORed
// with a function of the higher bits) so that the strided writes of the first
// passes and the unit-stride reads both hit 32 distinct 8-byte slots per 32
// lanes.  Twiddles are read from the plan's exp(2 pi i m / L) table.  The
// radix schedule is a compile-time list whose first entry is 16, so every
// pass is fully unrolled with constant strides.
//
// Inverse kernel (k_fixed_main): the wavelet spectrum of one frequency is
// non-zero only on a band of K consecutive bins (cyclically).  The workgroup
// first forms the K products X~[b] H[b] once, into LDS.  When K <= L/16 each
// radix-16 butterfly of the first Stockham pass sees at most one non-zero
// input, so that pass reduces to a gather: the second pass's inputs are the
// band products times exp(2 pi i jm (b - q) / L) (jm, q from the butterfly
// index).  Wider bands run the full set of passes.  The last pass stores
// natural-order rows straight from registers (thread t writes samples
// t + T m).
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

template <class RL>
struct Tail;
template <int R0, int... Rest>
struct Tail<RList<R0, Rest...>> {
    using type = RList<Rest...>;
};

}  // namespace

// ------------------------------------------------------------ inverse --

template <int MODE, int TWM, int... Rs>
__global__ void __launch_bounds__(RList<Rs...>::product / kV)
    __attribute__((amdgpu_waves_per_eu(
        (MODE != kOutBand && RList<Rs...>::product == 4096) ? 5 : 1)))
    k_fixed_main(MainParams p)
{
    using RL = RList<Rs...>;
    constexpr int L = RL::product;
    constexpr int T = L / kV;
    constexpr int R0 = RL::first;
    constexpr int S0 = L / R0;
    static_assert(R0 == kV, "the first pass must be radix 16");
    extern __shared__ cf lds[];
    const int t = threadIdx.x;
    const int N = p.N;
    const cf *tw = reinterpret_cast<const cf *>(p.tw);

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

    for (int q = qb; q < qe; ++q) {
        const int f = (MODE == kOutBand) ? p.grp_freq[q] : q;
        const BandDesc bd = p.band[f];
        const float *Hf = p.H + bd.off;
        const int K = bd.K;
        const int lo_u = bd.lo < 0 ? bd.lo + L : bd.lo;
        if (q != qb) __syncthreads();  // previous transform finished with lds
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
                const float h = Hf[kc];
                if (upper) xv.y = -xv.y;
                if (k < K) lds[k] = scale(xv, h);
            }
            if (K <= S0) {
                // roots of unity of order R0 R1 for the pruned gather below
                constexpr int NR = R0 * Tail<RL>::type::first;
                for (int m = t; m < NR; m += T) lds[S0 + m] = tw[m * (L / NR)];
            }
        }
        __syncthreads();
        cf v[kV];
        if (K <= S0) {
            // Pruned: gather the second pass's inputs directly.  Pass-1
            // butterfly j = R0 q + jm reads the in-band bins b = q + G r
            // (mod S0) times exp(2 pi i jm (b - q) / L); since b - q is a
            // multiple of G these are roots of unity of order R0 R1, staged
            // in lds[S0, S0 + R0 R1) next to the band products.
            constexpr int R1 = Tail<RL>::type::first;
            constexpr int S1 = L / R1;
            constexpr int NB = kV / R1;
            constexpr int G = S1 / R0;       // bin stride between the r inputs
            constexpr int NQ = S1 / R0;      // butterflies per jm
            constexpr int NR = R0 * R1;      // root order
            constexpr int LOG_S0 = __builtin_ctz(S0);
            static_assert(Tail<typename Tail<RL>::type>::type::count > 0,
                          "at least three passes");
#pragma unroll
            for (int kb = 0; kb < NB; ++kb) {
                // consecutive lanes take consecutive q (same jm), which keeps
                // the root reads to a few distinct LDS addresses per wave
                const int jj = t + kb * T;
                const int qq = jj & (NQ - 1);
                const int jm = jj / NQ;
                const int c0 = (qq - lo_u) & (S0 - 1);
                const int A = (lo_u - qq + c0) >> LOG_S0;  // exact multiple of S0
                const int acc = jm * R1 * A;
#pragma unroll
                for (int r = 0; r < R1; ++r) {
                    const int u = c0 + G * r;
                    const int o = u & (S0 - 1);
                    const int ri = (acc + jm * r - ((u >= S0) ? jm * R1 : 0)) & (NR - 1);
                    cf yw = mk(0.f, 0.f);
                    // whole 16-lane groups share o, so this branch is mostly
                    // uniform per wave and skips the out-of-band rows
                    if (o < K) yw = mul(lds[o], lds[S0 + ri]);
                    v[kb + r * NB] = yw;
                }
            }
            // second pass without its twiddle (folded into the gather)
#pragma unroll
            for (int kb = 0; kb < NB; ++kb) {
                cf e[R1];
#pragma unroll
                for (int r = 0; r < R1; ++r) e[r] = v[kb + r * NB];
                Dft<R1, 1>::run(e);
#pragma unroll
                for (int r = 0; r < R1; ++r) v[kb + r * NB] = e[r];
            }
            using After = typename Tail<typename Tail<RL>::type>::type;
            if constexpr (After::count > 0) {
                __syncthreads();  // every thread has read the band products and roots
#pragma unroll
                for (int kb = 0; kb < NB; ++kb) {
                    const int jj = t + kb * T;
                    const int qq = jj & (NQ - 1);
                    const int jm = jj / NQ;
                    const int base = NR * qq + jm;  // (j - jm) R1 + jm, j = R0 qq + jm
#pragma unroll
                    for (int r = 0; r < R1; ++r) lds[sw(base + r * R0)] = v[kb + r * NB];
                }
                __syncthreads();
                load_lds_columns<L>(v, t, lds);
                run_passes<1, L, R0 * R1, TWM>(v, t, tw, lds, After{});
            }
        } else {
#pragma unroll
            for (int m = 0; m < kV; ++m) {
                const int o = (t + T * m - lo_u) & (L - 1);
                const cf y = lds[o];
                v[m] = (o < K) ? y : mk(0.f, 0.f);
            }
            run_passes<1, L, 1, TWM>(v, t, tw, lds, RL{});
        }
        // epilogue: v[m] is sample t + T m
        float2 *ocx = reinterpret_cast<float2 *>(p.out) + ((int64_t)c * p.n_rows + f) * N;
        float *opw = reinterpret_cast<float *>(p.out) + ((int64_t)c * p.n_rows + f) * N;
        const bool first = (q == qb), final_f = (q == qe - 1);
#pragma unroll
        for (int m = 0; m < kV; ++m) {
            const int ts = t + T * m;
            if (ts < N) {
                const cf w = v[m];
                const float pw = w.x * w.x + w.y * w.y;
                if (MODE == kOutComplex) {
                    __builtin_nontemporal_store(f2v{w.x, w.y}, reinterpret_cast<f2v *>(ocx + ts));
                } else if (MODE == kOutPower) {
                    __builtin_nontemporal_store(pw, opw + ts);
                } else {
                    float a = first ? pw : orow_band[ts] + pw;
                    orow_band[ts] = final_f ? a * inv_n : a;
                }
            }
        }
    }
}

// ------------------------------------------------------------ forward --
// Two real channels packed as one complex sequence, forward transform in
// registers, then the separation X0 = (Z[b] + conj Z[-b]) / 2,
// X1 = (Z[b] - conj Z[-b]) / (2i) through LDS.

template <int... Rs>
__global__ void __launch_bounds__(RList<Rs...>::product / kV) k_fixed_forward(FwdParams p)
{
    using RL = RList<Rs...>;
    constexpr int L = RL::product;
    constexpr int T = L / kV;
    extern __shared__ cf lds[];
    const int t = threadIdx.x;
    const int c0 = 2 * blockIdx.x;
    const bool has1 = (c0 + 1) < p.C;
    const float *x0 = p.x + (int64_t)c0 * p.x_stride;
    const float *x1 = p.x + (int64_t)(c0 + 1) * p.x_stride;
    const cf *tw = reinterpret_cast<const cf *>(p.tw);
    const int N = p.N;
    cf v[kV];
#pragma unroll
    for (int m = 0; m < kV; ++m) {
        const int idx = t + T * m;
        cf z = mk(0.f, 0.f);
        if (idx < N) {
            z.x = x0[idx];
            if (has1) z.y = x1[idx];
        }
        v[m] = z;
    }
    run_passes<-1, L, 1, kTwPowers>(v, t, tw, lds, RL{});
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kV; ++m) lds[sw(t + T * m)] = v[m];
    __syncthreads();
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
static hipError_t launch_fixed_forward_t(const FwdParams &p, hipStream_t s)
{
    constexpr int L = RList<Rs...>::product;
    const size_t lds = (size_t)L * sizeof(cf);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_fixed_forward<Rs...>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
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
static hipError_t launch_fixed_t(const MainParams &p, hipStream_t s)
{
    constexpr int L = RList<Rs...>::product;
    const size_t lds = (size_t)L * sizeof(cf);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_fixed_main<MODE, TWM, Rs...>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fixed_main<MODE, TWM, Rs...>), dim3(p.C * p.n_rows), dim3(L / kV),
                       lds, s, p);
    return hipGetLastError();
}

template <int TWM, int... Rs>
static hipError_t launch_fixed_modes_t(const MainParams &p, hipStream_t s)
{
    switch (p.out_mode) {
    case kOutComplex: return launch_fixed_t<kOutComplex, TWM, Rs...>(p, s);
    case kOutPower: return launch_fixed_t<kOutPower, TWM, Rs...>(p, s);
    default: return launch_fixed_t<kOutBand, TWM, Rs...>(p, s);
    }
}

template <int... Rs>
static hipError_t launch_fixed_modes(const MainParams &p, hipStream_t s)
{
    return p.variant == 1 ? launch_fixed_modes_t<kTwPowers, Rs...>(p, s)
                          : launch_fixed_modes_t<kTwTable, Rs...>(p, s);
}

bool fixed_main_available(int L)
{
    return L == 1024 || L == 2048 || L == 4096 || L == 8192;
}

hipError_t launch_main_fixed(const MainParams &p, hipStream_t s)
{
    switch (p.rp.L) {
    case 1024: return launch_fixed_modes<16, 16, 4>(p, s);
    case 2048: return launch_fixed_modes<16, 16, 8>(p, s);
    case 4096: return launch_fixed_modes<16, 16, 16>(p, s);
    case 8192: return launch_fixed_modes<16, 16, 16, 2>(p, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace cwtk
