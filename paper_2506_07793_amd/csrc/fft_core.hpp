// Device building blocks of the LDS-resident mixed-radix FFT (gfx950, wave64).
//
// The transform is a Stockham autosort FFT: pass p with radix R and
// Ns = product of the radices of the earlier passes reads element
// j + r * (L / R) of butterfly j (r < R), multiplies it by the twiddle
// exp(SIGN 2 pi i (j mod Ns) r / (Ns R)), takes an R-point DFT and writes
// element r to (j div Ns) Ns R + (j mod Ns) + r Ns.  After the last pass the
// data is in natural order, so the last pass can store straight to global
// memory with consecutive threads on consecutive outputs.
//
// SIGN = +1 is the inverse direction exp(+2 pi i k t / L) (no 1/L here; the
// caller folds it into the wavelet spectrum), SIGN = -1 the forward one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cwtk {

// 8-byte aligned so that LDS and global accesses are single 64-bit operations
// (ds_read_b64 / global_load_dwordx2) rather than pairs of 32-bit ones.
struct alignas(8) cf {
    float x, y;
};

__device__ __forceinline__ cf mk(float a, float b) { return cf{a, b}; }

// Pointers into device (global) memory.  Out-of-line functions do not see
// where a plain pointer points and access it with flat instructions, whose
// completion is counted together with the LDS accesses', so that every wait
// for LDS data would also wait for the outstanding memory loads; pointers of
// the global address space keep those accesses on the global path.
template <class T>
using gptr = const __attribute__((address_space(1))) T *;
template <class T>
using gptr_mut = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(const T *p)
{
    return (gptr<T>)p;
}
template <class T>
__device__ __forceinline__ gptr_mut<T> as_global_mut(T *p)
{
    return (gptr_mut<T>)p;
}
// Complex values move through a two-float vector type, which (unlike a
// struct) copies out of and into a qualified address space directly.
typedef float f2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cf load_cf(gptr<cf> p)
{
    const f2_t v = *reinterpret_cast<gptr<f2_t>>(p);
    return cf{v.x, v.y};
}
__device__ __forceinline__ cf add(cf a, cf b) { return cf{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf sub(cf a, cf b) { return cf{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf mul(cf a, cf b)
{
    return cf{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cf scale(cf a, float s) { return cf{a.x * s, a.y * s}; }
// multiply by SIGN * i
template <int SIGN>
__device__ __forceinline__ cf mul_si(cf a)
{
    return SIGN > 0 ? cf{-a.y, a.x} : cf{a.y, -a.x};
}
template <int SIGN>
__device__ __forceinline__ cf conj_if(cf w)
{
    return SIGN > 0 ? w : cf{w.x, -w.y};
}

// ---------------------------------------------------------------- codelets --
// V[k] = sum_r v[r] exp(SIGN 2 pi i r k / R), natural order in and out.

template <int R, int SIGN>
struct Dft;

template <int SIGN>
struct Dft<1, SIGN> {  // length-1 transform (L == 1)
    static __device__ __forceinline__ void run(cf *) {}
};

template <int SIGN>
struct Dft<2, SIGN> {
    static __device__ __forceinline__ void run(cf *v)
    {
        cf a = v[0], b = v[1];
        v[0] = add(a, b);
        v[1] = sub(a, b);
    }
};

template <int SIGN>
struct Dft<4, SIGN> {
    static __device__ __forceinline__ void run(cf *v)
    {
        cf s02 = add(v[0], v[2]), d02 = sub(v[0], v[2]);
        cf s13 = add(v[1], v[3]), d13 = mul_si<SIGN>(sub(v[1], v[3]));
        v[0] = add(s02, s13);
        v[2] = sub(s02, s13);
        v[1] = add(d02, d13);
        v[3] = sub(d02, d13);
    }
};

template <int SIGN>
struct Dft<8, SIGN> {
    static __device__ __forceinline__ void run(cf *v)
    {
        const float h = 0.70710678118654752440f;
        cf e[4] = {v[0], v[2], v[4], v[6]};
        cf o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, SIGN>::run(e);
        Dft<4, SIGN>::run(o);
        // o[k] *= exp(SIGN 2 pi i k / 8)
        cf o1 = o[1], o3 = o[3];
        o[1] = scale(add(o1, mul_si<SIGN>(o1)), h);          // (1 + s i)/sqrt2
        o[2] = mul_si<SIGN>(o[2]);                           // s i
        o[3] = scale(sub(mul_si<SIGN>(o3), o3), h);          // (-1 + s i)/sqrt2
        for (int k = 0; k < 4; ++k) {
            v[k] = add(e[k], o[k]);
            v[k + 4] = sub(e[k], o[k]);
        }
    }
};

template <int SIGN>
struct Dft<16, SIGN> {
    // 16 = 4 x 4: DFT4 over r1 for each r2, twiddle exp(SIGN 2 pi i r2 k1 / 16),
    // DFT4 over r2 for each k1; output index k1 + 4 k2.
    static __device__ __forceinline__ void run(cf *v)
    {
        const float c1 = 0.92387953251128675613f;  // cos(pi/8)
        const float s1 = 0.38268343236508977173f;  // sin(pi/8)
        const float h = 0.70710678118654752440f;
        cf a[4][4];
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2) {
            cf t[4] = {v[r2], v[4 + r2], v[8 + r2], v[12 + r2]};
            Dft<4, SIGN>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) a[r2][k1] = t[k1];
        }
        const float sg = (float)SIGN;
        // r2 = 1: k1 = 1, 2, 3 -> angles pi/8, pi/4, 3pi/8
        a[1][1] = mul(a[1][1], mk(c1, sg * s1));
        a[1][2] = mul(a[1][2], mk(h, sg * h));
        a[1][3] = mul(a[1][3], mk(s1, sg * c1));
        // r2 = 2: angles pi/4, pi/2, 3pi/4
        a[2][1] = mul(a[2][1], mk(h, sg * h));
        a[2][2] = mul_si<SIGN>(a[2][2]);
        a[2][3] = mul(a[2][3], mk(-h, sg * h));
        // r2 = 3: angles 3pi/8, 3pi/4, 9pi/8
        a[3][1] = mul(a[3][1], mk(s1, sg * c1));
        a[3][2] = mul(a[3][2], mk(-h, sg * h));
        a[3][3] = mul(a[3][3], mk(-c1, -sg * s1));
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cf t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            Dft<4, SIGN>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    }
};

// Odd prime radices: V_k = a0 + sum_m cos(2 pi m k / R)(a_m + a_{R-m})
//                          + SIGN i sum_m sin(2 pi m k / R)(a_m - a_{R-m}).
template <int R>
struct OddConst;
template <>
struct OddConst<3> {
    static constexpr float c[1][1] = {{-0.5f}};
    static constexpr float s[1][1] = {{0.86602540378443864676f}};
};
template <>
struct OddConst<5> {
    // [k-1][m-1] for k, m in 1..2
    static constexpr float c[2][2] = {{0.30901699437494742410f, -0.80901699437494742410f},
                                      {-0.80901699437494742410f, 0.30901699437494742410f}};
    static constexpr float s[2][2] = {{0.95105651629515357212f, 0.58778525229247312917f},
                                      {0.58778525229247312917f, -0.95105651629515357212f}};
};
template <>
struct OddConst<7> {
    static constexpr float c[3][3] = {
        {0.62348980185873353053f, -0.22252093395631440429f, -0.90096886790241912624f},
        {-0.22252093395631440429f, -0.90096886790241912624f, 0.62348980185873353053f},
        {-0.90096886790241912624f, 0.62348980185873353053f, -0.22252093395631440429f}};
    static constexpr float s[3][3] = {
        {0.78183148246802980871f, 0.97492791218182360702f, 0.43388373911755812048f},
        {0.97492791218182360702f, -0.43388373911755812048f, -0.78183148246802980871f},
        {0.43388373911755812048f, -0.78183148246802980871f, 0.97492791218182360702f}};
};

template <int R, int SIGN>
struct DftOdd {
    static __device__ __forceinline__ void run(cf *v)
    {
        constexpr int H = (R - 1) / 2;
        cf sp[H], dm[H];
#pragma unroll
        for (int m = 1; m <= H; ++m) {
            sp[m - 1] = add(v[m], v[R - m]);
            dm[m - 1] = sub(v[m], v[R - m]);
        }
        cf a0 = v[0];
        cf sum = a0;
#pragma unroll
        for (int m = 0; m < H; ++m) sum = add(sum, sp[m]);
        v[0] = sum;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            cf re = a0, im = mk(0.f, 0.f);
#pragma unroll
            for (int m = 1; m <= H; ++m) {
                const float cc = OddConst<R>::c[k - 1][m - 1];
                const float ss = OddConst<R>::s[k - 1][m - 1];
                re = add(re, scale(sp[m - 1], cc));
                im = add(im, scale(dm[m - 1], ss));
            }
            cf sim = mul_si<SIGN>(im);
            v[k] = add(re, sim);
            v[R - k] = sub(re, sim);
        }
    }
};
template <int SIGN>
struct Dft<3, SIGN> : DftOdd<3, SIGN> {};
template <int SIGN>
struct Dft<5, SIGN> : DftOdd<5, SIGN> {};
template <int SIGN>
struct Dft<7, SIGN> : DftOdd<7, SIGN> {};

// Composite radices R = R1 R2 (small factors merged into one pass, so that a
// length does not spend an LDS round trip and two barriers on a radix-2 or
// radix-3 pass; 20, 21 and 24 only in plans of 24 values per thread): with r = R2 r1 + r2 and k = k1 + R1 k2,
//   V[k] = sum_r2 W_R2^(r2 k2) [ W_R^(r2 k1) sum_r1 v[R2 r1 + r2] W_R1^(r1 k1) ],
// W_M = exp(SIGN 2 pi i / M); wn[m] = W_R^m (table values, rounded once).
template <int R>
struct CompSplit {
    static constexpr int r1 = 0, r2 = 0;  // not composite
};
template <> struct CompSplit<6> { static constexpr int r1 = 2, r2 = 3; };
template <> struct CompSplit<9> { static constexpr int r1 = 3, r2 = 3; };
template <> struct CompSplit<10> { static constexpr int r1 = 2, r2 = 5; };
template <> struct CompSplit<12> { static constexpr int r1 = 4, r2 = 3; };
template <> struct CompSplit<14> { static constexpr int r1 = 2, r2 = 7; };
template <> struct CompSplit<15> { static constexpr int r1 = 3, r2 = 5; };
template <> struct CompSplit<20> { static constexpr int r1 = 4, r2 = 5; };
template <> struct CompSplit<21> { static constexpr int r1 = 3, r2 = 7; };
template <> struct CompSplit<24> { static constexpr int r1 = 8, r2 = 3; };

template <int R1, int R2, int SIGN>
struct DftC {
    static __device__ __forceinline__ void run(cf *v, const cf *wn)
    {
        constexpr int R = R1 * R2;
        cf a[R2][R1];
#pragma unroll
        for (int r2 = 0; r2 < R2; ++r2) {
            cf t[R1];
#pragma unroll
            for (int r1 = 0; r1 < R1; ++r1) t[r1] = v[R2 * r1 + r2];
            Dft<R1, SIGN>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1)
                a[r2][k1] = (r2 * k1 == 0) ? t[k1] : mul(t[k1], wn[(r2 * k1) % R]);
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cf t[R2];
#pragma unroll
            for (int r2 = 0; r2 < R2; ++r2) t[r2] = a[r2][k1];
            Dft<R2, SIGN>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
        }
    }
};

// The R-point transform of one butterfly, plain or composite.
template <int R, int SIGN>
__device__ __forceinline__ void codelet(cf *v, const cf *wn)
{
    if constexpr (CompSplit<R>::r1 > 0)
        DftC<CompSplit<R>::r1, CompSplit<R>::r2, SIGN>::run(v, wn);
    else
        Dft<R, SIGN>::run(v);
}

// LDS slot of element i in the buffer between the first and the second pass
// of a plan whose first radix is even: the low four bits are XORed with bits
// 4-7, so that the first pass's scatter to R j + r (R even) reaches 16
// distinct banks per 16-lane write group.  Stays inside i's aligned block of
// 16, so a buffer of L rounded up to 16 elements holds every slot.
__device__ __forceinline__ int first_pass_slot(int i) { return i ^ ((i >> 4) & 15); }

// Butterflies a thread may hold at once in one pass when it holds at most
// MAXV complex values.
template <int R, int MAXV>
struct MaxB {
    static constexpr int value = (MAXV / R) > 0 ? (MAXV / R) : 1;
};

// ------------------------------------------------------------- twiddles --
// w[r] = w1^r for r < R by balanced products (depth ceil(log2 r)), so the
// rounding error stays within a few FP32 ulps of the table value w1.
template <int R>
__device__ __forceinline__ void twiddle_powers(cf w1, cf *w)
{
    w[0] = mk(1.f, 0.f);
    if (R > 1) w[1] = w1;
#pragma unroll
    for (int r = 2; r < R; ++r) w[r] = mul(w[r / 2], w[r - r / 2]);
}

// --------------------------------------------------------------- one pass --
// Generic pass over the L/R butterflies of a workgroup of T threads; thread
// `tid` owns butterflies j = tid + k T.  `load(idx)` supplies input element
// idx, `store(slot, idx, value)` receives output element idx, where
// slot = k R + r numbers the values this thread holds.  When SYNC_MID is set
// a workgroup barrier separates all loads from all stores (in-place LDS use).
// Twiddles derive from tw[m] = exp(+2 pi i m / L) (conjugated for SIGN < 0).
// The pass is a separate (not inlined) function so that a kernel holding
// every radix keeps one pass's registers live at a time.
template <int R, int SIGN, int MAXV, bool SYNC_MID, class Load, class Store>
__device__ __attribute__((noinline)) void stockham_pass(int L, int Ns, int T, int tid,
                                                        gptr<cf> tw, Load load, Store store)
{
    constexpr int MB = MaxB<R, MAXV>::value;
    const int S = L / R;
    const int twstep = L / (Ns * R);
    cf v[MB][R];
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        const int j = tid + k * T;
        if (j < S) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[k][r] = load(j + r * S);
        }
    }
    if (SYNC_MID) __syncthreads();
    // internal twiddles of a composite radix: W_R^m = tw[m L / R]
    cf wn[CompSplit<R>::r1 > 0 ? R : 1];
    if constexpr (CompSplit<R>::r1 > 0) {
#pragma unroll
        for (int m = 0; m < R; ++m) wn[m] = conj_if<SIGN>(load_cf(tw + m * (L / R)));
    }
    // jm = j mod Ns for j = tid + k T, stepped by T mod Ns (one division per
    // pass instead of one per butterfly)
    const int dT = T % Ns;
    int jm = tid % Ns;
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        const int j = tid + k * T;
        if (k > 0) {
            jm += dT;
            if (jm >= Ns) jm -= Ns;
        }
        if (j < S) {
            if (Ns > 1) {
                cf w[R];
                twiddle_powers<R>(conj_if<SIGN>(load_cf(tw + (unsigned)(jm * twstep))), w);
#pragma unroll
                for (int r = 1; r < R; ++r) v[k][r] = mul(v[k][r], w[r]);
            }
            codelet<R, SIGN>(v[k], wn);
            const int base = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) store(k * R + r, base + r * Ns, v[k][r]);
        }
    }
}

// Dispatch one pass of runtime radix R to its compiled form.
template <int SIGN, int MAXV, bool SYNC_MID, class Load, class Store>
__device__ __forceinline__ void stockham_pass_rt(int R, int L, int Ns, int T, int tid,
                                                 gptr<cf> tw, Load load, Store store)
{
    switch (R) {
    case 16: stockham_pass<16, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 8: stockham_pass<8, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 4: stockham_pass<4, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 2: stockham_pass<2, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 3: stockham_pass<3, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 5: stockham_pass<5, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 7: stockham_pass<7, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 6: stockham_pass<6, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 9: stockham_pass<9, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 10: stockham_pass<10, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 12: stockham_pass<12, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 14: stockham_pass<14, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 15: stockham_pass<15, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    case 20:
        if constexpr (MAXV >= 20) stockham_pass<20, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store);
        break;
    case 21:
        if constexpr (MAXV >= 21) stockham_pass<21, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store);
        break;
    case 24:
        if constexpr (MAXV >= 24) stockham_pass<24, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store);
        break;
    case 1: stockham_pass<1, SIGN, MAXV, SYNC_MID>(L, Ns, T, tid, tw, load, store); break;
    default: break;
    }
}

}  // namespace cwtk
