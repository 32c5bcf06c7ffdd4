// Device building blocks of the gfx950 FFT: complex arithmetic, the small
// DFTs held in registers, the Stockham stage schedule and the block engine
// that runs the stages of one sub-FFT through LDS.
//
// Mathematics (paper section 3, Eq. 1): with N = M*K,
//   DFT_N = (DFT_K (x) I_M) D^N_M (I_K (x) DFT_M) Pi^N_K,
// Pi^N_K the stride-K gather and D^N_M the diagonal of twiddle factors
// w_N^(n2*k1), w_N = exp(-2 pi i / N).  A Stockham stage of radix R applies
// this once per butterfly: for butterfly j < L/R with k = j mod Ns,
//   u[r] = x[j + r*L/R] * w_(Ns*R)^(r*k)          (Mul(TwiddleCoe, X), Table 1)
//   u    = DFT_R(u)                               (FusedMKIV on strided data)
//   y[(j div Ns)*Ns*R + k + r*Ns] = u[r]           (FusedPKIV: self-sorting store)
// and Ns grows by R per stage.  After the last stage y is in natural order.
//
// All kernels compute the forward transform.  The inverse uses
// IDFT(x) = S DFT(S x), where S swaps the real and imaginary parts
// (S z = i conj(z), so S DFT(S x) = i conj(DFT(i conj(x))) = IDFT(x)): for
// split arrays the caller's real and imaginary pointers trade places, for
// interleaved data the two halves of each loaded pair do.  No arithmetic is
// added and one set of forward twiddle tables serves both directions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fftk {

// ---------------------------------------------------------------------------
// complex helpers, generic over the vector type V = float2 (FP32) or double2
// (FP64): (x, y) = (re, im)
// ---------------------------------------------------------------------------
template <class V> struct RealOf;
template <> struct RealOf<float2> { using type = float; };
template <> struct RealOf<double2> { using type = double; };
template <class R> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };
template <class R> using cplx_t = typename CplxOf<R>::type;

__device__ __forceinline__ float2 cmk(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ double2 cmk(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ float fmx(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmx(double a, double b, double c) { return fma(a, b, c); }

template <class V> __device__ __forceinline__ V c_add(V a, V b) { return cmk(a.x + b.x, a.y + b.y); }
template <class V> __device__ __forceinline__ V c_sub(V a, V b) { return cmk(a.x - b.x, a.y - b.y); }
// a * w
template <class V> __device__ __forceinline__ V c_mul(V a, V w) {
    return cmk(fmx(a.x, w.x, -(a.y * w.y)), fmx(a.x, w.y, a.y * w.x));
}
// a * (-i)
template <class V> __device__ __forceinline__ V c_mul_mi(V a) { return cmk(a.y, -a.x); }
template <class V> __device__ __forceinline__ V c_zero() { return cmk(typename RealOf<V>::type(0), typename RealOf<V>::type(0)); }

// exp(-2 pi i m / 16) for the register DFT_16 and DFT_8: cos(pi/8), sin(pi/8)
// and sqrt(2)/2 as correctly rounded literals of each precision.
template <class R> struct K16;
template <> struct K16<float> {
    static constexpr float C1 = 0.923879532511286756128f;  // cos(pi/8)
    static constexpr float S1 = 0.382683432365089771728f;  // sin(pi/8)
    static constexpr float R2 = 0.707106781186547524401f;  // sqrt(2)/2
};
template <> struct K16<double> {
    static constexpr double C1 = 0.923879532511286756128;
    static constexpr double S1 = 0.382683432365089771728;
    static constexpr double R2 = 0.707106781186547524401;
};

// a * exp(-2 pi i / 8) = a * (r, -r)
template <class V> __device__ __forceinline__ V c_mul_w8_1(V a) {
    constexpr auto r = K16<typename RealOf<V>::type>::R2;
    return cmk(r * (a.x + a.y), r * (a.y - a.x));
}
// a * exp(-2 pi i 3 / 8) = a * (-r, -r)
template <class V> __device__ __forceinline__ V c_mul_w8_3(V a) {
    constexpr auto r = K16<typename RealOf<V>::type>::R2;
    return cmk(r * (a.y - a.x), -r * (a.x + a.y));
}

// ---------------------------------------------------------------------------
// DFT_R in registers, forward, natural order in and out.
// DFT_8 and DFT_16 are themselves one step of Eq. 1 (K = 2 or 4, M = 4).
// ---------------------------------------------------------------------------
template <class V> __device__ __forceinline__ void dft2(V& a0, V& a1) {
    V t = a0;
    a0 = c_add(t, a1);
    a1 = c_sub(t, a1);
}

template <class V> __device__ __forceinline__ void dft4(V& a0, V& a1, V& a2, V& a3) {
    V t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
    V t2 = c_add(a1, a3), t3 = c_mul_mi(c_sub(a1, a3));
    a0 = c_add(t0, t2);
    a2 = c_sub(t0, t2);
    a1 = c_add(t1, t3);
    a3 = c_sub(t1, t3);
}

template <int R> struct Dft;

template <> struct Dft<1> {
    template <class V> __device__ __forceinline__ static void run(V*) {}
};
template <> struct Dft<2> {
    template <class V> __device__ __forceinline__ static void run(V* v) { dft2(v[0], v[1]); }
};
template <> struct Dft<4> {
    template <class V> __device__ __forceinline__ static void run(V* v) { dft4(v[0], v[1], v[2], v[3]); }
};
template <> struct Dft<8> {
    template <class V> __device__ __forceinline__ static void run(V* v) {
        // K = 2 sub-sequences of stride 2, DFT_4 each
        dft4(v[0], v[2], v[4], v[6]);
        dft4(v[1], v[3], v[5], v[7]);
        // v[n2 + 2 k1] = A[n2][k1]; twiddle w_8^(n2 k1)
        v[3] = c_mul_w8_1(v[3]);
        v[5] = c_mul_mi(v[5]);
        v[7] = c_mul_w8_3(v[7]);
        // DFT_2 across n2: X[k1 + 4 k2]
        V o[8];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            V a = v[2 * k1], b = v[2 * k1 + 1];
            o[k1] = c_add(a, b);
            o[k1 + 4] = c_sub(a, b);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = o[i];
    }
};
template <> struct Dft<16> {
    template <class V> __device__ __forceinline__ static void run(V* v) {
        // K = 4 sub-sequences x[4 n1 + n2], DFT_4 over n1
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
        // v[n2 + 4 k1] = A[n2][k1]; twiddle w_16^(n2 k1)
        using K = K16<typename RealOf<V>::type>;
        const V w1 = cmk(K::C1, -K::S1);
        const V w3 = cmk(K::S1, -K::C1);
        const V w9 = cmk(-K::C1, K::S1);
        v[5] = c_mul(v[5], w1);     // n2=1 k1=1
        v[9] = c_mul_w8_1(v[9]);    // n2=1 k1=2 (w^2)
        v[13] = c_mul(v[13], w3);   // n2=1 k1=3
        v[6] = c_mul_w8_1(v[6]);    // n2=2 k1=1 (w^2)
        v[10] = c_mul_mi(v[10]);    // n2=2 k1=2 (w^4)
        v[14] = c_mul_w8_3(v[14]);  // n2=2 k1=3 (w^6)
        v[7] = c_mul(v[7], w3);     // n2=3 k1=1
        v[11] = c_mul_w8_3(v[11]);  // n2=3 k1=2 (w^6)
        v[15] = c_mul(v[15], w9);   // n2=3 k1=3
        // DFT_4 across n2 for each k1 -> X[k1 + 4 k2] sits in v[4 k1 + k2]
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        V o[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = o[i];
    }
};

// cos(k pi / 16), k = 0 .. 8, correctly rounded in each precision
template <class R> struct K32;
#define FFTK_COS_PI16(T, s)                                                                                       \
    template <> struct K32<T> {                                                                                   \
        __host__ __device__ static constexpr T c(int k) {                                                         \
            return k == 0 ? T(1) : k == 1 ? 0.980785280403230449126##s : k == 2 ? 0.923879532511286756128##s      \
                 : k == 3 ? 0.831469612302545237079##s : k == 4 ? 0.707106781186547524401##s                         \
                 : k == 5 ? 0.555570233019602224743##s : k == 6 ? 0.382683432365089771728##s                         \
                 : k == 7 ? 0.195090322016128267848##s : T(0);                                                       \
        }                                                                                                         \
    };
FFTK_COS_PI16(float, f)
FFTK_COS_PI16(double, )
#undef FFTK_COS_PI16

// cos(m pi / 16) for any integer m, from the first octant by symmetry
template <class R>
__host__ __device__ constexpr R cos_pi16(int m) {
    m = ((m % 32) + 32) % 32;
    if (m > 16) m = 32 - m;
    return m > 8 ? -K32<R>::c(16 - m) : K32<R>::c(m);
}

// a * w_32^M, w_32 = exp(-2 pi i / 32) = (cos(pi/16), -sin(pi/16)); the
// multiples of w_8 take the cheaper forms
template <int M, class V>
__device__ __forceinline__ V c_mul_w32(V a) {
    using R = typename RealOf<V>::type;
    constexpr int m = M % 32;
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return c_mul_w8_1(a);
    else if constexpr (m == 8) return c_mul_mi(a);
    else if constexpr (m == 12) return c_mul_w8_3(a);
    else if constexpr (m == 16) return cmk(-a.x, -a.y);
    else {
        constexpr R c = cos_pi16<R>(m), s = cos_pi16<R>(8 - m);  // sin(m pi/16) = cos((8 - m) pi/16)
        return c_mul(a, cmk(c, -s));
    }
}

template <> struct Dft<32> {
    template <int N2, int K1, class V>
    __device__ __forceinline__ static void tw(V* v) {
        v[N2 + 4 * K1] = c_mul_w32<N2 * K1>(v[N2 + 4 * K1]);
        if constexpr (K1 + 1 < 8) tw<N2, K1 + 1>(v);
    }
    template <class V> __device__ __forceinline__ static void run(V* v) {
        // K = 4 sub-sequences x[4 n1 + n2], DFT_8 over n1 -> v[n2 + 4 k1] = A[n2][k1]
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            V u[8];
#pragma unroll
            for (int n1 = 0; n1 < 8; ++n1) u[n1] = v[n2 + 4 * n1];
            Dft<8>::run(u);
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) v[n2 + 4 * k1] = u[k1];
        }
        // twiddle w_32^(n2 k1)
        tw<1, 1>(v);
        tw<2, 1>(v);
        tw<3, 1>(v);
        // DFT_4 across n2 for each k1 -> X[k1 + 8 k2] sits in v[4 k1 + k2]
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        V o[32];
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) o[k1 + 8 * k2] = v[4 * k1 + k2];
#pragma unroll
        for (int i = 0; i < 32; ++i) v[i] = o[i];
    }
};

// ---------------------------------------------------------------------------
// Stage schedule of an L-point sub-FFT with E elements per thread.
// Stages of radix E, plus one stage of the remaining smaller radix (last, or
// first when REMFIRST).  Stage s reads twiddles w_(Ns*R)^(r*k) from a table
// laid out [k][r] (k < Ns, r < R) at offset twOff(s); stage 0 has Ns = 1 and
// needs none.
// ---------------------------------------------------------------------------
template <int LOG2L_, int LOG2E_, bool REMFIRST_>
struct Sched {
    static constexpr int LOG2L = LOG2L_;
    static constexpr bool REMFIRST = REMFIRST_;
    static constexpr int L = 1 << LOG2L;
    static constexpr int LE = (LOG2E_ < LOG2L) ? LOG2E_ : LOG2L;  // effective log2 E
    static constexpr int E = 1 << LE;
    static constexpr int T = L / E;  // threads per sub-FFT
    static constexpr int NFULL = LE ? LOG2L / LE : 0;
    static constexpr int REM = LE ? LOG2L % LE : 0;
    static constexpr int NST = NFULL + (REM ? 1 : 0);

    __host__ __device__ static constexpr int log2R(int s) {
        return REM == 0 ? LE : (REMFIRST ? (s == 0 ? REM : LE) : (s == NST - 1 ? REM : LE));
    }
    __host__ __device__ static constexpr int log2NS(int s) {
        int a = 0;
        for (int q = 0; q < s; ++q) a += log2R(q);
        return a;
    }
    __host__ __device__ static constexpr int twOff(int s) {
        int a = 0;
        for (int q = 1; q < s; ++q) a += 1 << (log2NS(q) + log2R(q));
        return a;
    }
    static constexpr int TW_SIZE = NST > 1 ? twOff(NST) : 0;
    // the recurrence form (TwRec): stage s keeps only w_(Ns*R)^k, k < Ns, in FP64
    __host__ __device__ static constexpr int recOff(int s) {
        int a = 0;
        for (int q = 1; q < s; ++q) a += 1 << log2NS(q);
        return a;
    }
    static constexpr int REC_SIZE = NST > 1 ? recOff(NST) : 0;
};

// LDS index of element i of group g: one element of padding every 16 elements
// breaks the power-of-two strides of the Stockham stores across banks.
template <int GS>
__device__ __forceinline__ int lds_at(int g, int i) { return g * GS + i + (i >> 4); }

// Synchronisation between stages: a workgroup barrier, or (when every
// sub-FFT lives inside one wavefront) only a wavefront-scope fence.  The
// fences order LDS only: stages exchange data through LDS alone (a thread's
// global stores go to addresses no other thread of the kernel reads), so
// global loads issued before a barrier - the next transform's data in the
// prefetching kernels - stay in flight across it.
template <bool WAVE>
__device__ __forceinline__ void stage_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
}

// ---------------------------------------------------------------------------
// Twiddle sources for the stages of an engine.  Stage S multiplies input r of
// butterfly j (j = t + b*T, k = j mod Ns) by w_(Ns*R)^(r*k), read from the
// stage table at twOff(S) + k*R + r.
//   TwMem  reads the table (L1/L2 resident) at every use.
//   TwReg  loads each thread's entries once into registers; persistent
//          kernels then reuse them for every transform they process, and no
//          table load competes with the streaming data loads.
// ---------------------------------------------------------------------------
template <class SC, class V = float2>
struct TwMem {
    const V* __restrict__ p;
    __device__ __forceinline__ explicit TwMem(const V* q) : p(q) {}
    __device__ __forceinline__ void init(int) {}

    template <int S, int R>
    __device__ __forceinline__ void apply(V (&u)[R], int /*b*/, int j) const {
        constexpr int LNS = SC::log2NS(S);
        const int k = j & ((1 << LNS) - 1);
        const V* q = p + SC::twOff(S) + k * R;
        if constexpr (R == 2 || !std::is_same<V, float2>::value) {
#pragma unroll
            for (int r = 1; r < R; ++r) u[r] = c_mul(u[r], q[r]);
        } else {
            // FP32: two twiddles per 16-byte load
            const float4* q4 = reinterpret_cast<const float4*>(q);
#pragma unroll
            for (int h = 0; h < R / 2; ++h) {
                const float4 w = q4[h];
                if (h > 0) u[2 * h] = c_mul(u[2 * h], make_float2(w.x, w.y));
                u[2 * h + 1] = c_mul(u[2 * h + 1], make_float2(w.z, w.w));
            }
        }
    }
};

template <class SC, class V = float2>
struct TwReg {
    static constexpr int E = SC::E;
    const V* __restrict__ p;
    V w[SC::NST > 1 ? SC::NST : 1][E];  // w[S][b*R + r]
    __device__ __forceinline__ explicit TwReg(const V* q) : p(q) {}

    // one stage's entries for the thread whose stage-S index is t (S > 0)
    template <int S>
    __device__ __forceinline__ void load_stage_only(int t) {
        constexpr int R = 1 << SC::log2R(S);
        constexpr int B = E / R;
        constexpr int LNS = SC::log2NS(S);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k = (t + b * SC::T) & ((1 << LNS) - 1);
            const V* q = p + SC::twOff(S) + k * R;
#pragma unroll
            for (int r = 1; r < R; ++r) w[S][b * R + r] = q[r];
        }
    }

    template <int S>
    __device__ __forceinline__ void load_stage(int t) {
        if constexpr (S < SC::NST) {
            if constexpr (S > 0) load_stage_only<S>(t);
            load_stage<S + 1>(t);
        }
    }
    __device__ __forceinline__ void init(int t) { load_stage<0>(t); }

    // variant for engines whose stages map threads differently: stage S takes
    // its t from ENG::map<S>(tid)
    template <class ENG, int S>
    __device__ __forceinline__ void load_stage_mapped(int tid) {
        if constexpr (S < SC::NST) {
            if constexpr (S > 0) {
                int g, t;
                ENG::template map<S>(tid, g, t);
                load_stage_only<S>(t);
            }
            load_stage_mapped<ENG, S + 1>(tid);
        }
    }
    template <class ENG>
    __device__ __forceinline__ void init_engine(int tid) { load_stage_mapped<ENG, 0>(tid); }

    template <int S, int R>
    __device__ __forceinline__ void apply(V (&u)[R], int b, int /*j*/) const {
#pragma unroll
        for (int r = 1; r < R; ++r) u[r] = c_mul(u[r], w[S][b * R + r]);
    }
};

// Registers for the last stage's twiddles (the largest table), the table for
// the stages before it: half the register cost of TwReg for three-stage
// schedules.  The earlier stages' tables are small and stay in L1.
template <class SC, class V = float2>
struct TwLast {
    TwReg<SC, V> reg;
    TwMem<SC, V> mem;
    __device__ __forceinline__ explicit TwLast(const V* q) : reg(q), mem(q) {}
    __device__ __forceinline__ void init(int t) {
        if constexpr (SC::NST > 1) reg.template load_stage_only<SC::NST - 1>(t);
    }
    template <int S, int R>
    __device__ __forceinline__ void apply(V (&u)[R], int b, int j) const {
        if constexpr (S == SC::NST - 1) reg.template apply<S, R>(u, b, j);
        else mem.template apply<S, R>(u, b, j);
    }
};

// ---------------------------------------------------------------------------
// Block engine: G independent L-point sub-FFTs per workgroup, T threads each.
// Thread -> (g, t) mapping per stage: "g-fast" (g = tid % G) or "t-fast"
// (t = tid % T).  The first stage uses FIRST_GFAST, the last LAST_GFAST, the
// ones between t-fast.  On entry v[m] holds input element t + T*m of sub-FFT
// g under the first mapping; on exit v[m] holds output element t + T*m of
// sub-FFT g under the last mapping.  GS is the LDS stride between groups.
// HALF: each exchange passes the real parts and then the imaginary parts
// through a buffer of G*GS reals (half the LDS of a complex exchange, two
// more barriers per exchange), so more workgroups fit on a compute unit.
// ---------------------------------------------------------------------------
template <class SC, int G, int GS, bool FIRST_GFAST, bool LAST_GFAST, bool WAVE, bool HALF = false>
struct Engine {
    static constexpr int E = SC::E;
    static constexpr int T = SC::T;
    static constexpr int NST = SC::NST;
    static_assert(NST >= 1, "empty schedule");
    static_assert(NST > 1 || FIRST_GFAST == LAST_GFAST, "one-stage engine cannot change mapping");

    template <int S>
    __device__ __forceinline__ static constexpr bool gfast() {
        return S == 0 ? FIRST_GFAST : (S == NST - 1 ? LAST_GFAST : false);
    }

    template <int S>
    __device__ __forceinline__ static void map(int tid, int& g, int& t) {
        if constexpr (gfast<S>()) {
            g = tid % G;
            t = tid / G;
        } else {
            t = tid % T;
            g = tid / T;
        }
    }

    // butterflies of stage S on registers; j = t + b*T
    template <int S, class V, class TW>
    __device__ __forceinline__ static void compute(V (&v)[E], int t, const TW& tw) {
        constexpr int LR = SC::log2R(S);
        constexpr int R = 1 << LR;
        constexpr int B = E / R;
        constexpr int NS = 1 << SC::log2NS(S);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            V u[R];
#pragma unroll
            for (int r = 0; r < R; ++r) u[r] = v[b + r * B];
            if constexpr (NS > 1) tw.template apply<S, R>(u, b, t + b * T);
            Dft<R>::run(u);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + r * B] = u[r];
        }
    }

    // store stage S's outputs into LDS at their self-sorting positions.  The
    // padded index i + (i >> 4) of base + r*Ns splits into a per-butterfly part
    // plus a constant whenever r*Ns is a multiple of 16 (Ns >= 16) or base is
    // a multiple of 16 (Ns = 1, R >= 16: then the padding of base + r is that
    // of base plus r >> 4), so each butterfly costs one address computation
    // instead of R.
    template <int S, class V>
    __device__ __forceinline__ static void write(const V (&v)[E], int g, int t, V* lds) {
        constexpr int LR = SC::log2R(S);
        constexpr int R = 1 << LR;
        constexpr int B = E / R;
        constexpr int LNS = SC::log2NS(S);
        constexpr int NS = 1 << LNS;
        constexpr bool SPLITS = NS >= 16 || (NS == 1 && R >= 16);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + b * T;
            const int k = j & (NS - 1);
            const int base = ((j >> LNS) << (LNS + LR)) + k;
            if constexpr (SPLITS) {
                V* p = lds + lds_at<GS>(g, base);
#pragma unroll
                for (int r = 0; r < R; ++r) p[NS >= 16 ? r * NS + ((r * NS) >> 4) : r + (r >> 4)] = v[b + r * B];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[lds_at<GS>(g, base + r * NS)] = v[b + r * B];
            }
        }
    }

    template <class V>
    __device__ __forceinline__ static void read(V (&v)[E], int g, int t, const V* lds) {
        if constexpr (T >= 16) {
            // T*m is a multiple of 16: padding of t + T*m = padding of t + T*m/16
            const V* p = lds + lds_at<GS>(g, t);
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = p[T * m + ((T * m) >> 4)];
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds[lds_at<GS>(g, t + T * m)];
        }
    }

    template <int S, class V, class TW>
    __device__ __forceinline__ static void stage(V (&v)[E], V* lds, const TW& tw, int tid) {
        int g, t;
        map<S>(tid, g, t);
        compute<S>(v, t, tw);
        if constexpr (S < NST - 1) {
            int g1, t1;
            map<S + 1>(tid, g1, t1);
            if constexpr (HALF) {
                using RV = typename RealOf<V>::type;
                RV* h = reinterpret_cast<RV*>(lds);
                RV part[E];
#pragma unroll
                for (int m = 0; m < E; ++m) part[m] = v[m].x;
                stage_sync<WAVE>();  // every thread has finished reading the previous exchange
                write<S>(part, g, t, h);
                stage_sync<WAVE>();  // the real parts are exchanged
                read(part, g1, t1, h);
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    v[m].x = part[m];  // next stage's layout
                    part[m] = v[m].y;  // still this stage's layout
                }
                stage_sync<WAVE>();  // every thread has read its real parts
                write<S>(part, g, t, h);
                stage_sync<WAVE>();  // the imaginary parts are exchanged
                read(part, g1, t1, h);
#pragma unroll
                for (int m = 0; m < E; ++m) v[m].y = part[m];
            } else {
                stage_sync<WAVE>();  // every thread has finished reading the previous exchange
                write<S>(v, g, t, lds);
                stage_sync<WAVE>();  // this exchange is complete
                read(v, g1, t1, lds);
            }
            stage<S + 1>(v, lds, tw, tid);
        }
    }

    template <class V, class TW>
    __device__ __forceinline__ static void run(V (&v)[E], V* lds, const TW& tw, int tid) {
        stage<0>(v, lds, tw, tid);
    }
};

// LDS complex elements needed by an engine with G groups of stride GS (0 if one stage)
template <class SC, int G, int GS>
constexpr int engine_lds_elems() { return SC::NST > 1 ? G * GS : 1; }

// ---------------------------------------------------------------------------
// Global memory access for the two layouts.  `a` is the interleaved array
// (as R*) or the real array; `b` the imaginary array (split only).
// ---------------------------------------------------------------------------
template <bool SPLIT, class R>
__device__ __forceinline__ cplx_t<R> gload(const R* a, const R* b, int64_t i) {
    if constexpr (SPLIT) {
        return cmk(a[i], b[i]);
    } else {
        return reinterpret_cast<const cplx_t<R>*>(a)[i];
    }
}

template <bool SPLIT, class R>
__device__ __forceinline__ void gstore(R* a, R* b, int64_t i, cplx_t<R> v) {
    if constexpr (SPLIT) {
        a[i] = v.x;
        b[i] = v.y;
    } else {
        reinterpret_cast<cplx_t<R>*>(a)[i] = v;
    }
}

// Streaming (nontemporal) variants for data that is read once and written
// once: the loads and stores carry the streaming cache hint.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
template <class R> struct NtVec;
template <> struct NtVec<float> { using type = f32x2_t; };
template <> struct NtVec<double> { using type = f64x2_t; };

template <bool SPLIT, class R>
__device__ __forceinline__ cplx_t<R> gload_nt(const R* a, const R* b, int64_t i) {
    if constexpr (SPLIT) {
        return cmk(__builtin_nontemporal_load(a + i), __builtin_nontemporal_load(b + i));
    } else {
        using NV = typename NtVec<R>::type;
        const NV x = __builtin_nontemporal_load(reinterpret_cast<const NV*>(a) + i);
        return cmk(R(x.x), R(x.y));
    }
}

template <bool SPLIT, class R>
__device__ __forceinline__ void gstore_nt(R* a, R* b, int64_t i, cplx_t<R> v) {
    if constexpr (SPLIT) {
        __builtin_nontemporal_store(v.x, a + i);
        __builtin_nontemporal_store(v.y, b + i);
    } else {
        using NV = typename NtVec<R>::type;
        NV x;
        x.x = v.x;
        x.y = v.y;
        __builtin_nontemporal_store(x, reinterpret_cast<NV*>(a) + i);
    }
}

// Wave priority while a batch of global loads is issued: the wavefront's
// loads leave ahead of the other wavefronts' arithmetic on its SIMD, so more
// reads are in flight while the rest of the workgroup computes.  Stores keep
// the normal priority (raising it there measured slower).
__device__ __forceinline__ void loads_begin() { __builtin_amdgcn_s_setprio(3); }
__device__ __forceinline__ void loads_end() { __builtin_amdgcn_s_setprio(0); }

// real/imaginary swap S of the inverse (free: a register renaming)
template <bool SWAP, class V>
__device__ __forceinline__ V swap_if(V a) {
    if constexpr (SWAP) return cmk(a.y, a.x);
    else return a;
}

// workgroup index -> tile index such that the workgroups one XCD receives
// (the dispatcher deals workgroups to the 8 XCDs in turn) take consecutive
// tiles, which then share L2 lines; identity when the count is not a
// multiple of 8.
__device__ __forceinline__ int64_t xcd_tile(int64_t wg, int64_t count) {
    if (count & 7) return wg;
    return (wg & 7) * (count >> 3) + (wg >> 3);
}

__device__ __forceinline__ double2 z_mul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}

// w_M^e in FP64 from the two tables below (not rounded)
__device__ __forceinline__ double2 twiddle_2level64(const double2* __restrict__ ta, const double2* __restrict__ tb,
                                                    int64_t e, int hbits) {
    return z_mul(ta[e >> hbits], tb[e & ((int64_t(1) << hbits) - 1)]);
}

// w_M^e = exp(-2 pi i e / M) from two FP64 tables, A[i] = w_M^(i << hbits) and
// B[i] = w_M^i (i < 2^hbits): the product is formed in FP64 and rounded once
// to the working precision.
__device__ __forceinline__ float2 round_to(double2 w, float2*) {
    return make_float2(static_cast<float>(w.x), static_cast<float>(w.y));
}
__device__ __forceinline__ double2 round_to(double2 w, double2*) { return w; }
template <class V>
__device__ __forceinline__ V cvt_tw(double2 w) { return round_to(w, static_cast<V*>(nullptr)); }

template <class V>
__device__ __forceinline__ V twiddle_2level(const double2* __restrict__ ta, const double2* __restrict__ tb,
                                           int64_t e, int hbits) {
    return cvt_tw<V>(twiddle_2level64(ta, tb, e, hbits));
}

// Stage twiddles by recurrence: butterfly j of stage S reads one FP64 value,
// w = w_(Ns*R)^k (k = j mod Ns, from a table of Ns entries at recOff(S)), and
// forms w^2 .. w^(R-1) by FP64 products (an error of a few FP64 ulps), each
// rounded once to the working precision: one load per butterfly instead of
// R - 1, for the sizes whose stage tables do not fit in registers.
template <class SC, class V = float2>
struct TwRec {
    const double2* __restrict__ p;
    __device__ __forceinline__ explicit TwRec(const double2* q) : p(q) {}
    __device__ __forceinline__ void init(int) {}

    template <int S, int R>
    __device__ __forceinline__ void apply(V (&u)[R], int /*b*/, int j) const {
        constexpr int LNS = SC::log2NS(S);
        const int k = j & ((1 << LNS) - 1);
        const double2 w = p[SC::recOff(S) + k];
        double2 x = w;
        u[1] = c_mul(u[1], cvt_tw<V>(x));
#pragma unroll
        for (int r = 2; r < R; ++r) {
            x = z_mul(x, w);
            u[r] = c_mul(u[r], cvt_tw<V>(x));
        }
    }
};

}  // namespace fftk
