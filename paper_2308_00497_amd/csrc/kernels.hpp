// Kernel templates of the gfx950 FFT and the host-side registry entries that
// describe every compiled instance.
//
//  k_single  one whole transform per sub-FFT (N up to the single-pass limit):
//            coalesced global load -> Stockham stages through LDS -> store.
//  k_pass    one pass of a multi-pass transform (N above the single-pass
//            limit): a radix-L Stockham pass over HBM whose DFT_L is itself a
//            register/LDS sub-FFT.  N = L_1 L_2 ... L_P; pass p has
//            Ns = L_1 ... L_(p-1) and, for butterfly column j < N/L_p with
//            k = j mod Ns, reads x[j + r N/L_p] (r < L_p), multiplies by
//            w_(Ns L_p)^(r k), transforms and writes
//            y[(j div Ns) Ns L_p + k + q Ns].  With P = 2 this is the
//            four-step scheme: Eq. 1 with M = L_1, K = L_2.
//  k_gen_*   FP64 twiddle generation on the GPU, rounded once to the working
//            precision.
//
// Every kernel is a template on the real type R (float or double); the FP64
// instances are the same code over double2.
#pragma once

#include <type_traits>

#include "fft_device.hpp"
#include "registry.hpp"

namespace fftk {

// ---------------------------------------------------------------------------
// twiddle generation (FP64 on the device)
// ---------------------------------------------------------------------------

// dst[k*R + r] = w_(Ns*R)^(r*k), k < Ns, r < R, computed as
// (cos, -sin)(2 pi m / M) = (cospi, -sinpi)(2m/M) with the exact rational
// argument 2m/M (M a power of two), then rounded once to V's precision.
template <class V>
__global__ void k_gen_stage_tw(V* dst, int log2NS, int log2R);

// dst[i] = w_M^(i*step) in FP64 for i < count.
__global__ void k_gen_pow64(double2* dst, int log2M, int64_t step, int64_t count);

// ---------------------------------------------------------------------------
// single-pass kernel
// ---------------------------------------------------------------------------
template <int LOG2N, int LOG2E, int WGT>
struct SingleShape {
    using SC = Sched<LOG2N, LOG2E, false>;
    static constexpr int G = SC::T >= WGT ? 1 : WGT / SC::T;  // transforms per workgroup
    static constexpr int THREADS = G * SC::T;
    static constexpr int GS = SC::L + (SC::L >> 4);
    static constexpr int LDS = engine_lds_elems<SC, G, GS>();
    static constexpr bool WAVE = SC::T <= 64;
};

// LDS elements (complex) of a single-pass workgroup: the engine's exchange,
// with staging the whole group (every group padded as in the engine), or with
// HALF exchanges (one real part at a time) half the engine's
template <int LOG2N, int LOG2E, int WGT, bool STG, bool HALF = false>
constexpr int single_lds() {
    using SH = SingleShape<LOG2N, LOG2E, WGT>;
    if constexpr (HALF) return (SH::LDS + 1) / 2;
    return STG && SH::G * SH::GS > SH::LDS ? SH::G * SH::GS : SH::LDS;
}

// Persistent: each workgroup loops over groups of G transforms
// (grp = blockIdx.x, blockIdx.x + gridDim.x, ...), so per-thread state such as
// register-resident twiddles is loaded once per workgroup.  Data is read and
// written with streaming (nontemporal) accesses.  SWAP exchanges the real and
// imaginary halves of each interleaved element on load and store (the inverse
// transform; split arrays get the same effect from swapped pointers).  With PF
// the loads of the workgroup's next group are issued before the stages of the
// current one run, so HBM reads overlap the LDS work (the stage barriers
// order LDS only and leave them in flight).  With STG (small transforms, each
// inside one wavefront) a wavefront's transforms, which are contiguous in
// memory, are read and written as one contiguous run (lane l takes elements
// l, l + 64, ...) and staged through LDS into the engine's layout, instead of
// each lane reading its own points at stride T.  With HALF the stages exchange
// real and imaginary parts one after the other through half the LDS, so more
// workgroups fit on a compute unit where LDS limits them.
template <class R, int LOG2N, int LOG2E, int WGT, bool SPLIT, bool SWAP, bool TWREG, bool PF = false,
          bool STG = false, bool HALF = false, bool TWREC = false>
__global__ void __launch_bounds__((SingleShape<LOG2N, LOG2E, WGT>::THREADS))
k_single(const R* ia, const R* ib, R* oa, R* ob, const cplx_t<R>* __restrict__ tw, int64_t batch) {
    using V = cplx_t<R>;
    using SH = SingleShape<LOG2N, LOG2E, WGT>;
    using SC = typename SH::SC;
    constexpr int E = SC::E, T = SC::T, L = SC::L, G = SH::G;
    static_assert(!(STG && PF), "staging and prefetching are separate variants");
    static_assert(!(STG && HALF), "staged transforms use the complex exchange");
    static_assert(!TWREC || (!TWREG && !STG), "the recurrence twiddles serve the unstaged table kernels");
    static_assert(!STG || (SH::WAVE && (64 % T) == 0 && SH::THREADS % 64 == 0),
                  "staging needs every transform inside one wavefront");
    __shared__ V lds[single_lds<LOG2N, LOG2E, WGT, STG, HALF>()];

    const int tid = threadIdx.x;
    TwReg<SC, V> twr(tw);
    if constexpr (TWREG) twr.init(tid % T);

    const int64_t groups = (batch + G - 1) / G;
    // Interleaved data: visit the groups of the two halves of the batch in
    // alternation (visit 2i -> group i, 2i + 1 -> group half + i), so the
    // workgroups in flight read two distant streams, as split data does by
    // itself; measured 1-2 % faster for interleaved, slower for split.
    const int64_t half = (groups + 1) / 2;
    auto group_of = [&](int64_t visit) {
        if constexpr (SPLIT) return visit;
        else return (visit & 1) ? half + (visit >> 1) : (visit >> 1);
    };
    // element index of this thread's first point in group grp (row >= batch: none)
    auto row_base = [&](int64_t visit, int tidl, bool& active) {
        const int64_t tr = group_of(visit) * G + tidl / T;
        active = tr < batch;
        return tr * L + tidl % T;
    };
    V nxt[PF ? E : 1];
    if constexpr (PF) {
        bool act;
        const int64_t base = row_base(blockIdx.x, tid, act);
        if (blockIdx.x < groups && act) {
            loads_begin();
#pragma unroll
            for (int m = 0; m < E; ++m) nxt[m] = swap_if<SWAP>(gload_nt<SPLIT>(ia, ib, base + T * m));
            loads_end();
        }
    }
    for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        // table reads stay inside the loop unless the registers were asked for:
        // the empty asm hides the pointer's loop invariance from the compiler
        // thread-derived addresses are recomputed each iteration instead of
        // being held in registers across the loop: the registers are worth more
        // as occupancy (N = 4096 fits 4 workgroups per CU this way)
        const V* twl = tw;
        int tidl = tid;
        asm volatile("" : "+v"(tidl));
        if constexpr (!TWREG) asm volatile("" : "+s"(twl));
        if constexpr (STG) {
            // this wavefront's transforms: elements w0 .. w0 + 64 E - 1 of the group
            const int lane = tidl & 63, w0 = (tidl >> 6) * 64 * E;
            const int64_t row0 = group_of(grp) * G;
            const int64_t ebase = row0 * L;
            V v[E];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int i = w0 + lane + 64 * m;
                v[m] = row0 + i / L < batch ? swap_if<SWAP>(gload_nt<SPLIT>(ia, ib, ebase + i)) : c_zero<V>();
            }
            stage_sync<true>();  // this wavefront's reads of the previous group are done
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int i = w0 + lane + 64 * m;
                lds[lds_at<SH::GS>(i / L, i % L)] = v[m];
            }
            stage_sync<true>();
            const int t = tidl % T, g = tidl / T;  // the engine's first mapping
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds[lds_at<SH::GS>(g, t + T * m)];
            if constexpr (TWREG) Engine<SC, G, SH::GS, false, false, true>::run(v, lds, twr, tidl);
            else Engine<SC, G, SH::GS, false, false, true>::run(v, lds, TwMem<SC, V>(twl), tidl);
            stage_sync<true>();  // the engine's (or the staging's) last reads are done
#pragma unroll
            for (int m = 0; m < E; ++m) lds[lds_at<SH::GS>(g, t + T * m)] = v[m];
            stage_sync<true>();
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int i = w0 + lane + 64 * m;
                if (row0 + i / L < batch)
                    gstore_nt<SPLIT>(oa, ob, ebase + i, swap_if<SWAP>(lds[lds_at<SH::GS>(i / L, i % L)]));
            }
            continue;
        }
        bool active;
        const int64_t base = row_base(grp, tidl, active);
        V v[E];
        if constexpr (PF) {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = active ? nxt[m] : c_zero<V>();
            bool act2;
            const int64_t base2 = row_base(grp + gridDim.x, tidl, act2);
            if (grp + gridDim.x < groups && act2) {
                loads_begin();
#pragma unroll
                for (int m = 0; m < E; ++m) nxt[m] = swap_if<SWAP>(gload_nt<SPLIT>(ia, ib, base2 + T * m));
                loads_end();
            }
        } else if (active) {
            // raised load priority: measured faster for interleaved data
            // (N = 4096: 97 -> 92 us) and for FP32 split data at N = 4096
            // (batch 1024: 15.2 -> 14.6 us; batch 8192: 0-1 %), slower for
            // split data at N = 8192
            constexpr bool PRIO = !SPLIT || (LOG2N == 12 && sizeof(R) == 4);
            if constexpr (PRIO) loads_begin();
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = swap_if<SWAP>(gload_nt<SPLIT>(ia, ib, base + T * m));
            if constexpr (PRIO) loads_end();
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = c_zero<V>();
        }
        if constexpr (TWREG) Engine<SC, G, SH::GS, false, false, SH::WAVE, HALF>::run(v, lds, twr, tidl);
        else if constexpr (TWREC)
            Engine<SC, G, SH::GS, false, false, SH::WAVE, HALF>::run(
                v, lds, TwRec<SC, V>(reinterpret_cast<const double2*>(twl)), tidl);
        else Engine<SC, G, SH::GS, false, false, SH::WAVE, HALF>::run(v, lds, TwMem<SC, V>(twl), tidl);
        if (active) {
#pragma unroll
            for (int m = 0; m < E; ++m) gstore_nt<SPLIT>(oa, ob, base + T * m, swap_if<SWAP>(v[m]));
        }
    }
}

template <class R, int LOG2N, int LOG2E, int WGT, bool SPLIT, bool SWAP, bool TWREG, bool PF = false, bool STG = false,
          bool HALF = false, bool TWREC = false>
hipError_t launch_single(const void* ia, const void* ib, void* oa, void* ob, const void* tw, int64_t batch, int grid,
                         hipStream_t s) {
    using SH = SingleShape<LOG2N, LOG2E, WGT>;
    const int64_t groups = (batch + SH::G - 1) / SH::G;
    const int64_t blocks = groups < grid ? groups : grid;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_single<R, LOG2N, LOG2E, WGT, SPLIT, SWAP, TWREG, PF, STG, HALF, TWREC>), dim3(static_cast<unsigned>(blocks)),
                       dim3(SH::THREADS), 0, s, static_cast<const R*>(ia), static_cast<const R*>(ib),
                       static_cast<R*>(oa), static_cast<R*>(ob), static_cast<const cplx_t<R>*>(tw), batch);
    return hipGetLastError();
}

// REC: the recurrence table (TwRec) - offsets and size in complex entries of
// the plan's precision, PAIR per FP64 pair (2 in a float2 buffer, which then
// holds it 16-byte aligned; 1 in a double2 buffer)
template <class SC, bool REC = false, int PAIR = 2>
EngineInfo engine_info() {
    EngineInfo e{};
    e.log2l = SC::LOG2L;
    e.log2e = SC::LE;
    e.remfirst = SC::REMFIRST;
    e.nst = SC::NST;
    e.rec = REC;
    e.tw_size = REC ? PAIR * SC::REC_SIZE : SC::TW_SIZE;
    for (int s = 0; s < SC::NST && s < kMaxStages; ++s) {
        e.log2ns[s] = SC::log2NS(s);
        e.log2r[s] = SC::log2R(s);
        e.tw_off[s] = REC ? PAIR * SC::recOff(s) : SC::twOff(s);
    }
    return e;
}

template <class R, int LOG2N, int LOG2E, int WGT, bool SPLIT, bool SWAP, bool TWREG, bool PF = false, bool STG = false,
          bool HALF = false, bool TWREC = false>
SingleKernel single_entry() {
    using SH = SingleShape<LOG2N, LOG2E, WGT>;
    SingleKernel k{};
    k.real_bytes = sizeof(R);
    k.log2n = LOG2N;
    k.log2e = SH::SC::LE;
    k.wgt = WGT;
    k.split = SPLIT;
    k.swap = SWAP;
    k.twreg = TWREG;
    k.pf = PF;
    k.stg = STG;
    k.half = HALF;
    k.twrec = TWREC;
    k.fn = &launch_single<R, LOG2N, LOG2E, WGT, SPLIT, SWAP, TWREG, PF, STG, HALF, TWREC>;
    k.kernel = reinterpret_cast<const void*>(&k_single<R, LOG2N, LOG2E, WGT, SPLIT, SWAP, TWREG, PF, STG, HALF, TWREC>);
    k.eng = engine_info<typename SH::SC, TWREC, sizeof(R) == 4 ? 2 : 1>();
    k.threads = SH::THREADS;
    k.per_wg = SH::G;
    k.lds_bytes = single_lds<LOG2N, LOG2E, WGT, STG, HALF>() * sizeof(cplx_t<R>);
    return k;
}

// ---------------------------------------------------------------------------
// pass kernel of the multi-pass scheme
// ---------------------------------------------------------------------------
template <int LOG2L, int LOG2E, int LOG2C>
struct PassShape {
    using SC = Sched<LOG2L, LOG2E, false>;
    static constexpr int C = 1 << LOG2C;                // columns per workgroup
    static constexpr int THREADS = C * SC::T;
    // group stride: the padded column plus an odd-ish skew so that the
    // column-fast first stage spreads its C lanes over distinct banks
    static constexpr int GS = SC::L + (SC::L >> 4) + 2;
    static constexpr int LDS = C * GS;
};

// FP32 first-pass tiles whose complex exchange would need more than 80 KB of
// LDS (one workgroup per CU) exchange the real and the imaginary parts in
// turn through half of it, so that two workgroups fit on a CU; their register
// allocation is then held to what two workgroups allow (the first pass forms
// no pass twiddles and fits; later passes would spill)
template <class R, int LOG2L, int LOG2E, int LOG2C, bool FIRST>
constexpr bool pass_half() {
    return FIRST && sizeof(R) == 4 && PassShape<LOG2L, LOG2E, LOG2C>::LDS * 8 > 80 * 1024;
}
template <class R, int LOG2L, int LOG2E, int LOG2C, bool FIRST>
constexpr int pass_lds() {
    constexpr int L = PassShape<LOG2L, LOG2E, LOG2C>::LDS;
    return pass_half<R, LOG2L, LOG2E, LOG2C, FIRST>() ? (L + 1) / 2 : L;
}
// minimum waves per SIMD for the launch bounds: two workgroups per CU with
// half-width exchanges, else no constraint
template <class R, int LOG2L, int LOG2E, int LOG2C, bool FIRST>
constexpr int pass_waves() {
    return pass_half<R, LOG2L, LOG2E, LOG2C, FIRST>() ? 2 * PassShape<LOG2L, LOG2E, LOG2C>::THREADS / 256 : 1;
}

// One tile of one pass: C consecutive butterfly columns j0 .. j0+C-1 of the
// transform starting at element tbase.  Shared by the pass kernel and the
// ragged persistent kernel.  `lds` holds PassShape::LDS complex elements; TW
// supplies the sub-FFT's stage twiddles.  `stream` (kStreamIn | kStreamOut)
// marks the loads and the stores that touch the caller's buffers: those use
// streaming (nontemporal) access, since they are read or written once.  The
// intermediate buffers between passes are accessed normally, so the next pass
// can find them in the memory-side cache.  R (float or double) is deduced
// from `ia`.
//
// The pass twiddle of input r of column j (k = j mod Ns) is w_M^(r k), M = Ns L.
// With twshift = s > 0 the low s bits of k are a column index that the
// twiddles must not see: w_M'^(r (k >> s)), M' = (Ns >> s) L (the column
// passes of a multi-dimensional plan, columns at stride 2^s, run as passes of
// a chain whose Ns starts at 2^s; the tables are then those of M').
// Addresses: input r of column j sits at
//   tbase + (j mod 2^ain) + ((j div 2^ain) 2^(ain + LOG2L)) + r 2^ain,
// and output q of a later pass at the same expression in aout.  The Stockham
// pass has ain = log2 N - LOG2L (j < 2^ain: x[j + r N/L]) and aout = log2 Ns
// (y[(j div Ns) Ns L + k + q Ns]); a negative argument selects these.  A pass
// with aout = ain writes its results over its own inputs (an in-place pass: a
// tile reads every address it writes, and all its loads are consumed before
// the engine's first barrier, so no tile overwrites data another still needs);
// the pass after an in-place penultimate pass finds its inputs with
// ain = log2 of that pass's Ns.
// A thread holds r = tp + T m (m < E), so w_M^(r k) = w_M^(tp k) (w_M^(T k))^m:
// two table lookups per thread and an FP64 running product, rounded once per
// element to the working precision (PASSTW = false leaves the factors out: a
// plain DFT_L down every column, the strided axes of multi-dimensional
// transforms) (the FP64 recurrence error over E <= 16
// steps stays near 1e-15: far below the rounding to FP32, and within a few
// units of FP64 rounding for the FP64 instances).
template <class T> struct nodeduce { using type = T; };

// The stream bits in KMASK are fixed at compile time to KVAL (the others come
// from `stream` at run time).  A run-time choice between a streaming and an
// ordinary access of the same address lets the compiler merge the two into one
// ordinary access when it simplifies this function before inlining it (it
// hoists identical scalar loads or stores out of both branches and drops the
// nontemporal hint), so callers fix the bits of the split-array sides, whose
// accesses are plain floats.
template <int LOG2L, int LOG2E, int LOG2C, bool FIRST, bool SPLIT_IN, bool SPLIT_OUT, bool SWAP_IN, bool SWAP_OUT,
          class TW, class R, bool PASSTW = true, int KMASK = 0, int KVAL = 0>
__device__ __forceinline__ void pass_tile(const R* ia, const typename nodeduce<R>::type* ib,
                                          typename nodeduce<R>::type* oa, typename nodeduce<R>::type* ob,
                                          const TW& tw, const double2* __restrict__ ta,
                                          const double2* __restrict__ tb, int log2N, int log2Ns, int hbits,
                                          int64_t tbase, int64_t j0, cplx_t<R>* lds, int tid, int stream,
                                          int twshift = 0, int ain = -1, int aout = -1) {
    using V = cplx_t<R>;
    using SH = PassShape<LOG2L, LOG2E, LOG2C>;
    using SC = typename SH::SC;
    constexpr int E = SC::E, T = SC::T, C = SH::C;
    static_assert(SC::NST >= 2, "a pass needs at least two stages to change the thread mapping");
    if (ain < 0) ain = log2N - LOG2L;
    if (aout < 0) aout = log2Ns;
    const int64_t stride = int64_t(1) << ain;  // distance between the L inputs of a column
    const int64_t NsMask = (int64_t(1) << log2Ns) - 1;

    // load: column-fast mapping, C consecutive columns form one contiguous run
    V v[E];
    {
        const int c = tid & (C - 1), tp = tid >> LOG2C;
        const int64_t j = j0 + c;
        const int64_t k = j & NsMask;
        const int64_t i0 = tbase + (j & (stride - 1)) + ((j >> ain) << (ain + LOG2L)) + tp * stride;
        if (stream & kLoadPrio) loads_begin();
        auto load_nt = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = swap_if<SWAP_IN>(gload_nt<SPLIT_IN>(ia, ib, i0 + T * m * stride));
        };
        auto load = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = swap_if<SWAP_IN>(gload<SPLIT_IN>(ia, ib, i0 + T * m * stride));
        };
        if constexpr ((KMASK & kStreamIn) != 0) {
            if constexpr ((KVAL & kStreamIn) != 0) load_nt();
            else load();
        } else {
            if (stream & kStreamIn) load_nt();
            else load();
        }
        if (stream & kLoadPrio) loads_end();
        if constexpr (!FIRST && PASSTW) {
            const int64_t kt = k >> twshift;
            double2 w = twiddle_2level64(ta, tb, kt * tp, hbits);
            const double2 step = twiddle_2level64(ta, tb, kt * T, hbits);
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m > 0) w = z_mul(w, step);
                v[m] = c_mul(v[m], cvt_tw<V>(w));
            }
        }
    }

    // first pass stores whole columns (thread-fast), later passes store runs of
    // C consecutive columns (column-fast)
    Engine<SC, C, SH::GS, true, !FIRST, false, pass_half<R, LOG2L, LOG2E, LOG2C, FIRST>()>::run(v, lds, tw, tid);

    if constexpr (FIRST) {
        const int t = tid % T, c = tid / T;
        const int64_t j = j0 + c;
        const int64_t obase = tbase + (j << LOG2L) + t;
        auto store_nt = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m) gstore_nt<SPLIT_OUT>(oa, ob, obase + T * m, swap_if<SWAP_OUT>(v[m]));
        };
        auto store = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m) gstore<SPLIT_OUT>(oa, ob, obase + T * m, swap_if<SWAP_OUT>(v[m]));
        };
        if constexpr ((KMASK & kStreamOut) != 0) {
            if constexpr ((KVAL & kStreamOut) != 0) store_nt();
            else store();
        } else {
            if (stream & kStreamOut) store_nt();
            else store();
        }
    } else {
        const int c = tid & (C - 1), tp = tid >> LOG2C;
        const int64_t j = j0 + c;
        const int64_t obase = tbase + ((j >> aout) << (aout + LOG2L)) + (j & ((int64_t(1) << aout) - 1));
        auto store_nt = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m)
                gstore_nt<SPLIT_OUT>(oa, ob, obase + (int64_t(tp + T * m) << aout), swap_if<SWAP_OUT>(v[m]));
        };
        auto store = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m)
                gstore<SPLIT_OUT>(oa, ob, obase + (int64_t(tp + T * m) << aout), swap_if<SWAP_OUT>(v[m]));
        };
        if constexpr ((KMASK & kStreamOut) != 0) {
            if constexpr ((KVAL & kStreamOut) != 0) store_nt();
            else store();
        } else {
            if (stream & kStreamOut) store_nt();
            else store();
        }
    }
}

// Persistent pass kernel: workgroup w takes tiles w, w + grid, ... (mapped
// so that the tiles one XCD works on are consecutive), with the sub-FFT's stage
// twiddles held in registers across tiles.  `stream` says which side is the
// caller's data (streaming access); the workspace between passes is not.
//
// The tile loop, with the stream bits in KMASK fixed at compile time to KVAL
// (pass_tile): the split-array sides take their stream bit as a constant.
// stage twiddles of a pass kernel in registers (else the recurrence table)
template <class R, int LOG2L, int LOG2E, int LOG2C>
constexpr bool pass_regtw() {
    return PassShape<LOG2L, LOG2E, LOG2C>::THREADS <= 512 && sizeof(R) == 4;
}

template <class R, int LOG2L, int LOG2E, int LOG2C, bool FIRST, bool SPLIT_IN, bool SPLIT_OUT, bool SWAP_IN,
          bool SWAP_OUT, int KMASK, int KVAL>
__device__ __forceinline__ void pass_loop(const R* ia, const R* ib, R* oa, R* ob, const cplx_t<R>* __restrict__ tw,
                                          const double2* __restrict__ ta, const double2* __restrict__ tb, int log2N,
                                          int log2Ns, int hbits, int64_t tiles, int stream, int twshift, int ain,
                                          int aout, cplx_t<R>* lds) {
    using V = cplx_t<R>;
    using SH = PassShape<LOG2L, LOG2E, LOG2C>;
    using SC = typename SH::SC;
    using ENG = Engine<SC, SH::C, SH::GS, true, !FIRST, false>;
    // stage twiddles in registers unless the workgroup is so large (1024
    // threads: at most 128 registers per lane) that they would spill, or the
    // elements are FP64 (twice the registers per entry); else one FP64 table
    // value per butterfly and its powers (TwRec)
    constexpr bool REGTW = pass_regtw<R, LOG2L, LOG2E, LOG2C>();
    const int tid = threadIdx.x;
    TwReg<SC, V> twr(tw);
    if constexpr (REGTW) twr.template init_engine<ENG>(tid);
    const int log2TilesPerT = log2N - LOG2L - LOG2C;  // tiles per transform (power of two)
    const int64_t slots = static_cast<int64_t>(gridDim.x);
    // load priority measured faster for FP32 tiles, slower for FP64 ones
    if constexpr (sizeof(R) == 4) stream |= kLoadPrio;
    for (int64_t lin = blockIdx.x; lin < tiles; lin += slots) {
        // consecutive tiles to the workgroups of one XCD (8 XCDs, dealt in turn)
        const int64_t tile = (slots & 7) ? lin : xcd_tile(lin, tiles);
        int tidl = tid;
        asm volatile("" : "+v"(tidl));  // keep per-tile addresses out of the loop-invariant set
        const int64_t b = tile >> log2TilesPerT;
        const int64_t j0 = (tile & ((int64_t(1) << log2TilesPerT) - 1)) << LOG2C;
        if constexpr (REGTW)
            pass_tile<LOG2L, LOG2E, LOG2C, FIRST, SPLIT_IN, SPLIT_OUT, SWAP_IN, SWAP_OUT, TwReg<SC, V>, R, true,
                      KMASK, KVAL>(ia, ib, oa, ob, twr, ta, tb, log2N, log2Ns, hbits, b << log2N, j0, lds, tidl,
                                   stream, twshift, ain, aout);
        else
            pass_tile<LOG2L, LOG2E, LOG2C, FIRST, SPLIT_IN, SPLIT_OUT, SWAP_IN, SWAP_OUT, TwRec<SC, V>, R, true,
                      KMASK, KVAL>(ia, ib, oa, ob, TwRec<SC, V>(reinterpret_cast<const double2*>(tw)), ta, tb, log2N,
                                   log2Ns, hbits, b << log2N, j0, lds, tidl, stream, twshift, ain, aout);
    }
}

template <class R, int LOG2L, int LOG2E, int LOG2C, bool FIRST, bool SPLIT_IN, bool SPLIT_OUT, bool SWAP_IN,
          bool SWAP_OUT>
__global__ void __launch_bounds__((PassShape<LOG2L, LOG2E, LOG2C>::THREADS), (pass_waves<R, LOG2L, LOG2E, LOG2C, FIRST>()))
k_pass(const R* ia, const R* ib, R* oa, R* ob, const cplx_t<R>* __restrict__ tw, const double2* __restrict__ ta,
       const double2* __restrict__ tb, int log2N, int log2Ns, int hbits, int64_t tiles, int stream, int twshift,
       int ain, int aout) {
    __shared__ cplx_t<R> lds[pass_lds<R, LOG2L, LOG2E, LOG2C, FIRST>()];
#define FFTK_PASS_LOOP(KM, KV)                                                                                   \
    pass_loop<R, LOG2L, LOG2E, LOG2C, FIRST, SPLIT_IN, SPLIT_OUT, SWAP_IN, SWAP_OUT, KM, KV>(                    \
        ia, ib, oa, ob, tw, ta, tb, log2N, log2Ns, hbits, tiles, stream, twshift, ain, aout, lds)
    if constexpr (SPLIT_IN) {
        if (stream & kStreamIn) FFTK_PASS_LOOP(kStreamIn, kStreamIn);
        else FFTK_PASS_LOOP(kStreamIn, 0);
    } else if constexpr (SPLIT_OUT) {
        // split output is always the caller's buffer (launch_pass checks)
        FFTK_PASS_LOOP(kStreamOut, kStreamOut);
    } else {
        FFTK_PASS_LOOP(0, 0);
    }
#undef FFTK_PASS_LOOP
}

template <class R, int LOG2L, int LOG2E, int LOG2C, bool FIRST, bool SPLIT_IN, bool SPLIT_OUT, bool SWAP_IN,
          bool SWAP_OUT>
hipError_t launch_pass(const void* ia, const void* ib, void* oa, void* ob, const void* tw, const double2* ta,
                       const double2* tb, int log2N, int log2Ns, int hbits, int64_t batch, int grid, int stream,
                       int twshift, int ain, int aout, hipStream_t s) {
    using SH = PassShape<LOG2L, LOG2E, LOG2C>;
    if (log2N < LOG2L + LOG2C) return hipErrorInvalidConfiguration;
    // runs of C columns must stay contiguous on both sides: ain, aout >= log2 C
    // (a first pass stores whole columns and takes no aout)
    if (ain >= 0 && (ain < LOG2C || ain > log2N - LOG2L)) return hipErrorInvalidConfiguration;
    if (aout >= 0 && (FIRST || aout < LOG2C || aout > log2N - LOG2L)) return hipErrorInvalidConfiguration;
    if (SPLIT_OUT && !(stream & kStreamOut)) return hipErrorInvalidValue;  // compiled for streaming stores only
    const int64_t tiles = (int64_t(1) << (log2N - LOG2L - LOG2C)) * batch;
    const int64_t blocks = tiles < grid ? tiles : grid;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_pass<R, LOG2L, LOG2E, LOG2C, FIRST, SPLIT_IN, SPLIT_OUT, SWAP_IN, SWAP_OUT>),
                       dim3(static_cast<unsigned>(blocks)), dim3(SH::THREADS), 0, s, static_cast<const R*>(ia),
                       static_cast<const R*>(ib), static_cast<R*>(oa), static_cast<R*>(ob),
                       static_cast<const cplx_t<R>*>(tw), ta, tb, log2N, log2Ns, hbits, tiles, stream, twshift, ain,
                       aout);
    return hipGetLastError();
}

template <class R, int LOG2L, int LOG2E, int LOG2C, bool FIRST, bool SPLIT_IN, bool SPLIT_OUT, bool SWAP_IN = false,
          bool SWAP_OUT = false>
PassKernel pass_entry() {
    using SH = PassShape<LOG2L, LOG2E, LOG2C>;
    PassKernel k{};
    k.real_bytes = sizeof(R);
    k.log2l = LOG2L;
    k.log2e = SH::SC::LE;
    k.log2c = LOG2C;
    k.first = FIRST;
    k.split_in = SPLIT_IN;
    k.split_out = SPLIT_OUT;
    k.swap_in = SWAP_IN;
    k.swap_out = SWAP_OUT;
    k.fn = &launch_pass<R, LOG2L, LOG2E, LOG2C, FIRST, SPLIT_IN, SPLIT_OUT, SWAP_IN, SWAP_OUT>;
    k.kernel =
        reinterpret_cast<const void*>(&k_pass<R, LOG2L, LOG2E, LOG2C, FIRST, SPLIT_IN, SPLIT_OUT, SWAP_IN, SWAP_OUT>);
    k.eng = engine_info<typename SH::SC, !pass_regtw<R, LOG2L, LOG2E, LOG2C>(), sizeof(R) == 4 ? 2 : 1>();
    k.threads = SH::THREADS;
    k.lds_bytes = pass_lds<R, LOG2L, LOG2E, LOG2C, FIRST>() * sizeof(cplx_t<R>);
    return k;
}

}  // namespace fftk
