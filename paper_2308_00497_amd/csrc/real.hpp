// Real-input transforms (R2C) and their inverse (C2R) for N = 2H real points,
// computed through the complex transform of half the length.
//
// R2C: the real row read as H complex pairs, z[n] = x[2n] + i x[2n+1], is one
// complex sequence; its DFT Z = DFT_H(z) holds the spectra of the even and
// the odd samples,
//     Ev[k] = (Z[k] + conj Z[H-k]) / 2,      Od[k] = -i (Z[k] - conj Z[H-k]) / 2
// (indices of Z mod H), and the DFT of x is X[k] = Ev[k] + w_N^k Od[k] for
// k = 0 .. H, with X[H-k] = conj(Ev[k] - w_N^k Od[k]).  A step of Eq. 1 with
// K = 2 on the real sequence, whose two half-length DFTs share one complex
// transform.
//
// C2R inverts it: with A = X[k] + conj X[H-k] and B = X[k] - conj X[H-k],
//     Z'[k] = A + i w_N^-k B,   k = 0 .. H-1,
// (the imaginary parts of X[0] and X[H] do not enter: the output is the real
// part of the inverse transform of the Hermitian extension), and the
// unnormalised inverse DFT_H of Z' is N (x[2n] + i x[2n+1]).
//
// Single-pass sizes run in one kernel: the half-length engine plus one more
// exchange through LDS that pairs k with H - k.  Larger sizes run the
// half-length multi-pass chain and one extra pass over HBM (k_r2c_post,
// k_c2r_pre).
//
// Adjoints (the backward of a real plan): with the real inner product on the
// complex side, the adjoint of R2C maps g (H + 1 values) to
// x[n] = Re sum_{k=0..H} g[k] w_N^-kn, which is C2R of g with the interior
// bins k = 1 .. H-1 halved; the adjoint of C2R is R2C with the interior bins
// doubled.  Every kernel below takes that interior scale (1 for the plain
// transforms).
#pragma once

#include "kernels.hpp"

namespace fftk {

template <class V>
__device__ __forceinline__ V c_scale(V a, typename RealOf<V>::type s) {
    return cmk(a.x * s, a.y * s);
}

// Ev[k] and w Od[k] for a = Z[k], mir = Z[(H-k) mod H], w = w_N^k:
// X[k] = ev + wo and X[H-k] = conj(ev - wo)
template <class V>
__device__ __forceinline__ void r2c_parts(V a, V mir, V w, V& ev, V& wo) {
    using R = typename RealOf<V>::type;
    const R h = R(0.5);
    ev = cmk(h * (a.x + mir.x), h * (a.y - mir.y));
    const V od = cmk(h * (a.y + mir.y), h * (mir.x - a.x));
    wo = c_mul(od, w);
}

// Z'[k] for a = X[k], mir = X[H-k], w = w_N^k
template <class V>
__device__ __forceinline__ V c2r_point(V a, V mir, V w) {
    const V c = cmk(mir.x, -mir.y);
    const V s = c_add(a, c), d = c_sub(a, c);
    const V wd = c_mul(d, cmk(w.x, -w.y));  // w^-k (a - conj mir)
    return cmk(s.x - wd.y, s.y + wd.x);      // s + i wd
}

template <class R, int LOG2H, int LOG2E, int WGT>
struct RealShape {
    using SH = SingleShape<LOG2H, LOG2E, WGT>;
    using SC = typename SH::SC;
    static constexpr int EX = SH::G * SH::GS;  // the pairing exchange: full group stride
    // a separate exchange region when both fit in 64 KB: the exchange then
    // needs no barrier against the engine's last LDS reads (the engine's own
    // stage barriers order one transform's exchange before the next one's)
    static constexpr bool SEP = SC::NST >= 2 && 2 * EX * sizeof(cplx_t<R>) <= 65536;
    static constexpr int LDS = SEP ? 2 * EX : EX;
};

// LDS elements of the real kernel: engine and pairing exchange, plus with
// staging one row of H + 1 complex values per transform of the workgroup
template <class R, int LOG2H, int LOG2E, int WGT, bool STG>
constexpr int real_lds() {
    using RS = RealShape<R, LOG2H, LOG2E, WGT>;
    return STG ? RS::LDS + SingleShape<LOG2H, LOG2E, WGT>::G * ((1 << LOG2H) + 1) : RS::LDS;
}

// One persistent single-pass kernel per direction.  `tw` is the engine's stage
// table, `twn` holds w_N^k for k < H.  R2C reads the real array as H complex
// pairs per row and writes H + 1 complex values per row; C2R the reverse.
// With STG (rows short enough that a wavefront holds whole rows) every
// wavefront reads and writes its rows as one contiguous run per side (lane l
// takes elements l, l + 64, ...), staged through LDS rows of H + 1 values, so
// that no access is a short strided one; C2R then pairs X[k] with X[H - k]
// straight from the staged rows.
template <class R, int LOG2H, int LOG2E, int WGT, bool C2R, bool SPLIT, bool TWREG, bool STG = false,
          bool TWREC = false>
__global__ void __launch_bounds__((SingleShape<LOG2H, LOG2E, WGT>::THREADS))
k_real_single(const R* ia, const R* ib, R* oa, R* ob, const cplx_t<R>* __restrict__ tw,
              const cplx_t<R>* __restrict__ twn, int64_t batch, R iscale) {
    using V = cplx_t<R>;
    using SH = SingleShape<LOG2H, LOG2E, WGT>;
    using SC = typename SH::SC;
    using RS = RealShape<R, LOG2H, LOG2E, WGT>;
    using ENG = Engine<SC, SH::G, SH::GS, false, false, SH::WAVE>;
    constexpr int E = SC::E, T = SC::T, H = SC::L, G = SH::G;
    static_assert(LOG2H >= 1, "H = 1 runs as a pre/post pass only");
    static_assert(!STG || (SH::WAVE && (64 % T) == 0 && SH::THREADS % 64 == 0),
                  "staging needs whole rows inside one wavefront");
    static_assert(!TWREC || (!TWREG && !STG), "the recurrence twiddles serve the unstaged table kernels");
    __shared__ V lds[real_lds<R, LOG2H, LOG2E, WGT, STG>()];
    V* const xch = RS::SEP ? lds + RS::EX : lds;  // pairing exchange region
    V* const stg = lds + RS::LDS;                 // staged rows (STG), stride H + 1
    constexpr int SGS = H + 1;
    constexpr int RPW = 64 / (T < 64 ? T : 64);   // rows per wavefront (STG)

    const int tid = threadIdx.x;
    TwReg<SC, V> twr(tw);
    if constexpr (TWREG) twr.init(tid % T);
    // w_N^k of this thread's points, loaded once per workgroup
    V wn[E];
#pragma unroll
    for (int m = 0; m < E; ++m) wn[m] = twn[tid % T + T * m];

    const int64_t groups = (batch + G - 1) / G;
    for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        const V* twl = tw;
        int tidl = tid;
        asm volatile("" : "+v"(tidl));
        if constexpr (!TWREG) asm volatile("" : "+s"(twl));
        const int tl = tidl % T, gl = tidl / T;
        const int64_t tr = grp * G + gl;
        const bool active = tr < batch;
        V v[E];
        if constexpr (STG) {
            const int lane = tidl & 63, r0 = (tidl >> 6) * RPW;  // this wavefront's first row in the group
            const int64_t grow0 = grp * G + r0;                  // ... and in the batch
            if constexpr (!C2R) {
                // the wavefront's real rows as H complex pairs each: 64 E pairs in a row
                loads_begin();
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = lane + 64 * m;
                    v[m] = grow0 + i / H < batch ? gload_nt<false>(ia, ia, grow0 * H + i) : c_zero<V>();
                }
                loads_end();
                stage_sync<true>();  // this wavefront's reads of its previous rows are done
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = lane + 64 * m;
                    stg[(r0 + i / H) * SGS + i % H] = v[m];
                }
                stage_sync<true>();
#pragma unroll
                for (int m = 0; m < E; ++m) v[m] = stg[gl * SGS + tl + T * m];
                if constexpr (TWREG) ENG::run(v, lds, twr, tidl);
                else if constexpr (TWREC) ENG::run(v, lds, TwRec<SC, V>(reinterpret_cast<const double2*>(twl)), tidl);
                else ENG::run(v, lds, TwMem<SC, V>(twl), tidl);
                if constexpr (!RS::SEP) stage_sync<true>();
#pragma unroll
                for (int m = 0; m < E; ++m) xch[lds_at<SH::GS>(gl, tl + T * m)] = v[m];
                stage_sync<true>();
                const V xh = cmk(v[0].x - v[0].y, R(0));  // X[H] (used by tl == 0)
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = tl + T * m;
                    const V mir = xch[lds_at<SH::GS>(gl, (H - k) & (H - 1))];
                    V ev, wo;
                    r2c_parts(v[m], mir, wn[m], ev, wo);
                    const V xk = c_add(ev, wo);
                    v[m] = k == 0 ? xk : c_scale(xk, iscale);
                }
#pragma unroll
                for (int m = 0; m < E; ++m) stg[gl * SGS + tl + T * m] = v[m];
                if (tl == 0) stg[gl * SGS + H] = xh;
                stage_sync<true>();
                // the wavefront's output rows: RPW (H + 1) values in a row
#pragma unroll
                for (int m = 0; m <= E; ++m) {
                    const int j = lane + 64 * m;
                    if (j < RPW * SGS && grow0 + j / SGS < batch)
                        gstore_nt<SPLIT>(oa, ob, grow0 * SGS + j, stg[r0 * SGS + j]);
                }
            } else {
                // the wavefront's complex rows: RPW (H + 1) values in a row
                V in[E + 1];
                loads_begin();
#pragma unroll
                for (int m = 0; m <= E; ++m) {
                    const int j = lane + 64 * m;
                    in[m] = j < RPW * SGS && grow0 + j / SGS < batch ? gload_nt<SPLIT>(ia, ib, grow0 * SGS + j)
                                                                      : c_zero<V>();
                }
                loads_end();
                stage_sync<true>();
#pragma unroll
                for (int m = 0; m <= E; ++m) {
                    const int j = lane + 64 * m;
                    if (j < RPW * SGS) stg[r0 * SGS + j] = in[m];
                }
                stage_sync<true>();
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = tl + T * m;
                    V a = stg[gl * SGS + k], mir;
                    if (k == 0) {
                        a = cmk(a.x, R(0));
                        mir = cmk(stg[gl * SGS + H].x, R(0));
                    } else {
                        mir = stg[gl * SGS + H - k];
                    }
                    const V zk = c2r_point(a, mir, wn[m]);
                    v[m] = swap_if<true>(k == 0 ? zk : c_scale(zk, iscale));
                }
                if constexpr (TWREG) ENG::run(v, lds, twr, tidl);
                else if constexpr (TWREC) ENG::run(v, lds, TwRec<SC, V>(reinterpret_cast<const double2*>(twl)), tidl);
                else ENG::run(v, lds, TwMem<SC, V>(twl), tidl);
                stage_sync<true>();  // every lane's reads of the staged input rows are done
#pragma unroll
                for (int m = 0; m < E; ++m) stg[gl * SGS + tl + T * m] = swap_if<true>(v[m]);
                stage_sync<true>();
                // the wavefront's real rows as pairs: 64 E in a row
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int i = lane + 64 * m;
                    if (grow0 + i / H < batch)
                        gstore_nt<false>(oa, oa, grow0 * H + i, stg[(r0 + i / H) * SGS + i % H]);
                }
            }
            continue;
        }
        if constexpr (!C2R) {
            const int64_t base = tr * H + tl;  // complex pair index in the real row
            loads_begin();
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = active ? gload_nt<false>(ia, ia, base + T * m) : c_zero<V>();
            loads_end();
            if constexpr (TWREG) ENG::run(v, lds, twr, tidl);
            else if constexpr (TWREC) ENG::run(v, lds, TwRec<SC, V>(reinterpret_cast<const double2*>(twl)), tidl);
            else ENG::run(v, lds, TwMem<SC, V>(twl), tidl);
            if constexpr (!RS::SEP) stage_sync<SH::WAVE>();  // the engine's last reads of LDS are done
#pragma unroll
            for (int m = 0; m < E; ++m) xch[lds_at<SH::GS>(gl, tl + T * m)] = v[m];
            stage_sync<SH::WAVE>();
            if (active) {
                const int64_t ob0 = tr * (H + 1);
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int k = tl + T * m;
                    const V mir = xch[lds_at<SH::GS>(gl, (H - k) & (H - 1))];
                    V ev, wo;
                    r2c_parts(v[m], mir, wn[m], ev, wo);
                    const V xk = c_add(ev, wo);
                    gstore_nt<SPLIT>(oa, ob, ob0 + k, k == 0 ? xk : c_scale(xk, iscale));
                }
                if (tl == 0) gstore_nt<SPLIT>(oa, ob, ob0 + H, cmk(v[0].x - v[0].y, R(0)));
            }
        } else {
            const int64_t ib0 = tr * (H + 1);
            V xh = c_zero<V>();
            loads_begin();
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = active ? gload_nt<SPLIT>(ia, ib, ib0 + tl + T * m) : c_zero<V>();
            if (active && tl == 0) xh = gload<SPLIT>(ia, ib, ib0 + H);
            loads_end();
            if constexpr (!RS::SEP) stage_sync<SH::WAVE>();  // the previous transform's reads of LDS are done
#pragma unroll
            for (int m = 0; m < E; ++m) xch[lds_at<SH::GS>(gl, tl + T * m)] = v[m];
            stage_sync<SH::WAVE>();
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int k = tl + T * m;
                V a = v[m], mir;
                if (k == 0) {
                    a = cmk(a.x, R(0));
                    mir = cmk(xh.x, R(0));
                } else {
                    mir = xch[lds_at<SH::GS>(gl, H - k)];
                }
                // inverse DFT_H = S DFT_H S: swap on the way in and out;
                // Z'[k], k > 0, is built from interior bins only
                const V zk = c2r_point(a, mir, wn[m]);
                v[m] = swap_if<true>(k == 0 ? zk : c_scale(zk, iscale));
            }
            if constexpr (TWREG) ENG::run(v, lds, twr, tidl);
            else if constexpr (TWREC) ENG::run(v, lds, TwRec<SC, V>(reinterpret_cast<const double2*>(twl)), tidl);
            else ENG::run(v, lds, TwMem<SC, V>(twl), tidl);
            if (active) {
                const int64_t base = tr * H + tl;
#pragma unroll
                for (int m = 0; m < E; ++m) gstore_nt<false>(oa, oa, base + T * m, swap_if<true>(v[m]));
            }
        }
    }
}

template <class R, int LOG2H, int LOG2E, int WGT, bool C2R, bool SPLIT, bool TWREG, bool STG = false,
          bool TWREC = false>
hipError_t launch_real_single(const void* ia, const void* ib, void* oa, void* ob, const void* tw, const void* twn,
                              int64_t batch, int grid, double iscale, hipStream_t s) {
    using SH = SingleShape<LOG2H, LOG2E, WGT>;
    const int64_t groups = (batch + SH::G - 1) / SH::G;
    const int64_t blocks = groups < grid ? groups : grid;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_real_single<R, LOG2H, LOG2E, WGT, C2R, SPLIT, TWREG, STG, TWREC>), dim3(static_cast<unsigned>(blocks)),
                       dim3(SH::THREADS), 0, s, static_cast<const R*>(ia), static_cast<const R*>(ib),
                       static_cast<R*>(oa), static_cast<R*>(ob), static_cast<const cplx_t<R>*>(tw),
                       static_cast<const cplx_t<R>*>(twn), batch, static_cast<R>(iscale));
    return hipGetLastError();
}

template <class R, int LOG2H, int LOG2E, int WGT, bool C2R, bool SPLIT, bool TWREG, bool STG = false,
          bool TWREC = false>
RealKernel real_entry() {
    using SH = SingleShape<LOG2H, LOG2E, WGT>;
    RealKernel k{};
    k.real_bytes = sizeof(R);
    k.log2h = LOG2H;
    k.log2e = SH::SC::LE;
    k.wgt = WGT;
    k.c2r = C2R;
    k.split = SPLIT;
    k.twreg = TWREG;
    k.stg = STG;
    k.twrec = TWREC;
    k.fn = &launch_real_single<R, LOG2H, LOG2E, WGT, C2R, SPLIT, TWREG, STG, TWREC>;
    k.kernel = reinterpret_cast<const void*>(&k_real_single<R, LOG2H, LOG2E, WGT, C2R, SPLIT, TWREG, STG, TWREC>);
    k.eng = engine_info<typename SH::SC, TWREC, sizeof(R) == 4 ? 2 : 1>();
    k.threads = SH::THREADS;
    k.per_wg = SH::G;
    k.lds_bytes = real_lds<R, LOG2H, LOG2E, WGT, STG>() * sizeof(cplx_t<R>);
    return k;
}

}  // namespace fftk
