// Strided-axis transforms for batched 2D/3D FFTs.  A d-dimensional DFT
// factorises over its axes (the exponential of a sum is a product), so a
// [batch][n_0]..[n_(d-1)] transform is the contiguous 1D transform along the
// last axis followed, for every other axis k, by DFT_(n_k) down the columns
// of stride s_k = n_(k+1) ... n_(d-1), in place.  A column pass is the pass
// kernel's tile (C consecutive columns, a radix-n_k Stockham sub-FFT through
// LDS) without the pass twiddles; columns of 16 points or fewer take one
// thread each with the DFT in registers.
#pragma once

#include "kernels.hpp"

namespace fftk {

// DFT_(2^LOG2L) down every column of stride 2^log2s, B column blocks
// (tiles = B * s / C), in place or out of place; the inverse swaps re/im of
// interleaved data in the kernel (split data: the caller swaps pointers).
template <class R, int LOG2L, int LOG2C, bool SPLIT, bool SWAP>
__global__ void __launch_bounds__((PassShape<LOG2L, 4, LOG2C>::THREADS), (pass_waves<R, LOG2L, 4, LOG2C, false>()))
k_strided(const R* ia, const R* ib, R* oa, R* ob, const cplx_t<R>* __restrict__ tw, int log2s, int64_t tiles) {
    using V = cplx_t<R>;
    using SH = PassShape<LOG2L, 4, LOG2C>;
    using SC = typename SH::SC;
    using ENG = Engine<SC, SH::C, SH::GS, true, true, false>;
    constexpr bool REGTW = pass_regtw<R, LOG2L, 4, LOG2C>();  // else the recurrence table
    __shared__ V lds[pass_lds<R, LOG2L, 4, LOG2C, false>()];
    const int tid = threadIdx.x;
    TwReg<SC, V> twr(tw);
    if constexpr (REGTW) twr.template init_engine<ENG>(tid);
    const int log2tpb = log2s - LOG2C;  // tiles per column block
    for (int64_t lin = blockIdx.x; lin < tiles; lin += gridDim.x) {
        int tidl = tid;
        asm volatile("" : "+v"(tidl));
        const int64_t b = lin >> log2tpb;
        const int64_t j0 = (lin & ((int64_t(1) << log2tpb) - 1)) << LOG2C;
        const int64_t tbase = b << (log2s + LOG2L);
        if constexpr (REGTW)
            pass_tile<LOG2L, 4, LOG2C, false, SPLIT, SPLIT, SWAP, SWAP, TwReg<SC, V>, R, false, 3, 0>(
                ia, ib, oa, ob, twr, nullptr, nullptr, log2s + LOG2L, log2s, 0, tbase, j0, lds, tidl, 0);
        else
            pass_tile<LOG2L, 4, LOG2C, false, SPLIT, SPLIT, SWAP, SWAP, TwRec<SC, V>, R, false, 3, 0>(
                ia, ib, oa, ob, TwRec<SC, V>(reinterpret_cast<const double2*>(tw)), nullptr, nullptr, log2s + LOG2L,
                log2s, 0, tbase, j0, lds, tidl, 0);
    }
}

// columns of 2^LOG2N <= 16 points: one thread per column
template <class R, int LOG2N, bool SPLIT, bool SWAP>
__global__ void __launch_bounds__(256) k_strided_small(const R* ia, const R* ib, R* oa, R* ob, int log2s,
                                                       int64_t cols) {
    using V = cplx_t<R>;
    constexpr int N = 1 << LOG2N;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < cols; t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = t >> log2s, c = t & ((int64_t(1) << log2s) - 1);
        const int64_t base = (b << (log2s + LOG2N)) + c;
        V u[N];
#pragma unroll
        for (int r = 0; r < N; ++r) u[r] = swap_if<SWAP>(gload<SPLIT>(ia, ib, base + (int64_t(r) << log2s)));
        Dft<N>::run(u);
#pragma unroll
        for (int r = 0; r < N; ++r) gstore<SPLIT>(oa, ob, base + (int64_t(r) << log2s), swap_if<SWAP>(u[r]));
    }
}

template <class R, int LOG2L, int LOG2C, bool SPLIT, bool SWAP>
hipError_t launch_strided(const void* ia, const void* ib, void* oa, void* ob, const void* tw, int log2s,
                          int64_t blocks_b, int grid, hipStream_t s) {
    using SH = PassShape<LOG2L, 4, LOG2C>;
    if (log2s < LOG2C) return hipErrorInvalidConfiguration;
    const int64_t tiles = blocks_b << (log2s - LOG2C);
    const int64_t blocks = tiles < grid ? tiles : grid;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_strided<R, LOG2L, LOG2C, SPLIT, SWAP>), dim3(static_cast<unsigned>(blocks)),
                       dim3(SH::THREADS), 0, s, static_cast<const R*>(ia), static_cast<const R*>(ib),
                       static_cast<R*>(oa), static_cast<R*>(ob), static_cast<const cplx_t<R>*>(tw), log2s, tiles);
    return hipGetLastError();
}

template <class R, int LOG2N, bool SPLIT, bool SWAP>
hipError_t launch_strided_small(const void* ia, const void* ib, void* oa, void* ob, const void*, int log2s,
                                int64_t blocks_b, int, hipStream_t s) {
    const int64_t cols = blocks_b << log2s;
    int64_t g = (cols + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL((k_strided_small<R, LOG2N, SPLIT, SWAP>), dim3(static_cast<unsigned>(g < 1 ? 1 : g)), dim3(256),
                       0, s, static_cast<const R*>(ia), static_cast<const R*>(ib), static_cast<R*>(oa),
                       static_cast<R*>(ob), log2s, cols);
    return hipGetLastError();
}

template <class R, int LOG2L, int LOG2C, bool SPLIT, bool SWAP>
StridedKernel strided_entry() {
    using SH = PassShape<LOG2L, 4, LOG2C>;
    StridedKernel k{};
    k.real_bytes = sizeof(R);
    k.log2l = LOG2L;
    k.log2c = LOG2C;
    k.split = SPLIT;
    k.swap = SWAP;
    k.fn = &launch_strided<R, LOG2L, LOG2C, SPLIT, SWAP>;
    k.kernel = reinterpret_cast<const void*>(&k_strided<R, LOG2L, LOG2C, SPLIT, SWAP>);
    k.eng = engine_info<typename SH::SC, !pass_regtw<R, LOG2L, 4, LOG2C>(), sizeof(R) == 4 ? 2 : 1>();
    k.threads = SH::THREADS;
    k.lds_bytes = pass_lds<R, LOG2L, 4, LOG2C, false>() * sizeof(cplx_t<R>);
    return k;
}

template <class R, int LOG2N, bool SPLIT, bool SWAP>
StridedKernel strided_small_entry() {
    StridedKernel k{};
    k.real_bytes = sizeof(R);
    k.log2l = LOG2N;
    k.log2c = 0;
    k.split = SPLIT;
    k.swap = SWAP;
    k.fn = &launch_strided_small<R, LOG2N, SPLIT, SWAP>;
    k.kernel = nullptr;  // elementwise grid, no occupancy query
    k.eng = EngineInfo{};
    k.threads = 256;
    k.lds_bytes = 0;
    return k;
}

}  // namespace fftk
