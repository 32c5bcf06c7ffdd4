// Host-side plan logic: decompositions, their text form and the plan object.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fft.h"
#include "registry.hpp"

namespace fftk {

// How one transform size is computed.
//   copy     N = 1
//   single   one persistent single-pass kernel (E = 2^log2e elements per
//            thread, workgroups of at least `wgt` threads, gmul workgroups per
//            compute unit, stage twiddles in registers when twreg)
//   multi    P passes of sub-FFT lengths 2^log2l[p] with 2^log2c[p] columns per
//            workgroup, sum of log2l = log2 N (Stockham radix-L passes)
//   ops      the per-operator baseline: Table 1's operators one kernel each,
//            radix 2^log2r (interleaved layout only; never chosen by default)
struct Decomp {
    enum Kind { COPY = 0, SINGLE = 1, MULTI = 2, OPS = 3 } kind = COPY;
    int log2r = 4;
    int log2e = 4;
    int wgt = 256;
    int gmul = 2;
    bool twreg = true;
    bool pf = false;  // single: the next transform's loads issued before the current one's stages
    bool stg = false; // single: contiguous loads/stores staged through LDS (small transforms)
    bool half = false; // single: stage exchanges one real part at a time (half the LDS)
    bool twrec = false; // single: stage twiddles from one FP64 value per butterfly ("r2")
    std::vector<int> log2l;
    std::vector<int> log2c;
    std::vector<int> inplace;  // per pass: 1 = writes over its own input ("i" suffix)
    bool in_place(size_t p) const { return p < inplace.size() && inplace[p] != 0; }

    std::string str() const;  // "copy" | "single:e4:w256:g2:r1[:p1|:s1|:h1]" | "multi:8c4,8c4i,8c4" | "ops:r4"
    static bool parse(const std::string& s, Decomp* out);
    bool operator==(const Decomp& o) const { return str() == o.str(); }
};

// Largest size, and the default (untuned) choice.  `rb` is the bytes of one
// real number: 4 (FP32) or 8 (FP64); the multi-pass choice depends on the
// layout of the caller's arrays.
constexpr int kMaxLog2N = 24;
// `batch` (0: unknown) refines the choice where a small batch measured
// faster with another shape.
Decomp default_decomposition(int log2n, int rb, fft_layout layout = FFT_LAYOUT_INTERLEAVED, int64_t batch = 0);

// every decomposition the library can run for log2n (autotuner candidates)
std::vector<Decomp> candidate_decompositions(int log2n, fft_layout layout, int rb);

// kernel lookup; nullptr when no such instance was compiled
const SingleKernel* find_single(int rb, int log2n, int log2e, int wgt, bool split, bool swap, bool twreg,
                                bool pf = false, bool stg = false, bool half = false, bool twrec = false);
const PassKernel* find_pass(int rb, int log2l, int log2c, bool first, bool split_in, bool split_out, bool swap_in,
                            bool swap_out);

// kernel of pass p (of P) for a layout and direction: the inverse swaps re/im
// (interleaved data in the kernel, split data by exchanging the pointers)
const PassKernel* pass_kernel_for(int rb, int log2l, int log2c, size_t p, size_t P, bool split, bool inverse);
const SingleKernel* single_kernel_for(int rb, int log2n, const Decomp& d, bool split, bool inverse);

// true when every kernel the decomposition needs exists for this layout
bool decomposition_available(const Decomp& d, int log2n, fft_layout layout, int rb);

// Real-input plans (R2C, or C2R when c2r) of N = 2^log2n real points run on
// the half length H = N/2: "copy" stands for H = 1 (the pre/post pass alone),
// "single:..." for the fused single-pass kernel, "multi:..." for the
// half-length pass chain plus one pre/post pass.  N = 1 has no decomposition.
const RealKernel* find_real(int rb, int log2h, int log2e, int wgt, bool c2r, bool split, bool twreg,
                            bool stg = false, bool twrec = false);
Decomp default_real_decomposition(int log2n, int rb);
bool real_decomposition_available(const Decomp& d, int log2n, fft_layout layout, int rb, bool c2r);

// Column kernel of a multi-dimensional plan for a strided axis of 2^log2l
// points at stride 2^log2s: the widest compiled column tile that fits the
// stride; nullptr if the axis is longer than 2^12 points.
const StridedKernel* strided_kernel_for(int rb, int log2l, int log2s, bool split, bool swap);
constexpr int kMaxStridedLog2 = 12;

// bytes of one real number for a precision (0 if invalid)
inline int real_bytes_of(fft_precision p) { return p == FFT_PRECISION_FP32 ? 4 : (p == FFT_PRECISION_FP64 ? 8 : 0); }

// radices (log2) of the per-operator baseline for N = 2^log2n, outermost first:
// radix 2^log2r at every level, the remainder innermost
std::vector<int> ops_radices(int log2n, int log2r);

int ilog2_exact(int64_t v);  // log2 of a power of two, -1 otherwise

}  // namespace fftk
