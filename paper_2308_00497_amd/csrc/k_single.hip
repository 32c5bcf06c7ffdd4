// Instances of the single-pass kernel: every N = 2^1 .. 2^14, both layouts,
// both directions, stage twiddles in registers or read from the table, 8, 16
// or 32 elements per thread, 64- or 256-thread workgroups for the sizes where
// several transforms share a workgroup.
#include "kernels.hpp"

namespace fftk {

// interleaved forward, interleaved inverse (re/im swapped), split (the inverse
// swaps the caller's pointers instead)
#define FFT_S1(n, e, w, r)                                                                          \
    single_entry<float, n, e, w, false, false, r>(), single_entry<float, n, e, w, false, true, r>(),   \
        single_entry<float, n, e, w, true, false, r>()
#define FFT_S(n, e, w) FFT_S1(n, e, w, false), FFT_S1(n, e, w, true)

static const SingleKernel kSingle[] = {
    // N <= 8: one thread per transform (E = N)
    FFT_S(1, 4, 64), FFT_S(1, 4, 256),
    FFT_S(2, 4, 64), FFT_S(2, 4, 256),
    FFT_S(3, 4, 64), FFT_S(3, 4, 256),
    FFT_S(4, 4, 64), FFT_S(4, 4, 256),
    FFT_S(4, 3, 64), FFT_S(4, 3, 256),
    FFT_S(5, 4, 64), FFT_S(5, 4, 256), FFT_S(5, 3, 64), FFT_S(5, 3, 256),
    FFT_S(6, 4, 64), FFT_S(6, 4, 256), FFT_S(6, 3, 64), FFT_S(6, 3, 256),
    FFT_S(7, 4, 64), FFT_S(7, 4, 256), FFT_S(7, 3, 64), FFT_S(7, 3, 256),
    FFT_S(8, 4, 64), FFT_S(8, 4, 256), FFT_S(8, 3, 64), FFT_S(8, 3, 256),
    FFT_S(9, 4, 64), FFT_S(9, 4, 256), FFT_S(9, 3, 64), FFT_S(9, 3, 256),
    FFT_S(10, 4, 64), FFT_S(10, 4, 256), FFT_S(10, 3, 256),
    FFT_S(11, 4, 256), FFT_S(11, 3, 256),
    FFT_S(12, 4, 256), FFT_S(12, 3, 256),
    FFT_S(13, 4, 256), FFT_S(13, 3, 256),
    FFT_S1(14, 4, 256, false),
    // one workgroup per CU at 2^14 (LDS): prefetching the next transform pays there
    single_entry<float, 14, 4, 256, false, false, false, true>(), single_entry<float, 14, 4, 256, false, true, false, true>(),
    single_entry<float, 14, 4, 256, true, false, false, true>(),
    single_entry<float, 13, 4, 256, false, false, true, true>(), single_entry<float, 13, 4, 256, false, true, true, true>(),
    single_entry<float, 13, 4, 256, true, false, true, true>(),
    // exchanges one real part at a time: half the LDS, so more workgroups per
    // CU at the sizes LDS limits (2^12: 4 -> 8, 2^13: 2 -> 4 by LDS)
#define FFT_SH(n, e, r)                                                                                     \
    single_entry<float, n, e, 256, false, false, r, false, false, true>(),                                  \
        single_entry<float, n, e, 256, false, true, r, false, false, true>(),                               \
        single_entry<float, n, e, 256, true, false, r, false, false, true>()
    FFT_SH(12, 4, true), FFT_SH(13, 4, true), FFT_SH(13, 4, false), FFT_SH(14, 4, false),
    // 32 points per thread (radix-32 stages): three stages and two exchanges
    // at 2^13 and 2^14 instead of four and three, half the threads per
    // transform; stage twiddles from the table (registers for them would spill)
    FFT_SH(13, 5, false), FFT_SH(14, 5, false),
#undef FFT_SH
    // stage twiddles from one FP64 value per butterfly (the sizes whose tables
    // do not fit in registers): half-width exchanges at 2^14, and 2^13
#define FFT_SR(n, e, h)                                                                                      \
    single_entry<float, n, e, 256, false, false, false, false, false, h, true>(),                            \
        single_entry<float, n, e, 256, false, true, false, false, false, h, true>(),                         \
        single_entry<float, n, e, 256, true, false, false, false, false, h, true>()
    FFT_SR(14, 4, true), FFT_SR(14, 5, true), FFT_SR(13, 4, false), FFT_SR(13, 5, true),
#undef FFT_SR
    // small transforms (each inside one wavefront): contiguous loads and
    // stores staged through LDS
#define FFT_ST(n, e)                                                                                        \
    single_entry<float, n, e, 256, false, false, true, false, true>(),                                      \
        single_entry<float, n, e, 256, false, true, true, false, true>(),                                   \
        single_entry<float, n, e, 256, true, false, true, false, true>()
    FFT_ST(1, 4), FFT_ST(2, 4), FFT_ST(3, 4),
    FFT_ST(4, 4), FFT_ST(4, 3), FFT_ST(5, 4), FFT_ST(5, 3), FFT_ST(6, 4), FFT_ST(6, 3),
    FFT_ST(7, 4), FFT_ST(7, 3), FFT_ST(8, 4), FFT_ST(8, 3), FFT_ST(9, 4), FFT_ST(9, 3),
#undef FFT_ST
};

#undef FFT_S
#undef FFT_S1

const SingleKernel* single_kernels(int* count) {
    *count = static_cast<int>(sizeof(kSingle) / sizeof(kSingle[0]));
    return kSingle;
}

}  // namespace fftk
