// FP64 instances of the single-pass kernel (the precision of the paper's
// evaluation, section 4): every N = 2^1 .. 2^13 (2^14 FP64 elements would not
// fit the 160 KB of LDS), both layouts, both directions.  Twice the register
// cost per element of the FP32 instances, so 8 elements per thread is offered
// everywhere and the twiddles-in-registers variants only where they fit.
#include "kernels.hpp"

namespace fftk {

// interleaved forward, interleaved inverse (re/im swapped), split
#define FFT_D1(n, e, w, r)                                                                             \
    single_entry<double, n, e, w, false, false, r>(), single_entry<double, n, e, w, false, true, r>(), \
        single_entry<double, n, e, w, true, false, r>()
#define FFT_D(n, e, w) FFT_D1(n, e, w, false), FFT_D1(n, e, w, true)

static const SingleKernel kSingle64[] = {
    FFT_D(1, 4, 64), FFT_D(1, 4, 256),
    FFT_D(2, 4, 64), FFT_D(2, 4, 256),
    FFT_D(3, 4, 64), FFT_D(3, 4, 256),
    FFT_D(4, 4, 64), FFT_D(4, 4, 256),
    FFT_D(4, 3, 64), FFT_D(4, 3, 256),
    FFT_D(5, 4, 64), FFT_D(5, 4, 256), FFT_D(5, 3, 64), FFT_D(5, 3, 256),
    FFT_D(6, 4, 64), FFT_D(6, 4, 256), FFT_D(6, 3, 64), FFT_D(6, 3, 256),
    FFT_D(7, 4, 64), FFT_D(7, 4, 256), FFT_D(7, 3, 64), FFT_D(7, 3, 256),
    FFT_D(8, 4, 64), FFT_D(8, 4, 256), FFT_D(8, 3, 64), FFT_D(8, 3, 256),
    FFT_D(9, 4, 256), FFT_D(9, 3, 64), FFT_D(9, 3, 256),
    FFT_D(10, 4, 256), FFT_D(10, 3, 256),
    FFT_D(11, 4, 256), FFT_D(11, 3, 256),
    FFT_D1(12, 4, 256, false), FFT_D(12, 3, 256),
    FFT_D1(13, 4, 256, false), FFT_D1(13, 3, 256, false),
    // prefetching variants where LDS allows one or two workgroups per CU
    single_entry<double, 13, 4, 256, false, false, false, true>(), single_entry<double, 13, 4, 256, false, true, false, true>(),
    single_entry<double, 13, 4, 256, true, false, false, true>(),
    single_entry<double, 12, 3, 256, false, false, true, true>(), single_entry<double, 12, 3, 256, false, true, true, true>(),
    single_entry<double, 12, 3, 256, true, false, true, true>(),
    // exchanges one real part at a time: half the LDS, twice the workgroups
    // per CU where LDS limits them
#define FFT_DH(n, e, r)                                                                                     \
    single_entry<double, n, e, 256, false, false, r, false, false, true>(),                                 \
        single_entry<double, n, e, 256, false, true, r, false, false, true>(),                              \
        single_entry<double, n, e, 256, true, false, r, false, false, true>()
    FFT_DH(12, 3, true), FFT_DH(12, 3, false), FFT_DH(12, 4, false), FFT_DH(13, 4, false), FFT_DH(13, 3, false),
#undef FFT_DH
    // stage twiddles from one FP64 table value per butterfly and its powers
#define FFT_DR(n, e, h)                                                                                     \
    single_entry<double, n, e, 256, false, false, false, false, false, h, true>(),                          \
        single_entry<double, n, e, 256, false, true, false, false, false, h, true>(),                       \
        single_entry<double, n, e, 256, true, false, false, false, false, h, true>()
    FFT_DR(13, 4, true), FFT_DR(13, 3, true), FFT_DR(12, 3, true),
#undef FFT_DR
};

#undef FFT_D
#undef FFT_D1

const SingleKernel* single_kernels64(int* count) {
    *count = static_cast<int>(sizeof(kSingle64) / sizeof(kSingle64[0]));
    return kSingle64;
}

}  // namespace fftk
