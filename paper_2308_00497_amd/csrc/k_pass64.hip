// FP64 instances of the multi-pass kernel.  LDS holds C columns of L FP64
// complex elements (16 bytes each), so the tiles are half the width of the
// FP32 ones for the same LDS: C = 8 FP64 columns give the same 128-byte runs
// as 16 FP32 columns.
#include "kernels.hpp"

namespace fftk {

#define FFT_PD(l, c)                                                                                       \
    pass_entry<double, l, 4, c, true, false, false, false, false>(),                                       \
        pass_entry<double, l, 4, c, true, false, false, true, false>(),                                    \
        pass_entry<double, l, 4, c, true, true, false, false, false>(),                                    \
        pass_entry<double, l, 4, c, false, false, false, false, false>(),                                  \
        pass_entry<double, l, 4, c, false, false, false, false, true>(),                                   \
        pass_entry<double, l, 4, c, false, false, true, false, false>()

static const PassKernel kPass64[] = {
    FFT_PD(6, 4), FFT_PD(6, 6), FFT_PD(6, 7),
    FFT_PD(7, 4), FFT_PD(7, 5), FFT_PD(7, 6),
    FFT_PD(8, 3), FFT_PD(8, 4), FFT_PD(8, 5),
    FFT_PD(9, 3), FFT_PD(9, 4),
    FFT_PD(10, 2), FFT_PD(10, 3),
    FFT_PD(11, 1), FFT_PD(11, 2),
    FFT_PD(12, 1),
    // the column passes of multi-dimensional plans (see the FP32 list)
#define FFT_PC(l, c)                                                                                       \
    pass_entry<double, l, 4, c, false, true, false, false, false>(),                                       \
        pass_entry<double, l, 4, c, false, false, false, true, false>()
#define FFT_PN(l, c)                                                                                       \
    pass_entry<double, l, 4, c, false, false, false, false, false>(),                                      \
        pass_entry<double, l, 4, c, false, false, false, false, true>(),                                   \
        pass_entry<double, l, 4, c, false, false, true, false, false>()
    FFT_PC(6, 6), FFT_PN(5, 7), FFT_PC(5, 7),
#undef FFT_PC
#undef FFT_PN
};

#undef FFT_PD

const PassKernel* pass_kernels64(int* count) {
    *count = static_cast<int>(sizeof(kPass64) / sizeof(kPass64[0]));
    return kPass64;
}

}  // namespace fftk
