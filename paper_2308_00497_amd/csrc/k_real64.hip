// FP64 instances of the single-pass R2C/C2R kernel (half lengths up to 2^13).
#include "real.hpp"

namespace fftk {

#define FFT_RD1(h, e, r)                                                                                       \
    real_entry<double, h, e, 256, false, false, r>(), real_entry<double, h, e, 256, false, true, r>(),        \
        real_entry<double, h, e, 256, true, false, r>(), real_entry<double, h, e, 256, true, true, r>()
#define FFT_RD(h, e) FFT_RD1(h, e, false), FFT_RD1(h, e, true)

static const RealKernel kReal64[] = {
    FFT_RD(1, 4), FFT_RD(2, 4), FFT_RD(3, 4),
    FFT_RD(4, 3), FFT_RD(5, 3), FFT_RD(6, 3), FFT_RD(7, 3), FFT_RD(8, 3), FFT_RD(9, 3), FFT_RD(10, 3),
    FFT_RD(11, 3), FFT_RD1(12, 3, false), FFT_RD1(13, 3, false),
    FFT_RD(4, 4), FFT_RD(5, 4), FFT_RD(6, 4), FFT_RD(7, 4), FFT_RD(8, 4), FFT_RD1(9, 4, false),
    FFT_RD1(10, 4, false), FFT_RD1(11, 4, false), FFT_RD1(12, 4, false), FFT_RD1(13, 4, false),
    // the largest half lengths: stage twiddles as one FP64 value per butterfly
#define FFT_RR(h, e)                                                                                          \
    real_entry<double, h, e, 256, false, false, false, false, true>(),                                        \
        real_entry<double, h, e, 256, false, true, false, false, true>(),                                     \
        real_entry<double, h, e, 256, true, false, false, false, true>(),                                     \
        real_entry<double, h, e, 256, true, true, false, false, true>()
    FFT_RR(12, 3), FFT_RR(12, 4), FFT_RR(13, 3), FFT_RR(13, 4),
#undef FFT_RR
    // short rows (whole rows inside one wavefront): staged through LDS
#define FFT_RT(h, e)                                                                                          \
    real_entry<double, h, e, 256, false, false, true, true>(), real_entry<double, h, e, 256, false, true, true, true>(), \
        real_entry<double, h, e, 256, true, false, true, true>(), real_entry<double, h, e, 256, true, true, true, true>()
    FFT_RT(1, 4), FFT_RT(2, 4), FFT_RT(3, 4), FFT_RT(4, 4), FFT_RT(4, 3), FFT_RT(5, 4), FFT_RT(5, 3),
    FFT_RT(6, 4), FFT_RT(6, 3), FFT_RT(7, 4), FFT_RT(7, 3),
#undef FFT_RT
};

#undef FFT_RD
#undef FFT_RD1

const RealKernel* real_kernels64(int* count) {
    *count = static_cast<int>(sizeof(kReal64) / sizeof(kReal64[0]));
    return kReal64;
}

}  // namespace fftk
