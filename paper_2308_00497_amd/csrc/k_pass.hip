// Instances of the multi-pass kernel: sub-FFT length L = 2^6 .. 2^12 with a
// few column-tile widths C each, in the four layout combinations a plan uses
// (first pass: user layout -> interleaved workspace; later passes:
// interleaved -> interleaved or -> user layout).
#include "kernels.hpp"

namespace fftk {

// first pass: interleaved in (plain or re/im-swapped) or split in, interleaved
// workspace out; later passes: interleaved workspace in, interleaved (plain or
// swapped) or split out
#define FFT_P(l, c)                                                                                        \
    pass_entry<float, l, 4, c, true, false, false, false, false>(),                                        \
        pass_entry<float, l, 4, c, true, false, false, true, false>(),                                     \
        pass_entry<float, l, 4, c, true, true, false, false, false>(),                                     \
        pass_entry<float, l, 4, c, false, false, false, false, false>(),                                   \
        pass_entry<float, l, 4, c, false, false, false, false, true>(),                                    \
        pass_entry<float, l, 4, c, false, false, true, false, false>()

static const PassKernel kPass[] = {
    FFT_P(6, 4), FFT_P(6, 6), FFT_P(6, 7),
    FFT_P(7, 4), FFT_P(7, 5), FFT_P(7, 6), FFT_P(7, 7),
    FFT_P(8, 3), FFT_P(8, 4), FFT_P(8, 5), FFT_P(8, 6),
    FFT_P(9, 3), FFT_P(9, 4),
    FFT_P(10, 2), FFT_P(10, 3),
    FFT_P(11, 2),
    FFT_P(12, 1), FFT_P(12, 2),
    // the column passes of multi-dimensional plans: later-pass variants whose
    // input is the caller's layout (split arrays, or re/im swapped), and a
    // 32-point pass with 256-column tiles
#define FFT_PC(l, c)                                                                                       \
    pass_entry<float, l, 4, c, false, true, false, false, false>(),                                        \
        pass_entry<float, l, 4, c, false, false, false, true, false>()
#define FFT_PN(l, c)                                                                                       \
    pass_entry<float, l, 4, c, false, false, false, false, false>(),                                       \
        pass_entry<float, l, 4, c, false, false, false, false, true>(),                                    \
        pass_entry<float, l, 4, c, false, false, true, false, false>()
    FFT_PC(6, 7), FFT_PN(5, 8), FFT_PC(5, 8),
#undef FFT_PC
#undef FFT_PN
};

#undef FFT_P

const PassKernel* pass_kernels(int* count) {
    *count = static_cast<int>(sizeof(kPass) / sizeof(kPass[0]));
    return kPass;
}

}  // namespace fftk
