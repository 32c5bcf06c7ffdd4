// Instances of the strided-axis kernels of multi-dimensional transforms:
// columns of 2..16 points (one thread each) and 32..4096 points (column
// tiles; C columns per workgroup, bounded by LDS), FP32 and FP64,
// interleaved (plain and re/im-swapped) and split.
#include "nd.hpp"

namespace fftk {

#define ND_S(R, n) strided_small_entry<R, n, false, false>(), strided_small_entry<R, n, false, true>(), \
                   strided_small_entry<R, n, true, false>()
#define ND_T(R, l, c) strided_entry<R, l, c, false, false>(), strided_entry<R, l, c, false, true>(), \
                      strided_entry<R, l, c, true, false>()

static const StridedKernel kStrided[] = {
    ND_S(float, 1), ND_S(float, 2), ND_S(float, 3), ND_S(float, 4),
    ND_T(float, 5, 0), ND_T(float, 5, 2), ND_T(float, 5, 4), ND_T(float, 5, 5),
    ND_T(float, 6, 0), ND_T(float, 6, 2), ND_T(float, 6, 4), ND_T(float, 6, 5),
    ND_T(float, 7, 0), ND_T(float, 7, 2), ND_T(float, 7, 4), ND_T(float, 7, 5),
    ND_T(float, 8, 0), ND_T(float, 8, 2), ND_T(float, 8, 4), ND_T(float, 8, 5),
    ND_T(float, 9, 0), ND_T(float, 9, 2), ND_T(float, 9, 4),
    ND_T(float, 10, 0), ND_T(float, 10, 2), ND_T(float, 10, 3),
    ND_T(float, 11, 0), ND_T(float, 11, 2),
    ND_T(float, 12, 0), ND_T(float, 12, 1),
    ND_S(double, 1), ND_S(double, 2), ND_S(double, 3), ND_S(double, 4),
    ND_T(double, 5, 0), ND_T(double, 5, 2), ND_T(double, 5, 3),
    ND_T(double, 6, 0), ND_T(double, 6, 2), ND_T(double, 6, 3),
    ND_T(double, 7, 0), ND_T(double, 7, 2), ND_T(double, 7, 3),
    ND_T(double, 8, 0), ND_T(double, 8, 2), ND_T(double, 8, 3),
    ND_T(double, 9, 0), ND_T(double, 9, 2), ND_T(double, 9, 3),
    ND_T(double, 10, 0), ND_T(double, 10, 2),
    ND_T(double, 11, 0), ND_T(double, 11, 1),
    ND_T(double, 12, 0),
};

#undef ND_S
#undef ND_T

const StridedKernel* strided_kernels(int* count) {
    *count = static_cast<int>(sizeof(kStrided) / sizeof(kStrided[0]));
    return kStrided;
}

}  // namespace fftk
