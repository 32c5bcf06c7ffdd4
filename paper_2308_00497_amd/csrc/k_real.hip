// FP32 instances of the single-pass R2C/C2R kernel, and the passes over HBM
// that surround the multi-pass half-length transform for large N (FP32 and
// FP64), plus the N = 1 case.
#include "real.hpp"

namespace fftk {

// R2C after the half-length transform: one thread per pair (k, H - k),
// k = 0 .. H/2, so each Z value is read once; w_N^k from the two FP64 tables
// (M = N = 2H), rounded once.
template <class R, bool SPLIT>
__global__ void __launch_bounds__(256) k_r2c_post(const R* __restrict__ z, R* oa, R* ob, const double2* __restrict__ ta,
                                                  const double2* __restrict__ tb, int hbits, int log2h,
                                                  int64_t batch, R iscale) {
    using V = cplx_t<R>;
    const int64_t H = int64_t(1) << log2h;
    const int64_t pairs = H / 2 + 1;
    const int64_t total = pairs * batch;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = i / pairs, k = i - b * pairs;
        const int64_t km = (H - k) & (H - 1);
        const V* zr = reinterpret_cast<const V*>(z) + b * H;
        const V a = zr[k], mir = zr[km];
        const V w = twiddle_2level<V>(ta, tb, k, hbits);
        V ev, wo;
        r2c_parts(a, mir, w, ev, wo);
        const int64_t o = b * (H + 1);
        if (k == 0) {
            gstore<SPLIT>(oa, ob, o, c_add(ev, wo));
            gstore<SPLIT>(oa, ob, o + H, cmk(a.x - a.y, R(0)));
        } else {
            // interior bins k and H - k (scaled for the adjoint of C2R)
            gstore<SPLIT>(oa, ob, o + k, c_scale(c_add(ev, wo), iscale));
            if (H - k != k) {
                const V d = c_sub(ev, wo);
                gstore<SPLIT>(oa, ob, o + H - k, c_scale(cmk(d.x, -d.y), iscale));
            }
        }
    }
}

// C2R before the half-length inverse transform: Z'[k] and Z'[H - k] from the
// pair X[k], X[H - k] (w_N^(H-k) = -conj(w_N^k)); interleaved output.
template <class R, bool SPLIT>
__global__ void __launch_bounds__(256) k_c2r_pre(const R* ia, const R* ib, R* __restrict__ z,
                                                 const double2* __restrict__ ta, const double2* __restrict__ tb,
                                                 int hbits, int log2h, int64_t batch, R iscale) {
    using V = cplx_t<R>;
    const int64_t H = int64_t(1) << log2h;
    const int64_t pairs = H / 2 + 1;
    const int64_t total = pairs * batch;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = i / pairs, k = i - b * pairs;
        const int64_t o = b * (H + 1);
        V* zr = reinterpret_cast<V*>(z) + b * H;
        const V w = twiddle_2level<V>(ta, tb, k, hbits);
        const V a = gload<SPLIT>(ia, ib, o + k);
        const V mir = gload<SPLIT>(ia, ib, o + H - k);
        if (k == 0) {
            zr[0] = c2r_point(cmk(a.x, R(0)), cmk(mir.x, R(0)), w);
        } else {
            // interior bins only (scaled for the adjoint of R2C)
            zr[k] = c_scale(c2r_point(a, mir, w), iscale);
            if (H - k != k) zr[H - k] = c_scale(c2r_point(mir, a, cmk(-w.x, w.y)), iscale);
        }
    }
}

// N = 1: X[0] = x[0] (R2C), x[0] = Re X[0] (C2R)
template <class R, bool C2R, bool SPLIT>
__global__ void __launch_bounds__(256) k_real1(const R* ia, const R* ib, R* oa, R* ob, int64_t batch) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < batch; i += int64_t(gridDim.x) * blockDim.x) {
        if constexpr (C2R) oa[i] = gload<SPLIT>(ia, ib, i).x;
        else gstore<SPLIT>(oa, ob, i, cmk(ia[i], R(0)));
    }
}

// dst[i] = w_M^i for i < count, from sincospi with the exact argument 2i/M,
// rounded once to V's precision
template <class V>
__global__ void k_gen_pow_round(V* dst, int log2M, int64_t count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t m = i & ((int64_t(1) << log2M) - 1);
    double s, c;
    sincospi(ldexp(static_cast<double>(m), 1 - log2M), &s, &c);
    dst[i] = cvt_tw<V>(make_double2(c, -s));
}

static unsigned elementwise_blocks(int64_t items) {
    int64_t b = (items + 255) / 256;
    if (b > 65536) b = 65536;  // grid-stride beyond this
    return static_cast<unsigned>(b < 1 ? 1 : b);
}

hipError_t launch_r2c_post(int rb, bool split, const void* z, void* oa, void* ob, const double2* ta,
                           const double2* tb, int hbits, int log2h, int64_t batch, double iscale, hipStream_t s) {
    const unsigned blocks = elementwise_blocks(((int64_t(1) << log2h) / 2 + 1) * batch);
#define FFT_POST(R, S)                                                                                          \
    hipLaunchKernelGGL((k_r2c_post<R, S>), dim3(blocks), dim3(256), 0, s, static_cast<const R*>(z),             \
                       static_cast<R*>(oa), static_cast<R*>(ob), ta, tb, hbits, log2h, batch, static_cast<R>(iscale))
    if (rb == 8) {
        if (split) FFT_POST(double, true);
        else FFT_POST(double, false);
    } else {
        if (split) FFT_POST(float, true);
        else FFT_POST(float, false);
    }
#undef FFT_POST
    return hipGetLastError();
}

hipError_t launch_c2r_pre(int rb, bool split, const void* ia, const void* ib, void* z, const double2* ta,
                          const double2* tb, int hbits, int log2h, int64_t batch, double iscale, hipStream_t s) {
    const unsigned blocks = elementwise_blocks(((int64_t(1) << log2h) / 2 + 1) * batch);
#define FFT_PRE(R, S)                                                                                           \
    hipLaunchKernelGGL((k_c2r_pre<R, S>), dim3(blocks), dim3(256), 0, s, static_cast<const R*>(ia),             \
                       static_cast<const R*>(ib), static_cast<R*>(z), ta, tb, hbits, log2h, batch, static_cast<R>(iscale))
    if (rb == 8) {
        if (split) FFT_PRE(double, true);
        else FFT_PRE(double, false);
    } else {
        if (split) FFT_PRE(float, true);
        else FFT_PRE(float, false);
    }
#undef FFT_PRE
    return hipGetLastError();
}

hipError_t launch_real1(int rb, bool c2r, bool split, const void* ia, const void* ib, void* oa, void* ob,
                        int64_t batch, hipStream_t s) {
    const unsigned blocks = elementwise_blocks(batch);
#define FFT_R1(R, C, S)                                                                                         \
    hipLaunchKernelGGL((k_real1<R, C, S>), dim3(blocks), dim3(256), 0, s, static_cast<const R*>(ia),            \
                       static_cast<const R*>(ib), static_cast<R*>(oa), static_cast<R*>(ob), batch)
    if (rb == 8) {
        if (c2r) {
            if (split) FFT_R1(double, true, true);
            else FFT_R1(double, true, false);
        } else {
            if (split) FFT_R1(double, false, true);
            else FFT_R1(double, false, false);
        }
    } else {
        if (c2r) {
            if (split) FFT_R1(float, true, true);
            else FFT_R1(float, true, false);
        } else {
            if (split) FFT_R1(float, false, true);
            else FFT_R1(float, false, false);
        }
    }
#undef FFT_R1
    return hipGetLastError();
}

hipError_t launch_gen_pow_round(void* dst, int rb, int log2M, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = static_cast<unsigned>((count + 255) / 256);
    if (rb == 8)
        hipLaunchKernelGGL(k_gen_pow_round<double2>, dim3(blocks), dim3(256), 0, s, static_cast<double2*>(dst), log2M,
                           count);
    else
        hipLaunchKernelGGL(k_gen_pow_round<float2>, dim3(blocks), dim3(256), 0, s, static_cast<float2*>(dst), log2M,
                           count);
    return hipGetLastError();
}

// Single-pass instances: 8 and 16 points per thread, stage twiddles in
// registers or from the table, both directions, both complex layouts.
#define FFT_RS1(h, e, r)                                                                                      \
    real_entry<float, h, e, 256, false, false, r>(), real_entry<float, h, e, 256, false, true, r>(),         \
        real_entry<float, h, e, 256, true, false, r>(), real_entry<float, h, e, 256, true, true, r>()
#define FFT_RS(h, e) FFT_RS1(h, e, false), FFT_RS1(h, e, true)

static const RealKernel kReal[] = {
    FFT_RS(1, 4), FFT_RS(2, 4), FFT_RS(3, 4),
    FFT_RS(4, 3), FFT_RS(5, 3), FFT_RS(6, 3), FFT_RS(7, 3), FFT_RS(8, 3), FFT_RS(9, 3), FFT_RS(10, 3),
    FFT_RS(11, 3), FFT_RS(12, 3), FFT_RS(13, 3),
    FFT_RS(4, 4), FFT_RS(5, 4), FFT_RS(6, 4), FFT_RS(7, 4), FFT_RS(8, 4), FFT_RS(9, 4), FFT_RS(10, 4),
    FFT_RS(11, 4), FFT_RS(12, 4), FFT_RS(13, 4),
    FFT_RS1(14, 4, false),
    // the largest half lengths: stage twiddles as one FP64 value per butterfly
#define FFT_RR(h, e)                                                                                          \
    real_entry<float, h, e, 256, false, false, false, false, true>(),                                         \
        real_entry<float, h, e, 256, false, true, false, false, true>(),                                      \
        real_entry<float, h, e, 256, true, false, false, false, true>(),                                      \
        real_entry<float, h, e, 256, true, true, false, false, true>()
    FFT_RR(13, 3), FFT_RR(13, 4), FFT_RR(14, 4),
#undef FFT_RR
    // short rows (whole rows inside one wavefront): staged through LDS
#define FFT_RT(h, e)                                                                                          \
    real_entry<float, h, e, 256, false, false, true, true>(), real_entry<float, h, e, 256, false, true, true, true>(), \
        real_entry<float, h, e, 256, true, false, true, true>(), real_entry<float, h, e, 256, true, true, true, true>()
    FFT_RT(1, 4), FFT_RT(2, 4), FFT_RT(3, 4), FFT_RT(4, 4), FFT_RT(4, 3), FFT_RT(5, 4), FFT_RT(5, 3),
    FFT_RT(6, 4), FFT_RT(6, 3), FFT_RT(7, 4), FFT_RT(7, 3),
#undef FFT_RT
};

#undef FFT_RS
#undef FFT_RS1

const RealKernel* real_kernels(int* count) {
    *count = static_cast<int>(sizeof(kReal) / sizeof(kReal[0]));
    return kReal;
}

}  // namespace fftk
