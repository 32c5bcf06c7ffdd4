// Twiddle generation (FP64 on the GPU, rounded once) and the streaming copy
// used as the practical HBM ceiling.
#include "kernels.hpp"

namespace fftk {

// The twiddle diagonal D^N_M of Eq. 1 (Table 1's TwiddleCoe): entries
// w_M^m = exp(-2 pi i m / M).  sincospi takes the exact rational argument 2m/M
// (M a power of two, m < M), so the only roundings are those of the FP64
// sine/cosine and the single rounding to float.
__global__ void k_gen_stage_tw(float2* dst, int log2NS, int log2R) {
    const int64_t count = int64_t(1) << (log2NS + log2R);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t k = i >> log2R;
    const int64_t r = i & ((int64_t(1) << log2R) - 1);
    const int64_t m = r * k;  // < Ns * R
    const double x = ldexp(static_cast<double>(m), 1 - (log2NS + log2R));  // 2m/M, exact
    double s, c;
    sincospi(x, &s, &c);
    dst[i] = make_float2(static_cast<float>(c), static_cast<float>(-s));
}

__global__ void k_gen_pow64(double2* dst, int log2M, int64_t step, int64_t count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t mask = (int64_t(1) << log2M) - 1;
    const int64_t m = (i * step) & mask;  // exponent reduced exactly modulo M
    const double x = ldexp(static_cast<double>(m), 1 - log2M);
    double s, c;
    sincospi(x, &s, &c);
    dst[i] = make_double2(c, -s);
}

hipError_t launch_gen_engine_tw(const EngineInfo& e, float2* dst, hipStream_t s) {
    for (int st = 1; st < e.nst; ++st) {
        const int64_t count = int64_t(1) << (e.log2ns[st] + e.log2r[st]);
        const unsigned blocks = static_cast<unsigned>((count + 255) / 256);
        hipLaunchKernelGGL(k_gen_stage_tw, dim3(blocks), dim3(256), 0, s, dst + e.tw_off[st], e.log2ns[st],
                           e.log2r[st]);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_gen_pow64(double2* dst, int log2M, int64_t step, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = static_cast<unsigned>((count + 255) / 256);
    hipLaunchKernelGGL(k_gen_pow64, dim3(blocks), dim3(256), 0, s, dst, log2M, step, count);
    return hipGetLastError();
}

// Grid-stride copy of 16-byte vectors.
__global__ void __launch_bounds__(256) k_copy16(const float4* __restrict__ src, float4* __restrict__ dst,
                                                int64_t n16) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const int64_t n16 = static_cast<int64_t>(bytes / 16);
    if (n16 == 0) return hipSuccess;
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;  // enough resident waves on 256 CUs
    hipLaunchKernelGGL(k_copy16, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace fftk
