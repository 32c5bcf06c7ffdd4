// Twiddle generation (FP64 on the GPU, rounded once) and the streaming copy
// used as the practical HBM ceiling.
#include "kernels.hpp"

namespace fftk {

// The twiddle diagonal D^N_M of Eq. 1 (Table 1's TwiddleCoe): entries
// w_M^m = exp(-2 pi i m / M).  sincospi takes the exact rational argument 2m/M
// (M a power of two, m < M), so the only roundings are those of the FP64
// sine/cosine and, for FP32 tables, the single rounding to float.
template <class V>
__global__ void k_gen_stage_tw(V* dst, int log2NS, int log2R) {
    const int64_t count = int64_t(1) << (log2NS + log2R);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t k = i >> log2R;
    const int64_t r = i & ((int64_t(1) << log2R) - 1);
    const int64_t m = r * k;  // < Ns * R
    const double x = ldexp(static_cast<double>(m), 1 - (log2NS + log2R));  // 2m/M, exact
    double s, c;
    sincospi(x, &s, &c);
    dst[i] = cvt_tw<V>(make_double2(c, -s));
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

hipError_t launch_gen_engine_tw(const EngineInfo& e, void* dst, int real_bytes, hipStream_t s) {
    if (e.rec) {
        // recurrence form: w_(Ns*R)^k for k < Ns per stage, FP64 pairs at
        // offsets counted in complex entries of the plan's precision
        const size_t entry = real_bytes == 8 ? sizeof(double2) : sizeof(float2);
        for (int st = 1; st < e.nst; ++st) {
            double2* t = reinterpret_cast<double2*>(static_cast<char*>(dst) + size_t(e.tw_off[st]) * entry);
            hipError_t err = launch_gen_pow64(t, e.log2ns[st] + e.log2r[st], 1, int64_t(1) << e.log2ns[st], s);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    }
    for (int st = 1; st < e.nst; ++st) {
        const int64_t count = int64_t(1) << (e.log2ns[st] + e.log2r[st]);
        const unsigned blocks = static_cast<unsigned>((count + 255) / 256);
        if (real_bytes == 8)
            hipLaunchKernelGGL(k_gen_stage_tw<double2>, dim3(blocks), dim3(256), 0, s,
                               static_cast<double2*>(dst) + e.tw_off[st], e.log2ns[st], e.log2r[st]);
        else
            hipLaunchKernelGGL(k_gen_stage_tw<float2>, dim3(blocks), dim3(256), 0, s,
                               static_cast<float2*>(dst) + e.tw_off[st], e.log2ns[st], e.log2r[st]);
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

// Streaming copy: each thread moves four 16-byte vectors spaced one
// workgroup-width apart (a 4 KiB block per workgroup step) with nontemporal
// loads and stores - the same access style as the FFT kernels; a grid-stride
// loop finishes the remainder.
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy16(const f32x4_t* __restrict__ src, f32x4_t* __restrict__ dst,
                                                int64_t n16) {
    // persistent: workgroup w copies 4 KiB blocks w, w + grid, ... (four
    // 16-byte streaming loads per thread, then four streaming stores)
    const int64_t full = n16 / 1024;  // complete 4 KiB blocks
    const int64_t tid = threadIdx.x;
    for (int64_t blk = blockIdx.x; blk < full; blk += gridDim.x) {
        const int64_t b = blk * 1024 + tid;
        f32x4_t a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = __builtin_nontemporal_load(src + b + 256 * i);
#pragma unroll
        for (int i = 0; i < 4; ++i) __builtin_nontemporal_store(a[i], dst + b + 256 * i);
    }
    for (int64_t i = full * 1024 + int64_t(blockIdx.x) * 256 + tid; i < n16; i += int64_t(gridDim.x) * 256)
        dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const int64_t n16 = static_cast<int64_t>(bytes / 16);
    if (n16 == 0) return hipSuccess;
    // one workgroup per compute unit measured fastest (256 MiB: 6.34 TB/s,
    // against 6.08 TB/s with one workgroup per 4 KiB block and 6.23-6.29 TB/s
    // with 4-16 per CU)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();  // only the failed query's own error
        cus = 256;
    }
    int64_t blocks = (n16 + 1023) / 1024;
    if (blocks > cus) blocks = cus;
    hipLaunchKernelGGL(k_copy16, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const f32x4_t*>(src), static_cast<f32x4_t*>(dst), n16);
    return hipGetLastError();
}

}  // namespace fftk
