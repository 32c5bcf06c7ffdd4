// Host-visible description of every compiled kernel instance.  The plan picks
// entries from these tables; the engine metadata (stage radices, twiddle
// table offsets) comes from the same constexpr schedule the kernels use, so
// the host-generated tables always match what the device reads.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fftk {

constexpr int kMaxStages = 32;

struct EngineInfo {
    int log2l;              // sub-FFT length L = 2^log2l
    int log2e;              // elements per thread
    bool remfirst;          // smaller radix first
    int nst;                // number of stages
    int tw_size;            // complex entries of the stage twiddle table
    int log2ns[kMaxStages];
    int log2r[kMaxStages];
    int tw_off[kMaxStages];
};

// Data pointers are float* / double* and the table float2* / double2* as
// `real_bytes` says; grid = number of persistent workgroups (clamped to the
// number of groups).
using single_fn = hipError_t (*)(const void* ia, const void* ib, void* oa, void* ob, const void* tw, int64_t batch,
                                 int grid, hipStream_t s);

struct SingleKernel {
    int real_bytes; // 4 (FP32) or 8 (FP64)
    int log2n;
    int log2e;
    int wgt;        // target threads per workgroup
    bool split;
    bool swap;      // swaps re/im of interleaved data on load and store (inverse)
    bool twreg;     // stage twiddles held in registers
    single_fn fn;
    const void* kernel;  // the __global__ function (occupancy queries)
    EngineInfo eng;
    int threads;    // actual threads per workgroup
    int per_wg;     // transforms per workgroup
    size_t lds_bytes;
};

// grid = number of persistent workgroups (clamped to the number of tiles)
using pass_fn = hipError_t (*)(const void* ia, const void* ib, void* oa, void* ob, const void* tw, const double2* ta,
                               const double2* tb, int log2N, int log2Ns, int hbits, int64_t batch, int grid,
                               hipStream_t s);

struct PassKernel {
    int real_bytes; // 4 (FP32) or 8 (FP64)
    int log2l;
    int log2e;
    int log2c;      // columns per workgroup
    bool first;
    bool split_in;
    bool split_out;
    bool swap_in;   // swap re/im of the interleaved input (inverse, first pass)
    bool swap_out;  // swap re/im of the interleaved output (inverse, last pass)
    pass_fn fn;
    const void* kernel;  // the __global__ function (occupancy queries)
    EngineInfo eng;
    int threads;
    size_t lds_bytes;
};

// tables defined in the kernel translation units (FP32 and FP64 instances)
const SingleKernel* single_kernels(int* count);
const PassKernel* pass_kernels(int* count);
const SingleKernel* single_kernels64(int* count);
const PassKernel* pass_kernels64(int* count);

// plain streaming copy (16-byte accesses), bytes % 16 == 0
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// twiddle generation launches; the stage table holds float2 (real_bytes 4) or
// double2 (real_bytes 8) entries
hipError_t launch_gen_engine_tw(const EngineInfo& e, void* dst, int real_bytes, hipStream_t s);
hipError_t launch_gen_pow64(double2* dst, int log2M, int64_t step, int64_t count, hipStream_t s);

}  // namespace fftk
