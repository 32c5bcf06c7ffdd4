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
    bool rec;               // recurrence form: per stage w_(Ns*R)^k, k < Ns, as FP64
                            // pairs (tw_size and tw_off then count FP32 complex
                            // entries, two per FP64 pair)
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
    bool pf;        // next transform's loads issued before the current one's stages
    bool stg;       // small transforms: contiguous loads/stores staged through LDS
    bool half;      // stage exchanges one real part at a time (half the LDS)
    bool twrec;     // stage twiddles formed from one FP64 table value per butterfly
    single_fn fn;
    const void* kernel;  // the __global__ function (occupancy queries)
    EngineInfo eng;
    int threads;    // actual threads per workgroup
    int per_wg;     // transforms per workgroup
    size_t lds_bytes;
};

// Per-launch access flags of a pass tile (the `stream` argument).  kStreamIn /
// kStreamOut: the side is the caller's buffer, read or written once, with
// streaming (nontemporal) access.  kLoadPrio: raise the wave priority while
// the tile's loads are issued (set inside the FP32 pass kernel itself, not by
// callers).
constexpr int kStreamIn = 1, kStreamOut = 2;
constexpr int kLoadPrio = 4;

// grid = number of persistent workgroups (clamped to the number of tiles);
// stream = kStreamIn | kStreamOut for the sides that are the caller's buffers
// (streaming access), 0 for workspace on both sides; twshift = low bits of
// the column index hidden from the pass twiddles (0 for 1D chains); ain/aout
// = the address maps of the pass tile (-1: the Stockham pass's own; equal
// values: an in-place pass)
using pass_fn = hipError_t (*)(const void* ia, const void* ib, void* oa, void* ob, const void* tw, const double2* ta,
                               const double2* tb, int log2N, int log2Ns, int hbits, int64_t batch, int grid,
                               int stream, int twshift, int ain, int aout, hipStream_t s);

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

// Single-pass real-input kernel (R2C, or C2R when c2r): half length
// H = 2^log2h; `tw` is the engine stage table and `twn` holds w_N^k, k < H,
// N = 2H, both in the kernel's precision.
// iscale multiplies the interior bins k = 1 .. H-1 of the complex side (1 for
// the transforms themselves; 1/2 and 2 give the adjoints of R2C and C2R).
using real_fn = hipError_t (*)(const void* ia, const void* ib, void* oa, void* ob, const void* tw, const void* twn,
                               int64_t batch, int grid, double iscale, hipStream_t s);

struct RealKernel {
    int real_bytes;
    int log2h;
    int log2e;
    int wgt;
    bool c2r;
    bool split;     // complex side split into re/im arrays
    bool twreg;
    bool stg;       // short rows: contiguous loads/stores staged through LDS
    bool twrec;     // stage twiddles as one FP64 value per butterfly and its powers
    real_fn fn;
    const void* kernel;
    EngineInfo eng;
    int threads;
    int per_wg;
    size_t lds_bytes;
};

// Column transforms of multi-dimensional plans: DFT_(2^log2l) down every
// column of stride 2^log2s, over blocks_b column blocks, C = 2^log2c columns
// per workgroup (log2l <= 4: one thread per column, no table, log2c 0).
using strided_fn = hipError_t (*)(const void* ia, const void* ib, void* oa, void* ob, const void* tw, int log2s,
                                  int64_t blocks_b, int grid, hipStream_t s);

struct StridedKernel {
    int real_bytes;
    int log2l;
    int log2c;
    bool split;
    bool swap;
    strided_fn fn;
    const void* kernel;  // nullptr for the one-thread-per-column kernels
    EngineInfo eng;
    int threads;
    size_t lds_bytes;
};

// tables defined in the kernel translation units (FP32 and FP64 instances)
const SingleKernel* single_kernels(int* count);
const PassKernel* pass_kernels(int* count);
const SingleKernel* single_kernels64(int* count);
const PassKernel* pass_kernels64(int* count);
const RealKernel* real_kernels(int* count);
const RealKernel* real_kernels64(int* count);
const StridedKernel* strided_kernels(int* count);

// passes over HBM around the multi-pass half-length transform of real plans
// (z: interleaved half-length data; ta/tb: FP64 tables of w_N, N = 2^(log2h+1))
// (iscale: the interior-bin scale of real_fn)
hipError_t launch_r2c_post(int rb, bool split, const void* z, void* oa, void* ob, const double2* ta,
                           const double2* tb, int hbits, int log2h, int64_t batch, double iscale, hipStream_t s);
hipError_t launch_c2r_pre(int rb, bool split, const void* ia, const void* ib, void* z, const double2* ta,
                          const double2* tb, int hbits, int log2h, int64_t batch, double iscale, hipStream_t s);
// per-operator baseline (Table 1 operators, one kernel each; interleaved data)
hipError_t launch_op_kron(int rb, int log2r, const void* x, void* y, int64_t a, int64_t b, bool swap_in,
                          bool swap_out, hipStream_t s);
hipError_t launch_op_mul(int rb, const void* x, void* y, const void* d, int64_t a, int log2n, hipStream_t s);
hipError_t launch_op_perm(int rb, const void* x, void* y, int64_t a, int log2m, int log2n, bool swap_in,
                          hipStream_t s);
hipError_t launch_gen_diag(int rb, void* dst, int log2n, int log2m, hipStream_t s);
// N = 1 real transforms
hipError_t launch_real1(int rb, bool c2r, bool split, const void* ia, const void* ib, void* oa, void* ob,
                        int64_t batch, hipStream_t s);
// dst[i] = w_M^i rounded once to the precision of rb, i < count
hipError_t launch_gen_pow_round(void* dst, int rb, int log2M, int64_t count, hipStream_t s);

// plain streaming copy (16-byte accesses), bytes % 16 == 0
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// twiddle generation launches; the stage table holds float2 (real_bytes 4) or
// double2 (real_bytes 8) entries
hipError_t launch_gen_engine_tw(const EngineInfo& e, void* dst, int real_bytes, hipStream_t s);
hipError_t launch_gen_pow64(double2* dst, int log2M, int64_t step, int64_t count, hipStream_t s);

}  // namespace fftk
