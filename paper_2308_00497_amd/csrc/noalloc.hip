// fft_execute_no_alloc: fft_execute of a created plan with the workspace of
// its multi-pass kernels taken from a static device array of this file
// instead of the plan's own allocation, so the call itself allocates nothing
// (no hipMalloc, hipFree or allocating library routine): for callers that
// cannot allocate, such as code under stream capture or tight serving loops.
//
// The array lives in the code object and every GPU the library is loaded on
// holds its own copy for the life of the process.  Host code never uses the
// array's name as an address: on the first call on a device, with that device
// current, hipGetSymbolAddress gives that copy's device address, which is kept
// per device and passed to the kernels like any workspace.  Every call on one
// GPU shares that GPU's array; calls that overlap in time on one GPU (other
// streams, other threads) race on it.  The kernels write every workspace
// element before reading it, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fft.h"
#include "scratch.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // FFT_NO_ALLOC_SCRATCH_BYTES
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device (null until set up)

// `dev` must be current.  Looks the address up once per device.
fft_status scratch_on(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        fftk::set_error_detail("device index beyond the scratch table");
        return FFT_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            fftk::set_error_detail(e != hipSuccess ? hipGetErrorString(e) : "scratch address is null");
            return FFT_ERR_HIP;
        }
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return FFT_OK;
}

}  // namespace

extern "C" {

size_t fft_no_alloc_scratch_bytes(void) { return kScratchBytes; }

fft_status fft_execute_no_alloc(fft_plan p, const void* in_re_or_z, const void* in_im, void* out_re_or_z,
                                void* out_im, void* stream) {
    size_t need = 0;
    int dev = 0;
    fft_status st = fftk::plan_scratch_need(p, &need, &dev);
    if (st != FFT_OK) return st;
    if (need > kScratchBytes) {
        fftk::set_error_detail("plan needs more workspace than the 64 MiB static scratch buffer; use fft_execute");
        return FFT_ERR_INVALID_SIZE;
    }
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) {
        (void)hipGetLastError();
        fftk::set_error_detail("hipGetDevice failed");
        return FFT_ERR_HIP;
    }
    if (cur != dev && hipSetDevice(dev) != hipSuccess) {
        (void)hipGetLastError();
        fftk::set_error_detail("hipSetDevice failed");
        return FFT_ERR_HIP;
    }
    void* ws = nullptr;
    st = scratch_on(dev, &ws);
    if (st == FFT_OK) st = fftk::execute_with_workspace(p, in_re_or_z, in_im, out_re_or_z, out_im, stream, ws);
    if (cur != dev) (void)hipSetDevice(cur);
    return st;
}

}  // extern "C"
