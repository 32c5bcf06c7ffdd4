// Internal hooks of the plan layer (capi.cpp) for the entry point that runs a
// plan on the library's static scratch buffer (noalloc.hip).
#pragma once

#include <stddef.h>

#include "../../include/fft.h"

namespace fftk {

// Workspace bytes one execution of `p` needs (0: none) and the plan's device.
// FFT_ERR_NOT_SUPPORTED for ragged plans, FFT_ERR_INVALID_ARG for a bad handle.
fft_status plan_scratch_need(fft_plan p, size_t* bytes, int* device);

// fft_execute with `ws` (device memory of at least plan_scratch_need bytes)
// in place of the plan's own workspace.  Allocates nothing.
fft_status execute_with_workspace(fft_plan p, const void* ia, const void* ib, void* oa, void* ob, void* stream,
                                  void* ws);

// text returned by fft_last_error_detail on this thread
void set_error_detail(const char* what);

}  // namespace fftk
