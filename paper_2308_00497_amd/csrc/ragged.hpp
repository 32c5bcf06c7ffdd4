// Ragged batches: transforms of different power-of-two sizes, packed back to
// back, computed by one persistent kernel launch replayed from a HIP graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fft.h"

namespace fftk {

struct RaggedPlan;

fft_status ragged_create(const int64_t* sizes, int64_t count, fft_layout layout, RaggedPlan** out,
                         std::string* detail);
// swap: exchange re/im of interleaved data in the kernel (the inverse); split
// callers already exchanged their pointers
fft_status ragged_execute(RaggedPlan* r, const float* ia, const float* ib, float* oa, float* ob, bool swap,
                          hipStream_t s, std::string* detail);
void ragged_destroy(RaggedPlan* r);
size_t ragged_workspace_bytes(const RaggedPlan* r);
fft_status ragged_set_workspace(RaggedPlan* r, void* dev_ptr, std::string* detail);
std::string ragged_describe(const RaggedPlan* r);

}  // namespace fftk
