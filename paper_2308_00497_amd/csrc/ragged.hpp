// Ragged batches: transforms of different power-of-two sizes, packed back to
// back, computed by one persistent kernel launch replayed from a HIP graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fft.h"

namespace fftk {

struct RaggedPlan;

// The tunable choices of a ragged plan (the autotuner times combinations):
//   max_pass_log2   longest pass sub-FFT of the multi-pass transforms, 2^6 .. 2^8
//                   (more, shorter passes trade HBM passes for wider column tiles)
//   grid_eighths    persistent workgroups per launch, in eighths of the number
//                   that can be resident at once
//   smallest_first  order of the multi-pass transforms within a level
//   group_mib       0: every multi-pass transform's pass p in level p.  Else
//                   the multi-pass transforms are cut into groups of at most
//                   this many MiB of workspace, and group g's pass p runs in
//                   level g + p (a software pipeline over levels): what one
//                   level writes to the workspace is read by the next while it
//                   can still be in the memory-side cache, and the workspace
//                   is a ring of two group-sized slots
//   single_max_log2 largest size run as one single-pass tile, 2^14 (radix-32
//                   stages) or 2^13 (2^14 then takes two passes)
struct RaggedConfig {
    int max_pass_log2 = 8;
    int grid_eighths = 8;
    // largest first measured equal or up to 1 % faster on the 2^6..2^16 mix
    // since 2^14 runs single-pass (smallest first led while 2^14 took two passes)
    bool smallest_first = false;
    int group_mib = 128;  // measured best on the 2^6..2^16 mix (two 128 MiB slots)
    int single_max_log2 = 14;
    std::string str() const;  // "ragged:p8:g8:o0", "ragged:p8:g8:o0:w128", "ragged:p8:g8:o0:w128:s13"
    static bool parse(const std::string& s, RaggedConfig* out);
};

// every configuration the autotuner tries
std::vector<RaggedConfig> ragged_candidates();

fft_status ragged_create(const int64_t* sizes, int64_t count, fft_layout layout, const RaggedConfig& cfg,
                         RaggedPlan** out, std::string* detail);
// average time of one execution on scratch buffers of the plan's size
fft_status ragged_time(RaggedPlan* r, float* ms, std::string* detail);
const RaggedConfig& ragged_config(const RaggedPlan* r);
// swap: exchange re/im of interleaved data in the kernel (the inverse); split
// callers already exchanged their pointers
fft_status ragged_execute(RaggedPlan* r, const float* ia, const float* ib, float* oa, float* ob, bool swap,
                          hipStream_t s, std::string* detail);
void ragged_destroy(RaggedPlan* r);
size_t ragged_workspace_bytes(const RaggedPlan* r);
fft_status ragged_set_workspace(RaggedPlan* r, void* dev_ptr, std::string* detail);
std::string ragged_describe(const RaggedPlan* r);

}  // namespace fftk
