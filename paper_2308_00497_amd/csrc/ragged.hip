#include "ragged.hpp"
namespace fftk {
struct RaggedPlan { int dummy; };
fft_status ragged_create(const int64_t*, int64_t, fft_layout, RaggedPlan** out, std::string* detail) {
    *out = nullptr; *detail = "ragged plans not built yet"; return FFT_ERR_NOT_SUPPORTED; }
fft_status ragged_execute(RaggedPlan*, const float*, const float*, float*, float*, uint32_t, hipStream_t, std::string*) { return FFT_ERR_NOT_SUPPORTED; }
void ragged_destroy(RaggedPlan*) {}
size_t ragged_workspace_bytes(const RaggedPlan*) { return 0; }
fft_status ragged_set_workspace(RaggedPlan*, void*, std::string*) { return FFT_ERR_NOT_SUPPORTED; }
std::string ragged_describe(const RaggedPlan*) { return ""; }
}
