// Autotuner: times every compiled decomposition of a size on the device and
// remembers the fastest in a JSON cache keyed by (GPU architecture, HIP
// runtime version, log2 N, batch class, layout, precision); ragged batches
// by their size histogram instead of N.
#pragma once

#include <string>

#include "../../include/fft.h"
#include "plan.hpp"

namespace fftk {

struct TuneKey {
    std::string s;
};

TuneKey make_key(int device, int log2n, int64_t batch, fft_layout layout, int rb);
TuneKey make_ragged_key(int device, const int64_t* sizes, int64_t count, fft_layout layout);
bool autotune_enabled();                                   // FFT_AUTOTUNE=1
std::string autotune_cache_path();                         // FFT_AUTOTUNE_CACHE or the default
bool autotune_lookup(const TuneKey& key, Decomp* out);     // in-memory copy of the cache file
void autotune_store(const TuneKey& key, const Decomp& d);  // updates memory and file
bool autotune_lookup_text(const TuneKey& key, std::string* out);        // any cached value
void autotune_store_text(const TuneKey& key, const std::string& value);  // e.g. a ragged configuration
fft_status autotune_run(fft_plan p, const TuneKey& key, Decomp* best, std::string* detail);

// provided by the plan code
fft_status plan_time_decomposition(fft_plan p, const Decomp& d, void* in, void* out, float* ms, std::string* detail);
const Decomp& plan_decomposition(fft_plan p);
int64_t plan_elements(fft_plan p);
fft_layout plan_layout(fft_plan p);
int plan_log2n(fft_plan p);
int plan_real_bytes(fft_plan p);

// cache text <-> entries (exposed for tests through the C ABI helpers)
bool parse_cache_text(const std::string& text, std::vector<std::pair<std::string, std::string>>* entries);
std::string format_cache_text(const std::vector<std::pair<std::string, std::string>>& entries);

}  // namespace fftk
