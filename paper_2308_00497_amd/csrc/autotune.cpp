// Autotuner and its JSON cache.
//
// The paper picks radices by hand and names a runtime planner that measures
// candidate decompositions (as FFTW's exhaustive mode does) as future work
// (sections 4 and 6); loop-tile sizes were hyperparameters it set by hand
// (section 3, step 4).  Here every compiled decomposition of a size is timed
// with HIP events on scratch buffers and the winner is cached on disk.
#include "autotune.hpp"
#include "ragged.hpp"

#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <map>
#include <mutex>

namespace fftk {

namespace {

std::mutex g_mu;
std::string g_loaded_path;  // cache file the in-memory entries came from
bool g_loaded = false;
std::map<std::string, std::string> g_entries;

std::string read_file(const std::string& path) {
    FILE* f = fopen(path.c_str(), "rb");
    if (!f) return std::string();
    std::string s;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
    fclose(f);
    return s;
}

// one JSON string starting at s[i] == '"'; returns false on malformed input
bool read_string(const std::string& s, size_t& i, std::string* out) {
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
        if (s[i] == '\\') {
            if (i + 1 >= s.size()) return false;
            ++i;
        }
        out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
}

void skip_ws(const std::string& s, size_t& i) {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\t' || s[i] == '\r')) ++i;
}

void load_locked() {
    const std::string path = autotune_cache_path();
    if (g_loaded && path == g_loaded_path) return;
    g_loaded = true;
    g_loaded_path = path;
    g_entries.clear();
    std::vector<std::pair<std::string, std::string>> e;
    if (parse_cache_text(read_file(path), &e))
        for (auto& kv : e) g_entries[kv.first] = kv.second;
}

}  // namespace

// Format: {"version": 1, "entries": {"<key>": "<decomposition>", ...}}
bool parse_cache_text(const std::string& s, std::vector<std::pair<std::string, std::string>>* entries) {
    entries->clear();
    const size_t v = s.find("\"version\"");
    if (v == std::string::npos) return false;
    size_t i = s.find(':', v);
    if (i == std::string::npos) return false;
    ++i;
    skip_ws(s, i);
    if (s.compare(i, 1, "1") != 0) return false;  // unknown version: ignore the file
    const size_t e = s.find("\"entries\"");
    if (e == std::string::npos) return false;
    i = s.find('{', e);
    if (i == std::string::npos) return false;
    ++i;
    std::vector<std::pair<std::string, std::string>> tmp;
    while (true) {
        skip_ws(s, i);
        if (i < s.size() && s[i] == '}') break;
        std::string k, val;
        if (!read_string(s, i, &k)) return false;
        skip_ws(s, i);
        if (i >= s.size() || s[i] != ':') return false;
        ++i;
        skip_ws(s, i);
        if (!read_string(s, i, &val)) return false;
        Decomp d;
        RaggedConfig rc;
        if (!Decomp::parse(val, &d) && !RaggedConfig::parse(val, &rc)) return false;
        tmp.emplace_back(k, val);
        skip_ws(s, i);
        if (i < s.size() && s[i] == ',') {
            ++i;
            continue;
        }
        if (i < s.size() && s[i] == '}') break;
        return false;
    }
    *entries = tmp;
    return true;
}

std::string format_cache_text(const std::vector<std::pair<std::string, std::string>>& entries) {
    std::string s = "{\"version\": 1, \"entries\": {";
    for (size_t i = 0; i < entries.size(); ++i) {
        s += (i ? ",\n  \"" : "\n  \"") + entries[i].first + "\": \"" + entries[i].second + "\"";
    }
    s += "\n}}\n";
    return s;
}

TuneKey make_key(int device, int log2n, int64_t batch, fft_layout layout, int rb) {
    hipDeviceProp_t prop;
    char arch[64] = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
        char* colon = strchr(arch, ':');
        if (colon) *colon = '\0';
    }
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    int bclass = 0;
    while ((int64_t(1) << bclass) < batch) ++bclass;
    char buf[160];
    snprintf(buf, sizeof buf, "%s|hip%d|n%d|b%d|%s|%s", arch, rt, log2n, bclass,
             layout == FFT_LAYOUT_SPLIT ? "split" : "interleaved", rb == 8 ? "fp64" : "fp32");
    return TuneKey{buf};
}

// Ragged batches are keyed by their size histogram (FNV-1a over the count of
// each log2 size), not by the order of the transforms.
TuneKey make_ragged_key(int device, const int64_t* sizes, int64_t count, fft_layout layout) {
    int64_t hist[kMaxLog2N + 1] = {};
    for (int64_t i = 0; i < count; ++i) {
        const int k = ilog2_exact(sizes[i]);
        if (k >= 0 && k <= kMaxLog2N) ++hist[k];
    }
    uint64_t h = 1469598103934665603ull;
    for (int k = 0; k <= kMaxLog2N; ++k)
        for (int b = 0; b < 8; ++b) {
            h ^= uint64_t(hist[k] >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    TuneKey base = make_key(device, 0, count, layout, 4);
    char buf[64];
    snprintf(buf, sizeof buf, "|ragged%016llx", static_cast<unsigned long long>(h));
    return TuneKey{base.s + buf};
}

bool autotune_enabled() {
    const char* s = getenv("FFT_AUTOTUNE");
    return s && s[0] == '1';
}

std::string autotune_cache_path() {
    const char* s = getenv("FFT_AUTOTUNE_CACHE");
    if (s && *s) return s;
    const char* home = getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/fft_mi355x_autotune.json";
}

bool autotune_lookup_text(const TuneKey& key, std::string* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_entries.find(key.s);
    if (it == g_entries.end()) return false;
    *out = it->second;
    return true;
}

bool autotune_lookup(const TuneKey& key, Decomp* out) {
    std::string v;
    return autotune_lookup_text(key, &v) && Decomp::parse(v, out);
}

void autotune_store(const TuneKey& key, const Decomp& d) { autotune_store_text(key, d.str()); }

void autotune_store_text(const TuneKey& key, const std::string& value) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_entries[key.s] = value;
    std::vector<std::pair<std::string, std::string>> e(g_entries.begin(), g_entries.end());
    const std::string path = autotune_cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        // create the parent directory if missing (one level; no shell)
        (void)mkdir(path.substr(0, slash).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string(getpid());
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    const std::string text = format_cache_text(e);
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    fclose(f);
    if (ok) (void)rename(tmp.c_str(), path.c_str());
    else (void)remove(tmp.c_str());
}

fft_status autotune_run(fft_plan p, const TuneKey& key, Decomp* best, std::string* detail) {
    const int log2n = plan_log2n(p);
    const auto cands = candidate_decompositions(log2n, plan_layout(p), plan_real_bytes(p));
    *best = plan_decomposition(p);
    if (cands.size() <= 1) return FFT_OK;
    const size_t bytes = size_t(plan_elements(p)) * 2 * size_t(plan_real_bytes(p));
    void *in = nullptr, *out = nullptr;
    if (hipMalloc(&in, bytes) != hipSuccess || hipMalloc(&out, bytes) != hipSuccess) {
        if (in) (void)hipFree(in);
        *detail = "autotune scratch allocation failed";
        return FFT_ERR_ALLOC;
    }
    (void)hipMemset(in, 0, bytes);
    float best_ms = 1e30f;
    for (const Decomp& d : cands) {
        float ms = 0.f;
        std::string det;
        if (plan_time_decomposition(p, d, in, out, &ms, &det) != FFT_OK) continue;
        if (getenv("FFT_LOG")) fprintf(stderr, "[fft autotune] %s %s %.4f ms\n", key.s.c_str(), d.str().c_str(), ms);
        if (ms < best_ms) {
            best_ms = ms;
            *best = d;
        }
    }
    (void)hipFree(in);
    (void)hipFree(out);
    autotune_store(key, *best);
    return FFT_OK;
}

}  // namespace fftk
