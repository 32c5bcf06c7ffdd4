// Ragged batches: transforms of different power-of-two sizes packed back to
// back, computed by persistent kernels captured in ONE HIP graph (one host
// launch for the whole batch).
//
// The work is cut into tiles of (at most) 8192 complex elements, one tile per
// visit of a 512-thread workgroup:
//   copy tile     up to 512 transforms of size 1
//   single tile   G = 512/T whole transforms of size N <= 8192 (T = N/E
//                 threads each, E = 8 points per thread up to 2^12, 16 at
//                 2^13), the single-pass Stockham engine; one transform of
//                 2^14 points at 32 points per thread (radix-32 stages, the
//                 exchanges one real part at a time so the LDS stays that of
//                 8192 complex elements), unless the configuration sets the
//                 single-pass limit to 2^13
//   pass tile     C = 8192/L columns of one pass of a transform above the
//                 single-pass limit, split into P = ceil(log2 N / 8) passes of
//                 L <= 256 points (the multi-pass scheme of Eq. 1 with M, K
//                 the pass lengths)
// Tiles are grouped in levels: level 0 holds every first-pass tile and then
// every single/copy tile, level p > 0 the p-th pass tiles.  With pipelined
// groups (RaggedConfig::group_mib) the multi-pass transforms are cut into
// groups and level k holds pass p of group k - p, so each level's workspace
// output is consumed by the next level.  Each level is one launch of the
// persistent kernel; the kernel boundary orders pass p - 1 before pass p, so
// no workgroup ever waits for another.  Within a level the
// tiles are sorted by class and dealt round-robin to the resident workgroups
// (tile w, w + grid, ...), and a workgroup keeps running one class's code, with
// that class's stage twiddles in registers, while its next tile is of the same
// class.  Descriptors carry every offset a tile needs, so a tile's data loads
// depend on one descriptor read at most.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "ragged.hpp"

namespace fftk {

namespace {

constexpr int kThreads = 512;
constexpr int kTileLog2 = 13;  // 8192 elements per tile
constexpr int kSingleMaxLog2 = 14;  // largest single-pass class
constexpr int kMinPassLog2 = 5, kMaxPassLog2 = 8;
constexpr int kMaxPasses = 3;  // passes of one multi-pass transform

enum : uint32_t { CODE_COPY = 0, CODE_PASS_FIRST = 16, CODE_PASS_MID = 20, CODE_PASS_LAST = 24 };

struct RaggedTile {
    uint32_t code;    // CODE_COPY, log2 N (single, 1..13) or CODE_PASS_* + (log2 L - 5)
    uint32_t first;   // copy/single: index into the tile-slot offset list
    uint32_t count;   // copy/single: transforms in the tile
    uint32_t col;     // pass: first butterfly column j0
    int32_t log2n, log2ns, hbits;
    uint32_t tw_eng;  // float2 offset of the engine stage table
    uint32_t ta, tb;  // double2 offsets of the pass twiddle tables
    uint32_t src, dst;  // 0 input, 1 workspace A, 2 workspace B, 3 output
    int64_t uoff;     // pass: element offset of the transform in the caller's buffers
    int64_t woff;     // pass: element offset of the transform in the workspaces
};
static_assert(sizeof(RaggedTile) == 64, "one cache line per descriptor");

struct RaggedArgs {
    const float* ia;
    const float* ib;
    float* oa;
    float* ob;
    float* wsa;  // interleaved workspaces
    float* wsb;
    const RaggedTile* tiles;  // this level's tiles
    uint32_t ntiles;
    const int64_t* toffs;     // element offsets of the transforms of copy/single tiles
    const float2* tw32;
    const double2* tw64;
};

// points per thread of the single-pass classes: 8 up to 2^12, 16 for 2^13
// (the shapes measured fastest for the plain kernels), 32 for 2^14 (the
// whole transform on the 512 threads)
constexpr int single_log2e(int log2n) { return log2n <= 12 ? 3 : (log2n == 13 ? 4 : 5); }
// the 2^14 class exchanges real and imaginary parts in turn (half the LDS)
constexpr bool single_half(int log2n) { return log2n == 14; }
// classes whose stage twiddles come from one FP64 value per butterfly
// (TwRec): 2^13 and 2^14, whose stage tables do not fit in registers
constexpr bool single_rec(int log2n) { return log2n >= 13; }

template <int LOG2N>
using RSingle = SingleShape<LOG2N, single_log2e(LOG2N), kThreads>;

template <int LOG2L>
using RPass = PassShape<LOG2L, 4, kTileLog2 - LOG2L>;

constexpr int lds_max() {
    int m = 1;
    m = std::max(m, (RSingle<14>::LDS + 1) / 2);
    m = std::max(m, RSingle<13>::LDS);
    m = std::max(m, RSingle<12>::LDS);
    m = std::max(m, RSingle<11>::LDS);
    m = std::max(m, RSingle<5>::LDS);
    m = std::max(m, RPass<5>::LDS);
    m = std::max(m, RPass<6>::LDS);
    m = std::max(m, RPass<7>::LDS);
    m = std::max(m, RPass<8>::LDS);
    return m;
}
constexpr int kLds = lds_max();

// Tiles are dealt to the persistent workgroups round-robin (tile w, w + grid,
// ...); a tile carries 4096 to 16384 elements (8192 for every pass tile).
__device__ __forceinline__ bool same_class(const RaggedArgs& a, uint32_t ti, uint32_t code) {
    return ti < a.ntiles && a.tiles[ti].code == code;
}

// Whole transforms of one size class, tile after tile while this workgroup's
// next tile is of the same class; the stage twiddles (same table for every
// tile of the class) stay in registers.  Returns the workgroup's first tile of
// another class (or past the end).
template <int LOG2N, bool SPLIT, bool SWAP>
__device__ __forceinline__ uint32_t run_single(const RaggedArgs& a, uint32_t ti, float2* lds, int tid) {
    using SH = RSingle<LOG2N>;
    using SC = typename SH::SC;
    static_assert(SH::THREADS == kThreads, "single tiles use the whole workgroup");
    constexpr int E = SC::E, T = SC::T;
    // all stage twiddles in registers when they are few, else only the last
    // stage's (the 128-register budget of two 512-thread workgroups per CU);
    // also all of them for 2^10 - 2^12 (24 pairs: a batch of 2^12 transforms
    // 121 -> 102 us for 2^25 elements, 2^10 and 2^11 15 % faster too; they
    // fit since the one-transform tiles address through rebased pointers); for
    // 2^13 and 2^14 (tables too large for registers) one FP64 value per
    // butterfly and its powers (TwRec)
    constexpr bool RECTW = single_rec(LOG2N);
    constexpr bool ALLREG = !RECTW && (SC::NST - 1) * E <= (E == 8 && LOG2N >= 10 ? 32 : 16);
    constexpr bool MEMTW = !RECTW && ((SPLIT && !ALLREG && E == 16) || E == 32);
    using ENG = Engine<SC, SH::G, SH::GS, false, false, SH::WAVE, single_half(LOG2N)>;
    const uint32_t code = static_cast<uint32_t>(LOG2N);
    const float2* tw = a.tw32 + a.tiles[ti].tw_eng;
    using TWT = typename std::conditional<ALLREG, TwReg<SC>, TwLast<SC>>::type;
    TWT twr(tw);
    if constexpr (!MEMTW && !RECTW) twr.init(tid % T);
    do {
        const RaggedTile d = a.tiles[ti];
        int tidl = tid;
        asm volatile("" : "+v"(tidl));
        const int t = tidl % T, g = tidl / T;
        const bool active = static_cast<uint32_t>(g) < d.count;
        float2 v[E];
        if constexpr (SH::G == 1) {
            // one transform per tile: pointers rebased on it (workgroup-
            // uniform) and 32-bit offsets per lane, so the loads need no
            // 64-bit address pair each (register budget)
            const int64_t toff = a.toffs[d.first];
            const float* ia = a.ia + (SPLIT ? toff : 2 * toff);
            const float* ib = SPLIT ? a.ib + toff : nullptr;
            if constexpr (!SPLIT) loads_begin();
#pragma unroll
            for (int m = 0; m < E; ++m)
                v[m] = swap_if<SWAP>(gload_nt<SPLIT>(ia, ib, static_cast<uint32_t>(t + T * m)));
            if constexpr (!SPLIT) loads_end();
        } else {
            const int64_t base = (active ? a.toffs[d.first + g] : 0) + t;
            // raised load priority for interleaved data, as in the plain kernel
            if constexpr (!SPLIT) loads_begin();
#pragma unroll
            for (int m = 0; m < E; ++m)
                v[m] = active ? swap_if<SWAP>(gload_nt<SPLIT>(a.ia, a.ib, base + T * m)) : make_float2(0.f, 0.f);
            if constexpr (!SPLIT) loads_end();
        }
        if constexpr (RECTW) {
            const float2* twl = tw;
            asm volatile("" : "+v"(twl));  // keep the table reads inside the loop
            ENG::run(v, lds, TwRec<SC>(reinterpret_cast<const double2*>(twl)), tidl);
        } else if constexpr (MEMTW) {
            const float2* twl = tw;
            asm volatile("" : "+v"(twl));  // keep the table reads inside the loop
            ENG::run(v, lds, TwMem<SC>(twl), tidl);
        } else {
            ENG::run(v, lds, twr, tidl);
        }
        if constexpr (SH::G == 1) {
            const int64_t toff = a.toffs[d.first];
            float* oa = a.oa + (SPLIT ? toff : 2 * toff);
            float* ob = SPLIT ? a.ob + toff : nullptr;
            // the lane offsets are formed again here rather than kept from the
            // loads across the stages (32 points per thread leave no registers
            // for them)
            int tids = tid;
            asm volatile("" : "+v"(tids));
            const int ts = tids % T;
#pragma unroll
            for (int m = 0; m < E; ++m) gstore_nt<SPLIT>(oa, ob, static_cast<uint32_t>(ts + T * m), swap_if<SWAP>(v[m]));
        } else if (active) {
            const int64_t base = a.toffs[d.first + g] + t;
#pragma unroll
            for (int m = 0; m < E; ++m) gstore_nt<SPLIT>(a.oa, a.ob, base + T * m, swap_if<SWAP>(v[m]));
        }
        ti += gridDim.x;
    } while (same_class(a, ti, code));
    return ti;
}

// size-1 transforms are the identity in both directions
template <bool SPLIT>
__device__ __forceinline__ uint32_t run_copy(const RaggedArgs& a, uint32_t ti, int tid) {
    do {
        const RaggedTile d = a.tiles[ti];
        if (static_cast<uint32_t>(tid) < d.count) {
            const int64_t i = a.toffs[d.first + tid];
            if (SPLIT) {
                a.oa[i] = a.ia[i];
                a.ob[i] = a.ib[i];
            } else {
                reinterpret_cast<float2*>(a.oa)[i] = reinterpret_cast<const float2*>(a.ia)[i];
            }
        }
        ti += gridDim.x;
    } while (same_class(a, ti, CODE_COPY));
    return ti;
}

// Pass tiles of one (pass kind, sub-length) class; the sub-FFT's stage
// twiddles stay in registers across tiles.  Interleaved workspace between
// passes, the caller's layout at the ends.  REGALL: the later passes of 64
// to 256 points keep their stage twiddles in registers too (the pass-only
// kernel, whose register budget is not shared with the single-pass classes;
// the 32-point passes would spill there).
template <int LOG2L, uint32_t KIND, bool SPLIT, bool SWAP, bool REGALL>
__device__ __forceinline__ uint32_t run_pass(const RaggedArgs& a, uint32_t ti, float2* lds, int tid) {
    constexpr int LOG2C = kTileLog2 - LOG2L;
    constexpr bool FIRST = KIND == CODE_PASS_FIRST, LAST = KIND == CODE_PASS_LAST;
    using SH = RPass<LOG2L>;
    using SC = typename SH::SC;
    static_assert(SH::THREADS == kThreads, "pass tiles use the whole workgroup");
    using ENG = Engine<SC, SH::C, SH::GS, true, !FIRST, false>;
    const uint32_t code = KIND + static_cast<uint32_t>(LOG2L - kMinPassLog2);
    // later passes also form FP64 pass twiddles; in the kernel that serves
    // every class their stage twiddles come from the (L1-resident) table to
    // stay inside the register budget (registers measured 8 % faster)
    constexpr bool REG = FIRST || (REGALL && LOG2L >= 6);
    using TWT = typename std::conditional<REG, TwReg<SC>, TwMem<SC>>::type;
    TWT twr(a.tw32 + a.tiles[ti].tw_eng);
    if constexpr (REG) twr.template init_engine<ENG>(tid);
    do {
        const RaggedTile d = a.tiles[ti];
        int tidl = tid;
        asm volatile("" : "+v"(tidl));
        const int64_t uoff = d.uoff;
        const int64_t woff = d.woff;
        // element offsets folded into the base pointers (interleaved: 2 floats each)
        const int64_t u = SPLIT ? uoff : 2 * uoff;
        const float* ia = a.ia + u;
        const float* ib = SPLIT ? a.ib + uoff : nullptr;
        float* oa = a.oa + u;
        float* ob = SPLIT ? a.ob + uoff : nullptr;
        float* wsrc = (d.src == 2 ? a.wsb : a.wsa) + 2 * woff;
        float* wdst = (d.dst == 2 ? a.wsb : a.wsa) + 2 * woff;
        const double2* ta = a.tw64 + d.ta;
        const double2* tb = a.tw64 + d.tb;
        // the caller's data is streamed; the workspace between levels is not,
        // so the next level can find it in the memory-side cache
        // (stream bits fixed at compile time: the split sides' streaming
        // accesses would otherwise be merged into ordinary ones); raised wave
        // priority while the loads are issued, as in the plain pass kernel
        // (C4 split 0.2714-0.2724 -> 0.2652-0.2660 ms, interleaved 0.5 %)
        if constexpr (FIRST) {
            pass_tile<LOG2L, 4, LOG2C, true, SPLIT, false, SWAP, false, TWT, float, true, 3, kStreamIn>(
                ia, ib, wdst, nullptr, twr, ta, tb, d.log2n, d.log2ns, d.hbits, 0, d.col, lds, tidl, kStreamIn | kLoadPrio);
        } else if constexpr (LAST) {
            pass_tile<LOG2L, 4, LOG2C, false, false, SPLIT, false, SWAP, TWT, float, true, 3, kStreamOut>(
                wsrc, nullptr, oa, ob, twr, ta, tb, d.log2n, d.log2ns, d.hbits, 0, d.col, lds, tidl, kStreamOut | kLoadPrio);
        } else {
            pass_tile<LOG2L, 4, LOG2C, false, false, false, false, false, TWT, float, true, 3, 0>(
                wsrc, nullptr, wdst, nullptr, twr, ta, tb, d.log2n, d.log2ns, d.hbits, 0, d.col, lds, tidl, kLoadPrio);
        }
        ti += gridDim.x;
    } while (same_class(a, ti, code));
    return ti;
}

// PASSONLY: an instance for the levels that hold pass tiles only (every level
// after the first); it leaves out the single-pass and copy classes.
template <bool SPLIT, bool SWAP, bool PASSONLY>
__global__ void __launch_bounds__(kThreads, 4) k_ragged(RaggedArgs a) {
    __shared__ float2 lds[kLds];
    const int tid = threadIdx.x;
    uint32_t ti = blockIdx.x;
    while (ti < a.ntiles) {
        // Each pass of this loop starts a run of another class.  The engines
        // of classes whose transforms fit in one wavefront order LDS with
        // wavefront fences only, and their LDS regions differ from those of
        // the class before, so a wavefront could write the new class's first
        // exchange while another is still reading the previous class's last
        // one: one workgroup barrier per class change rules that out.
        stage_sync<false>();
        const uint32_t code = a.tiles[ti].code;
        if constexpr (!PASSONLY) {
            if (code < CODE_PASS_FIRST) {
                switch (code) {
                    case CODE_COPY: ti = run_copy<SPLIT>(a, ti, tid); break;
#define FFT_RS(n) \
    case n: ti = run_single<n, SPLIT, SWAP>(a, ti, lds, tid); break;
                    FFT_RS(1) FFT_RS(2) FFT_RS(3) FFT_RS(4) FFT_RS(5) FFT_RS(6) FFT_RS(7)
                    FFT_RS(8) FFT_RS(9) FFT_RS(10) FFT_RS(11) FFT_RS(12) FFT_RS(13) FFT_RS(14)
#undef FFT_RS
                    default: ti += gridDim.x; break;
                }
                continue;
            }
        }
        switch (code) {
#define FFT_RP(kind)                                                                    \
    case kind + 0: ti = run_pass<5, kind, SPLIT, SWAP, PASSONLY>(a, ti, lds, tid); break; \
    case kind + 1: ti = run_pass<6, kind, SPLIT, SWAP, PASSONLY>(a, ti, lds, tid); break; \
    case kind + 2: ti = run_pass<7, kind, SPLIT, SWAP, PASSONLY>(a, ti, lds, tid); break; \
    case kind + 3: ti = run_pass<8, kind, SPLIT, SWAP, PASSONLY>(a, ti, lds, tid); break;
            FFT_RP(CODE_PASS_FIRST)
            FFT_RP(CODE_PASS_MID)
            FFT_RP(CODE_PASS_LAST)
#undef FFT_RP
            default: ti += gridDim.x; break;
        }
    }
}

template <class SC>
int engine_tw_size() {
    return (SC::TW_SIZE + 1) & ~1;
}

}  // namespace

struct RaggedPlan {
    RaggedConfig cfg;
    int64_t count = 0, total = 0;
    fft_layout layout = FFT_LAYOUT_INTERLEAVED;
    int device = 0;
    int grid = 0;
    std::vector<RaggedTile> htiles;
    RaggedTile* tiles = nullptr;
    int64_t* toffs = nullptr;      // offsets of the transforms of copy/single tiles
    float2* tw32 = nullptr;
    double2* tw64 = nullptr;
    void* ws_own = nullptr;
    void* ws_user = nullptr;
    size_t ws_half = 0;            // bytes of one workspace region
    int ws_regions = 0;
    hipStream_t cap = nullptr;     // capture stream
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    static constexpr int kMaxLevels = 24;  // pass levels of the pipelined groups
    int nlevels = 0;
    uint32_t level_begin[kMaxLevels + 1] = {};     // tile index ranges of the levels
    int level_grid[kMaxLevels] = {};
    bool level_pass_only[kMaxLevels] = {};         // launched with the pass-only kernel
    hipGraphNode_t node[2][kMaxLevels] = {};
    RaggedArgs args[2][kMaxLevels];
    int nsingle_tiles = 0, npass_tiles = 0, ncopy_tiles = 0, nmulti = 0, ngroups = 0;
    std::string classes;

    void* ws() const { return ws_user ? ws_user : ws_own; }
};

namespace {

fft_status hip_err(hipError_t e, const char* what, std::string* detail) {
    *detail = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    return FFT_ERR_HIP;
}

void free_all(RaggedPlan* r) {
    for (int i = 0; i < 2; ++i) {
        if (r->exec[i]) (void)hipGraphExecDestroy(r->exec[i]);
        if (r->graph[i]) (void)hipGraphDestroy(r->graph[i]);
    }
    if (r->cap) (void)hipStreamDestroy(r->cap);
    void* bufs[] = {r->tiles, r->toffs, r->tw32, r->tw64, r->ws_own};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
    if (e != hipSuccess) return e;
    if (src.empty()) return hipSuccess;
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

std::vector<int> even_parts(int log2n, int parts) {
    std::vector<int> v(parts, log2n / parts);
    for (int i = 0; i < log2n % parts; ++i) v[i] += 1;
    return v;
}

void* kernel_for(bool split, bool swap, bool pass_only) {
    if (pass_only) {
        if (split) return reinterpret_cast<void*>(&k_ragged<true, false, true>);
        return swap ? reinterpret_cast<void*>(&k_ragged<false, true, true>)
                    : reinterpret_cast<void*>(&k_ragged<false, false, true>);
    }
    if (split) return reinterpret_cast<void*>(&k_ragged<true, false, false>);
    return swap ? reinterpret_cast<void*>(&k_ragged<false, true, false>)
                : reinterpret_cast<void*>(&k_ragged<false, false, false>);
}

// Capture one persistent launch per level into a graph.
fft_status build_graph(RaggedPlan* r, int variant, std::string* detail) {
    const bool split = r->layout == FFT_LAYOUT_SPLIT;
    const bool swap = variant == 1;
    hipError_t e = hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_err(e, "graph capture begin", detail);
    for (int l = 0; l < r->nlevels && e == hipSuccess; ++l) {
        RaggedArgs& a = r->args[variant][l];
        void* kparams[] = {&a};
        void* fn = kernel_for(split, swap, r->level_pass_only[l]);
        e = hipLaunchKernel(fn, dim3(r->level_grid[l]), dim3(kThreads), kparams, 0, r->cap);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(r->cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_err(e, "ragged launch capture", detail);
    }
    if (e2 != hipSuccess) return hip_err(e2, "graph capture end", detail);
    r->graph[variant] = g;
    size_t nn = 0;
    e = hipGraphGetNodes(g, nullptr, &nn);
    std::vector<hipGraphNode_t> nodes(nn);
    if (e == hipSuccess) e = hipGraphGetNodes(g, nodes.data(), &nn);
    if (e != hipSuccess) return hip_err(e, "graph nodes", detail);
    // match each persistent-kernel node to its level by the tile pointer it carries
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        if (hipGraphKernelNodeGetParams(nd, &kp) != hipSuccess || !kp.kernelParams) continue;
        const bool ours = kp.func == kernel_for(split, swap, false) || kp.func == kernel_for(split, swap, true);
        if (!ours) continue;
        const RaggedArgs* ka = static_cast<const RaggedArgs*>(kp.kernelParams[0]);
        for (int l = 0; l < r->nlevels; ++l)
            if (ka->tiles == r->args[variant][l].tiles && kp.func == kernel_for(split, swap, r->level_pass_only[l]))
                r->node[variant][l] = nd;
    }
    for (int l = 0; l < r->nlevels; ++l)
        if (!r->node[variant][l]) {
            *detail = "persistent kernel node not found in the captured graph";
            return FFT_ERR_HIP;
        }
    e = hipGraphInstantiate(&r->exec[variant], g, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_err(e, "graph instantiate", detail);
    return FFT_OK;
}

}  // namespace

std::string RaggedConfig::str() const {
    char buf[64];
    int k = snprintf(buf, sizeof buf, "ragged:p%d:g%d:o%d", max_pass_log2, grid_eighths, smallest_first ? 1 : 0);
    if (group_mib > 0) k += snprintf(buf + k, sizeof buf - k, ":w%d", group_mib);
    if (single_max_log2 != kSingleMaxLog2) snprintf(buf + k, sizeof buf - k, ":s%d", single_max_log2);
    return buf;
}

bool RaggedConfig::parse(const std::string& s, RaggedConfig* out) {
    int p = 0, g = 0, o = 0, w = 0, sm = kSingleMaxLog2, used = 0;
    if (sscanf(s.c_str(), "ragged:p%d:g%d:o%d%n", &p, &g, &o, &used) != 3) return false;
    size_t at = static_cast<size_t>(used);
    // optional ":w<W>", then optional ":s<S>"
    if (s.compare(at, 2, ":w") == 0) {
        used = 0;
        if (sscanf(s.c_str() + at, ":w%d%n", &w, &used) != 1 || used == 0) return false;
        at += static_cast<size_t>(used);
        if (w < 8 || w > 65536) return false;
    }
    if (s.compare(at, 2, ":s") == 0) {
        used = 0;
        if (sscanf(s.c_str() + at, ":s%d%n", &sm, &used) != 1 || used == 0) return false;
        at += static_cast<size_t>(used);
        if (sm != kTileLog2 && sm != kSingleMaxLog2) return false;
    }
    if (at != s.size()) return false;
    if (p < 6 || p > kMaxPassLog2 || g < 1 || g > 8 || (o != 0 && o != 1)) return false;
    out->max_pass_log2 = p;
    out->grid_eighths = g;
    out->smallest_first = o == 1;
    out->group_mib = w;
    out->single_max_log2 = sm;
    return true;
}

std::vector<RaggedConfig> ragged_candidates() {
    std::vector<RaggedConfig> v;
    for (int w : {128, 0, 64, 192, 256})
        for (int p : {8, 7, 6})
            for (int g : {8, 6, 4})
                for (int o : {0, 1})
                    for (int sm : {kSingleMaxLog2, kTileLog2}) {
                        if (sm != kSingleMaxLog2 && w != 128) continue;  // the 2^13 limit at one group size
                        RaggedConfig c;
                        c.max_pass_log2 = p;
                        c.grid_eighths = g;
                        c.smallest_first = o == 1;
                        c.group_mib = w;
                        c.single_max_log2 = sm;
                        v.push_back(c);
                    }
    return v;
}

const RaggedConfig& ragged_config(const RaggedPlan* r) { return r->cfg; }

fft_status ragged_create(const int64_t* sizes, int64_t count, fft_layout layout, const RaggedConfig& cfg,
                         RaggedPlan** out, std::string* detail) {
    *out = nullptr;
    RaggedPlan* r = new (std::nothrow) RaggedPlan;
    if (!r) return FFT_ERR_ALLOC;
    r->cfg = cfg;
    r->count = count;
    r->layout = layout;
    hipError_t e = hipGetDevice(&r->device);
    int cus = 256;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, r->device);
    if (e != hipSuccess) {
        delete r;
        return hip_err(e, "device query", detail);
    }

    // ---- items and classes ------------------------------------------------
    std::vector<int> lg(count);
    std::vector<int64_t> offs(count);
    int64_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        lg[i] = ilog2_exact(sizes[i]);
        offs[i] = total;
        total += sizes[i];
    }
    r->total = total;

    // engine tables: single classes 1..14 and pass lengths 5..8
    const int smax = cfg.single_max_log2;
    EngineInfo eng_single[kSingleMaxLog2 + 1] = {};
    eng_single[1] = engine_info<RSingle<1>::SC>();
    eng_single[2] = engine_info<RSingle<2>::SC>();
    eng_single[3] = engine_info<RSingle<3>::SC>();
    eng_single[4] = engine_info<RSingle<4>::SC>();
    eng_single[5] = engine_info<RSingle<5>::SC>();
    eng_single[6] = engine_info<RSingle<6>::SC>();
    eng_single[7] = engine_info<RSingle<7>::SC>();
    eng_single[8] = engine_info<RSingle<8>::SC>();
    eng_single[9] = engine_info<RSingle<9>::SC>();
    eng_single[10] = engine_info<RSingle<10>::SC>();
    eng_single[11] = engine_info<RSingle<11>::SC>();
    eng_single[12] = engine_info<RSingle<12>::SC>();
    static_assert(single_rec(13) && single_rec(14) && !single_rec(12), "recurrence tables for 2^13, 2^14");
    eng_single[13] = engine_info<RSingle<13>::SC, true>();  // recurrence tables (TwRec)
    eng_single[14] = engine_info<RSingle<14>::SC, true>();
    EngineInfo eng_pass[kMaxPassLog2 + 1] = {};
    eng_pass[5] = engine_info<RPass<5>::SC>();
    eng_pass[6] = engine_info<RPass<6>::SC>();
    eng_pass[7] = engine_info<RPass<7>::SC>();
    eng_pass[8] = engine_info<RPass<8>::SC>();
    uint32_t off_single[kSingleMaxLog2 + 1] = {}, off_pass[kMaxPassLog2 + 1] = {};
    size_t tw32_n = 0;
    for (int n = 1; n <= smax; ++n) {
        off_single[n] = static_cast<uint32_t>(tw32_n);
        tw32_n += (eng_single[n].tw_size + 1) & ~1;
    }
    for (int l = kMinPassLog2; l <= kMaxPassLog2; ++l) {
        off_pass[l] = static_cast<uint32_t>(tw32_n);
        tw32_n += (eng_pass[l].tw_size + 1) & ~1;
    }

    // multi-pass items: passes, workspace offsets, FP64 pass tables per (size, pass)
    struct PassTab {
        int log2m, hbits;
        uint32_t ta, tb;
    };
    std::vector<std::vector<int>> parts(kMaxLog2N + 1);
    std::vector<std::vector<PassTab>> ptab(kMaxLog2N + 1);
    size_t tw64_n = 0;
    std::vector<int64_t> wsoff(count, 0);
    int max_passes = 0;
    std::vector<int64_t> multi;
    for (int64_t i = 0; i < count; ++i) {
        if (lg[i] <= smax) continue;
        multi.push_back(i);
        const int n = lg[i];
        if (parts[n].empty()) {
            // passes of at most 2^max_pass_log2 points (and at least 2^5, at most
            // three passes, at most 2^8 points)
            int np = std::max((n + cfg.max_pass_log2 - 1) / cfg.max_pass_log2, (n + kMaxPassLog2 - 1) / kMaxPassLog2);
            np = std::min(np, std::min(kMaxPasses, n / kMinPassLog2));
            parts[n] = even_parts(n, np);
            int log2ns = 0;
            for (size_t p = 0; p < parts[n].size(); ++p) {
                PassTab t{};
                if (p > 0) {
                    t.log2m = log2ns + parts[n][p];
                    t.hbits = (t.log2m + 1) / 2;
                    t.ta = static_cast<uint32_t>(tw64_n);
                    tw64_n += size_t(1) << (t.log2m - t.hbits);
                    t.tb = static_cast<uint32_t>(tw64_n);
                    tw64_n += size_t(1) << t.hbits;
                }
                ptab[n].push_back(t);
                log2ns += parts[n][p];
            }
        }
        max_passes = std::max<int>(max_passes, static_cast<int>(parts[n].size()));
    }
    r->nmulti = static_cast<int>(multi.size());

    // ---- tiles in queue order ------------------------------------------------
    std::vector<RaggedTile>& tiles = r->htiles;
    std::vector<int64_t> toffs;
    // largest transforms first within each phase
    std::stable_sort(multi.begin(), multi.end(), [&](int64_t a, int64_t b) {
        return cfg.smallest_first ? lg[a] < lg[b] : lg[a] > lg[b];
    });
    // groups of consecutive multi-pass transforms with at most group_mib MiB
    // of workspace each (one group without pipelining); so many groups that
    // the levels would not fit are merged by growing the group size
    std::vector<size_t> group_begin;  // index into `multi` of each group's first transform
    int64_t slot_elems = 0;           // workspace elements of the largest group
    for (int64_t cap = cfg.group_mib > 0 ? (int64_t(cfg.group_mib) << 20) / int64_t(sizeof(float2)) : INT64_MAX;;
         cap *= 2) {
        group_begin.clear();
        slot_elems = 0;
        int64_t cur = 0;
        for (size_t m = 0; m < multi.size(); ++m) {
            const int64_t sz = sizes[multi[m]];
            if (group_begin.empty() || (cur > 0 && cur + sz > cap)) {
                group_begin.push_back(m);
                cur = 0;
            }
            wsoff[multi[m]] = cur;  // offset inside the group's slot
            cur += sz;
            slot_elems = std::max(slot_elems, cur);
        }
        if (group_begin.size() + std::max(max_passes, 1) - 1 <= size_t(RaggedPlan::kMaxLevels)) break;
    }
    const int ngroups = static_cast<int>(group_begin.size());
    const int slots = ngroups > 1 ? 2 : 1;  // ring: group g uses slot g % 2
    for (int gi = 0; gi < ngroups; ++gi) {
        const size_t end = gi + 1 < ngroups ? group_begin[gi + 1] : multi.size();
        for (size_t m = group_begin[gi]; m < end; ++m) wsoff[multi[m]] += int64_t(gi % 2) * slot_elems;
    }
    r->ngroups = ngroups;
    auto pass_tiles = [&](size_t p, int gi) {
        const size_t mbeg = group_begin[gi], mend = gi + 1 < ngroups ? group_begin[gi + 1] : multi.size();
        for (size_t m = mbeg; m < mend; ++m) {
            const int64_t i = multi[m];
            const int n = lg[i];
            if (p >= parts[n].size()) continue;
            const int l = parts[n][p];
            const size_t P = parts[n].size();
            int log2ns = 0;
            for (size_t q = 0; q < p; ++q) log2ns += parts[n][q];
            const uint32_t kind = p == 0 ? CODE_PASS_FIRST : (p + 1 == P ? CODE_PASS_LAST : CODE_PASS_MID);
            const int64_t ntile = int64_t(1) << (n - kTileLog2);  // columns / C = N / 8192
            const int log2c = kTileLog2 - l;
            for (int64_t c = 0; c < ntile; ++c) {
                RaggedTile t{};
                t.code = kind + static_cast<uint32_t>(l - kMinPassLog2);
                t.first = static_cast<uint32_t>(i);
                t.col = static_cast<uint32_t>(c << log2c);
                t.log2n = n;
                t.log2ns = log2ns;
                t.hbits = ptab[n][p].hbits;
                t.tw_eng = off_pass[l];
                t.ta = ptab[n][p].ta;
                t.tb = ptab[n][p].tb;
                t.uoff = offs[i];
                t.woff = wsoff[i];
                t.src = p == 0 ? 0u : ((p - 1) % 2 == 0 ? 1u : 2u);
                t.dst = p + 1 == P ? 3u : (p % 2 == 0 ? 1u : 2u);
                tiles.push_back(t);
                ++r->npass_tiles;
            }
        }
    };
    // level 0: first passes (of group 0), then the whole small transforms
    r->level_begin[0] = 0;
    if (ngroups > 0) pass_tiles(0, 0);
    for (int n = smax; n >= 0; --n) {
        std::vector<uint32_t> cls;
        for (int64_t i = 0; i < count; ++i)
            if (lg[i] == n) cls.push_back(static_cast<uint32_t>(i));
        if (cls.empty()) continue;
        const int le = std::min(single_log2e(n), n);
        const int T = 1 << (n - le);  // threads per transform
        const int G = kThreads / T;   // transforms per tile
        for (size_t s = 0; s < cls.size(); s += G) {
            RaggedTile t{};
            t.code = n == 0 ? CODE_COPY : static_cast<uint32_t>(n);
            t.first = static_cast<uint32_t>(toffs.size() + s);
            t.count = static_cast<uint32_t>(std::min<size_t>(G, cls.size() - s));
            t.log2n = n;
            t.tw_eng = n >= 1 ? off_single[n] : 0;
            tiles.push_back(t);
            if (n == 0) ++r->ncopy_tiles;
            else ++r->nsingle_tiles;
        }
        for (uint32_t i : cls) toffs.push_back(offs[i]);
        char buf[48];
        snprintf(buf, sizeof buf, "%s\"2^%d\": %zu", r->classes.empty() ? "" : ", ", n, cls.size());
        r->classes += buf;
    }
    // level k > 0: pass p of group k - p, later passes first
    r->nlevels = 1;
    const int nlev = ngroups > 0 ? ngroups + max_passes - 1 : 1;
    for (int k = 1; k < nlev; ++k) {
        r->level_begin[k] = static_cast<uint32_t>(tiles.size());
        for (int p = std::min(k, max_passes - 1); p >= 0; --p)
            if (k - p < ngroups) pass_tiles(size_t(p), k - p);
        r->nlevels = k + 1;
    }
    // the last group may lack the longest chains: drop empty trailing levels
    // (every level then has tiles, and a distinct first descriptor)
    while (r->nlevels > 1 && r->level_begin[r->nlevels - 1] == tiles.size()) --r->nlevels;
    r->level_begin[r->nlevels] = static_cast<uint32_t>(tiles.size());
    for (int l = 0; l < r->nlevels; ++l) {
        bool only = true;
        for (uint32_t i = r->level_begin[l]; i < r->level_begin[l + 1]; ++i) only = only && tiles[i].code >= CODE_PASS_FIRST;
        r->level_pass_only[l] = only;
    }
    for (int n = smax + 1; n <= kMaxLog2N; ++n) {
        int64_t c = 0;
        for (int64_t i : multi) c += lg[i] == n;
        if (!c) continue;
        char buf[48];
        snprintf(buf, sizeof buf, "%s\"2^%d\": %lld", r->classes.empty() ? "" : ", ", n, (long long)c);
        r->classes += buf;
    }

    // ---- device state ---------------------------------------------------------
    fft_status st = FFT_OK;
    e = upload(&r->tiles, tiles);
    if (e == hipSuccess) e = upload(&r->toffs, toffs);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&r->tw32), std::max<size_t>(2, tw32_n) * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&r->tw64), std::max<size_t>(2, tw64_n) * sizeof(double2));
    r->ws_half = size_t(slot_elems) * slots * sizeof(float2);
    r->ws_regions = max_passes >= 3 ? 2 : (max_passes == 2 ? 1 : 0);
    if (e == hipSuccess && r->ws_half) e = hipMalloc(&r->ws_own, r->ws_half * r->ws_regions);
    if (e != hipSuccess) {
        *detail = std::string("ragged plan allocation: ") + hipGetErrorString(e);
        (void)hipGetLastError();
        free_all(r);
        delete r;
        return FFT_ERR_ALLOC;
    }
    for (int n = 1; n <= smax && e == hipSuccess; ++n) e = launch_gen_engine_tw(eng_single[n], r->tw32 + off_single[n], 4, nullptr);
    for (int l = kMinPassLog2; l <= kMaxPassLog2 && e == hipSuccess; ++l)
        e = launch_gen_engine_tw(eng_pass[l], r->tw32 + off_pass[l], 4, nullptr);
    for (int n = smax + 1; n <= kMaxLog2N && e == hipSuccess; ++n)
        for (size_t p = 1; p < ptab[n].size() && e == hipSuccess; ++p) {
            const PassTab& t = ptab[n][p];
            e = launch_gen_pow64(r->tw64 + t.ta, t.log2m, int64_t(1) << t.hbits, int64_t(1) << (t.log2m - t.hbits),
                                 nullptr);
            if (e == hipSuccess) e = launch_gen_pow64(r->tw64 + t.tb, t.log2m, 1, int64_t(1) << t.hbits, nullptr);
        }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        st = hip_err(e, "ragged twiddle generation", detail);
        free_all(r);
        delete r;
        return st;
    }

    // persistent grids: as many workgroups as can be resident, at most one per tile
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel_for(layout == FFT_LAYOUT_SPLIT, false, false)),
                                                     kThreads, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    const int64_t want = std::max<int64_t>(1, int64_t(per_cu) * cus * cfg.grid_eighths / 8);
    for (int l = 0; l < r->nlevels; ++l) {
        const int64_t nt = int64_t(r->level_begin[l + 1]) - r->level_begin[l];
        r->level_grid[l] = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, nt)));
    }
    r->grid = r->level_grid[0];
    e = hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        st = hip_err(e, "capture stream", detail);
        free_all(r);
        delete r;
        return st;
    }
    for (int v = 0; v < 2; ++v)
        for (int l = 0; l < r->nlevels; ++l) {
            RaggedArgs& a = r->args[v][l];
            a = RaggedArgs{};
            a.tiles = r->tiles + r->level_begin[l];
            a.ntiles = r->level_begin[l + 1] - r->level_begin[l];
            a.toffs = r->toffs;
            a.tw32 = r->tw32;
            a.tw64 = r->tw64;
        }
    *out = r;
    return FFT_OK;
}

fft_status ragged_execute(RaggedPlan* r, const float* ia, const float* ib, float* oa, float* ob, bool swap,
                          hipStream_t s, std::string* detail) {
    const int v = swap ? 1 : 0;
    if (r->ws_half && !r->ws()) {
        *detail = "no workspace";
        return FFT_ERR_INVALID_ARG;
    }
    if (!r->exec[v]) {
        fft_status st = build_graph(r, v, detail);
        if (st != FFT_OK) return st;
    }
    float* wsa = static_cast<float*>(r->ws());
    float* wsb = r->ws_regions == 2 ? reinterpret_cast<float*>(static_cast<char*>(r->ws()) + r->ws_half) : wsa;
    for (int l = 0; l < r->nlevels; ++l) {
        RaggedArgs& a = r->args[v][l];
        if (a.ia == ia && a.ib == ib && a.oa == oa && a.ob == ob && a.wsa == wsa && a.wsb == wsb) continue;
        a.ia = ia;
        a.ib = ib;
        a.oa = oa;
        a.ob = ob;
        a.wsa = wsa;
        a.wsb = wsb;
        hipKernelNodeParams kp;
        hipError_t e = hipGraphKernelNodeGetParams(r->node[v][l], &kp);
        void* kparams[] = {&a};
        kp.kernelParams = kparams;
        kp.extra = nullptr;
        if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(r->exec[v], r->node[v][l], &kp);
        if (e != hipSuccess) return hip_err(e, "graph parameter update", detail);
    }
    hipError_t e = hipGraphLaunch(r->exec[v], s);
    if (e != hipSuccess) return hip_err(e, "graph launch", detail);
    return FFT_OK;
}

fft_status ragged_time(RaggedPlan* r, float* ms, std::string* detail) {
    const size_t bytes = size_t(r->total) * sizeof(float2);
    void *in = nullptr, *out = nullptr;
    hipError_t e = hipMalloc(&in, bytes);
    if (e == hipSuccess) e = hipMalloc(&out, bytes);
    if (e == hipSuccess) e = hipMemset(in, 0, bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    fft_status st = e == hipSuccess ? FFT_OK : hip_err(e, "ragged autotune scratch", detail);
    const bool split = r->layout == FFT_LAYOUT_SPLIT;
    const float* ia = static_cast<const float*>(in);
    const float* ib = split ? ia + r->total : nullptr;
    float* oa = static_cast<float*>(out);
    float* ob = split ? oa + r->total : nullptr;
    for (int i = 0; i < 2 && st == FFT_OK; ++i) st = ragged_execute(r, ia, ib, oa, ob, false, nullptr, detail);
    const int reps = 5;
    if (st == FFT_OK) {
        e = hipEventRecord(e0, nullptr);
        for (int i = 0; i < reps && st == FFT_OK; ++i) st = ragged_execute(r, ia, ib, oa, ob, false, nullptr, detail);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        *ms = t / reps;
        if (st == FFT_OK && e != hipSuccess) st = hip_err(e, "ragged autotune timing", detail);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
    return st;
}

void ragged_destroy(RaggedPlan* r) {
    if (!r) return;
    (void)hipDeviceSynchronize();
    free_all(r);
    delete r;
}

size_t ragged_workspace_bytes(const RaggedPlan* r) { return r->ws_half * r->ws_regions; }

fft_status ragged_set_workspace(RaggedPlan* r, void* dev_ptr, std::string* detail) {
    if (dev_ptr) {
        if (r->ws_own) {
            (void)hipDeviceSynchronize();
            (void)hipFree(r->ws_own);
            r->ws_own = nullptr;
        }
        r->ws_user = dev_ptr;
        return FFT_OK;
    }
    r->ws_user = nullptr;
    if (!r->ws_own && r->ws_half) {
        hipError_t e = hipMalloc(&r->ws_own, r->ws_half * r->ws_regions);
        if (e != hipSuccess) {
            *detail = "workspace allocation failed";
            (void)hipGetLastError();
            return FFT_ERR_ALLOC;
        }
    }
    return FFT_OK;
}

std::string ragged_describe(const RaggedPlan* r) {
    char buf[512];
    snprintf(buf, sizeof buf,
             "\"kernel\": \"ragged persistent\", \"transforms\": %lld, \"elements\": %lld, \"tiles\": %zu, "
             "\"single_tiles\": %d, \"pass_tiles\": %d, \"copy_tiles\": %d, \"multi_pass_transforms\": %d, "
             "\"levels\": %d, \"groups\": %d, \"workgroups\": %d, \"threads\": %d, \"lds_bytes\": %zu, "
             "\"workspace_bytes\": %zu, \"classes\": {",
             (long long)r->count, (long long)r->total, r->htiles.size(), r->nsingle_tiles, r->npass_tiles,
             r->ncopy_tiles, r->nmulti, r->nlevels, r->ngroups, r->grid, kThreads, size_t(kLds) * sizeof(float2),
             r->ws_half * r->ws_regions);
    int pass_only = 0;
    for (int l = 0; l < r->nlevels; ++l) pass_only += r->level_pass_only[l];
    return std::string(buf) + r->classes + "}, \"pass_only_levels\": " + std::to_string(pass_only) +
           ", \"config\": \"" + r->cfg.str() + "\"";
}

}  // namespace fftk
