// C ABI of the library: argument checking, plan construction (twiddle
// tables, workspace), execution and introspection.  Every entry point returns
// an fft_status; nothing throws across the boundary.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "../../include/fft.h"
#include "autotune.hpp"
#include "plan.hpp"
#include "ragged.hpp"
#include "registry.hpp"

using fftk::Decomp;

namespace {

thread_local std::string g_detail;

constexpr uint64_t kPlanMagic = 0x46465450'4c414e31ull;  // "FFTPLAN1"
constexpr uint64_t kDeadMagic = 0x44454144'504c414eull;

fft_status fail_hip(hipError_t e, const char* what) {
    g_detail = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();  // clear the sticky launch error, if any
    return FFT_ERR_HIP;
}

// Test hook: FFT_TEST_FAIL_ALLOC=k makes the k-th device allocation of the
// process (counting from 1) fail as if the device were out of memory.
hipError_t dev_malloc(void** p, size_t bytes) {
    static long countdown = [] {
        const char* s = getenv("FFT_TEST_FAIL_ALLOC");
        return s ? atol(s) : 0L;
    }();
    if (countdown > 0 && --countdown == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

struct PassStep {
    const fftk::PassKernel* k;      // forward
    const fftk::PassKernel* k_inv;  // inverse (re/im swapped at the ends)
    int log2ns;
    int hbits;
    size_t twe_off;   // engine stage table (complex entries of the plan's precision)
    size_t ta_off;    // FP64 tables (double2 entries)
    size_t tb_off;
    int src;  // 0 = caller input, 1 = workspace A, 2 = workspace B
    int dst;  // 3 = caller output, 1, 2 as above
    int grid; // persistent workgroups: resident per CU x CUs
    int ain = -1, aout = -1;  // address maps of the pass tile (-1: Stockham's own)
};

// One strided axis of a multi-dimensional plan: DFT down the columns of
// stride 2^log2s, in place on the output.
struct NdStep {
    const fftk::StridedKernel* k = nullptr;      // forward (one column pass)
    const fftk::StridedKernel* k_inv = nullptr;  // inverse (interleaved re/im swap)
    int log2s = 0;
    int64_t blocks = 0;  // column blocks: batch x the axes before this one
    size_t twe_off = 0;  // engine stage table (complex entries)
    int grid = 0;
    // long columns (l = log2 length > 0): two passes of the pass kernel along
    // the column, DFT_L with L = 2^l1 2^l2 as a Stockham chain whose Ns starts
    // at the column stride 2^log2s (the column index hidden from the pass
    // twiddles), through the plan's workspace and back
    int l = 0, l1 = 0, l2 = 0;
    const fftk::PassKernel *pa = nullptr, *pa_inv = nullptr, *pb = nullptr, *pb_inv = nullptr;
    size_t twe_a = 0, twe_b = 0, ta_off = 0, tb_off = 0;
    int hbits = 0, grid_a = 0, grid_b = 0;
};

// Column lengths that run as two passes of the pass kernel (their one-pass
// tiles would hold 8 columns or fewer): {l1, c1, l2, c2} for l = 10, 11, 12.
// Measured on MI355X: two passes win from 2^11 on, and at 2^10 for split
// arrays and FP64; interleaved FP32 columns of 2^10 are faster in one pass
// of 8-column tiles.
bool nd_two_pass_shape(int rb, int l, bool split, int* t) {
    static const int f32[3][4] = {{5, 8, 5, 8}, {6, 7, 5, 8}, {6, 7, 6, 7}};
    static const int f64[3][4] = {{5, 7, 5, 7}, {6, 6, 5, 7}, {6, 6, 6, 6}};
    if (l < 10 || l > 12 || (l == 10 && rb == 4 && !split)) return false;
    for (int i = 0; i < 4; ++i) t[i] = (rb == 8 ? f64 : f32)[l - 10][i];
    return true;
}

bool valid_layout(int l) { return l == FFT_LAYOUT_INTERLEAVED || l == FFT_LAYOUT_SPLIT; }
bool valid_dir(int d) { return d == FFT_FORWARD || d == FFT_INVERSE; }

bool overlaps(uintptr_t a, size_t na, uintptr_t b, size_t nb) { return na && nb && a < b + nb && b < a + na; }

}  // namespace

struct fft_plan_s {
    uint64_t magic = kPlanMagic;
    int device = 0;
    int64_t n = 0, batch = 0;
    int log2n = 0;
    fft_layout layout = FFT_LAYOUT_INTERLEAVED;
    fft_direction dir = FFT_FORWARD;
    int rb = 4;                                      // bytes per real: 4 (FP32) or 8 (FP64)
    Decomp dec;
    int cus = 256;                                   // compute units of the device
    const fftk::SingleKernel* single = nullptr;      // forward kernel
    const fftk::SingleKernel* single_inv = nullptr;  // inverse kernel
    std::vector<PassStep> steps;
    std::vector<int> ops_r;        // per-operator baseline: radices (log2), outermost first
    std::vector<size_t> ops_doff;  // offsets (complex entries) of the Mul diagonals in twe
    void* twe = nullptr;   // engine stage tables (float2 or double2)
    size_t twe_n = 0;
    double2* tw64 = nullptr;
    size_t tw64_n = 0;
    void* ws_own = nullptr;
    void* ws_user = nullptr;
    size_t ws_bytes = 0;
    int64_t elements = 0;
    double flops = 0.0;
    fftk::RaggedPlan* ragged = nullptr;
    std::string source;  // "default" | "cache" | "autotune"
    // real-input plans: R2C (dir FORWARD) or C2R (dir INVERSE) of n real points
    // through the half length H = n/2 (log2h); `dec` describes the half length
    bool real = false;
    int log2h = 0;
    const fftk::RealKernel* rk = nullptr;      // single-pass kernel
    const fftk::RealKernel* rk_adj = nullptr;  // the same shape in the other direction (backward)
    void* twn = nullptr;                   // w_n^k, k < H, in the plan's precision
    size_t rta_off = 0, rtb_off = 0;       // FP64 tables of w_n (pre/post pass)
    int rhbits = 0;
    // multi-dimensional plans: the last axis by `inner` (a 1D plan over
    // batch x the other axes), every other axis by a column pass in place
    int rank = 1;
    int64_t dims[3] = {0, 0, 0};
    fft_plan_s* inner = nullptr;
    std::vector<NdStep> nd;

    void* ws() const { return ws_user ? ws_user : ws_own; }
    size_t cbytes() const { return 2 * size_t(rb); }  // bytes per complex element
    bool nd_own_ws() const {  // a multi-dimensional plan whose column passes need a workspace
        for (const NdStep& q : nd)
            if (q.l) return true;
        return false;
    }
};

namespace {

bool plan_ok(fft_plan p) { return p && p->magic == kPlanMagic; }

void free_plan_memory(fft_plan p) {
    if (p->twe) (void)hipFree(p->twe);
    if (p->tw64) (void)hipFree(p->tw64);
    if (p->ws_own) (void)hipFree(p->ws_own);
    p->twe = nullptr;
    p->tw64 = nullptr;
    p->ws_own = nullptr;
    if (p->twn) (void)hipFree(p->twn);
    p->twn = nullptr;
    if (p->inner) {
        free_plan_memory(p->inner);
        p->inner->magic = kDeadMagic;
        delete p->inner;
        p->inner = nullptr;
    }
    if (p->ragged) fftk::ragged_destroy(p->ragged);
    p->ragged = nullptr;
}

// Pass i of the P-pass chain `dec` (sub-FFT Ns = 2^log2ns): kernels for the
// two directions, persistent grid, and the table offsets it appends to the
// plan's engine and FP64 twiddle tables.  src/dst are left to the caller.
fft_status make_pass_step(fft_plan p, const Decomp& dec, size_t i, int log2ns, bool split, bool inverse_only,
                          PassStep* st) {
    const size_t P = dec.log2l.size();
    *st = PassStep{};
    st->k = fftk::pass_kernel_for(p->rb, dec.log2l[i], dec.log2c[i], i, P, split, inverse_only);
    st->k_inv = inverse_only ? st->k : fftk::pass_kernel_for(p->rb, dec.log2l[i], dec.log2c[i], i, P, split, true);
    if (!st->k || !st->k_inv) return FFT_ERR_NOT_SUPPORTED;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, st->k->kernel, st->k->threads, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    st->grid = per_cu * p->cus;
    st->log2ns = log2ns;
    st->twe_off = p->twe_n;
    p->twe_n += (st->k->eng.tw_size + 1) & ~size_t(1);  // keep 16-byte alignment
    if (i > 0) {
        const int log2m = log2ns + dec.log2l[i];
        st->hbits = (log2m + 1) / 2;
        st->ta_off = p->tw64_n;
        p->tw64_n += size_t(1) << (log2m - st->hbits);
        st->tb_off = p->tw64_n;
        p->tw64_n += size_t(1) << st->hbits;
    }
    return FFT_OK;
}

// Resolve kernels, lay out the tables and the workspace for `dec`.
fft_status resolve(fft_plan p, const Decomp& dec) {
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    p->dec = dec;
    p->single = nullptr;
    p->single_inv = nullptr;
    p->steps.clear();
    p->twe_n = 0;
    p->tw64_n = 0;
    p->ws_bytes = 0;
    p->ops_r.clear();
    p->ops_doff.clear();
    switch (dec.kind) {
        case Decomp::COPY:
            break;
        case Decomp::OPS: {
            // one Mul diagonal of n_l entries per level l < L - 1
            p->ops_r = fftk::ops_radices(p->log2n, dec.log2r);
            int log2nl = p->log2n;
            for (size_t l = 0; l + 1 < p->ops_r.size(); ++l) {
                p->ops_doff.push_back(p->twe_n);
                p->twe_n += size_t(1) << log2nl;
                log2nl -= p->ops_r[l];
            }
            p->ws_bytes = 2 * size_t(p->n) * size_t(p->batch) * p->cbytes();
            break;
        }
        case Decomp::SINGLE:
            p->single = fftk::single_kernel_for(p->rb, p->log2n, dec, split, false);
            p->single_inv = fftk::single_kernel_for(p->rb, p->log2n, dec, split, true);
            if (!p->single || !p->single_inv) return FFT_ERR_NOT_SUPPORTED;
            p->twe_n = p->single->eng.tw_size;
            break;
        case Decomp::MULTI: {
            const size_t P = dec.log2l.size();
            int log2ns = 0, halves = 0;
            for (size_t i = 0; i < P; ++i) {
                PassStep st;
                const bool first = i == 0, last = i == P - 1;
                const fft_status rs = make_pass_step(p, dec, i, log2ns, split, false, &st);
                if (rs != FFT_OK) return rs;
                // ping-pong between two workspace halves; the last pass writes
                // the output.  An in-place penultimate pass (P >= 3) writes
                // over its own input, and the last pass reads it with the
                // address map of that layout (ain = log2 of the penultimate
                // pass's Ns), so a three-pass chain needs one half only.
                const int prev_dst = i == 0 ? 0 : p->steps.back().dst;
                st.src = prev_dst;
                if (dec.in_place(i)) {
                    if (P < 3 || i + 2 != P) return FFT_ERR_NOT_SUPPORTED;
                    st.dst = st.src;
                    st.ain = p->log2n - dec.log2l[i];
                    st.aout = st.ain;
                } else {
                    st.dst = last ? 3 : (prev_dst == 1 ? 2 : 1);
                }
                if (i > 0 && dec.in_place(i - 1)) st.ain = p->steps.back().log2ns;
                if (st.dst == 2 || st.src == 2) halves = 2;
                else if (halves == 0 && (st.dst == 1 || st.src == 1)) halves = 1;
                p->steps.push_back(st);
                log2ns += dec.log2l[i];
            }
            const size_t half = size_t(p->n) * size_t(p->batch) * p->cbytes();
            p->ws_bytes = size_t(halves) * half;
            break;
        }
    }
    return FFT_OK;
}

// Real plans: the half-length chain (interleaved data; R2C forward, C2R
// inverse), the fused single-pass kernel, or H = 1 (pre/post pass alone).
// Kernels of both directions are resolved: the backward (adjoint) of an R2C
// plan runs the C2R kernels and vice versa, on the same tables.
fft_status resolve_real(fft_plan p, const Decomp& dec) {
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    const bool c2r = p->dir == FFT_INVERSE;
    p->dec = dec;
    p->rk = nullptr;
    p->rk_adj = nullptr;
    p->steps.clear();
    p->twe_n = 0;
    p->tw64_n = 0;
    p->ws_bytes = 0;
    if (p->log2n == 0) return FFT_OK;  // N = 1
    const int log2nn = p->log2n;      // w_N tables, N = 2H
    auto add_wn_tables = [&]() {
        p->rhbits = (log2nn + 1) / 2;
        p->rta_off = p->tw64_n;
        p->tw64_n += size_t(1) << (log2nn - p->rhbits);
        p->rtb_off = p->tw64_n;
        p->tw64_n += size_t(1) << p->rhbits;
    };
    switch (dec.kind) {
        case Decomp::OPS:
            return FFT_ERR_NOT_SUPPORTED;
        case Decomp::COPY:
            add_wn_tables();
            break;
        case Decomp::SINGLE:
            p->rk = fftk::find_real(p->rb, p->log2h, dec.log2e, dec.wgt, c2r, split, dec.twreg, dec.stg, dec.twrec);
            p->rk_adj =
                fftk::find_real(p->rb, p->log2h, dec.log2e, dec.wgt, !c2r, split, dec.twreg, dec.stg, dec.twrec);
            if (!p->rk || !p->rk_adj) return FFT_ERR_NOT_SUPPORTED;
            p->twe_n = p->rk->eng.tw_size;
            break;
        case Decomp::MULTI: {
            const size_t P = dec.log2l.size();
            int log2ns = 0;
            for (size_t i = 0; i < P; ++i) {
                PassStep st;
                // forward kernels (R2C) and inverse kernels (C2R) of each pass;
                // the buffers of each pass are chosen at execution (run_real)
                const fft_status rs = make_pass_step(p, dec, i, log2ns, false, false, &st);
                if (rs != FFT_OK) return rs;
                // an in-place penultimate pass (src = dst at execution) and the
                // address map of the pass after it, as in complex chains
                if (dec.in_place(i)) st.ain = st.aout = p->log2h - dec.log2l[i];
                if (i > 0 && dec.in_place(i - 1)) st.ain = p->steps.back().log2ns;
                p->steps.push_back(st);
                log2ns += dec.log2l[i];
            }
            add_wn_tables();
            p->ws_bytes = 2 * (size_t(1) << p->log2h) * size_t(p->batch) * p->cbytes();
            break;
        }
    }
    return FFT_OK;
}

// Allocate and fill the twiddle tables (FP64 on the GPU, rounded once to the
// plan's precision).
fft_status build_tables(fft_plan p, hipStream_t s) {
    hipError_t e;
    if (p->twe_n) {
        e = dev_malloc(&p->twe, p->twe_n * p->cbytes());
        if (e != hipSuccess) {
            g_detail = "twiddle table allocation failed";
            return FFT_ERR_ALLOC;
        }
    }
    if (p->tw64_n) {
        e = dev_malloc(reinterpret_cast<void**>(&p->tw64), p->tw64_n * sizeof(double2));
        if (e != hipSuccess) {
            g_detail = "FP64 twiddle table allocation failed";
            return FFT_ERR_ALLOC;
        }
    }
    if (p->single && p->single->eng.tw_size) {
        e = fftk::launch_gen_engine_tw(p->single->eng, p->twe, p->rb, s);
        if (e != hipSuccess) return fail_hip(e, "twiddle generation");
    }
    {
        int log2nl = p->log2n;
        for (size_t l = 0; l < p->ops_doff.size(); ++l) {
            e = fftk::launch_gen_diag(p->rb, static_cast<char*>(p->twe) + p->ops_doff[l] * p->cbytes(), log2nl,
                                      log2nl - p->ops_r[l], s);
            if (e != hipSuccess) return fail_hip(e, "diagonal generation");
            log2nl -= p->ops_r[l];
        }
    }
    if (p->rk) {
        if (p->rk->eng.tw_size) {
            e = fftk::launch_gen_engine_tw(p->rk->eng, p->twe, p->rb, s);
            if (e != hipSuccess) return fail_hip(e, "twiddle generation");
        }
        const int64_t h = int64_t(1) << p->log2h;
        e = dev_malloc(&p->twn, size_t(h) * p->cbytes());
        if (e != hipSuccess) {
            p->twn = nullptr;
            g_detail = "twiddle table allocation failed";
            return FFT_ERR_ALLOC;
        }
        e = fftk::launch_gen_pow_round(p->twn, p->rb, p->log2n, h, s);
        if (e != hipSuccess) return fail_hip(e, "twiddle generation");
    }
    if (p->real && p->rhbits > 0) {
        e = fftk::launch_gen_pow64(p->tw64 + p->rta_off, p->log2n, int64_t(1) << p->rhbits,
                                   int64_t(1) << (p->log2n - p->rhbits), s);
        if (e == hipSuccess) e = fftk::launch_gen_pow64(p->tw64 + p->rtb_off, p->log2n, 1, int64_t(1) << p->rhbits, s);
        if (e != hipSuccess) return fail_hip(e, "FP64 twiddle generation");
    }
    for (const PassStep& st : p->steps) {
        if (st.k->eng.tw_size) {
            e = fftk::launch_gen_engine_tw(st.k->eng, static_cast<char*>(p->twe) + st.twe_off * p->cbytes(), p->rb,
                                           s);
            if (e != hipSuccess) return fail_hip(e, "twiddle generation");
        }
        if (st.log2ns > 0) {
            const int log2m = st.log2ns + st.k->log2l;
            e = fftk::launch_gen_pow64(p->tw64 + st.ta_off, log2m, int64_t(1) << st.hbits,
                                       int64_t(1) << (log2m - st.hbits), s);
            if (e == hipSuccess) e = fftk::launch_gen_pow64(p->tw64 + st.tb_off, log2m, 1, int64_t(1) << st.hbits, s);
            if (e != hipSuccess) return fail_hip(e, "FP64 twiddle generation");
        }
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "twiddle generation sync");
    return FFT_OK;
}

fft_status alloc_workspace(fft_plan p) {
    if (p->ws_bytes == 0 || p->ws_user) return FFT_OK;
    hipError_t e = dev_malloc(&p->ws_own, p->ws_bytes);
    if (e != hipSuccess) {
        p->ws_own = nullptr;
        g_detail = "workspace allocation failed";
        return FFT_ERR_ALLOC;
    }
    return FFT_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess) prev = cur;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Checks shared by execute and execute_backward (before any HIP call).
// Real plans: the real array and the complex array(s) must not overlap at all.
fft_status check_real_buffers(fft_plan p, const void* ia, const void* ib, const void* oa, const void* ob,
                              bool c2r) {
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    const void* ca = c2r ? ia : oa;  // complex side
    const void* cb = c2r ? ib : ob;
    const void* ra = c2r ? oa : ia;  // real side
    if (!ca || !ra || (split && !cb)) return FFT_ERR_NULL_POINTER;
    auto mis = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) != 0; };
    if (mis(ca) || mis(ra) || (split && mis(cb))) return FFT_ERR_MISALIGNED;
    const size_t hc = (p->n / 2 + 1) * size_t(p->batch);  // complex values per array
    const size_t rbytes = size_t(p->n) * size_t(p->batch) * size_t(p->rb);
    const size_t cbytes = split ? hc * size_t(p->rb) : hc * p->cbytes();
    if (overlaps(uintptr_t(ra), rbytes, uintptr_t(ca), cbytes)) return FFT_ERR_INVALID_ARG;
    if (split && (overlaps(uintptr_t(ra), rbytes, uintptr_t(cb), cbytes) ||
                  overlaps(uintptr_t(ca), cbytes, uintptr_t(cb), cbytes)))
        return FFT_ERR_INVALID_ARG;
    return FFT_OK;
}

// One real transform in direction c2r (the plan's own, or the other one for
// the backward); iscale scales the interior bins of the complex side (1, or
// 1/2 and 2 for the adjoints of R2C and C2R).
fft_status run_real(fft_plan p, void* wsp, const void* ia, const void* ib, void* oa, void* ob, bool c2r, double iscale,
                    hipStream_t s) {
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    hipError_t e = hipSuccess;
    if (p->log2n == 0) {
        e = fftk::launch_real1(p->rb, c2r, split, ia, ib, oa, ob, p->batch, s);
        return e == hipSuccess ? FFT_OK : fail_hip(e, "real N=1 launch");
    }
    const double2* ta = p->tw64 ? p->tw64 + p->rta_off : nullptr;
    const double2* tb = p->tw64 ? p->tw64 + p->rtb_off : nullptr;
    switch (p->dec.kind) {
        case Decomp::OPS:
            return FFT_ERR_NOT_SUPPORTED;
        case Decomp::COPY:  // H = 1: the pre/post pass is the whole transform (no interior bins)
            e = c2r ? fftk::launch_c2r_pre(p->rb, split, ia, ib, oa, ta, tb, p->rhbits, 0, p->batch, iscale, s)
                    : fftk::launch_r2c_post(p->rb, split, ia, oa, ob, ta, tb, p->rhbits, 0, p->batch, iscale, s);
            return e == hipSuccess ? FFT_OK : fail_hip(e, "real pre/post launch");
        case Decomp::SINGLE: {
            const fftk::RealKernel* k = c2r == p->rk->c2r ? p->rk : p->rk_adj;
            e = k->fn(ia, ib, oa, ob, p->twe, p->twn, p->batch, p->dec.gmul * p->cus, iscale, s);
            return e == hipSuccess ? FFT_OK : fail_hip(e, "real single-pass launch");
        }
        case Decomp::MULTI: {
            if (!wsp) {
                g_detail = "no workspace";
                return FFT_ERR_INVALID_ARG;
            }
            const size_t half = (size_t(1) << p->log2h) * size_t(p->batch) * p->cbytes();
            void* ws[3] = {nullptr, wsp, static_cast<char*>(wsp) + half};
            // buffers: 0 the caller's input, 1/2 the workspace halves, 3 the
            // caller's output; C2R starts from the pre pass's output in half 1
            int prev = 0;
            if (c2r) {
                e = fftk::launch_c2r_pre(p->rb, split, ia, ib, ws[1], ta, tb, p->rhbits, p->log2h, p->batch, iscale, s);
                if (e != hipSuccess) return fail_hip(e, "C2R pre-pass launch");
                prev = 1;
            }
            for (size_t i = 0; i < p->steps.size(); ++i) {
                const PassStep& st = p->steps[i];
                const bool in_place = st.aout >= 0 && st.aout == st.ain;  // the penultimate pass only, prev is a half
                const int dst = (c2r && i + 1 == p->steps.size()) ? 3 : in_place ? prev : (prev == 1 ? 2 : 1);
                const void* src = prev == 0 ? ia : ws[prev];
                void* out = dst == 3 ? oa : ws[dst];
                const int stream = (prev == 0 ? fftk::kStreamIn : 0) | (dst == 3 ? fftk::kStreamOut : 0);
                const fftk::PassKernel* k = c2r ? st.k_inv : st.k;
                e = k->fn(src, nullptr, out, nullptr, static_cast<const char*>(p->twe) + st.twe_off * p->cbytes(),
                          p->tw64 + st.ta_off, p->tw64 + st.tb_off, p->log2h, st.log2ns, st.hbits, p->batch,
                          st.grid, stream, 0, st.ain, st.aout, s);
                if (e != hipSuccess) return fail_hip(e, "pass launch");
                prev = dst;
            }
            if (!c2r) {
                e = fftk::launch_r2c_post(p->rb, split, ws[prev], oa, ob, ta, tb, p->rhbits, p->log2h, p->batch,
                                          iscale, s);
                if (e != hipSuccess) return fail_hip(e, "R2C post-pass launch");
            }
            return FFT_OK;
        }
    }
    return FFT_ERR_INVALID_ARG;
}

fft_status check_buffers(fft_plan p, const void* ia, const void* ib, const void* oa, const void* ob,
                         bool adjoint) {
    if (!plan_ok(p)) return FFT_ERR_INVALID_ARG;
    if (p->real) return check_real_buffers(p, ia, ib, oa, ob, (p->dir == FFT_INVERSE) != adjoint);
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    if (!ia || !oa || (split && (!ib || !ob))) return FFT_ERR_NULL_POINTER;
    auto mis = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) != 0; };
    if (mis(ia) || mis(oa) || (split && (mis(ib) || mis(ob)))) return FFT_ERR_MISALIGNED;
    const size_t elems = size_t(p->elements);
    const size_t bytes = split ? elems * size_t(p->rb) : elems * p->cbytes();
    const uintptr_t ua = uintptr_t(ia), ub = split ? uintptr_t(ib) : 0, va = uintptr_t(oa),
                    vb = split ? uintptr_t(ob) : 0;
    const size_t nb = split ? bytes : 0;
    // input/output pairs may coincide exactly (in place) or be disjoint
    if (overlaps(ua, bytes, va, bytes) && ua != va) return FFT_ERR_INVALID_ARG;
    if (split) {
        if (overlaps(ub, nb, vb, nb) && ub != vb) return FFT_ERR_INVALID_ARG;
        if (overlaps(ua, bytes, vb, nb) || overlaps(ub, nb, va, bytes)) return FFT_ERR_INVALID_ARG;
        if (overlaps(va, bytes, vb, nb)) return FFT_ERR_INVALID_ARG;
    }
    return FFT_OK;
}

// `wsp`: the workspace the passes use (the plan's own, or one the caller
// supplies for this call only: the scratch-buffer entry point)
fft_status run(fft_plan p, const void* ia, const void* ib, void* oa, void* ob, void* stream, bool adjoint,
               void* wsp = nullptr);

// Multi-dimensional: the last axis (inner 1D plan, in -> out), then the
// column passes in place on the output, last-but-one axis first.
fft_status run_nd(fft_plan p, void* wsp, const void* ia, const void* ib, void* oa, void* ob, void* stream,
                  bool adjoint, bool ws_given) {
    fft_status st = run(p->inner, ia, ib, oa, ob, stream, adjoint, ws_given ? wsp : nullptr);
    if (st != FFT_OK) return st;
    const bool inverse = (p->dir == FFT_INVERSE) != adjoint;
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    void* a = oa;
    void* b = ob;
    if (inverse && split) std::swap(a, b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (const NdStep& stp : p->nd) {
        if (stp.l) {
            // out -> workspace -> out; the pass twiddles see the column's own index only
            if (!wsp) {
                g_detail = "no workspace";
                return FFT_ERR_INVALID_ARG;
            }
            const fftk::PassKernel* ka = inverse && !split ? stp.pa_inv : stp.pa;
            const fftk::PassKernel* kb = inverse && !split ? stp.pb_inv : stp.pb;
            const char* twe = static_cast<const char*>(p->twe);
            const double2* ta = p->tw64 + stp.ta_off;
            const double2* tb = p->tw64 + stp.tb_off;
            const int log2n = stp.l + stp.log2s;
            // the first column step reads what the last-axis plan has just
            // streamed out (not cached): streaming loads there measured
            // faster (4096 x 4096 interleaved: 307 -> 277 us); a later step
            // reads what the step before it left in the cache
            const int in_stream = &stp == &p->nd.front() ? fftk::kStreamIn : 0;
            hipError_t e = ka->fn(a, b, wsp, nullptr, twe + stp.twe_a * p->cbytes(), ta, tb, log2n, stp.log2s,
                                  stp.hbits, stp.blocks, stp.grid_a, in_stream, stp.log2s, -1, -1, s);
            if (e == hipSuccess)
                e = kb->fn(wsp, nullptr, a, b, twe + stp.twe_b * p->cbytes(), ta, tb, log2n, stp.log2s + stp.l1,
                           stp.hbits, stp.blocks, stp.grid_b, fftk::kStreamOut, stp.log2s, -1, -1, s);
            if (e != hipSuccess) return fail_hip(e, "column pass launch");
            continue;
        }
        const fftk::StridedKernel* k = inverse && !split ? stp.k_inv : stp.k;
        const hipError_t e = k->fn(a, b, a, b, static_cast<const char*>(p->twe) + stp.twe_off * p->cbytes(), stp.log2s,
                                   stp.blocks, stp.grid, s);
        if (e != hipSuccess) return fail_hip(e, "column pass launch");
    }
    return FFT_OK;
}

fft_status run(fft_plan p, const void* ia, const void* ib, void* oa, void* ob, void* stream, bool adjoint,
               void* wsp) {
    fft_status st = check_buffers(p, ia, ib, oa, ob, adjoint);
    if (st != FFT_OK) return st;
    DeviceGuard guard(p->device);
    const bool ws_given = wsp != nullptr;
    if (!ws_given) wsp = p->ws();
    if (p->rank > 1) return run_nd(p, wsp, ia, ib, oa, ob, stream, adjoint, ws_given);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->real) {
        // the backward of R2C is C2R with the interior bins halved, of C2R
        // R2C with them doubled (the adjoints under the real inner product)
        const bool c2r = (p->dir == FFT_INVERSE) != adjoint;
        return run_real(p, wsp, ia, ib, oa, ob, c2r, adjoint ? (c2r ? 0.5 : 2.0) : 1.0, s);
    }
    // forward kernels everywhere; the inverse swaps re and im on the way in and
    // out: split arrays by exchanging the pointers, interleaved data in-kernel
    const bool inverse = (p->dir == FFT_INVERSE) != adjoint;
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    const void* fa = ia;
    const void* fb = ib;
    void* ga = oa;
    void* gb = ob;
    if (inverse && split) {
        std::swap(fa, fb);
        std::swap(ga, gb);
    }
    hipError_t e = hipSuccess;

    if (p->ragged)
        return fftk::ragged_execute(p->ragged, static_cast<const float*>(fa), static_cast<const float*>(fb),
                                    static_cast<float*>(ga), static_cast<float*>(gb), inverse && !split, s,
                                    &g_detail);

    switch (p->dec.kind) {
        case Decomp::COPY: {
            if (ia == oa && (!split || ib == ob)) return FFT_OK;
            const size_t bytes = size_t(p->elements) * (split ? size_t(p->rb) : p->cbytes());
            e = hipMemcpyAsync(oa, ia, bytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && split) e = hipMemcpyAsync(ob, ib, bytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail_hip(e, "copy");
            return FFT_OK;
        }
        case Decomp::OPS: {
            // Permute for l = 0 .. L-2, innermost DFT blocks, then Mul and
            // FusedMKIV for l = L-2 .. 0; ping-pong through the workspace
            if (!wsp) {
                g_detail = "no workspace";
                return FFT_ERR_INVALID_ARG;
            }
            const size_t full = size_t(p->n) * size_t(p->batch) * p->cbytes();
            void* buf[2] = {wsp, static_cast<char*>(wsp) + full};
            const int L = static_cast<int>(p->ops_r.size());
            const int nops = 3 * L - 2;
            int done = 0, cur = -1;  // cur = -1: the caller's input
            auto src = [&]() -> const void* { return cur < 0 ? ia : buf[cur]; };
            auto dst = [&]() -> void* { return done + 1 == nops ? oa : buf[cur < 0 ? 0 : 1 - cur]; };
            auto step = [&]() { cur = cur < 0 ? 0 : 1 - cur; ++done; };
            int64_t a = p->batch;
            int log2nl = p->log2n;
            for (int l = 0; l + 1 < L; ++l) {
                e = fftk::launch_op_perm(p->rb, src(), dst(), a, log2nl - p->ops_r[l], p->ops_r[l],
                                         inverse && done == 0, s);
                if (e != hipSuccess) return fail_hip(e, "Permute launch");
                step();
                a <<= p->ops_r[l];
                log2nl -= p->ops_r[l];
            }
            e = fftk::launch_op_kron(p->rb, p->ops_r[L - 1], src(), dst(), a, 1, inverse && done == 0,
                                     inverse && done + 1 == nops, s);
            if (e != hipSuccess) return fail_hip(e, "FusedIKMV launch");
            step();
            for (int l = L - 2; l >= 0; --l) {
                a >>= p->ops_r[l];
                log2nl += p->ops_r[l];
                e = fftk::launch_op_mul(p->rb, src(), dst(), static_cast<const char*>(p->twe) + p->ops_doff[l] * p->cbytes(),
                                        a, log2nl, s);
                if (e != hipSuccess) return fail_hip(e, "Mul launch");
                step();
                e = fftk::launch_op_kron(p->rb, p->ops_r[l], src(), dst(), a, int64_t(1) << (log2nl - p->ops_r[l]),
                                         false, inverse && done + 1 == nops, s);
                if (e != hipSuccess) return fail_hip(e, "FusedMKIV launch");
                step();
            }
            return FFT_OK;
        }
        case Decomp::SINGLE: {
            const fftk::SingleKernel* k = inverse ? p->single_inv : p->single;
            e = k->fn(fa, fb, ga, gb, p->twe, p->batch, p->dec.gmul * p->cus, s);
            if (e != hipSuccess) return fail_hip(e, "single-pass launch");
            return FFT_OK;
        }
        case Decomp::MULTI: {
            if (!wsp) {
                g_detail = "no workspace";
                return FFT_ERR_INVALID_ARG;
            }
            const size_t half = size_t(p->n) * size_t(p->batch) * p->cbytes();
            void* wsa = wsp;
            void* wsb = static_cast<char*>(wsp) + half;
            const size_t P = p->steps.size();
            for (size_t i = 0; i < P; ++i) {
                const PassStep& stp = p->steps[i];
                const void *sa = nullptr, *sb = nullptr;
                void *da = nullptr, *db = nullptr;
                if (stp.src == 0) {
                    sa = fa;
                    sb = fb;
                } else {
                    sa = stp.src == 1 ? wsa : wsb;
                }
                if (stp.dst == 3) {
                    da = ga;
                    db = gb;
                } else {
                    da = stp.dst == 1 ? wsa : wsb;
                }
                const fftk::PassKernel* k = inverse ? stp.k_inv : stp.k;
                // the caller's buffers are streamed; the workspace between
                // passes stays cacheable for the next pass
                const int stream = (stp.src == 0 ? fftk::kStreamIn : 0) | (stp.dst == 3 ? fftk::kStreamOut : 0);
                e = k->fn(sa, sb, da, db, static_cast<const char*>(p->twe) + stp.twe_off * p->cbytes(),
                          p->tw64 ? p->tw64 + stp.ta_off : nullptr,
                          p->tw64 ? p->tw64 + stp.tb_off : nullptr, p->log2n, stp.log2ns, stp.hbits, p->batch,
                          stp.grid, stream, 0, stp.ain, stp.aout, s);
                if (e != hipSuccess) return fail_hip(e, "pass launch");
            }
            (void)split;
            return FFT_OK;
        }
    }
    return FFT_ERR_INVALID_ARG;
}

std::string describe(fft_plan p) {
    char buf[512];
    std::string s = "{";
    snprintf(buf, sizeof buf,
             "\"n\": %lld, \"batch\": %lld, \"layout\": \"%s\", \"direction\": \"%s\", \"precision\": \"%s\", ",
             (long long)p->n, (long long)p->batch, p->layout == FFT_LAYOUT_SPLIT ? "split" : "interleaved",
             p->dir == FFT_FORWARD ? "forward" : "inverse", p->rb == 8 ? "fp64" : "fp32");
    s += buf;
    if (p->ragged) {
        s += fftk::ragged_describe(p->ragged);
        s += ", \"source\": \"" + p->source + "\"}";
        return s;
    }
    if (p->rank > 1) {
        std::string d, cols;
        for (int i = 0; i < p->rank; ++i) d += (i ? ", " : "") + std::to_string(p->dims[i]);
        for (size_t i = 0; i < p->nd.size(); ++i) {
            const NdStep& st = p->nd[i];
            if (st.l)
                snprintf(buf, sizeof buf,
                         "%s{\"length\": %d, \"stride\": %lld, \"passes\": [\"%dc%d\", \"%dc%d\"]}", i ? ", " : "",
                         1 << st.l, (long long)(int64_t(1) << st.log2s), st.l1, st.pa->log2c, st.l2, st.pb->log2c);
            else
                snprintf(buf, sizeof buf, "%s{\"length\": %d, \"stride\": %lld, \"columns_per_wg\": %d}",
                         i ? ", " : "", 1 << st.k->log2l, (long long)(int64_t(1) << st.log2s), 1 << st.k->log2c);
            cols += buf;
        }
        s += "\"rank\": " + std::to_string(p->rank) + ", \"dims\": [" + d + "], \"last_axis\": " + describe(p->inner) +
             ", \"column_passes\": [" + cols + "], \"workspace_bytes\": " + std::to_string(p->ws_bytes) + "}";
        return s;
    }
    if (p->real) {
        snprintf(buf, sizeof buf, "\"real\": \"%s\", \"half_length\": %lld, ", p->dir == FFT_INVERSE ? "c2r" : "r2c",
                 (long long)(p->log2n ? int64_t(1) << p->log2h : 0));
        s += buf;
    }
    snprintf(buf, sizeof buf, "\"decomposition\": \"%s\", \"source\": \"%s\", \"workspace_bytes\": %zu",
             p->log2n == 0 && p->real ? "n1" : p->dec.str().c_str(), p->source.c_str(), p->ws_bytes);
    s += buf;
    if (p->rk) {
        std::string radices;
        for (int i = 0; i < p->rk->eng.nst; ++i) radices += (i ? "," : "") + std::to_string(1 << p->rk->eng.log2r[i]);
        snprintf(buf, sizeof buf,
                 ", \"kernel\": \"real-single\", \"radices\": [%s], \"threads\": %d, \"transforms_per_wg\": %d, "
                 "\"lds_bytes\": %zu",
                 radices.c_str(), p->rk->threads, p->rk->per_wg, p->rk->lds_bytes);
        s += buf;
    }
    if (p->single) {
        std::string radices;
        for (int i = 0; i < p->single->eng.nst; ++i)
            radices += (i ? "," : "") + std::to_string(1 << p->single->eng.log2r[i]);
        snprintf(buf, sizeof buf,
                 ", \"kernel\": \"single\", \"radices\": [%s], \"threads\": %d, \"transforms_per_wg\": %d, "
                 "\"lds_bytes\": %zu",
                 radices.c_str(), p->single->threads, p->single->per_wg, p->single->lds_bytes);
        s += buf;
    }
    if (!p->steps.empty()) {
        s += ", \"passes\": [";
        for (size_t i = 0; i < p->steps.size(); ++i) {
            const auto& st = p->steps[i];
            std::string radices;
            for (int j = 0; j < st.k->eng.nst; ++j) radices += (j ? "," : "") + std::to_string(1 << st.k->eng.log2r[j]);
            snprintf(buf, sizeof buf,
                     "%s{\"L\": %d, \"columns\": %d, \"Ns\": %lld, \"radices\": [%s], \"threads\": %d, "
                     "\"lds_bytes\": %zu}",
                     i ? ", " : "", 1 << st.k->log2l, 1 << st.k->log2c, (long long)(int64_t(1) << st.log2ns),
                     radices.c_str(), st.k->threads, st.k->lds_bytes);
            s += buf;
        }
        s += "]";
    }
    s += "}";
    return s;
}

fft_status copy_out(const std::string& s, char* buf, size_t len) {
    if (!buf || len == 0) return FFT_ERR_NULL_POINTER;
    const size_t n = s.size() < len - 1 ? s.size() : len - 1;
    memcpy(buf, s.data(), n);
    buf[n] = '\0';
    return FFT_OK;
}

double nominal_flops(int64_t n) {
    int k = fftk::ilog2_exact(n);
    return k <= 0 ? 0.0 : 5.0 * double(n) * double(k);
}

}  // namespace

extern "C" {

static fft_status create_impl(fft_plan* out, int64_t n, int64_t batch, fft_layout layout, fft_direction dir,
                              fft_precision precision, const char* explicit_dec) {
    if (!out) return FFT_ERR_NULL_POINTER;
    *out = nullptr;
    const int log2n = fftk::ilog2_exact(n);
    if (log2n < 0 || log2n > fftk::kMaxLog2N) return FFT_ERR_INVALID_SIZE;
    const int rb = fftk::real_bytes_of(precision);
    if (batch < 1 || !valid_layout(layout) || !valid_dir(dir) || rb == 0) return FFT_ERR_INVALID_ARG;
    if (batch > (int64_t(1) << 40) / n) return FFT_ERR_INVALID_ARG;  // element count bound
    Decomp forced;
    if (explicit_dec) {
        if (!Decomp::parse(explicit_dec, &forced)) return FFT_ERR_INVALID_ARG;
        if (!fftk::decomposition_available(forced, log2n, layout, rb)) return FFT_ERR_NOT_SUPPORTED;
    }

    fft_plan p = new (std::nothrow) fft_plan_s;
    if (!p) return FFT_ERR_ALLOC;
    p->n = n;
    p->batch = batch;
    p->log2n = log2n;
    p->layout = layout;
    p->dir = dir;
    p->rb = rb;
    p->elements = n * batch;
    p->flops = nominal_flops(n) * double(batch);
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "hipGetDevice");
    }

    Decomp dec = fftk::default_decomposition(log2n, rb, layout, batch);
    p->source = "default";
    fftk::TuneKey key = fftk::make_key(p->device, log2n, batch, layout, rb);
    Decomp cached;
    if (explicit_dec) {
        dec = forced;
        p->source = "explicit";
    } else if (fftk::autotune_lookup(key, &cached) && fftk::decomposition_available(cached, log2n, layout, rb)) {
        dec = cached;
        p->source = "cache";
    }
    fft_status st = resolve(p, dec);
    if (st == FFT_OK) st = build_tables(p, nullptr);
    if (st == FFT_OK) st = alloc_workspace(p);
    if (st == FFT_OK && !explicit_dec && fftk::autotune_enabled() && p->source != "cache") {
        // time every candidate on scratch buffers and keep the fastest
        Decomp best;
        st = fftk::autotune_run(p, key, &best, &g_detail);
        if (st == FFT_OK && !(best == p->dec)) {
            free_plan_memory(p);
            st = resolve(p, best);
            if (st == FFT_OK) st = build_tables(p, nullptr);
            if (st == FFT_OK) st = alloc_workspace(p);
        }
        p->source = "autotune";
    }
    if (st != FFT_OK) {
        free_plan_memory(p);
        p->magic = kDeadMagic;
        delete p;
        return st;
    }
    *out = p;
    return FFT_OK;
}

fft_status fft_plan_create(fft_plan* out, int64_t n, int64_t batch, fft_layout layout, fft_direction dir) {
    return create_impl(out, n, batch, layout, dir, FFT_PRECISION_FP32, nullptr);
}

fft_status fft_plan_create_explicit(fft_plan* out, int64_t n, int64_t batch, fft_layout layout, fft_direction dir,
                                    const char* decomposition) {
    if (!decomposition) return FFT_ERR_NULL_POINTER;
    return create_impl(out, n, batch, layout, dir, FFT_PRECISION_FP32, decomposition);
}

fft_status fft_plan_create_ex(fft_plan* out, int64_t n, int64_t batch, fft_layout layout, fft_direction dir,
                              fft_precision precision, const char* decomposition) {
    return create_impl(out, n, batch, layout, dir, precision, decomposition);
}

fft_status fft_plan_create_nd(fft_plan* out, int rank, const int64_t* dims, int64_t batch, fft_layout layout,
                              fft_direction dir, fft_precision precision) {
    if (!out) return FFT_ERR_NULL_POINTER;
    *out = nullptr;
    if (!dims) return FFT_ERR_NULL_POINTER;
    if (rank < 1 || rank > 3) return FFT_ERR_INVALID_ARG;
    int log2d[3] = {0, 0, 0};
    int log2total = 0;
    for (int i = 0; i < rank; ++i) {
        log2d[i] = fftk::ilog2_exact(dims[i]);
        if (log2d[i] < 0) return FFT_ERR_INVALID_SIZE;
        if (i + 1 < rank && log2d[i] > fftk::kMaxStridedLog2) return FFT_ERR_INVALID_SIZE;
        if (i + 1 == rank && log2d[i] > fftk::kMaxLog2N) return FFT_ERR_INVALID_SIZE;
        log2total += log2d[i];
    }
    const int rb = fftk::real_bytes_of(precision);
    if (batch < 1 || !valid_layout(layout) || !valid_dir(dir) || rb == 0) return FFT_ERR_INVALID_ARG;
    if (log2total > 40 || batch > (int64_t(1) << (40 - log2total))) return FFT_ERR_INVALID_ARG;
    if (rank == 1) return create_impl(out, dims[0], batch, layout, dir, precision, nullptr);
    const bool split = layout == FFT_LAYOUT_SPLIT;
    // kernels of the strided axes (checked before any allocation)
    std::vector<NdStep> steps;
    for (int k = rank - 2; k >= 0; --k) {
        if (log2d[k] == 0) continue;
        int log2s = 0;
        for (int j = k + 1; j < rank; ++j) log2s += log2d[j];
        NdStep st{};
        int sh[4];
        const int l = log2d[k];
        if (nd_two_pass_shape(rb, l, split, sh) && l + log2s >= sh[0] + sh[1] && l + log2s >= sh[2] + sh[3]) {
            st.pa = fftk::find_pass(rb, sh[0], sh[1], false, split, false, false, false);
            st.pa_inv = split ? st.pa : fftk::find_pass(rb, sh[0], sh[1], false, false, false, true, false);
            st.pb = fftk::find_pass(rb, sh[2], sh[3], false, false, split, false, false);
            st.pb_inv = split ? st.pb : fftk::find_pass(rb, sh[2], sh[3], false, false, false, false, true);
            if (st.pa && st.pa_inv && st.pb && st.pb_inv) {
                st.l = l;
                st.l1 = sh[0];
                st.l2 = sh[2];
            }
        }
        if (!st.l) {
            st.k = fftk::strided_kernel_for(rb, log2d[k], log2s, split, false);
            st.k_inv = split ? st.k : fftk::strided_kernel_for(rb, log2d[k], log2s, split, true);
            if (!st.k || !st.k_inv) return FFT_ERR_NOT_SUPPORTED;
        }
        st.log2s = log2s;
        st.blocks = batch;
        for (int j = 0; j < k; ++j) st.blocks *= dims[j];
        steps.push_back(st);
    }
    fft_plan p = new (std::nothrow) fft_plan_s;
    if (!p) return FFT_ERR_ALLOC;
    p->rank = rank;
    for (int i = 0; i < rank; ++i) p->dims[i] = dims[i];
    p->n = int64_t(1) << log2total;
    p->log2n = log2total;
    p->batch = batch;
    p->layout = layout;
    p->dir = dir;
    p->rb = rb;
    p->elements = p->n * batch;
    p->flops = nominal_flops(p->n) * double(batch);
    p->source = "nd";
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "hipGetDevice");
    }
    fft_status st = create_impl(&p->inner, dims[rank - 1], p->elements / dims[rank - 1], layout, dir, precision,
                                nullptr);
    if (st == FFT_OK) {
        auto occupancy_grid = [&](const void* kernel, int threads) {
            int per_cu = 1;
            if (kernel && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
                           per_cu < 1))
                per_cu = 1;
            return per_cu * p->cus;
        };
        bool two_pass = false;
        for (NdStep& stp : steps) {
            if (stp.l) {
                two_pass = true;
                stp.twe_a = p->twe_n;
                p->twe_n += (stp.pa->eng.tw_size + 1) & ~size_t(1);
                stp.twe_b = p->twe_n;
                p->twe_n += (stp.pb->eng.tw_size + 1) & ~size_t(1);
                stp.hbits = (stp.l + 1) / 2;  // pass twiddles w_L^e = A[e >> hbits] B[e & mask]
                stp.ta_off = p->tw64_n;
                p->tw64_n += size_t(1) << (stp.l - stp.hbits);
                stp.tb_off = p->tw64_n;
                p->tw64_n += size_t(1) << stp.hbits;
                stp.grid_a = occupancy_grid(stp.pa->kernel, stp.pa->threads);
                stp.grid_b = occupancy_grid(stp.pb->kernel, stp.pb->threads);
                continue;
            }
            stp.twe_off = p->twe_n;
            p->twe_n += (stp.k->eng.tw_size + 1) & ~size_t(1);
            stp.grid = occupancy_grid(stp.k->kernel, stp.k->threads);
        }
        p->nd = steps;
        if (p->twe_n) {
            e = dev_malloc(&p->twe, p->twe_n * p->cbytes());
            if (e != hipSuccess) {
                p->twe = nullptr;
                g_detail = "twiddle table allocation failed";
                st = FFT_ERR_ALLOC;
            }
        }
        if (st == FFT_OK && p->tw64_n) {
            e = dev_malloc(reinterpret_cast<void**>(&p->tw64), p->tw64_n * sizeof(double2));
            if (e != hipSuccess) {
                p->tw64 = nullptr;
                g_detail = "twiddle table allocation failed";
                st = FFT_ERR_ALLOC;
            }
        }
        char* twe = static_cast<char*>(p->twe);
        for (size_t i = 0; st == FFT_OK && i < p->nd.size(); ++i) {
            const NdStep& q = p->nd[i];
            if (q.l) {
                if (q.pa->eng.tw_size) e = fftk::launch_gen_engine_tw(q.pa->eng, twe + q.twe_a * p->cbytes(), rb, nullptr);
                if (e == hipSuccess && q.pb->eng.tw_size)
                    e = fftk::launch_gen_engine_tw(q.pb->eng, twe + q.twe_b * p->cbytes(), rb, nullptr);
                if (e == hipSuccess)
                    e = fftk::launch_gen_pow64(p->tw64 + q.ta_off, q.l, int64_t(1) << q.hbits,
                                               int64_t(1) << (q.l - q.hbits), nullptr);
                if (e == hipSuccess) e = fftk::launch_gen_pow64(p->tw64 + q.tb_off, q.l, 1, int64_t(1) << q.hbits, nullptr);
            } else if (q.k->eng.tw_size) {
                e = fftk::launch_gen_engine_tw(q.k->eng, twe + q.twe_off * p->cbytes(), rb, nullptr);
            }
            if (e != hipSuccess) st = fail_hip(e, "twiddle generation");
        }
        if (st == FFT_OK) {
            e = hipStreamSynchronize(nullptr);
            if (e != hipSuccess) st = fail_hip(e, "twiddle generation sync");
        }
        // the workspace: the last-axis plan's, or with two-pass columns one of
        // the whole array that the last-axis plan shares (it runs first)
        p->ws_bytes = p->inner ? p->inner->ws_bytes : 0;
        if (st == FFT_OK && two_pass) {
            p->ws_bytes = std::max(p->ws_bytes, size_t(p->elements) * p->cbytes());
            st = alloc_workspace(p);
            if (st == FFT_OK && p->inner->ws_bytes) st = fft_plan_set_workspace(p->inner, p->ws());
        }
    }
    if (st != FFT_OK) {
        free_plan_memory(p);
        p->magic = kDeadMagic;
        delete p;
        return st;
    }
    *out = p;
    return FFT_OK;
}

fft_status fft_plan_create_real(fft_plan* out, int64_t n, int64_t batch, fft_layout layout, fft_direction dir,
                                fft_precision precision, const char* decomposition) {
    if (!out) return FFT_ERR_NULL_POINTER;
    *out = nullptr;
    const int log2n = fftk::ilog2_exact(n);
    if (log2n < 0 || log2n > fftk::kMaxLog2N) return FFT_ERR_INVALID_SIZE;
    const int rb = fftk::real_bytes_of(precision);
    if (batch < 1 || !valid_layout(layout) || !valid_dir(dir) || rb == 0) return FFT_ERR_INVALID_ARG;
    if (batch > (int64_t(1) << 40) / n) return FFT_ERR_INVALID_ARG;
    const bool c2r = dir == FFT_INVERSE;
    Decomp dec;
    if (log2n >= 1) {
        if (decomposition) {
            if (!Decomp::parse(decomposition, &dec)) return FFT_ERR_INVALID_ARG;
            if (!fftk::real_decomposition_available(dec, log2n, layout, rb, c2r)) return FFT_ERR_NOT_SUPPORTED;
        } else {
            dec = fftk::default_real_decomposition(log2n, rb);
            if (!fftk::real_decomposition_available(dec, log2n, layout, rb, c2r)) return FFT_ERR_NOT_SUPPORTED;
        }
    } else if (decomposition) {
        return FFT_ERR_NOT_SUPPORTED;  // N = 1 has no decomposition
    }
    fft_plan p = new (std::nothrow) fft_plan_s;
    if (!p) return FFT_ERR_ALLOC;
    p->n = n;
    p->batch = batch;
    p->log2n = log2n;
    p->log2h = log2n > 0 ? log2n - 1 : 0;
    p->layout = layout;
    p->dir = dir;
    p->rb = rb;
    p->real = true;
    p->elements = n * batch;
    p->flops = 0.5 * nominal_flops(n) * double(batch);
    p->source = decomposition ? "explicit" : "default";
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "hipGetDevice");
    }
    fft_status st = resolve_real(p, dec);
    if (st == FFT_OK) st = build_tables(p, nullptr);
    if (st == FFT_OK) st = alloc_workspace(p);
    if (st != FFT_OK) {
        free_plan_memory(p);
        p->magic = kDeadMagic;
        delete p;
        return st;
    }
    *out = p;
    return FFT_OK;
}

fft_status fft_execute(fft_plan p, const void* in_re_or_z, const void* in_im, void* out_re_or_z, void* out_im,
                       void* stream) {
    return run(p, in_re_or_z, in_im, out_re_or_z, out_im, stream, false);
}

fft_status fft_execute_backward(fft_plan p, const void* grad_out_re_or_z, const void* grad_out_im,
                                void* grad_in_re_or_z, void* grad_in_im, void* stream) {
    return run(p, grad_out_re_or_z, grad_out_im, grad_in_re_or_z, grad_in_im, stream, true);
}

fft_status fft_plan_destroy(fft_plan p) {
    if (!p) return FFT_OK;
    if (!plan_ok(p)) return FFT_ERR_INVALID_ARG;
    DeviceGuard guard(p->device);
    (void)hipDeviceSynchronize();
    free_plan_memory(p);
    p->magic = kDeadMagic;
    delete p;
    return FFT_OK;
}

static fft_status create_ragged_impl(fft_plan* out, const int64_t* sizes, int64_t count, fft_layout layout,
                                     fft_direction dir, const char* config) {
    if (!out) return FFT_ERR_NULL_POINTER;
    *out = nullptr;
    if (!sizes) return FFT_ERR_NULL_POINTER;
    if (count < 1 || !valid_layout(layout) || !valid_dir(dir)) return FFT_ERR_INVALID_ARG;
    fftk::RaggedConfig explicit_cfg;
    if (config && !fftk::RaggedConfig::parse(config, &explicit_cfg)) {
        g_detail = std::string("unknown ragged configuration: ") + config;
        return FFT_ERR_INVALID_ARG;
    }
    int64_t total = 0;
    double flops = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        const int k = fftk::ilog2_exact(sizes[i]);
        if (k < 0 || k > fftk::kMaxLog2N) return FFT_ERR_INVALID_SIZE;
        total += sizes[i];
        flops += nominal_flops(sizes[i]);
        if (total > (int64_t(1) << 40)) return FFT_ERR_INVALID_ARG;
    }
    fft_plan p = new (std::nothrow) fft_plan_s;
    if (!p) return FFT_ERR_ALLOC;
    p->n = 0;
    p->batch = count;
    p->layout = layout;
    p->dir = dir;
    p->elements = total;
    p->flops = flops;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "hipGetDevice");
    }
    // configuration: the cached winner for this size histogram, else the
    // default; FFT_AUTOTUNE=1 times every candidate and caches the fastest
    fftk::RaggedConfig cfg;
    const fftk::TuneKey key = fftk::make_ragged_key(p->device, sizes, count, layout);
    std::string cached;
    p->source = "default";
    if (config) {
        cfg = explicit_cfg;
        p->source = "explicit";
    } else if (fftk::autotune_lookup_text(key, &cached) && fftk::RaggedConfig::parse(cached, &cfg)) {
        p->source = "cache";
    } else if (fftk::autotune_enabled()) {
        float best_ms = 1e30f;
        fftk::RaggedConfig best = cfg;
        for (const fftk::RaggedConfig& c : fftk::ragged_candidates()) {
            fftk::RaggedPlan* trial = nullptr;
            std::string det;
            if (fftk::ragged_create(sizes, count, layout, c, &trial, &det) != FFT_OK) continue;
            float ms = 0.f;
            const fft_status ts = fftk::ragged_time(trial, &ms, &det);
            fftk::ragged_destroy(trial);
            if (ts != FFT_OK) continue;
            if (getenv("FFT_LOG")) fprintf(stderr, "[fft autotune] %s %s %.4f ms\n", key.s.c_str(), c.str().c_str(), ms);
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        cfg = best;
        fftk::autotune_store_text(key, cfg.str());
        p->source = "autotune";
    }
    fft_status st = fftk::ragged_create(sizes, count, layout, cfg, &p->ragged, &g_detail);
    if (st != FFT_OK) {
        p->magic = kDeadMagic;
        delete p;
        return st;
    }
    p->ws_bytes = fftk::ragged_workspace_bytes(p->ragged);
    *out = p;
    return FFT_OK;
}

fft_status fft_plan_create_ragged(fft_plan* out, const int64_t* sizes, int64_t count, fft_layout layout,
                                  fft_direction dir) {
    return create_ragged_impl(out, sizes, count, layout, dir, nullptr);
}

fft_status fft_plan_create_ragged_ex(fft_plan* out, const int64_t* sizes, int64_t count, fft_layout layout,
                                     fft_direction dir, const char* config) {
    return create_ragged_impl(out, sizes, count, layout, dir, config);
}

fft_status fft_plan_workspace_bytes(fft_plan p, size_t* bytes) {
    if (!plan_ok(p)) return FFT_ERR_INVALID_ARG;
    if (!bytes) return FFT_ERR_NULL_POINTER;
    *bytes = p->ws_bytes;
    return FFT_OK;
}

fft_status fft_plan_set_workspace(fft_plan p, void* dev_ptr) {
    if (!plan_ok(p)) return FFT_ERR_INVALID_ARG;
    if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) & 15u)) return FFT_ERR_MISALIGNED;
    DeviceGuard guard(p->device);
    if (p->ragged) return fftk::ragged_set_workspace(p->ragged, dev_ptr, &g_detail);
    if (p->inner && !p->nd_own_ws()) return fft_plan_set_workspace(p->inner, dev_ptr);
    if (p->inner) {
        // a multi-dimensional plan with two-pass columns: one workspace for
        // both stages (they run one after the other)
        if (dev_ptr) {
            if (p->ws_own) {
                (void)hipDeviceSynchronize();
                (void)hipFree(p->ws_own);
                p->ws_own = nullptr;
            }
            p->ws_user = dev_ptr;
        } else {
            p->ws_user = nullptr;
            const fft_status st = alloc_workspace(p);
            if (st != FFT_OK) return st;
        }
        return p->inner->ws_bytes ? fft_plan_set_workspace(p->inner, p->ws()) : FFT_OK;
    }
    if (dev_ptr) {
        if (p->ws_own) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p->ws_own);
            p->ws_own = nullptr;
        }
        p->ws_user = dev_ptr;
        return FFT_OK;
    }
    p->ws_user = nullptr;
    return alloc_workspace(p);
}

fft_status fft_plan_sizes(fft_plan p, int64_t* transforms, int64_t* elements, double* flops) {
    if (!plan_ok(p)) return FFT_ERR_INVALID_ARG;
    if (transforms) *transforms = p->batch;
    if (elements) *elements = p->elements;
    if (flops) *flops = p->flops;
    return FFT_OK;
}

fft_status fft_plan_describe(fft_plan p, char* buf, size_t len) {
    if (!plan_ok(p)) return FFT_ERR_INVALID_ARG;
    return copy_out(describe(p), buf, len);
}

fft_status fft_query_decomposition(int64_t n, fft_layout layout, fft_precision precision, char* buf, size_t len) {
    const int log2n = fftk::ilog2_exact(n);
    if (log2n < 0 || log2n > fftk::kMaxLog2N) return FFT_ERR_INVALID_SIZE;
    const int rb = fftk::real_bytes_of(precision);
    if (!valid_layout(layout) || rb == 0) return FFT_ERR_INVALID_ARG;
    const Decomp d = fftk::default_decomposition(log2n, rb, layout);
    std::string s = "{\"n\": " + std::to_string(n) + ", \"precision\": \"" + (rb == 8 ? "fp64" : "fp32") +
                    "\", \"default\": \"" + d.str() + "\", \"available\": " +
                    (fftk::decomposition_available(d, log2n, layout, rb) ? "true" : "false") + ", \"candidates\": [";
    const auto cands = fftk::candidate_decompositions(log2n, layout, rb);
    for (size_t i = 0; i < cands.size(); ++i) s += (i ? ", \"" : "\"") + cands[i].str() + "\"";
    s += "]}";
    return copy_out(s, buf, len);
}

fft_status fft_copy_device(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst) return FFT_ERR_NULL_POINTER;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | bytes) & 15u) return FFT_ERR_MISALIGNED;
    if (overlaps(uintptr_t(src), bytes, uintptr_t(dst), bytes)) return FFT_ERR_INVALID_ARG;
    hipError_t e = fftk::launch_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "copy launch");
    return FFT_OK;
}

const char* fft_status_string(fft_status s) {
    switch (s) {
        case FFT_OK: return "FFT_OK";
        case FFT_ERR_INVALID_SIZE: return "FFT_ERR_INVALID_SIZE: size is not a power of two in [1, 2^24]";
        case FFT_ERR_INVALID_ARG: return "FFT_ERR_INVALID_ARG: invalid argument";
        case FFT_ERR_NULL_POINTER: return "FFT_ERR_NULL_POINTER: required pointer is NULL";
        case FFT_ERR_MISALIGNED: return "FFT_ERR_MISALIGNED: pointer not 16-byte aligned";
        case FFT_ERR_ALLOC: return "FFT_ERR_ALLOC: allocation failed";
        case FFT_ERR_HIP: return "FFT_ERR_HIP: HIP runtime error";
        case FFT_ERR_NOT_SUPPORTED: return "FFT_ERR_NOT_SUPPORTED: no kernel for this configuration";
    }
    return "unknown fft_status";
}

const char* fft_last_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// hooks for the autotuner (same translation unit as the plan layout)
// ---------------------------------------------------------------------------
namespace fftk {

fft_status plan_time_decomposition(fft_plan p, const Decomp& d, void* in, void* out, float* ms, std::string* detail) {
    // build a throw-away plan with the candidate decomposition and time it
    fft_plan_s tmp;
    tmp.device = p->device;
    tmp.cus = p->cus;
    tmp.n = p->n;
    tmp.batch = p->batch;
    tmp.log2n = p->log2n;
    tmp.layout = p->layout;
    tmp.rb = p->rb;
    tmp.dir = FFT_FORWARD;
    tmp.elements = p->elements;
    fft_status st = resolve(&tmp, d);
    if (st == FFT_OK) st = build_tables(&tmp, nullptr);
    if (st == FFT_OK) st = alloc_workspace(&tmp);
    if (st != FFT_OK) {
        free_plan_memory(&tmp);
        tmp.magic = kDeadMagic;
        return st;
    }
    const bool split = p->layout == FFT_LAYOUT_SPLIT;
    const size_t half = size_t(p->elements) * size_t(p->rb);
    void* ib = split ? static_cast<char*>(in) + half : nullptr;
    void* ob = split ? static_cast<char*>(out) + half : nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // warm up twice, then time a few launches
    for (int i = 0; i < 2 && st == FFT_OK; ++i) st = run(&tmp, in, ib, out, ob, nullptr, false);
    const int reps = 5;
    if (st == FFT_OK && e == hipSuccess) {
        e = hipEventRecord(e0, nullptr);
        for (int i = 0; i < reps && st == FFT_OK; ++i) st = run(&tmp, in, ib, out, ob, nullptr, false);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        *ms = t / reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    free_plan_memory(&tmp);
    tmp.magic = kDeadMagic;
    if (st == FFT_OK && e != hipSuccess) {
        *detail = std::string("autotune timing: ") + hipGetErrorString(e);
        return FFT_ERR_HIP;
    }
    return st;
}

const Decomp& plan_decomposition(fft_plan p) { return p->dec; }
int64_t plan_elements(fft_plan p) { return p->elements; }
fft_layout plan_layout(fft_plan p) { return p->layout; }
int plan_log2n(fft_plan p) { return p->log2n; }
int plan_real_bytes(fft_plan p) { return p->rb; }

}  // namespace fftk

// ---------------------------------------------------------------------------
// hooks for the entry point that runs on the library's static scratch buffer
// ---------------------------------------------------------------------------
namespace fftk {

fft_status plan_scratch_need(fft_plan p, size_t* bytes, int* device) {
    if (!plan_ok(p)) return FFT_ERR_INVALID_ARG;
    if (p->ragged) {
        g_detail = "ragged plans keep their own workspace ring; use fft_execute";
        return FFT_ERR_NOT_SUPPORTED;
    }
    size_t need = p->ws_bytes;
    if (p->inner && p->inner->ws_bytes > need) need = p->inner->ws_bytes;
    *bytes = need;
    *device = p->device;
    return FFT_OK;
}

fft_status execute_with_workspace(fft_plan p, const void* ia, const void* ib, void* oa, void* ob, void* stream,
                                  void* ws) {
    return run(p, ia, ib, oa, ob, stream, false, ws);
}

void set_error_detail(const char* what) { g_detail = what; }

}  // namespace fftk
