// Decompositions of a power-of-two size into GPU kernels (host only).
//
// Eq. 1 of the paper (section 3) factors DFT_N for any N = M K; applied
// recursively it turns a power-of-two N into a chain of radix stages.  The
// paper notes (section 4) that the choice of radices decides speed (radix-2
// N = 128 is slow, N = 256 as 16 x 16 is fast) and that a runtime planner is
// future work; this file enumerates the choices and picks a default, and the
// autotuner times them.
#include "plan.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

namespace fftk {

int ilog2_exact(int64_t v) {
    if (v <= 0 || (v & (v - 1))) return -1;
    int k = 0;
    while ((int64_t(1) << k) < v) ++k;
    return k;
}

std::string Decomp::str() const {
    char buf[64];
    switch (kind) {
        case COPY:
            return "copy";
        case SINGLE:
            snprintf(buf, sizeof buf, "single:e%d:w%d:g%d:r%d%s", log2e, wgt, gmul, twreg ? 1 : (twrec ? 2 : 0),
                     pf ? ":p1" : (stg ? ":s1" : (half ? ":h1" : "")));
            return buf;
        case OPS:
            snprintf(buf, sizeof buf, "ops:r%d", log2r);
            return buf;
        case MULTI: {
            std::string s = "multi:";
            for (size_t p = 0; p < log2l.size(); ++p) {
                snprintf(buf, sizeof buf, "%s%dc%d%s", p ? "," : "", log2l[p], log2c[p], in_place(p) ? "i" : "");
                s += buf;
            }
            return s;
        }
    }
    return "?";
}

bool Decomp::parse(const std::string& s, Decomp* out) {
    Decomp d;
    if (s == "copy") {
        d.kind = COPY;
        *out = d;
        return true;
    }
    int e = 0, w = 0, g = 0, r = 0, used = 0;
    if (sscanf(s.c_str(), "single:e%d:w%d:g%d:r%d%n", &e, &w, &g, &r, &used) == 4) {
        // r: stage twiddles read from the table (0), held in registers (1), or
        // formed from one FP64 table value per butterfly (2); optional variant:
        // ":p1" prefetching, ":s1" staged, ":h1" half-width exchanges
        // (":p0"/":s0"/":h0" are spelled by leaving the field out)
        const std::string rest = s.substr(used);
        if (!rest.empty() && rest != ":p1" && rest != ":s1" && rest != ":h1") return false;
        if (g < 1 || g > 64 || r < 0 || r > 2) return false;
        d.kind = SINGLE;
        d.log2e = e;
        d.wgt = w;
        d.gmul = g;
        d.twreg = r == 1;
        d.twrec = r == 2;
        d.pf = rest == ":p1";
        d.stg = rest == ":s1";
        d.half = rest == ":h1";
        *out = d;
        return true;
    }
    int rr = 0;
    if (sscanf(s.c_str(), "ops:r%d%n", &rr, &used) == 1 && used == (int)s.size()) {
        if (rr < 1 || rr > 4) return false;
        d.kind = OPS;
        d.log2r = rr;
        *out = d;
        return true;
    }
    if (s.compare(0, 6, "multi:") == 0) {
        d.kind = MULTI;
        const char* p = s.c_str() + 6;
        while (*p) {
            int l = 0, c = 0, used = 0;
            if (sscanf(p, "%dc%d%n", &l, &c, &used) != 2) return false;
            d.log2l.push_back(l);
            d.log2c.push_back(c);
            p += used;
            d.inplace.push_back(*p == 'i' ? 1 : 0);
            if (*p == 'i') ++p;
            if (*p == ',') ++p;
            else if (*p) return false;
        }
        if (d.log2l.empty()) return false;
        *out = d;
        return true;
    }
    return false;
}

const SingleKernel* find_single(int rb, int log2n, int log2e, int wgt, bool split, bool swap, bool twreg, bool pf,
                                bool stg, bool half, bool twrec) {
    int cnt = 0;
    const SingleKernel* t = rb == 8 ? single_kernels64(&cnt) : single_kernels(&cnt);
    const int le = log2e < log2n ? log2e : log2n;
    for (int i = 0; i < cnt; ++i)
        if (t[i].log2n == log2n && t[i].log2e == le && t[i].wgt == wgt && t[i].split == split && t[i].swap == swap &&
            t[i].twreg == twreg && t[i].pf == pf && t[i].stg == stg && t[i].half == half && t[i].twrec == twrec)
            return &t[i];
    return nullptr;
}

const PassKernel* find_pass(int rb, int log2l, int log2c, bool first, bool split_in, bool split_out, bool swap_in,
                            bool swap_out) {
    int cnt = 0;
    const PassKernel* t = rb == 8 ? pass_kernels64(&cnt) : pass_kernels(&cnt);
    for (int i = 0; i < cnt; ++i)
        if (t[i].log2l == log2l && t[i].log2c == log2c && t[i].first == first && t[i].split_in == split_in &&
            t[i].split_out == split_out && t[i].swap_in == swap_in && t[i].swap_out == swap_out)
            return &t[i];
    return nullptr;
}

const PassKernel* pass_kernel_for(int rb, int log2l, int log2c, size_t p, size_t P, bool split, bool inverse) {
    const bool first = p == 0, last = p + 1 == P;
    return find_pass(rb, log2l, log2c, first, first && split, last && split, first && inverse && !split,
                     last && inverse && !split);
}

const SingleKernel* single_kernel_for(int rb, int log2n, const Decomp& d, bool split, bool inverse) {
    return find_single(rb, log2n, d.log2e, d.wgt, split, inverse && !split, d.twreg, d.pf, d.stg, d.half, d.twrec);
}

// column tile for a sub-FFT length: the widest compiled one up to 128-byte
// runs of interleaved data (16 FP32 or 8 FP64 columns), else the narrowest
// compiled one
static int default_log2c(int rb, int log2l) {
    const int cap = rb == 8 ? 3 : 4;
    int best = -1, min_any = 99;
    int cnt = 0;
    const PassKernel* t = rb == 8 ? pass_kernels64(&cnt) : pass_kernels(&cnt);
    for (int i = 0; i < cnt; ++i) {
        if (t[i].log2l != log2l) continue;
        const int c = t[i].log2c;
        if (c <= cap && c > best) best = c;
        if (c < min_any) min_any = c;
    }
    return best >= 0 ? best : (min_any == 99 ? -1 : min_any);
}

static bool pass_chain_available(const std::vector<int>& ls, const std::vector<int>& cs, fft_layout layout, int rb) {
    const bool split = layout == FFT_LAYOUT_SPLIT;
    const size_t P = ls.size();
    if (P < 2) return false;
    for (size_t p = 0; p < P; ++p)
        for (bool inv : {false, true})
            if (!pass_kernel_for(rb, ls[p], cs[p], p, P, split, inv)) return false;
    return true;
}

std::vector<int> ops_radices(int log2n, int log2r) {
    std::vector<int> r(log2n / log2r, log2r);
    if (log2n % log2r) r.push_back(log2n % log2r);
    return r;
}

bool decomposition_available(const Decomp& d, int log2n, fft_layout layout, int rb) {
    if (rb != 4 && rb != 8) return false;
    switch (d.kind) {
        case Decomp::OPS:
            return log2n >= 1 && layout == FFT_LAYOUT_INTERLEAVED && d.log2r >= 1 && d.log2r <= 4;
        case Decomp::COPY:
            return log2n == 0;
        case Decomp::SINGLE: {
            const bool split = layout == FFT_LAYOUT_SPLIT;
            return log2n >= 1 && single_kernel_for(rb, log2n, d, split, false) != nullptr &&
                   single_kernel_for(rb, log2n, d, split, true) != nullptr;
        }
        case Decomp::MULTI: {
            int sum = 0;
            for (int l : d.log2l) sum += l;
            if (sum != log2n || d.log2l.size() != d.log2c.size()) return false;
            // every pass needs at least 2^log2c columns
            const size_t P = d.log2l.size();
            for (size_t p = 0; p < P; ++p)
                if (log2n - d.log2l[p] < d.log2c[p]) return false;
            // only the penultimate pass of a chain of three or more may run in
            // place, and the last pass then reads runs of 2^(l_1 + .. + l_(P-2))
            // elements, which must hold its 2^log2c columns
            for (size_t p = 0; p < P; ++p)
                if (d.in_place(p) && (P < 3 || p + 2 != P)) return false;
            if (P >= 3 && d.in_place(P - 2)) {
                int ns = 0;
                for (size_t p = 0; p + 2 < P; ++p) ns += d.log2l[p];
                if (ns < d.log2c[P - 1]) return false;
            }
            return pass_chain_available(d.log2l, d.log2c, layout, rb);
        }
    }
    return false;
}

// Split log2n into `parts` near-equal sub-lengths, largest first.
static std::vector<int> even_split(int log2n, int parts) {
    std::vector<int> v(parts, log2n / parts);
    for (int i = 0; i < log2n % parts; ++i) v[i] += 1;
    return v;
}

// FP64 defaults, measured on MI355X (batches of 2^24 elements): single-pass
// up to 2^13 (the faster on average over both layouts), then pass chains per
// layout, timed on inputs that are not in any cache; three-pass chains run
// their middle pass in place (2^24 split: 351 -> 287 us)
static Decomp default_decomposition64(int log2n, fft_layout layout) {
    // 2^13: half-width exchanges (two workgroups per CU instead of one;
    // 2^25 elements: interleaved 269 -> 256 us, split 279 -> 280 us), and the
    // stage twiddles from one table value per butterfly (tw 2: interleaved
    // 260-269 -> 200 us, split 289 -> 228 us; tw 1 = registers, 0 = table)
    static const struct { int log2e, wgt, gmul, tw, pf, half; } single[14] = {
        {4, 256, 1, 1, 0, 0}, {4, 256, 2, 0, 0, 0}, {4, 64, 3, 0, 0, 0}, {4, 64, 1, 0, 0, 0}, {3, 256, 8, 1, 0, 0},
        {3, 256, 8, 1, 0, 0}, {3, 256, 1, 1, 0, 0}, {3, 64, 3, 1, 0, 0}, {3, 64, 3, 1, 0, 0}, {3, 64, 4, 1, 0, 0},
        {3, 256, 2, 1, 0, 0}, {3, 256, 2, 1, 0, 0}, {3, 256, 1, 1, 1, 0}, {4, 256, 3, 2, 0, 1},  // 2^10 .. 2^13
    };
    static const char* multi_il[kMaxLog2N + 1] = {
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, nullptr,
        "multi:7c5,7c5",          // 2^14
        "multi:8c4,7c5",          // 2^15
        "multi:8c4,8c4",          // 2^16
        "multi:9c3,8c4",          // 2^17
        "multi:10c3,8c5",         // 2^18
        "multi:10c3,9c4",         // 2^19
        "multi:10c3,10c3",        // 2^20
        "multi:11c2,10c3",        // 2^21
        "multi:8c4,8c5i,6c6",     // 2^22
        "multi:8c4,8c4i,7c5",     // 2^23
        "multi:8c4,8c5i,8c5",     // 2^24
    };
    static const char* multi_sp[kMaxLog2N + 1] = {
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, nullptr,
        "multi:7c4,7c4",          // 2^14
        "multi:8c4,7c4",          // 2^15
        "multi:8c5,8c5",          // 2^16
        "multi:9c4,8c5",          // 2^17
        "multi:9c4,9c4",          // 2^18
        "multi:10c3,9c4",         // 2^19
        "multi:7c5,7c6i,6c6",     // 2^20
        "multi:7c6,7c5i,7c5",     // 2^21
        "multi:8c4,7c5i,7c5",     // 2^22
        "multi:8c4,8c4i,7c5",     // 2^23
        "multi:8c4,8c5i,8c5",     // 2^24
    };
    const char* const* multi = layout == FFT_LAYOUT_SPLIT ? multi_sp : multi_il;
    Decomp d;
    if (log2n <= 0) {
        d.kind = Decomp::COPY;
    } else if (log2n <= 13) {
        d.kind = Decomp::SINGLE;
        d.log2e = single[log2n].log2e;
        d.wgt = single[log2n].wgt;
        d.gmul = single[log2n].gmul;
        d.twreg = single[log2n].tw == 1;
        d.twrec = single[log2n].tw == 2;
        d.pf = single[log2n].pf == 1;
        d.half = single[log2n].half == 1;
        // split 2^12: half-width exchanges and the recurrence twiddles at 8
        // workgroups per CU's worth of grid (231 -> 195 us for 2^25 elements;
        // interleaved the prefetching kernel stays ahead, 177 against 190 us)
        if (log2n == 12 && layout == FFT_LAYOUT_SPLIT) {
            d.gmul = 8;
            d.twreg = false;
            d.twrec = true;
            d.pf = false;
            d.half = true;
        }
    } else {
        Decomp::parse(multi[log2n], &d);
    }
    return d;
}

Decomp default_decomposition(int log2n, int rb, fft_layout layout, int64_t batch) {
    if (rb == 8) return default_decomposition64(log2n, layout);
    Decomp d;
    if (log2n <= 0) {
        d.kind = Decomp::COPY;
        return d;
    }
    if (log2n <= 14) {
        // single-pass shapes measured fastest on MI355X (batches of 2^25
        // elements from inputs that are not cached, the mean over both
        // layouts); up to 2^7 the staged kernel, whose loads and stores are
        // contiguous runs; at 2^14 half-width exchanges (two workgroups per
        // CU instead of one: 151.5 -> 136.3 us interleaved, 149.5 -> 142.2 us
        // split); at 2^13 and 2^14 stage twiddles from one FP64 value per
        // butterfly (tw 2: 2^13 106.6-114.8 -> 97.4-98.5 us, 2^14 136-137 ->
        // 111 us interleaved, 128 -> 102-105 us split; tw 1 = registers, 0 =
        // the table); the autotuner refines them per device
        static const struct { int log2e, gmul, tw, pf, stg, half; } table[15] = {
            {4, 1, 1, 0, 0, 0}, {4, 4, 1, 0, 1, 0}, {4, 3, 1, 0, 1, 0}, {4, 2, 1, 0, 1, 0}, {4, 8, 1, 0, 1, 0},  // 2^0 .. 2^4
            {4, 8, 1, 0, 1, 0}, {4, 8, 1, 0, 1, 0}, {4, 8, 1, 0, 1, 0}, {3, 2, 1, 0, 0, 0}, {3, 2, 1, 0, 0, 0},  // 2^5 .. 2^9
            {3, 2, 1, 0, 0, 0}, {3, 2, 1, 0, 0, 0}, {4, 2, 1, 0, 0, 0}, {5, 8, 2, 0, 0, 1}, {4, 8, 2, 0, 0, 1},  // 2^10 .. 2^14
        };
        d.kind = Decomp::SINGLE;
        d.log2e = table[log2n].log2e;
        d.wgt = 256;
        d.gmul = table[log2n].gmul;
        d.twreg = table[log2n].tw == 1;
        d.twrec = table[log2n].tw == 2;
        d.pf = table[log2n].pf == 1;
        d.stg = table[log2n].stg == 1;
        d.half = table[log2n].half == 1;
        // N = 4096 at most 1024 transforms (every group resident at once):
        // radix-8 stages measured faster (1024 split rows not cached:
        // e3 15.2-15.7 us against e4 16.4-16.7 us; e4 leads from 8192 rows)
        if (log2n == 12 && batch > 0 && batch <= 1024) d.log2e = 3;
        // split data at 2^14: 32 points per thread (radix-32, 32, 16 stages)
        // at 4 workgroups per CU's worth of grid, 102-105 us against 113-115
        // for 16 points per thread; interleaved the 16-point shape leads
        // (110.8-111.1 against 111.8-112.5 us)
        if (log2n == 14 && layout == FFT_LAYOUT_SPLIT) {
            d.log2e = 5;
            d.gmul = 4;
        }
        return d;
    }
    // multi-pass chains measured fastest on MI355X per layout (batches of 2^25
    // elements from inputs not in any cache; the workspace between passes is
    // read back through the memory-side cache, which favours two passes for
    // interleaved 2^18 .. 2^20, and an in-place middle pass for three-pass
    // chains: one workspace half instead of two, 15-25 % faster at every size;
    // split chains re-measured once their first and last passes stream the
    // caller's arrays: the interleaved shapes win there too, 2^18 by 22 %;
    // first passes of 1024-thread tiles since they exchange through half the
    // LDS (two workgroups per CU): interleaved 2^22 8c6,8c5i,6c7 132.2-132.5
    // against 135.4-135.9 us and split 2^20 7c7,7c4i,6c6 139.1-139.3 against
    // 141.4-141.9 (2^24 elements); for 2^25 elements interleaved 2^15
    // 165-166 against 173-179, split 2^15 168.8 against 171.7, interleaved
    // 2^16 164.6-164.9 against 166.5-166.9, split 2^19 261.6-262.0 against
    // 272.5-272.7, split 2^21 258.3-259.2 against 264.2-264.9, interleaved
    // 2^23 256.6-256.8 against 265.0-265.6; interleaved 2^21 keeps its chain,
    // 250 against 254 us)
    static const char* measured_il[kMaxLog2N + 1] = {
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, nullptr, nullptr,
        "multi:8c6,7c5",          // 2^15
        "multi:8c6,8c5",          // 2^16
        "multi:9c4,8c5",          // 2^17
        "multi:9c4,9c4",          // 2^18
        "multi:10c3,9c4",         // 2^19
        "multi:10c3,10c3",        // 2^20
        "multi:7c6,7c6i,7c6",     // 2^21
        "multi:8c6,8c5i,6c7",     // 2^22
        "multi:8c6,8c5i,7c6",     // 2^23
        "multi:8c5,8c5i,8c5",     // 2^24
    };
    static const char* measured_sp[kMaxLog2N + 1] = {
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
        nullptr, nullptr, nullptr, nullptr, nullptr,
        "multi:8c6,7c5",          // 2^15
        "multi:8c5,8c5",          // 2^16
        "multi:9c4,8c5",          // 2^17
        "multi:9c4,9c4",          // 2^18
        "multi:7c7,6c6i,6c6",     // 2^19
        "multi:7c7,7c4i,6c6",     // 2^20
        "multi:7c7,7c6i,7c6",     // 2^21
        "multi:8c6,8c5i,6c7",     // 2^22
        "multi:8c6,8c5i,7c6",     // 2^23
        "multi:8c5,8c5i,8c5",     // 2^24
    };
    const char* const* measured = layout == FFT_LAYOUT_SPLIT ? measured_sp : measured_il;
    if (measured[log2n] && Decomp::parse(measured[log2n], &d)) return d;
    // otherwise passes of at most 2^9 points with 16-column tiles (128-byte runs)
    int parts = (log2n + 8) / 9;
    if (parts < 2) parts = 2;
    d = Decomp();
    d.kind = Decomp::MULTI;
    d.log2l = even_split(log2n, parts);
    for (int l : d.log2l) d.log2c.push_back(default_log2c(rb, l));
    return d;
}

const RealKernel* find_real(int rb, int log2h, int log2e, int wgt, bool c2r, bool split, bool twreg, bool stg,
                            bool twrec) {
    int cnt = 0;
    const RealKernel* t = rb == 8 ? real_kernels64(&cnt) : real_kernels(&cnt);
    const int le = log2e < log2h ? log2e : log2h;
    for (int i = 0; i < cnt; ++i)
        if (t[i].log2h == log2h && t[i].log2e == le && t[i].wgt == wgt && t[i].c2r == c2r && t[i].split == split &&
            t[i].twreg == twreg && t[i].stg == stg && t[i].twrec == twrec)
            return &t[i];
    return nullptr;
}

bool real_decomposition_available(const Decomp& d, int log2n, fft_layout layout, int rb, bool c2r) {
    if ((rb != 4 && rb != 8) || log2n < 1) return false;
    const int log2h = log2n - 1;
    const bool split = layout == FFT_LAYOUT_SPLIT;
    switch (d.kind) {
        case Decomp::OPS:
            return false;
        case Decomp::COPY:
            return log2h == 0;
        case Decomp::SINGLE:
            return log2h >= 1 && !d.pf && !d.half &&
                   find_real(rb, log2h, d.log2e, d.wgt, c2r, split, d.twreg, d.stg, d.twrec) != nullptr;
        case Decomp::MULTI: {
            // the half-length chain runs on interleaved data in both directions
            int sum = 0;
            for (int l : d.log2l) sum += l;
            if (sum != log2h || d.log2l.size() != d.log2c.size() || d.log2l.size() < 2) return false;
            for (size_t q = 0; q < d.log2l.size(); ++q)
                if (d.in_place(q) && (d.log2l.size() < 3 || q + 2 != d.log2l.size())) return false;
            if (d.log2l.size() >= 3 && d.in_place(d.log2l.size() - 2)) {
                int ns = 0;
                for (size_t q = 0; q + 2 < d.log2l.size(); ++q) ns += d.log2l[q];
                if (ns < d.log2c.back()) return false;
            }
            const size_t P = d.log2l.size();
            for (size_t q = 0; q < P; ++q) {
                if (log2h - d.log2l[q] < d.log2c[q]) return false;
                if (!pass_kernel_for(rb, d.log2l[q], d.log2c[q], q, P, false, c2r)) return false;
            }
            return true;
        }
    }
    return false;
}

// Real plans: single-pass shapes measured on MI355X (2^25 FP32 or 2^24 FP64
// reals, the faster of R2C + C2R; up to 2^8 on inputs that are not cached,
// both layouts, where the staged kernel wins; N = 4096 re-measured on rows
// not in any cache: e3 g3 49.6 us against e4 g2 52-54 us for 8192 rows),
// indexed by log2 N; above the single-pass limit, the half length's complex
// pass chain.  tw: stage twiddles from the table (0), in registers (1), or as
// one FP64 value per butterfly (2: the two largest sizes of each precision,
// R2C + C2R FP32 2^14 152-165 -> 131 us interleaved and 183 -> 133 us split,
// 2^15 186 -> 154 and 200 -> 166 us; FP64 2^13 138-146 -> 107-109 and 139 ->
// 112 us, 2^14 173 -> 138 and 177 -> 143 us).
struct RealShapeChoice {
    int log2e, gmul, tw, stg;
};

Decomp default_real_decomposition(int log2n, int rb) {
    static const RealShapeChoice r32[16] = {
        {4, 1, 1, 0}, {4, 1, 1, 0}, {3, 4, 1, 1}, {4, 4, 1, 1}, {3, 3, 1, 1}, {3, 3, 1, 1}, {3, 3, 1, 1},  // 2^0 .. 2^6
        {3, 3, 1, 1}, {3, 3, 1, 1}, {3, 2, 1, 0}, {3, 2, 1, 0}, {4, 2, 1, 0}, {3, 3, 1, 0}, {3, 2, 1, 0},  // 2^7 .. 2^13
        {4, 8, 2, 0}, {4, 1, 2, 0},                                                                        // 2^14 .. 2^15
    };
    static const RealShapeChoice r64[15] = {
        {4, 1, 1, 0}, {4, 1, 1, 0}, {3, 3, 1, 1}, {3, 8, 1, 1}, {3, 8, 1, 1}, {3, 2, 1, 1}, {3, 2, 1, 1},  // 2^0 .. 2^6
        {3, 2, 1, 1}, {3, 2, 1, 1}, {3, 2, 1, 0}, {3, 2, 1, 0}, {3, 2, 1, 0}, {3, 2, 1, 0}, {4, 8, 2, 0},  // 2^7 .. 2^13
        {4, 1, 2, 0},                                                                                      // 2^14
    };
    const int log2h = log2n - 1;
    Decomp d;
    if (log2h <= 0) {
        d.kind = Decomp::COPY;
        return d;
    }
    const int lim = rb == 8 ? 14 : 15;
    if (log2n > lim) return default_decomposition(log2h, rb);
    const RealShapeChoice& t = rb == 8 ? r64[log2n] : r32[log2n];
    d.kind = Decomp::SINGLE;
    d.log2e = t.log2e;
    d.wgt = 256;
    d.gmul = t.gmul;
    d.twreg = t.tw == 1;
    d.twrec = t.tw == 2;
    d.stg = t.stg == 1;
    return d;
}

const StridedKernel* strided_kernel_for(int rb, int log2l, int log2s, bool split, bool swap) {
    int cnt = 0;
    const StridedKernel* t = strided_kernels(&cnt);
    const StridedKernel* best = nullptr;
    for (int i = 0; i < cnt; ++i) {
        const StridedKernel& k = t[i];
        if (k.real_bytes != rb || k.log2l != log2l || k.split != split || k.swap != swap || k.log2c > log2s) continue;
        if (!best || k.log2c > best->log2c) best = &k;
    }
    return best;
}

std::vector<Decomp> candidate_decompositions(int log2n, fft_layout layout, int rb) {
    std::vector<Decomp> out;
    if (log2n <= 0) {
        Decomp d;
        d.kind = Decomp::COPY;
        out.push_back(d);
        return out;
    }
    // single-pass variants: kernel shape x grid size x twiddle source
    std::vector<const SingleKernel*> shapes;
    for (int e : {4, 3, 5})  // 5 last: below 2^5 it names the same kernels as 4
        for (int w : {256, 64})
            for (int r : {1, 0, 2})  // registers, table, recurrence
                for (int var : {0, 1, 2, 3}) {  // plain, prefetching, staged, half-width exchanges
                    const bool pf = var == 1, stg = var == 2, half = var == 3;
                    const SingleKernel* k = find_single(rb, log2n, e, w, false, false, r == 1, pf, stg, half, r == 2);
                    if (!k) continue;
                    bool dup = false;
                    for (auto* o : shapes) dup |= (o == k);
                    if (dup) continue;
                    shapes.push_back(k);
                    for (int g : {1, 2, 3, 4, 8}) {
                        Decomp d;
                        d.kind = Decomp::SINGLE;
                        d.log2e = e;
                        d.wgt = w;
                        d.gmul = g;
                        d.twreg = r == 1;
                        d.twrec = r == 2;
                        d.pf = pf;
                        d.stg = stg;
                        d.half = half;
                        if (decomposition_available(d, log2n, layout, rb)) out.push_back(d);
                    }
                }
    // multi-pass chains with 2 or 3 passes, every sub-length and tile compiled
    int cnt = 0;
    const PassKernel* t = rb == 8 ? pass_kernels64(&cnt) : pass_kernels(&cnt);
    std::vector<std::pair<int, int>> lc;  // distinct (log2l, log2c)
    for (int i = 0; i < cnt; ++i) {
        std::pair<int, int> x(t[i].log2l, t[i].log2c);
        bool seen = false;
        for (auto& y : lc) seen |= (y == x);
        if (!seen) lc.push_back(x);
    }
    for (int parts = 2; parts <= 3; ++parts) {
        // enumerate ordered tuples of (l, c)
        std::vector<size_t> idx(parts, 0);
        while (true) {
            int sum = 0;
            for (int p = 0; p < parts; ++p) sum += lc[idx[p]].first;
            if (sum == log2n) {
                Decomp d;
                d.kind = Decomp::MULTI;
                for (int p = 0; p < parts; ++p) {
                    d.log2l.push_back(lc[idx[p]].first);
                    d.log2c.push_back(lc[idx[p]].second);
                }
                // keep sub-lengths non-increasing to bound the search
                bool sorted = true;
                for (int p = 1; p < parts; ++p) sorted &= d.log2l[p] <= d.log2l[p - 1];
                if (sorted && decomposition_available(d, log2n, layout, rb)) out.push_back(d);
                if (sorted && parts >= 3) {
                    // the same chain with an in-place penultimate pass
                    d.inplace.assign(parts, 0);
                    d.inplace[parts - 2] = 1;
                    if (decomposition_available(d, log2n, layout, rb)) out.push_back(d);
                }
            }
            int p = parts - 1;
            while (p >= 0 && ++idx[p] == lc.size()) idx[p--] = 0;
            if (p < 0) break;
        }
    }
    return out;
}

}  // namespace fftk
