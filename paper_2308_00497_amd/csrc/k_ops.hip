// Per-operator baseline: the FFT as the paper's compiler maps it to a GPU,
// one kernel per operator of Table 1 (its GPU path lowers each affine loop
// nest to its own kernel, section 3.2), every operator a full pass over HBM.
// It exists to measure what fusing the operators into Stockham stages buys on
// this device; it is not the fast path.
//
// Eq. 1 with K = R (radix) and M = N/R, applied recursively to DFT_M:
//     DFT_N = (DFT_R (x) I_M) D^N_M (I_R (x) DFT_M) Pi^N_R.
// Over a batch of B transforms (and at depth l, a = B R_0 ... R_(l-1)
// independent sub-transforms of length n_l) the operators are
//     Permute    y = (I_a (x) Pi^(n_l)_(R_l)) x     z[M n2 + n1] = x[R n1 + n2]
//     FusedIKMV  y = (I_a (x) DFT_R) x              innermost level
//     Mul        y = (I_a (x) D^(n_l)_(n_(l+1))) x  entry M n2 + k1: w_(n_l)^(n2 k1)
//     FusedMKIV  y = (I_a (x) DFT_R (x) I_M) x
// executed as: Permute for l = 0 .. L-2, the innermost DFT blocks, then
// Mul and FusedMKIV for l = L-2 .. 0: 3L - 2 kernels for N = R^L.  The
// inverse swaps real and imaginary parts in the first and last operator.
#include "kernels.hpp"

namespace fftk {

// y = (I_a (x) DFT_R (x) I_b) x over interleaved complex data
template <class R, int RADIX>
__global__ void __launch_bounds__(256) k_op_kron(const cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ y,
                                                 int64_t a, int64_t b, int swap_in, int swap_out) {
    using V = cplx_t<R>;
    const int64_t total = a * b;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = t / b, j = t - i * b;
        const int64_t base = i * RADIX * b + j;
        V u[RADIX];
#pragma unroll
        for (int r = 0; r < RADIX; ++r) {
            const V v = x[base + r * b];
            u[r] = swap_in ? cmk(v.y, v.x) : v;
        }
        Dft<RADIX>::run(u);
#pragma unroll
        for (int r = 0; r < RADIX; ++r) y[base + r * b] = swap_out ? cmk(u[r].y, u[r].x) : u[r];
    }
}

// y = (I_a (x) D) x with the diagonal D (n entries) from a table
template <class R>
__global__ void __launch_bounds__(256) k_op_mul(const cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ y,
                                                const cplx_t<R>* __restrict__ d, int64_t a, int log2n) {
    const int64_t total = a << log2n;
    const int64_t mask = (int64_t(1) << log2n) - 1;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
        y[t] = c_mul(x[t], d[t & mask]);
}

// y = (I_a (x) Pi^(mn)_m) x, Permute(m, mn) of Table 1: Y[i + m j] = X[n i + j]
template <class R>
__global__ void __launch_bounds__(256) k_op_perm(const cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ y,
                                                 int64_t a, int log2m, int log2n, int swap_in) {
    using V = cplx_t<R>;
    const int log2mn = log2m + log2n;
    const int64_t total = a << log2mn;
    const int64_t mmask = (int64_t(1) << log2m) - 1, nmask = (int64_t(1) << log2n) - 1;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t blk = t >> log2mn;
        const int64_t o = t & ((int64_t(1) << log2mn) - 1);  // o = i + m j
        const int64_t i = o & mmask, j = o >> log2m;
        const V v = x[(blk << log2mn) + (i << log2n) + (j & nmask)];
        y[t] = swap_in ? cmk(v.y, v.x) : v;
    }
}

// D^n_m: entry m n2 + k1 = w_n^(n2 k1), n2 < n/m, k1 < m; FP64, rounded once
template <class V>
__global__ void k_gen_diag(V* dst, int log2n, int log2m) {
    const int64_t n = int64_t(1) << log2n;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t n2 = i >> log2m, k1 = i & ((int64_t(1) << log2m) - 1);
    const int64_t e = (n2 * k1) & (n - 1);
    double s, c;
    sincospi(ldexp(static_cast<double>(e), 1 - log2n), &s, &c);
    dst[i] = cvt_tw<V>(make_double2(c, -s));
}

static unsigned op_blocks(int64_t items) {
    int64_t b = (items + 255) / 256;
    if (b > 65536) b = 65536;
    return static_cast<unsigned>(b < 1 ? 1 : b);
}

template <class R>
static hipError_t launch_kron_t(int log2r, const void* x, void* y, int64_t a, int64_t b, bool si, bool so,
                                hipStream_t s) {
    using V = cplx_t<R>;
    const unsigned g = op_blocks(a * b);
    const V* xi = static_cast<const V*>(x);
    V* yo = static_cast<V*>(y);
    switch (log2r) {
        case 1: hipLaunchKernelGGL((k_op_kron<R, 2>), dim3(g), dim3(256), 0, s, xi, yo, a, b, int(si), int(so)); break;
        case 2: hipLaunchKernelGGL((k_op_kron<R, 4>), dim3(g), dim3(256), 0, s, xi, yo, a, b, int(si), int(so)); break;
        case 3: hipLaunchKernelGGL((k_op_kron<R, 8>), dim3(g), dim3(256), 0, s, xi, yo, a, b, int(si), int(so)); break;
        case 4: hipLaunchKernelGGL((k_op_kron<R, 16>), dim3(g), dim3(256), 0, s, xi, yo, a, b, int(si), int(so)); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_op_kron(int rb, int log2r, const void* x, void* y, int64_t a, int64_t b, bool swap_in,
                          bool swap_out, hipStream_t s) {
    return rb == 8 ? launch_kron_t<double>(log2r, x, y, a, b, swap_in, swap_out, s)
                   : launch_kron_t<float>(log2r, x, y, a, b, swap_in, swap_out, s);
}

hipError_t launch_op_mul(int rb, const void* x, void* y, const void* d, int64_t a, int log2n, hipStream_t s) {
    const unsigned g = op_blocks(a << log2n);
    if (rb == 8)
        hipLaunchKernelGGL(k_op_mul<double>, dim3(g), dim3(256), 0, s, static_cast<const double2*>(x),
                           static_cast<double2*>(y), static_cast<const double2*>(d), a, log2n);
    else
        hipLaunchKernelGGL(k_op_mul<float>, dim3(g), dim3(256), 0, s, static_cast<const float2*>(x),
                           static_cast<float2*>(y), static_cast<const float2*>(d), a, log2n);
    return hipGetLastError();
}

hipError_t launch_op_perm(int rb, const void* x, void* y, int64_t a, int log2m, int log2n, bool swap_in,
                          hipStream_t s) {
    const unsigned g = op_blocks(a << (log2m + log2n));
    if (rb == 8)
        hipLaunchKernelGGL(k_op_perm<double>, dim3(g), dim3(256), 0, s, static_cast<const double2*>(x),
                           static_cast<double2*>(y), a, log2m, log2n, int(swap_in));
    else
        hipLaunchKernelGGL(k_op_perm<float>, dim3(g), dim3(256), 0, s, static_cast<const float2*>(x),
                           static_cast<float2*>(y), a, log2m, log2n, int(swap_in));
    return hipGetLastError();
}

hipError_t launch_gen_diag(int rb, void* dst, int log2n, int log2m, hipStream_t s) {
    const int64_t n = int64_t(1) << log2n;
    const unsigned g = static_cast<unsigned>((n + 255) / 256);
    if (rb == 8)
        hipLaunchKernelGGL(k_gen_diag<double2>, dim3(g), dim3(256), 0, s, static_cast<double2*>(dst), log2n, log2m);
    else
        hipLaunchKernelGGL(k_gen_diag<float2>, dim3(g), dim3(256), 0, s, static_cast<float2*>(dst), log2n, log2m);
    return hipGetLastError();
}

}  // namespace fftk
