/*
 * fft.h - C ABI of the MI355X (gfx950) batched 1D complex-to-complex FFT.
 *
 * The library computes, for power-of-two N, the unnormalised DFT
 *
 *     X[k] = sum_{n<N} x[n] exp(s * 2 pi i k n / N),  s = -1 forward, +1 inverse
 *
 * by the radix factorisation of Eq. 1 of the paper (section 3): every GPU
 * stage is one instance of DFT_N = (DFT_K (x) I_M) D^N_M (I_K (x) DFT_M) Pi^N_K,
 * evaluated as a Stockham (self-sorting) stage so the output comes out in
 * natural order.  Complex arrays are either interleaved (re, im adjacent) or
 * split into separate real and imaginary arrays, the two layouts of section 3,
 * step 3.  The paper packages its generated kernels as a precompiled library
 * with an FFTW-like plan/execute API (section 4); this is that boundary.
 *
 * Conventions for every function below
 *  - All functions return fft_status and never throw or abort.
 *  - Data pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors on
 *    the current HIP device).  Arrays hold the plan's real type (float32, or
 *    float64 for FFT_PRECISION_FP64 plans); a transform occupies N
 *    consecutive elements and transform b starts at element b*N ("[batch][N]").
 *    Interleaved: one array of 2*N*batch reals (re0, im0, re1, im1, ...).
 *    Split: two arrays of N*batch reals each (re, im).
 *  - Pointers must be 16-byte aligned (FFT_ERR_MISALIGNED otherwise) and
 *    non-null (FFT_ERR_NULL_POINTER); split layout needs both arrays.
 *  - In-place (input pointers equal to output pointers) is allowed; a partial
 *    overlap between input and output is FFT_ERR_INVALID_ARG.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    execution is asynchronous on that stream; the caller keeps every buffer
 *    alive until the work completes.  Device faults surface at the caller's
 *    next synchronisation.
 *  - Argument checks happen before any HIP call, so invalid arguments are
 *    reported even on a machine without a GPU.
 */
#ifndef FFT_MI355X_H
#define FFT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque plan, owned by the library: created by fft_plan_create* and released
 * by fft_plan_destroy.  A plan is immutable after creation apart from the
 * workspace pointer (fft_plan_set_workspace) and a ragged plan's cached graph. */
typedef struct fft_plan_s *fft_plan;

/* Complex layout (paper section 3, step 3: interleaved or split arrays). */
typedef enum {
    FFT_LAYOUT_INTERLEAVED = 0,
    FFT_LAYOUT_SPLIT = 1
} fft_layout;

/* Real type of the data.  FP32 is the default everywhere; FP64 is the
 * precision of the paper's evaluation (section 4).  Twiddles of FP64 plans are
 * evaluated in FP64 and used unrounded. */
typedef enum {
    FFT_PRECISION_FP32 = 0,
    FFT_PRECISION_FP64 = 1
} fft_precision;

/* Sign of the exponent. */
typedef enum {
    FFT_FORWARD = -1,
    FFT_INVERSE = 1
} fft_direction;

typedef enum {
    FFT_OK = 0,
    FFT_ERR_INVALID_SIZE = 1,   /* N not a power of two, or outside [1, 2^24] */
    FFT_ERR_INVALID_ARG = 2,    /* bad batch/count/enum, partial overlap, bad plan */
    FFT_ERR_NULL_POINTER = 3,
    FFT_ERR_MISALIGNED = 4,     /* a data pointer not 16-byte aligned */
    FFT_ERR_ALLOC = 5,          /* device or host allocation failed */
    FFT_ERR_HIP = 6,            /* a HIP runtime call failed; see fft_last_error_detail */
    FFT_ERR_NOT_SUPPORTED = 7
} fft_status;

/* Create a plan for `batch` contiguous transforms of size n (paper section 4:
 * powers of two only; 1 <= n <= 2^24, batch >= 1) in `layout`, direction
 * `dir`.  Builds the twiddle tables on the current device: every factor
 * exp(-2 pi i m / M) is evaluated in FP64 on the GPU and rounded once to FP32
 * (the diagonal D^N_M of Eq. 1 and Table 1's Mul(TwiddleCoe, X)).  Plans for
 * n above the single-pass limit also own a workspace (see
 * fft_plan_workspace_bytes).  On failure *out is set to NULL.
 * Environment: FFT_AUTOTUNE=1 times candidate decompositions at creation and
 * records the winner in the cache file named by FFT_AUTOTUNE_CACHE (default
 * $HOME/.cache/fft_mi355x_autotune.json); without it the cache is only read. */
fft_status fft_plan_create(fft_plan *out, int64_t n, int64_t batch,
                           fft_layout layout, fft_direction dir);

/* As fft_plan_create, with the decomposition given explicitly instead of
 * chosen: "single:e<log2 E>:w<threads>:g<G>:r<0|1|2>[:p1|:s1|:h1]"
 * (persistent single-pass kernel, 2^E elements per thread, workgroups of at
 * least <threads> threads, G workgroups per compute unit; stage twiddles read
 * from the table (r0), held in registers (r1), or formed from one FP64 table
 * value per butterfly (r2); optionally the prefetching (p1), LDS-staged short
 * transform (s1) or half-width-exchange (h1) variant) or
 * "multi:<log2 L1>c<log2 C1>,<log2 L2>c<log2 C2>,..." (one pass per sub-FFT
 * length L_p with C_p columns per workgroup; the log2 L_p sum to log2 n; an
 * "i" after the penultimate pass of three or more runs it in place), or
 * "copy" for n = 1 - the strings fft_plan_describe and
 * fft_query_decomposition report - or "ops:r<log2 R>", the per-operator
 * baseline (Table 1's Permute, FusedIKMV, Mul and FusedMKIV as one kernel each,
 * composed by Eq. 1 with radix R; interleaved only; never chosen by
 * default).  FFT_ERR_NOT_SUPPORTED if no compiled kernel matches,
 * FFT_ERR_INVALID_ARG if the string does not parse. */
fft_status fft_plan_create_explicit(fft_plan *out, int64_t n, int64_t batch,
                                    fft_layout layout, fft_direction dir,
                                    const char *decomposition);

/* General form of the two above: `precision` selects float32 or float64
 * data (and twiddles), `decomposition` is an explicit decomposition string
 * or NULL to let the library choose (default table, autotune cache, or the
 * autotuner as for fft_plan_create).  FP64 plans run the same kernels over
 * double2 elements: single-pass up to n = 2^13 (the LDS holds 2^13 FP64
 * complex elements per workgroup), multi-pass above.  FFT_ERR_INVALID_ARG for
 * an unknown precision. */
fft_status fft_plan_create_ex(fft_plan *out, int64_t n, int64_t batch,
                              fft_layout layout, fft_direction dir,
                              fft_precision precision,
                              const char *decomposition);

/* Real-input plan: `batch` rows of n real values (n a power of two in
 * [1, 2^24]).  dir FFT_FORWARD is real-to-complex (R2C): row b of the real
 * input maps to the n/2 + 1 values X[k] = sum_m x[m] exp(-2 pi i k m / n),
 * k = 0 .. n/2, the half of the DFT of a real sequence that determines the
 * rest (X[n-k] = conj X[k]).  dir FFT_INVERSE is complex-to-real (C2R): rows
 * of n/2 + 1 values map to y[m] = Re sum_{k<n} Xe[k] exp(+2 pi i k m / n),
 * Xe the Hermitian extension (Xe[k] = X[k] for k <= n/2, conj X[n-k] above),
 * unnormalised, so C2R(R2C(x)) = n x; the imaginary parts of X[0] and X[n/2]
 * do not contribute.  Computed through the complex transform of length n/2
 * (Eq. 1 with K = 2 splits x into even and odd samples, which form one
 * complex sequence): single-pass for n/2 up to the complex single-pass limit,
 * else the half-length multi-pass chain plus one pass that separates (R2C) or
 * merges (C2R) the two spectra.
 *   Buffers of fft_execute: R2C in_re_or_z = real array [batch][n], in_im
 *   ignored; out = complex array(s) [batch][n/2 + 1] in `layout`.  C2R in =
 *   complex array(s) [batch][n/2 + 1], out_re_or_z = real array [batch][n],
 *   out_im ignored.  The real and complex buffers may not overlap (no in-place).
 *   fft_execute_backward applies the adjoint under the real inner products
 *   (sum x y on the real side, Re sum conj(X) Y on the complex side), the
 *   vector-Jacobian product of the plan: for R2C it maps a complex gradient
 *   g (n/2 + 1 values per row, same layout) to the real
 *   x[m] = Re sum_{k<=n/2} g[k] exp(+2 pi i k m / n), which is C2R of g with
 *   the bins k = 1 .. n/2-1 halved; for C2R it maps a real gradient to R2C of
 *   it with those bins doubled.  Its buffers are those of fft_execute with the
 *   roles exchanged (R2C backward: in = complex, out = real).  fft_plan_sizes
 *   reports n*batch elements and 2.5 n log2 n flops per row.
 * `decomposition` is NULL (default) or a decomposition string of the half
 * length ("copy" for n = 2); n = 1 takes none. */
fft_status fft_plan_create_real(fft_plan *out, int64_t n, int64_t batch,
                                fft_layout layout, fft_direction dir,
                                fft_precision precision,
                                const char *decomposition);

/* Multi-dimensional plan: `batch` arrays of shape dims[0] x ... x
 * dims[rank-1] (row-major, the last axis contiguous; rank 1, 2 or 3; every
 * dim a power of two, the last up to 2^24, the others up to 2^12), the DFT
 * over all `rank` axes:
 *     X[k] = sum_n x[n] exp(-+ 2 pi i sum_j k_j n_j / dims[j]),
 * unnormalised, in `layout` and `dir` and `precision`.  The exponential
 * factorises over the axes, so it runs as the batched 1D transform of the last
 * axis (a plan as from fft_plan_create_ex, in -> out) followed by one pass per
 * other axis, in place on the output, each a DFT down the columns of that
 * axis's stride.  In-place execution, the adjoint (fft_execute_backward) and a
 * caller workspace (that of the last-axis plan) work as for 1D plans.
 * fft_plan_sizes counts batch x prod(dims) elements and 5 M log2 M flops per
 * array, M = prod(dims).  rank 1 returns an ordinary 1D plan. */
fft_status fft_plan_create_nd(fft_plan *out, int rank, const int64_t *dims,
                              int64_t batch, fft_layout layout,
                              fft_direction dir, fft_precision precision);

/* Apply the plan's transform to `batch` transforms: in -> out.
 * Defined by: the DFT_N of Eq. 1 (section 3), applied through the plan/execute
 * call of the precompiled library with an FFTW-like API (section 4), whose
 * arguments are plain pointers in place of the paper's memref structs; the
 * two pointer pairs are the layout flag of section 3, step 3.
 * in_re_or_z / out_re_or_z: interleaved array, or the real array (split).
 * in_im / out_im: the imaginary arrays (split), ignored (may be NULL) when
 * interleaved.  For a ragged plan the transforms are packed back to back in
 * creation order. */
fft_status fft_execute(fft_plan p, const void *in_re_or_z, const void *in_im,
                       void *out_re_or_z, void *out_im, void *stream);

/* Apply the adjoint of the plan's transform, unnormalised: F^H (the inverse
 * transform) for a forward plan, F for an inverse plan.
 * Defined by: the conjugate transpose of DFT_N in Eq. 1 (section 3); the
 * factorisation is unitary up to the scale N, so F^H = N F^-1 is the same
 * stages with conjugated twiddles.  This is the vector-
 * Jacobian product of fft_execute, so fft_execute followed by
 * fft_execute_backward multiplies the input by N.  Same buffers and rules as
 * fft_execute (real-input plans: see fft_plan_create_real). */
fft_status fft_execute_backward(fft_plan p, const void *grad_out_re_or_z,
                                const void *grad_out_im, void *grad_in_re_or_z,
                                void *grad_in_im, void *stream);

/* Release the plan and everything it owns (tables, workspace it allocated,
 * graphs).  NULL is a no-op.  Waits for the device to finish work that may
 * still use the plan's memory.
 * Defined by: the plan lifetime of the FFTW-like library API (section 4). */
fft_status fft_plan_destroy(fft_plan p);

/* Ragged plan (FP32): `count` transforms of sizes sizes[0..count) (each a
 * power of two in [1, 2^24]) packed back to back, transform i starting at
 * element sum_{j<i} sizes[j].  Executed as ONE HIP graph launch: persistent
 * kernels over fixed-size tiles (whole small transforms, or one pass of a
 * large one), one launch per pass level so that pass p - 1 of a large
 * transform finishes before pass p starts.  `sizes` is a host array, read
 * during the call only.  The plan's choices (pass lengths of the large
 * transforms, persistent grid size, tile order) come from the autotune cache
 * for this size histogram if present; FFT_AUTOTUNE=1 times every candidate
 * configuration at creation and records the fastest, as for fft_plan_create. */
/* Defined by: not a call of the paper - the batched form grows the method
 * toward serving systems; its per-size radix split and tile sizes are the
 * tiling hyperparameters of section 3, step 4, chosen by measuring candidate
 * plans, the runtime planner section 6 names as future work.  Every transform
 * of the batch is the DFT of Eq. 1. */
fft_status fft_plan_create_ragged(fft_plan *out, const int64_t *sizes,
                                  int64_t count, fft_layout layout,
                                  fft_direction dir);

/* fft_plan_create_ragged with an explicit configuration (the autotuner's
 * choices, bypassing cache and tuning): "ragged:p<P>:g<G>:o<O>[:w<W>][:s<S>]" with
 *   P  longest pass sub-FFT of the multi-pass transforms, 2^6 .. 2^8 (6..8)
 *   G  persistent workgroups per level, in eighths of the resident maximum (1..8)
 *   O  1: smallest multi-pass transforms first within a level, 0: largest
 *   W  pipelined groups of at most W MiB of workspace (8..65536): group g's
 *      pass p runs in level g + p, so each level reads what the previous one
 *      wrote while it can still be cached; the workspace is a ring of two
 *      group-sized slots.  Absent: every pass p in level p.
 *   S  largest size computed as one single-pass tile: 14 (2^14 on one
 *      workgroup, 32 points per thread) or 13 (2^14 then takes two passes).
 *      Absent: 14.
 * config NULL behaves as fft_plan_create_ragged.  A string that does not
 * parse is FFT_ERR_INVALID_ARG. */
fft_status fft_plan_create_ragged_ex(fft_plan *out, const int64_t *sizes,
                                     int64_t count, fft_layout layout,
                                     fft_direction dir, const char *config);

/* Bytes of device workspace the plan uses (0 for single-pass plans).
 * Defined by: the buffers between the passes of a multi-pass plan, Eq. 1
 * applied with M and K both larger than one pass (section 3), exposed
 * through the plan/execute API of section 4. */
fft_status fft_plan_workspace_bytes(fft_plan p, size_t *bytes);

/* Defined by: as fft_plan_workspace_bytes; the caller owns the memory, as the
 * caller owns every data pointer handed to the library (section 4).
 * Hand the plan a caller-owned device workspace of at least
 * fft_plan_workspace_bytes bytes (16-byte aligned); the plan frees its own.
 * NULL returns the plan to a workspace it allocates itself.  Executions of one
 * plan that overlap in time (different streams) race on the workspace. */
fft_status fft_plan_set_workspace(fft_plan p, void *dev_ptr);

/* Number of transforms, total complex elements per execution and the nominal
 * flop count (sum of 5 N log2 N, the paper's model in section 4). */
fft_status fft_plan_sizes(fft_plan p, int64_t *transforms, int64_t *elements,
                          double *nominal_flops);

/* For callers that cannot allocate device memory during execution (code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * fft_execute with the workspace of the multi-pass kernels taken from a static
 * device array of the library (fft_no_alloc_scratch_bytes() = 64 MiB per GPU,
 * held by every GPU the library is loaded on until the process ends) instead
 * of the plan's own.  The call allocates and frees nothing.  Arguments, layout,
 * ownership and results are those of fft_execute (bitwise the same output).
 * Plans whose workspace exceeds the scratch size return FFT_ERR_INVALID_SIZE,
 * ragged plans FFT_ERR_NOT_SUPPORTED, both before any launch.  All calls on one
 * GPU share its array: calls that overlap in time on one GPU (other streams,
 * other threads) race on it and must be ordered by the caller. */
fft_status fft_execute_no_alloc(fft_plan p, const void *in_re_or_z,
                                const void *in_im, void *out_re_or_z,
                                void *out_im, void *stream);

/* Size in bytes of the static scratch array behind fft_execute_no_alloc. */
size_t fft_no_alloc_scratch_bytes(void);

/* Human-readable JSON description of the chosen decomposition (kernel kind,
 * radices, passes, tiles) into buf (NUL-terminated, truncated to len). */
fft_status fft_plan_describe(fft_plan p, char *buf, size_t len);

/* Decomposition that fft_plan_create_ex would choose by default for
 * (n, layout, precision), and the autotuner's candidates, computed on the
 * host only (no GPU needed), as JSON into buf. */
fft_status fft_query_decomposition(int64_t n, fft_layout layout,
                                   fft_precision precision, char *buf,
                                   size_t len);

/* Plain streaming copy of `bytes` bytes (multiple of 16, 16-byte aligned
 * pointers; nontemporal 16-byte accesses): the practical HBM ceiling the
 * benchmark reports beside the FFT. */
fft_status fft_copy_device(const void *src, void *dst, size_t bytes, void *stream);

/* Static description of a status code.  Not defined by the paper: the
 * error reporting of this boundary (every entry point returns a status and
 * none aborts). */
const char *fft_status_string(fft_status s);

/* Detail of the most recent FFT_ERR_HIP / FFT_ERR_ALLOC on this thread
 * (the HIP error text), or "" if none. */
const char *fft_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* FFT_MI355X_H */
