/*
 * FP64 CPU oracle for the 1D complex-to-complex DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP path.
 *
 * What it computes (the paper, section 3, Eq. 1 and the surrounding text):
 * the DFT of size N, which Eq. 1 factors exactly into radix stages.  The paper
 * never prints the DFT formula; the sign and normalisation follow the library
 * it compares against in section 4 (forward exponent -2*pi*i*k*n/N, no
 * scaling; inverse exponent +2*pi*i*k*n/N, no scaling):
 *
 *     X[k] = sum_{n=0}^{N-1} x[n] * exp(sign * 2*pi*i * k*n / N)
 *
 * with sign = -1 (forward) or +1 (inverse).  All arithmetic is IEEE double.
 *
 * Routines
 *   oracle_dft          O(N^2) definition, the dense form the paper started
 *                       from (section 3, step 1; section 4).
 *   oracle_fft_r2       recursive radix-2 decimation in time: Eq. 1 with
 *                       K = 2 applied recursively (section 3).
 *   oracle_fft_r2_batch the same over a batch, optionally on several threads.
 *   oracle_wpower_loss  L = sum_k w_k |(F x)_k|^2 (the differentiable workload).
 *   oracle_wpower_grad  dL/dRe(x) + i dL/dIm(x) = 2 F^H (w .* F x).
 *   oracle_rfft_batch   the DFT of real sequences, its non-redundant half
 *                       k = 0 .. N/2 (real-to-complex).
 *   oracle_irfft_batch  the unnormalised inverse DFT of the Hermitian
 *                       extension of such a half, real part
 *                       (complex-to-real).
 *
 * Error behaviour: every routine returns 0 on success, -1 on a bad argument
 * (N not positive, N not a power of two where one is required, sign not +-1)
 * and -2 when memory cannot be allocated.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* 2*pi to more digits than a double holds. */
static const double ORACLE_TWO_PI = 6.28318530717958647692528676655900577;

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* Unit-circle table: c[m] = cos(2 pi m / n), s[m] = sin(2 pi m / n), m < n.
 * Each entry comes straight from libm with the exact rational argument m/n,
 * so no error accumulates across entries. */
static int unit_circle(int64_t n, double **c, double **s)
{
    *c = (double *)malloc(sizeof(double) * (size_t)n);
    *s = (double *)malloc(sizeof(double) * (size_t)n);
    if (!*c || !*s) {
        free(*c);
        free(*s);
        *c = *s = NULL;
        return -2;
    }
    for (int64_t m = 0; m < n; ++m) {
        double a = ORACLE_TWO_PI * (double)m / (double)n;
        (*c)[m] = cos(a);
        (*s)[m] = sin(a);
    }
    return 0;
}

/* ---- O(N^2) definition ------------------------------------------------ */

int oracle_dft(int64_t n, int sign, const double *xr, const double *xi,
               double *yr, double *yi)
{
    if (n <= 0 || (sign != 1 && sign != -1))
        return -1;
    double *c, *s;
    int rc = unit_circle(n, &c, &s);
    if (rc)
        return rc;
    for (int64_t k = 0; k < n; ++k) {
        double acc_r = 0.0, acc_i = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            /* exponent reduced exactly in integers: k*j mod n */
            int64_t m = (int64_t)(((unsigned __int128)k * (unsigned __int128)j) % (unsigned __int128)n);
            double wr = c[m];
            double wi = (double)sign * s[m];
            acc_r += xr[j] * wr - xi[j] * wi;
            acc_i += xr[j] * wi + xi[j] * wr;
        }
        yr[k] = acc_r;
        yi[k] = acc_i;
    }
    free(c);
    free(s);
    return 0;
}

/* ---- recursive radix-2 decimation in time ----------------------------- */

/* Transform the n samples x[0], x[stride], x[2*stride], ... into y[0..n).
 * The DFT of size n is split into the DFTs E and O of the even and odd
 * samples (Eq. 1 with K = 2, M = n/2), recombined as
 *     y[k]       = E[k] + w^k O[k]
 *     y[k + n/2] = E[k] - w^k O[k],      w = exp(sign 2 pi i / n),
 * where w^k is entry k*tstep of the size-N unit-circle table. */
static void r2_rec(const double *xr, const double *xi, int64_t stride, int64_t n,
                   double *yr, double *yi, const double *c, const double *s,
                   int64_t tstep, double sign)
{
    if (n == 1) {
        yr[0] = xr[0];
        yi[0] = xi[0];
        return;
    }
    int64_t h = n / 2;
    r2_rec(xr, xi, 2 * stride, h, yr, yi, c, s, 2 * tstep, sign);
    r2_rec(xr + stride, xi + stride, 2 * stride, h, yr + h, yi + h, c, s, 2 * tstep, sign);
    for (int64_t k = 0; k < h; ++k) {
        double wr = c[k * tstep];
        double wi = sign * s[k * tstep];
        double er = yr[k], ei = yi[k];
        double orr = yr[h + k] * wr - yi[h + k] * wi;
        double oi = yr[h + k] * wi + yi[h + k] * wr;
        yr[k] = er + orr;
        yi[k] = ei + oi;
        yr[h + k] = er - orr;
        yi[h + k] = ei - oi;
    }
}

int oracle_fft_r2(int64_t n, int sign, const double *xr, const double *xi,
                  double *yr, double *yi)
{
    if (!is_pow2(n) || (sign != 1 && sign != -1))
        return -1;
    double *c, *s;
    int rc = unit_circle(n, &c, &s);
    if (rc)
        return rc;
    r2_rec(xr, xi, 1, n, yr, yi, c, s, 1, (double)sign);
    free(c);
    free(s);
    return 0;
}

/* ---- batch over threads ------------------------------------------------ */

typedef struct {
    int64_t n, first, count;
    double sign;
    const double *xr, *xi;
    double *yr, *yi;
    const double *c, *s;
} r2_job;

static void *r2_worker(void *arg)
{
    r2_job *jb = (r2_job *)arg;
    for (int64_t b = jb->first; b < jb->first + jb->count; ++b) {
        int64_t off = b * jb->n;
        r2_rec(jb->xr + off, jb->xi + off, 1, jb->n, jb->yr + off, jb->yi + off,
               jb->c, jb->s, 1, jb->sign);
    }
    return NULL;
}

/* Batch of `batch` contiguous transforms of size n (row b at offset b*n).
 * nthreads <= 1 runs on the calling thread. */
int oracle_fft_r2_batch(int64_t n, int64_t batch, int sign, const double *xr,
                        const double *xi, double *yr, double *yi, int nthreads)
{
    if (!is_pow2(n) || batch < 0 || (sign != 1 && sign != -1))
        return -1;
    if (batch == 0)
        return 0;
    double *c, *s;
    int rc = unit_circle(n, &c, &s);
    if (rc)
        return rc;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > batch)
        nthreads = (int)batch;
    r2_job *jobs = (r2_job *)calloc((size_t)nthreads, sizeof(r2_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        free(c);
        free(s);
        return -2;
    }
    int64_t per = batch / nthreads, extra = batch % nthreads, first = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].n = n;
        jobs[t].first = first;
        jobs[t].count = per + (t < extra ? 1 : 0);
        jobs[t].sign = (double)sign;
        jobs[t].xr = xr;
        jobs[t].xi = xi;
        jobs[t].yr = yr;
        jobs[t].yi = yi;
        jobs[t].c = c;
        jobs[t].s = s;
        first += jobs[t].count;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t) {
        if (pthread_create(&tids[t], NULL, r2_worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    r2_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        pthread_join(tids[t], NULL);
    /* any job whose thread could not start runs here */
    for (int t = started + 1; t < nthreads; ++t)
        r2_worker(&jobs[t]);
    free(jobs);
    free(tids);
    free(c);
    free(s);
    return 0;
}

/* ---- the differentiable workload --------------------------------------- */

/* L(x) = sum_k w[k] * |X[k]|^2 with X = F x (forward DFT). */
int oracle_wpower_loss(int64_t n, const double *xr, const double *xi,
                       const double *w, double *loss)
{
    if (!is_pow2(n))
        return -1;
    double *yr = (double *)malloc(sizeof(double) * (size_t)n);
    double *yi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!yr || !yi) {
        free(yr);
        free(yi);
        return -2;
    }
    int rc = oracle_fft_r2(n, -1, xr, xi, yr, yi);
    if (rc == 0) {
        double acc = 0.0;
        for (int64_t k = 0; k < n; ++k)
            acc += w[k] * (yr[k] * yr[k] + yi[k] * yi[k]);
        *loss = acc;
    }
    free(yr);
    free(yi);
    return rc;
}

/* Gradient of L with respect to the real pair (Re x, Im x), packed as
 * g = dL/dRe(x) + i dL/dIm(x).  With X = F x and L = sum_k w_k |X_k|^2,
 * dL/dRe(X_k) + i dL/dIm(X_k) = 2 w_k X_k, and the chain rule through the
 * linear map F gives g = F^H (2 w .* X), F^H being the unnormalised inverse. */
int oracle_wpower_grad(int64_t n, const double *xr, const double *xi,
                       const double *w, double *gr, double *gi)
{
    if (!is_pow2(n))
        return -1;
    double *yr = (double *)malloc(sizeof(double) * (size_t)n);
    double *yi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!yr || !yi) {
        free(yr);
        free(yi);
        return -2;
    }
    int rc = oracle_fft_r2(n, -1, xr, xi, yr, yi);
    if (rc == 0) {
        for (int64_t k = 0; k < n; ++k) {
            yr[k] *= 2.0 * w[k];
            yi[k] *= 2.0 * w[k];
        }
        rc = oracle_fft_r2(n, +1, yr, yi, gr, gi);
    }
    free(yr);
    free(yi);
    return rc;
}

/* ---- real sequences: the non-redundant half ---------------------------- */

/* Real-to-complex.  For real x of length n the DFT satisfies
 * X[n - k] = conj(X[k]), so X[0 .. n/2] carries all of it.  This computes
 * exactly those n/2 + 1 values of the forward DFT of (x, 0): the complex
 * transform of the real row with a zero imaginary part, truncated.  Output
 * row b starts at b * (n/2 + 1). */
int oracle_rfft_batch(int64_t n, int64_t batch, const double *x, double *yr,
                      double *yi, int nthreads)
{
    if (!is_pow2(n) || batch < 0)
        return -1;
    if (batch == 0)
        return 0;
    const int64_t h = n / 2 + 1;
    const size_t total = (size_t)n * (size_t)batch;
    double *zi = (double *)calloc(total, sizeof(double));
    double *fr = (double *)malloc(total * sizeof(double));
    double *fi = (double *)malloc(total * sizeof(double));
    int rc = -2;
    if (zi && fr && fi)
        rc = oracle_fft_r2_batch(n, batch, -1, x, zi, fr, fi, nthreads);
    if (rc == 0) {
        for (int64_t b = 0; b < batch; ++b) {
            for (int64_t k = 0; k < h; ++k) {
                yr[b * h + k] = fr[b * n + k];
                yi[b * h + k] = fi[b * n + k];
            }
        }
    }
    free(zi);
    free(fr);
    free(fi);
    return rc;
}

/* Complex-to-real.  Input rows X[0 .. n/2] (n/2 + 1 values each).  The
 * Hermitian extension is Xe[k] = X[k] for k <= n/2 and conj(X[n - k]) for
 * k > n/2; the output is the real part of its unnormalised inverse DFT,
 *     y[m] = Re sum_{k<n} Xe[k] exp(+2 pi i k m / n),
 * so that C2R(R2C(x)) = n x.  Imaginary parts of X[0] and X[n/2] drop out
 * of the real part. */
int oracle_irfft_batch(int64_t n, int64_t batch, const double *xr,
                       const double *xi, double *y, int nthreads)
{
    if (!is_pow2(n) || batch < 0)
        return -1;
    if (batch == 0)
        return 0;
    const int64_t h = n / 2 + 1;
    const size_t total = (size_t)n * (size_t)batch;
    double *er = (double *)malloc(total * sizeof(double));
    double *ei = (double *)malloc(total * sizeof(double));
    double *fr = (double *)malloc(total * sizeof(double));
    double *fi = (double *)malloc(total * sizeof(double));
    int rc = -2;
    if (er && ei && fr && fi) {
        for (int64_t b = 0; b < batch; ++b) {
            for (int64_t k = 0; k < n; ++k) {
                if (k <= n / 2) {
                    er[b * n + k] = xr[b * h + k];
                    ei[b * n + k] = xi[b * h + k];
                } else {
                    er[b * n + k] = xr[b * h + (n - k)];
                    ei[b * n + k] = -xi[b * h + (n - k)];
                }
            }
        }
        rc = oracle_fft_r2_batch(n, batch, 1, er, ei, fr, fi, nthreads);
        if (rc == 0)
            memcpy(y, fr, total * sizeof(double));
    }
    free(er);
    free(ei);
    free(fr);
    free(fi);
    return rc;
}
