/*
 * FP64 O(N^2) DFT oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU library never includes,
 * links or calls anything here, and nothing here is shared with it.
 *
 * What it computes (paper, Section II "Background", definition of DFT_N):
 *     y[k] = sum_{n=0}^{N-1} DFT_N[k,n] x[n],   DFT_N[k,n] = w_N^{k n},
 *     w_N = exp(-2 pi i / N)                    (forward, unnormalised)
 * i.e. the dense matrix-vector product that the paper calls the direct
 * DFT, with the same loop shape as its lowering of the matrix product to a
 * triple affine loop of complex multiply/add in complex<f64> (Listing 3).
 * The inverse (not defined by the paper) uses w_N^{-1}, also unnormalised.
 *
 * Precision choices (the paper computes in complex<f64> throughout):
 *  - twiddles: the table w[m] = exp(s 2 pi i m / N), m in [0,N), is built
 *    from libm cos/sin of an angle reduced to the first octant, with the
 *    eight multiples of pi/4 set exactly; this keeps w[N-m] = conj(w[m]) and
 *    w[m+N/2] = -w[m] exact.
 *  - the exponent k*n is reduced modulo N in exact integer arithmetic.
 *  - complex multiply is 4 mul + 2 add; build with -ffp-contract=off.
 *  - each of the real and imaginary sums is Neumaier-compensated.
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* cos and sin of 2 pi m / N for m in [0, N), N >= 1. */
static void unit_root(int64_t m, int64_t n, double *c, double *s)
{
    /* exact values at the multiples of pi/4, octant o = 8m/N */
    static const double ec[8] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440,
                                 -1.0, -0.70710678118654752440, 0.0, 0.70710678118654752440};
    static const double es[8] = {0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440,
                                 0.0, -0.70710678118654752440, -1.0, -0.70710678118654752440};
    const int64_t p = 8 * m;       /* angle = 2 pi p / (8N) */
    const int64_t o = p / n;       /* octant 0..7           */
    const int64_t e = p - o * n;   /* offset inside octant  */
    if (e == 0) {
        *c = ec[o];
        *s = es[o];
        return;
    }
    /* phi in (0, pi/4): for even octants measured up from o*pi/4, for odd
     * octants measured down from (o+1)*pi/4.                              */
    const int64_t q = (o & 1) ? (n - e) : e;
    const double phi = (M_PI * (double)q) / (4.0 * (double)n);
    const double cp = cos(phi), sp = sin(phi);
    switch (o) {
    case 0: *c = cp;  *s = sp;  break;  /* phi              */
    case 1: *c = sp;  *s = cp;  break;  /* pi/2 - phi       */
    case 2: *c = -sp; *s = cp;  break;  /* pi/2 + phi       */
    case 3: *c = -cp; *s = sp;  break;  /* pi - phi         */
    case 4: *c = -cp; *s = -sp; break;  /* pi + phi         */
    case 5: *c = -sp; *s = -cp; break;  /* 3pi/2 - phi      */
    case 6: *c = sp;  *s = -cp; break;  /* 3pi/2 + phi      */
    default: *c = cp; *s = -sp; break;  /* 2pi - phi        */
    }
}

/* Fill wr/wi with exp(sign * 2 pi i m / N), m in [0, N). */
int oracle_twiddles(int64_t n, int sign, double *wr, double *wi)
{
    if (n < 1 || (sign != 1 && sign != -1) || !wr || !wi)
        return -1;
    for (int64_t m = 0; m < n; ++m) {
        double c, s;
        unit_root(m, n, &c, &s);
        wr[m] = c;
        wi[m] = (double)sign * s;
    }
    return 0;
}

/* Neumaier step: sum += v with running compensation comp. */
static inline void neumaier(double *sum, double *comp, double v)
{
    const double t = *sum + v;
    if (fabs(*sum) >= fabs(v))
        *comp += (*sum - t) + v;
    else
        *comp += (v - t) + *sum;
    *sum = t;
}

/*
 * Batched DFT of `batch` contiguous transforms of length n.
 *   in, out : interleaved (re, im) doubles, element (b, j) at [2 (b n + j)]
 *   sign    : -1 forward (w_N = exp(-2 pi i/N)), +1 inverse; no scaling
 *   threads : OpenMP threads (<= 0: runtime default)
 * Returns 0, or -1 on a bad argument, -2 if the table cannot be allocated.
 * in and out must not overlap.
 */
int oracle_dft(const double *in, double *out, int64_t n, int64_t batch, int sign, int threads)
{
    if (n < 1 || batch < 0 || (sign != 1 && sign != -1) || (!in && batch) || (!out && batch))
        return -1;
    if (batch == 0)
        return 0;
    double *wr = (double *)malloc(sizeof(double) * (size_t)n);
    double *wi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!wr || !wi) {
        free(wr);
        free(wi);
        return -2;
    }
    oracle_twiddles(n, sign, wr, wi);
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    const int64_t total = batch * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t bk = 0; bk < total; ++bk) {
        const int64_t b = bk / n, k = bk - b * n;
        const double *x = in + 2 * b * n;
        double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
        int64_t idx = 0; /* (j k) mod n */
        for (int64_t j = 0; j < n; ++j) {
            const double a = x[2 * j], bb = x[2 * j + 1];
            const double c = wr[idx], d = wi[idx];
            const double pr = a * c - bb * d;
            const double pi = a * d + bb * c;
            neumaier(&sr, &cr, pr);
            neumaier(&si, &ci, pi);
            idx += k;
            if (idx >= n)
                idx -= n;
        }
        out[2 * bk] = sr + cr;
        out[2 * bk + 1] = si + ci;
    }
    free(wr);
    free(wi);
    return 0;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Selected outputs of one transform, straight from the definition:
 *   out[i] = sum_j x[j] w_N^{j k_i},  k_i = ks[i],  i < nk
 * (same table, exponent reduction, products and compensated sums as
 * oracle_dft).  For checking long transforms one output at a time.
 * Returns 0, -1 on a bad argument (k outside [0, n)), -2 on allocation failure.
 */
int oracle_dft_points(const double *in, int64_t n, int sign, const int64_t *ks, int64_t nk,
                      double *out, int threads)
{
    if (n < 1 || nk < 0 || (sign != 1 && sign != -1) || !in || (nk && (!ks || !out)))
        return -1;
    for (int64_t i = 0; i < nk; ++i)
        if (ks[i] < 0 || ks[i] >= n)
            return -1;
    double *wr = (double *)malloc(sizeof(double) * (size_t)n);
    double *wi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!wr || !wi) {
        free(wr);
        free(wi);
        return -2;
    }
    oracle_twiddles(n, sign, wr, wi);
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nk; ++i) {
        const int64_t k = ks[i];
        double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
        int64_t idx = 0;
        for (int64_t j = 0; j < n; ++j) {
            const double a = in[2 * j], bb = in[2 * j + 1];
            const double c = wr[idx], d = wi[idx];
            neumaier(&sr, &cr, a * c - bb * d);
            neumaier(&si, &ci, a * d + bb * c);
            idx += k;
            if (idx >= n)
                idx -= n;
        }
        out[2 * i] = sr + cr;
        out[2 * i + 1] = si + ci;
    }
    free(wr);
    free(wi);
    return 0;
}
