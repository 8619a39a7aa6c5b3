/*
 * oracle_fft.c -- FP64 reference 1-D DFT for the oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the oracle package loads it (through ctypes) for tests, the
 * smoke check and the benchmark's CPU-baseline leg.
 *
 * What it computes: the 1-D DFT of the paper's Eq. (1),
 *     Xbar(k) = sum_{j=0}^{n-1} w_n^{jk} X(j),   w_n = exp(sign * 2*pi*i / n),
 * with sign = -1 for the forward transform (the paper's w_N = e^{-2 pi i/N},
 * no normalisation factor) and sign = +1 for the unscaled backward sum.
 *
 * How: plain recursive decimation in time.  Let r be the smallest prime factor
 * of n and m = n / r.  The r interleaved subsequences X(q + r j), j < m, are
 * transformed recursively (Y_q), and then
 *     Xbar(K) = sum_{q<r} w_n^{q K} Y_q(K mod m),   K = 0..n-1,
 * which is Eq. (1) with j = q + r j' regrouped.  A prime n is summed directly
 * from Eq. (1).  Every exponent is reduced modulo n in exact integer
 * arithmetic before sin/cos are called.  No blocking, no special-cased radix
 * butterflies: it is meant to be read against Eq. (1), not to be fast.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double ORACLE_TWO_PI = 6.283185307179586476925286766559;

/* w_n^e with e already reduced into [0, n). */
static cplx root_of_unity(int64_t e, int64_t n, int sign)
{
    double ang = ORACLE_TWO_PI * (double)e / (double)n;
    return cos(ang) + (double)sign * sin(ang) * I;
}

static int64_t smallest_prime_factor(int64_t n)
{
    for (int64_t p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* Direct evaluation of Eq. (1) for one sequence (stride in elements). */
static void dft_direct(const cplx *in, int64_t stride, int64_t n, cplx *out, int sign)
{
    for (int64_t k = 0; k < n; ++k) {
        cplx s = 0;
        for (int64_t j = 0; j < n; ++j)
            s += root_of_unity((j * k) % n, n, sign) * in[j * stride];
        out[k] = s;
    }
}

/*
 * out[0..n) = DFT of in[0], in[stride], ..., in[(n-1) stride].
 * scratch must hold 2n elements (this level uses n, the children use the rest).
 */
static void fft_rec(const cplx *in, int64_t stride, int64_t n, cplx *out,
                    int sign, cplx *scratch)
{
    if (n == 1) { out[0] = in[0]; return; }
    int64_t r = smallest_prime_factor(n);
    if (r == n) { dft_direct(in, stride, n, out, sign); return; }
    int64_t m = n / r;

    /* Y_q occupies out[q*m .. q*m+m). */
    for (int64_t q = 0; q < r; ++q)
        fft_rec(in + q * stride, stride * r, m, out + q * m, sign, scratch + n);

    cplx *tmp = scratch;
    for (int64_t K = 0; K < n; ++K) {
        cplx s = 0;
        for (int64_t q = 0; q < r; ++q)
            s += root_of_unity((q * K) % n, n, sign) * out[q * m + (K % m)];
        tmp[K] = s;
    }
    memcpy(out, tmp, (size_t)n * sizeof(cplx));
}

/*
 * Transform nrows contiguous rows of length n in place.  data holds
 * interleaved (re, im) doubles.  Rows are independent, so they are spread
 * over OpenMP threads when the library is built with -fopenmp.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_fft_rows(double *data, int64_t nrows, int64_t n, int sign)
{
    if (!data || nrows < 0 || n < 1 || (sign != 1 && sign != -1)) return -1;
    int failed = 0;
#pragma omp parallel
    {
        cplx *row = (cplx *)malloc((size_t)n * sizeof(cplx));
        cplx *res = (cplx *)malloc((size_t)n * sizeof(cplx));
        cplx *scr = (cplx *)malloc((size_t)(2 * n) * sizeof(cplx));
        if (!row || !res || !scr) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t b = 0; b < nrows; ++b) {
                cplx *src = (cplx *)(data + 2 * b * n);
                memcpy(row, src, (size_t)n * sizeof(cplx));
                fft_rec(row, 1, n, res, sign, scr);
                memcpy(src, res, (size_t)n * sizeof(cplx));
            }
        }
        free(row); free(res); free(scr);
    }
    return failed ? -1 : 0;
}

/* Threads for later OpenMP regions (no effect without OpenMP). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of threads an OpenMP region would use (1 without OpenMP). */
int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
