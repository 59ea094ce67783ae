/*
 * Oracle for the tall-and-skinny products of TSM2X (Rivera, Chen, Xiong,
 * Zhang, Song, Tao).  TEST INFRASTRUCTURE ONLY: the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may call it; the library
 * under paper_2002_03258_amd/ never does, and this file shares no code,
 * header or constant with it.
 *
 * Everything here is plain, unblocked, sequential-sum double precision C.
 *
 *  - tsm_oracle_matmul: the problem statement of the paper (Background,
 *    "Tall-and-Skinny Input for GEMM"): C = A*B with A m-by-k and B k-by-n,
 *    C[i,p] = sum over j of A[i,j]*B[j,p].  The sum is taken in increasing j,
 *    which is the order of the per-thread loop of the outer-product design
 *    (Design of TSM2R, Algorithm 2).  Element (i,j) of a matrix X lives at
 *    X[i*rs + j*cs], so column-major, row-major and transposed views are all
 *    the same routine.
 *  - tsm_oracle_grad: for the scalar L(A,B) = <dC, A*B> the gradients are
 *    dA = dC*B^T and dB = A^T*dC; both are the same definition applied to
 *    transposed views.
 *  - tsm_oracle_round: round-to-nearest, ties-to-even, of a real number to a
 *    binary floating-point format with p significand bits, minimum normal
 *    exponent emin and largest finite value max (IEEE 754 definition of
 *    roundTiesToEven, with gradual underflow).  bfloat16 is (8, -126),
 *    binary16 is (11, -14).
 *  - tsm_oracle_split: the storage form of A used by the low-precision path:
 *    hi = round(a), lo = round(a - hi).  a - hi is formed in double, where it
 *    is exact.
 *  - tsm_oracle_matmul_dot2: the same product with each sum taken by
 *    Dot2 (Ogita, Rump, Oishi, "Accurate sum and dot product", SIAM J. Sci.
 *    Comput. 26(6), 2005): every product is split exactly into its rounded
 *    value and error (TwoProduct, by fma), every addition likewise (TwoSum),
 *    and the errors are summed apart, so the result is as accurate as if the
 *    sum were taken in twice double precision and then rounded.  It measures
 *    the rounding error of the sequential sums at full size.
 *  - tsm_oracle_kmeans_assign: the assignment step of K-means, the
 *    application the paper's Introduction names as a tall-and-skinny GEMM
 *    user (many points, few centroids): each point goes to the centroid at
 *    the smallest squared Euclidean distance, sum over j of
 *    (x[i,j] - mu[j,c])^2, taken here as that definition (not expanded).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

void tsm_oracle_matmul(int64_t m, int64_t k, int64_t n,
                       const double* A, int64_t a_rs, int64_t a_cs,
                       const double* B, int64_t b_rs, int64_t b_cs,
                       double* C, int64_t c_rs, int64_t c_cs)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        for (int64_t p = 0; p < n; ++p) {
            double s = 0.0;
            for (int64_t j = 0; j < k; ++j)
                s += A[i * a_rs + j * a_cs] * B[j * b_rs + p * b_cs];
            C[i * c_rs + p * c_cs] = s;
        }
    }
}

/* TwoSum (Knuth): s + e == a + b exactly, s = fl(a + b). */
static void two_sum(double a, double b, double* s, double* e)
{
    const double x = a + b;
    const double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* C = A*B with each C[i,p] by Dot2: sum of the TwoProduct/TwoSum errors
 * carried beside the running sum, added once at the end. */
void tsm_oracle_matmul_dot2(int64_t m, int64_t k, int64_t n,
                            const double* A, int64_t a_rs, int64_t a_cs,
                            const double* B, int64_t b_rs, int64_t b_cs,
                            double* C, int64_t c_rs, int64_t c_cs)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        for (int64_t p = 0; p < n; ++p) {
            double s = 0.0, c = 0.0;
            for (int64_t j = 0; j < k; ++j) {
                const double x = A[i * a_rs + j * a_cs], y = B[j * b_rs + p * b_cs];
                const double h = x * y;
                const double r = fma(x, y, -h);         /* x*y == h + r exactly */
                double t, q;
                two_sum(s, h, &t, &q);
                s = t;
                c += q + r;
            }
            C[i * c_rs + p * c_cs] = s + c;
        }
    }
}

/* Column-major inputs: A m-by-k (lda), dC m-by-n (lddc), B k-by-n (ldb).
 * Writes dA m-by-k (ldda) = dC*B^T and dB k-by-n (lddb) = A^T*dC.
 * Either output pointer may be NULL to skip it. */
void tsm_oracle_grad(int64_t m, int64_t k, int64_t n,
                     const double* A, int64_t lda,
                     const double* B, int64_t ldb,
                     const double* dC, int64_t lddc,
                     double* dA, int64_t ldda,
                     double* dB, int64_t lddb)
{
    /* dA[i,j] = sum_p dC[i,p] * B^T[p,j],  B^T[p,j] = B[j,p] */
    if (dA)
        tsm_oracle_matmul(m, n, k, dC, 1, lddc, B, ldb, 1, dA, 1, ldda);
    /* dB[j,p] = sum_i A^T[j,i] * dC[i,p],  A^T[j,i] = A[i,j] */
    if (dB)
        tsm_oracle_matmul(k, m, n, A, lda, 1, dC, 1, lddc, dB, 1, lddb);
}

/* Round x to the nearest value with p significand bits, ties to even, for a
 * format whose smallest normal number is 2^emin and whose largest finite
 * number is maxval.  Overflow gives +-inf, NaN stays NaN, the sign of zero
 * is kept. */
double tsm_oracle_round(double x, int p, int emin, double maxval)
{
    if (isnan(x) || isinf(x) || x == 0.0)
        return x;
    int e;
    frexp(fabs(x), &e);          /* |x| = f * 2^e, f in [0.5, 1) */
    int ex = e - 1;              /* |x| in [2^ex, 2^(ex+1)) */
    if (ex < emin)
        ex = emin;               /* gradual underflow: fixed spacing */
    double ulp = ldexp(1.0, ex - (p - 1));
    double q = x / ulp;          /* exact: a power-of-two scaling */
    double r = nearbyint(q);     /* default mode is ties-to-even */
    double v = r * ulp;
    /* Values at or above max + ulp/2 overflow; max itself is representable. */
    if (fabs(v) > maxval)
        return x > 0 ? INFINITY : -INFINITY;
    return v;
}

static double fmt_max(int fmt)
{
    /* bfloat16: (2 - 2^-7) * 2^127 ; binary16: (2 - 2^-10) * 2^15 */
    return fmt == 0 ? ldexp(2.0 - ldexp(1.0, -7), 127)
                    : ldexp(2.0 - ldexp(1.0, -10), 15);
}

double tsm_oracle_round_fmt(double x, int fmt)
{
    return fmt == 0 ? tsm_oracle_round(x, 8, -126, fmt_max(0))
                    : tsm_oracle_round(x, 11, -14, fmt_max(1));
}

/* Encode a value that is exactly representable in the format into its
 * 16-bit pattern. */
uint16_t tsm_oracle_encode(double v, int fmt)
{
    if (fmt == 0) {
        float f = (float)v;      /* exact: bfloat16 values are binary32 values */
        uint32_t u;
        memcpy(&u, &f, 4);
        if (isnan(v))
            return (uint16_t)(((u >> 16) & 0x8000u) | 0x7FC0u);
        return (uint16_t)(u >> 16);
    }
    uint16_t sign = signbit(v) ? 0x8000u : 0u;
    if (isnan(v))
        return 0x7E00u;
    double a = fabs(v);
    if (isinf(a))
        return sign | 0x7C00u;
    if (a == 0.0)
        return sign;
    if (a < ldexp(1.0, -14))                      /* subnormal: a = m * 2^-24 */
        return sign | (uint16_t)(a / ldexp(1.0, -24));
    int e;
    double f = frexp(a, &e);                      /* a = f * 2^e, f in [0.5,1) */
    uint16_t bexp = (uint16_t)(e - 1 + 15);
    uint16_t mant = (uint16_t)((f * 2.0 - 1.0) * 1024.0);
    return sign | (uint16_t)(bexp << 10) | mant;
}

double tsm_oracle_decode(uint16_t h, int fmt)
{
    if (fmt == 0) {
        uint32_t u = (uint32_t)h << 16;
        float f;
        memcpy(&f, &u, 4);
        return (double)f;
    }
    int sign = (h >> 15) & 1, bexp = (h >> 10) & 31, mant = h & 1023;
    double v;
    if (bexp == 0)
        v = ldexp((double)mant, -24);
    else if (bexp == 31)
        v = mant ? NAN : INFINITY;
    else
        v = ldexp(1.0 + mant / 1024.0, bexp - 15);
    return sign ? -v : v;
}

/* hi[i] = round(a[i]); lo[i] = round(a[i] - hi[i]) when lo != NULL. */
void tsm_oracle_split(const float* a, int64_t count, int fmt,
                      uint16_t* hi, uint16_t* lo)
{
    for (int64_t i = 0; i < count; ++i) {
        double x = (double)a[i];
        double h = tsm_oracle_round_fmt(x, fmt);
        hi[i] = tsm_oracle_encode(h, fmt);
        if (lo) {
            double r = (isinf(h) || isnan(h)) ? h : x - h;   /* exact */
            lo[i] = tsm_oracle_encode(tsm_oracle_round_fmt(r, fmt), fmt);
        }
    }
}

int tsm_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the row loops from now on (timing only; results do not depend
   on it: each output is summed by one thread in j order). */
void tsm_oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Points X (m-by-k, element (i,j) at X[i*x_rs + j*x_cs]) and centroids
 * (k-by-n, centroid c is column c, element (j,c) at Mu[j*m_rs + c*m_cs]).
 * label[i] = the smallest c with the smallest D[i,c] = sum_j (x_ij - mu_jc)^2
 * (NaN distances never compare smaller; a row with no non-NaN distance gets
 * label 0); dist[i] = D[i, label[i]] (dist may be NULL). */
void tsm_oracle_kmeans_assign(int64_t m, int64_t k, int64_t n,
                              const double* X, int64_t x_rs, int64_t x_cs,
                              const double* Mu, int64_t m_rs, int64_t m_cs,
                              int32_t* label, double* dist)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        int64_t best = -1;
        double bd = 0.0;
        for (int64_t c = 0; c < n; ++c) {
            double d = 0.0;
            for (int64_t j = 0; j < k; ++j) {
                const double e = X[i * x_rs + j * x_cs] - Mu[j * m_rs + c * m_cs];
                d += e * e;
            }
            if (d != d) continue;
            if (best < 0 || d < bd) {
                best = c;
                bd = d;
            }
        }
        if (best < 0) {                 /* every distance is NaN */
            double d = 0.0;
            for (int64_t j = 0; j < k; ++j) {
                const double e = X[i * x_rs + j * x_cs] - Mu[j * m_rs];
                d += e * e;
            }
            best = 0;
            bd = d;
        }
        label[i] = (int32_t)best;
        if (dist) dist[i] = bd;
    }
}
