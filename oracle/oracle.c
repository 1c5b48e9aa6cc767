/*
 * Strassen GEMM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU code that states what the GPU path must
 * compute.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product library never does, and this file
 * shares no code, header, table or constant with the HIP path.
 *
 * Problem (Introduction, eq. "prime"):   C := alpha * A * B + beta * C
 *   A is m x k, B is k x n, C is m x n, all row-major with leading
 *   dimensions lda, ldb, ldc (element (i,j) of X lives at X[i*ldX + j]).
 *
 * Functions
 *   oracle_gemm_f64      the classical definition, evaluated in fp64.
 *   oracle_strassen      the paper's seven-product scheme (Method section,
 *                        eq. "gpu_allops") applied recursively `levels`
 *                        times on quadrants of ceil(dim/2) (eq.
 *                        "strassenpart"), with explicit zero-padded copies for
 *                        odd dimensions, and the classical product below the
 *                        last level.  round32 = 0 runs it in fp64; round32 = 1
 *                        rounds every sum and product to IEEE binary32, which
 *                        predicts the rounding level of an fp32 implementation
 *                        of the same scheme (used only to calibrate the
 *                        tolerance of parity tests).
 *
 * Conventions (readings of the paper, which fixes alpha = beta = 1):
 *   - beta == 0 means C is write-only: its old contents are never read.
 *   - alpha == 0 or k == 0 means C := beta * C; A and B are not read.
 *   - The scheme accumulates C += M_i; alpha and beta are applied once at the
 *     top: C := beta*C, then C += alpha * (A*B evaluated by the scheme).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math, no
 * contraction, so every operation rounds exactly as written).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;

/* ------------------------------------------------------------------ */
/* Classical product, the plain definition of eq. "prime".             */
/* ------------------------------------------------------------------ */

/* C[i,j] := alpha * sum_l A[i,l] * B[l,j] + beta * C[i,j], summed in order
 * l = 0, 1, ..., k-1 in fp64.  Rows of C are independent and are spread over
 * OpenMP threads. Returns 0, or -1 if scratch memory could not be allocated. */
int oracle_gemm_f64(i64 m, i64 n, i64 k,
                    const double *A, i64 lda,
                    const double *B, i64 ldb,
                    double *C, i64 ldc,
                    double alpha, double beta)
{
    int failed = 0;
    if (m <= 0 || n <= 0) return 0;
    const int use_product = (k > 0 && alpha != 0.0);
#pragma omp parallel
    {
        double *acc = (double *)malloc((size_t)n * sizeof(double));
        if (!acc) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (i64 i = 0; i < m; ++i) {
            if (!acc) continue;
            for (i64 j = 0; j < n; ++j) acc[j] = 0.0;
            if (use_product) {
                for (i64 l = 0; l < k; ++l) {
                    const double a = A[i * lda + l];
                    const double *b = B + l * ldb;
                    for (i64 j = 0; j < n; ++j) acc[j] += a * b[j];
                }
            }
            double *c = C + i * ldc;
            for (i64 j = 0; j < n; ++j) {
                const double old = (beta == 0.0) ? 0.0 : beta * c[j];
                c[j] = (use_product ? alpha * acc[j] : 0.0) + old;
            }
        }
        free(acc);
    }
    return failed ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Strassen recursion (Method section).                                */
/* ------------------------------------------------------------------ */

/* Rounds x to binary32 when emulating fp32 arithmetic.  Sums and products of
 * two binary32 values formed in binary64 and then rounded to binary32 equal
 * the correctly rounded binary32 result (binary64 carries more than twice the
 * binary32 precision plus two bits), so this emulates fp32 exactly. */
static inline double rnd(double x, int round32)
{
    return round32 ? (double)(float)x : x;
}

/* The seven products of eq. "gpu_allops".  Quadrant q of a matrix (eq.
 * "strassenpart") is row half q / 2, column half q % 2:
 *   0 = top-left, 1 = top-right, 2 = bottom-left, 3 = bottom-right.
 * Each product lists its signed A quadrants (summed into the left factor),
 * its signed B quadrants (summed into the right factor) and the signed C
 * quadrants it is added into. */
typedef struct {
    int na, a[2], sa[2];
    int nb, b[2], sb[2];
    int nc, c[2], sc[2];
} product_t;

static const product_t SEVEN[7] = {
    /* M0 = (A0 + A3)(B0 + B3);  C0 += M0;  C3 += M0 */
    {2, {0, 3}, {+1, +1}, 2, {0, 3}, {+1, +1}, 2, {0, 3}, {+1, +1}},
    /* M1 = (A2 + A3) B0;        C2 += M1;  C3 -= M1 */
    {2, {2, 3}, {+1, +1}, 1, {0, 0}, {+1, 0}, 2, {2, 3}, {+1, -1}},
    /* M2 = A0 (B1 - B3);        C1 += M2;  C3 += M2 */
    {1, {0, 0}, {+1, 0}, 2, {1, 3}, {+1, -1}, 2, {1, 3}, {+1, +1}},
    /* M3 = A3 (B2 - B0);        C0 += M3;  C2 += M3 */
    {1, {3, 0}, {+1, 0}, 2, {2, 0}, {+1, -1}, 2, {0, 2}, {+1, +1}},
    /* M4 = (A0 + A1) B3;        C1 += M4;  C0 -= M4 */
    {2, {0, 1}, {+1, +1}, 1, {3, 0}, {+1, 0}, 2, {1, 0}, {+1, -1}},
    /* M5 = (A2 - A0)(B0 + B1);  C3 += M5 */
    {2, {2, 0}, {+1, -1}, 2, {0, 1}, {+1, +1}, 1, {3, 0}, {+1, 0}},
    /* M6 = (A1 - A3)(B2 + B3);  C0 += M6 */
    {2, {1, 3}, {+1, -1}, 2, {2, 3}, {+1, +1}, 1, {0, 0}, {+1, 0}},
};

/* Classical C += A*B (C is accumulated into, never scaled), with every
 * product and every partial sum rounded when round32 is set. */
static void classical_acc(i64 m, i64 n, i64 k,
                          const double *A, i64 lda, const double *B, i64 ldb,
                          double *C, i64 ldc, int round32)
{
    for (i64 i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        for (i64 l = 0; l < k; ++l) {
            const double a = A[i * lda + l];
            const double *b = B + l * ldb;
            for (i64 j = 0; j < n; ++j)
                c[j] = rnd(c[j] + rnd(a * b[j], round32), round32);
        }
    }
}

/* Copies quadrant q (of size hr x hc, origin (q/2)*hr, (q%2)*hc) of the
 * r x c matrix X into the dense hr x hc buffer Q, writing zeros where the
 * quadrant extends past the matrix (padding for odd dimensions). */
static void take_quadrant(const double *X, i64 ldx, i64 r, i64 c,
                          int q, i64 hr, i64 hc, double *Q)
{
    const i64 r0 = (i64)(q / 2) * hr, c0 = (i64)(q % 2) * hc;
    for (i64 i = 0; i < hr; ++i)
        for (i64 j = 0; j < hc; ++j) {
            const i64 gi = r0 + i, gj = c0 + j;
            Q[i * hc + j] = (gi < r && gj < c) ? X[gi * ldx + gj] : 0.0;
        }
}

/* C += A*B by `levels` levels of the seven-product scheme. Returns 0, or -1
 * on allocation failure. */
static int strassen_acc(i64 m, i64 n, i64 k,
                        const double *A, i64 lda, const double *B, i64 ldb,
                        double *C, i64 ldc, int levels, int round32)
{
    if (levels == 0 || m == 0 || n == 0 || k == 0) {
        classical_acc(m, n, k, A, lda, B, ldb, C, ldc, round32);
        return 0;
    }
    const i64 hm = (m + 1) / 2, hn = (n + 1) / 2, hk = (k + 1) / 2;
    const size_t sa = (size_t)(hm * hk), sb = (size_t)(hk * hn),
                 sc = (size_t)(hm * hn);
    double *Aq = (double *)malloc(4 * sa * sizeof(double));
    double *Bq = (double *)malloc(4 * sb * sizeof(double));
    double *P = (double *)malloc(sa * sizeof(double));
    double *Q = (double *)malloc(sb * sizeof(double));
    double *M = (double *)malloc(sc * sizeof(double));
    int rc = 0;
    if (!Aq || !Bq || !P || !Q || !M) {
        rc = -1;
        goto done;
    }
    for (int q = 0; q < 4; ++q) {
        take_quadrant(A, lda, m, k, q, hm, hk, Aq + q * sa);
        take_quadrant(B, ldb, k, n, q, hk, hn, Bq + q * sb);
    }
    for (int p = 0; p < 7; ++p) {
        const product_t *t = &SEVEN[p];
        /* left factor: sum of signed A quadrants */
        for (size_t e = 0; e < sa; ++e) {
            double s = t->sa[0] * Aq[t->a[0] * sa + e];
            if (t->na == 2) s = rnd(s + t->sa[1] * Aq[t->a[1] * sa + e], round32);
            P[e] = s;
        }
        /* right factor: sum of signed B quadrants */
        for (size_t e = 0; e < sb; ++e) {
            double s = t->sb[0] * Bq[t->b[0] * sb + e];
            if (t->nb == 2) s = rnd(s + t->sb[1] * Bq[t->b[1] * sb + e], round32);
            Q[e] = s;
        }
        /* M = P*Q, one level further down */
        memset(M, 0, sc * sizeof(double));
        rc = strassen_acc(hm, hn, hk, P, hk, Q, hn, M, hn, levels - 1, round32);
        if (rc) goto done;
        /* signed scatter of M into its C quadrants, clipped to C's extent */
        for (int o = 0; o < t->nc; ++o) {
            const int q = t->c[o];
            const double g = (double)t->sc[o];
            const i64 r0 = (i64)(q / 2) * hm, c0 = (i64)(q % 2) * hn;
            for (i64 i = 0; i < hm && r0 + i < m; ++i)
                for (i64 j = 0; j < hn && c0 + j < n; ++j) {
                    double *cij = C + (r0 + i) * ldc + (c0 + j);
                    *cij = rnd(*cij + g * M[i * hn + j], round32);
                }
        }
    }
done:
    free(Aq);
    free(Bq);
    free(P);
    free(Q);
    free(M);
    return rc;
}

/* C := alpha * (A*B by `levels` levels of Strassen) + beta * C.
 * levels >= 0; round32 in {0, 1}.  Returns 0 on success, -1 on allocation
 * failure, -2 on a bad argument. */
int oracle_strassen(i64 m, i64 n, i64 k,
                    const double *A, i64 lda,
                    const double *B, i64 ldb,
                    double *C, i64 ldc,
                    double alpha, double beta, int levels, int round32)
{
    if (m < 0 || n < 0 || k < 0 || levels < 0) return -2;
    if (m == 0 || n == 0) return 0;
    const int use_product = (k > 0 && alpha != 0.0);
    double *T = NULL;
    if (use_product) {
        T = (double *)calloc((size_t)(m * n), sizeof(double));
        if (!T) return -1;
        const int rc = strassen_acc(m, n, k, A, lda, B, ldb, T, n, levels, round32);
        if (rc) {
            free(T);
            return rc;
        }
    }
    for (i64 i = 0; i < m; ++i)
        for (i64 j = 0; j < n; ++j) {
            double *cij = C + i * ldc + j;
            const double old = (beta == 0.0) ? 0.0 : rnd(beta * *cij, round32);
            const double prod = use_product ? rnd(alpha * T[i * n + j], round32) : 0.0;
            *cij = rnd(prod + old, round32);
        }
    free(T);
    return 0;
}
