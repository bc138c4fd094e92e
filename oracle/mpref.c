/*
 * mpref.c -- plain CPU oracle for multiple-precision dense C := AB.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the GPU library, and the
 * GPU library never calls it.
 *
 * Everything here is deliberately written as the textbook definition, with
 * no blocking, fusion or reordering:
 *
 *   - Error-free transforms: Knuth's TwoSum, Dekker's FastTwoSum and
 *     Dekker's TwoProduct (Veltkamp splitting, no FMA), plus the FMA
 *     TwoProduct used only as a cross-check.
 *   - Double-double (DD) multiply and accurate add (the "QD library"
 *     arithmetic the paper builds on, Section 1; the DD product is the
 *     classic Dekker product followed by FastTwoSum, the add is the
 *     accurate two-TwoSum form).
 *   - Quad-double (QD) add and multiply: all partial terms are produced
 *     exactly (TwoSum / TwoProduct), then distilled by repeated error-free
 *     VecSum passes and peeled into four limbs.
 *   - The simple algorithm, Eq. (1): c_ij = sum_k a_ik b_kj with k in order,
 *     each step acc <- add(acc, mul(a_ik, b_kj)).
 *   - Strassen, Eq. (3) (classic 7-product form) and the Winograd variant
 *     (same products, 15 additions), recursive to a fixed depth with zero
 *     padding of odd dimensions.
 *   - The exact product: Eq. (1) evaluated with no rounding at all in a
 *     fixed-point super-accumulator, then rounded limb by limb to nearest.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Error-free transforms                                              */
/* ------------------------------------------------------------------ */

/* Knuth TwoSum: s + e == a + b exactly, s == fl(a + b). */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    double eb = b - bv;
    double ea = a - av;
    *s = x;
    *e = ea + eb;
}

/* Dekker FastTwoSum: exact when a == 0 or exponent(a) >= exponent(b). */
static void fast_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    *e = b - (x - a);
    *s = x;
}

/* Veltkamp split: a == h + l, each half fits in 26 bits. */
static void veltkamp_split(double a, double *h, double *l)
{
    const double c = 134217729.0; /* 2^27 + 1 */
    double t = c * a;
    double hi = t - (t - a);
    *h = hi;
    *l = a - hi;
}

/* Dekker TwoProduct: p + e == a * b exactly, p == fl(a * b). */
static void two_prod_dekker(double a, double b, double *p, double *e)
{
    double ah, al, bh, bl;
    double x = a * b;
    veltkamp_split(a, &ah, &al);
    veltkamp_split(b, &bh, &bl);
    *p = x;
    *e = (((ah * bh - x) + ah * bl) + al * bh) + al * bl;
}

/* FMA TwoProduct (cross-check only). */
static void two_prod_fma(double a, double b, double *p, double *e)
{
    double x = a * b;
    *p = x;
    *e = fma(a, b, -x);
}

/* ------------------------------------------------------------------ */
/* Double-double arithmetic                                           */
/* ------------------------------------------------------------------ */

typedef struct { double hi, lo; } dd_t;

/* DD product: TwoProduct of the heads, cross terms added to the error,
 * renormalised with FastTwoSum. */
static dd_t dd_mul(dd_t a, dd_t b)
{
    double p, e, s, t;
    two_prod_dekker(a.hi, b.hi, &p, &e);
    e = e + (a.hi * b.lo + a.lo * b.hi);
    fast_two_sum(p, e, &s, &t);
    dd_t r = { s, t };
    return r;
}

/* Accurate DD sum: TwoSum of heads and of tails, two renormalisations. */
static dd_t dd_add(dd_t a, dd_t b)
{
    double s, e, t, f;
    two_sum(a.hi, b.hi, &s, &e);
    two_sum(a.lo, b.lo, &t, &f);
    e = e + t;
    fast_two_sum(s, e, &s, &e);
    e = e + f;
    fast_two_sum(s, e, &s, &e);
    dd_t r = { s, e };
    return r;
}

static dd_t dd_neg(dd_t a) { dd_t r = { -a.hi, -a.lo }; return r; }
static dd_t dd_sub(dd_t a, dd_t b) { return dd_add(a, dd_neg(b)); }

/* ------------------------------------------------------------------ */
/* Quad-double arithmetic                                             */
/* ------------------------------------------------------------------ */

typedef struct { double x[4]; } qd_t;

/* Turn a list of doubles (exact sum T) into four limbs whose sum is T up to
 * the size of the discarded tail.  For each limb, bottom-up VecSum passes
 * (each step a TwoSum, so the sum never changes) are repeated until a pass
 * changes nothing; then fl(x[k] + x[k+1]) == x[k] for every neighbour pair,
 * so x[k] is within about half an ulp of the remaining sum. */
static qd_t qd_from_terms(double *x, int n)
{
    qd_t r;
    for (int k = 0; k < 4; ++k) {
        if (k >= n) { r.x[k] = 0.0; continue; }
        for (int pass = 0; pass < 200; ++pass) {
            int changed = 0;
            for (int i = n - 1; i > k; --i) {
                double s, e;
                two_sum(x[i - 1], x[i], &s, &e);
                if (s != x[i - 1] || e != x[i]) changed = 1;
                x[i - 1] = s;
                x[i] = e;
            }
            if (!changed) break;
        }
        r.x[k] = x[k];
    }
    return r;
}

static qd_t qd_add(qd_t a, qd_t b)
{
    double t[8];
    for (int i = 0; i < 4; ++i) { t[i] = a.x[i]; t[4 + i] = b.x[i]; }
    return qd_from_terms(t, 8);
}

static qd_t qd_neg(qd_t a)
{
    qd_t r;
    for (int i = 0; i < 4; ++i) r.x[i] = -a.x[i];
    return r;
}

static qd_t qd_sub(qd_t a, qd_t b) { return qd_add(a, qd_neg(b)); }

/* QD product: every limb product a_i b_j with i + j <= 3 is split exactly
 * by TwoProduct, those with i + j == 4 are rounded products (their errors
 * sit near 2^-265 relative), those with i + j >= 5 are dropped. */
static qd_t qd_mul(qd_t a, qd_t b)
{
    double t[32];
    int n = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            if (i + j <= 3) {
                double p, e;
                two_prod_dekker(a.x[i], b.x[j], &p, &e);
                t[n++] = p;
                t[n++] = e;
            } else if (i + j == 4) {
                t[n++] = a.x[i] * b.x[j];
            }
        }
    return qd_from_terms(t, n);
}

/* ------------------------------------------------------------------ */
/* Generic "number with L limbs" helpers (L = 2 for DD, 4 for QD)     */
/* ------------------------------------------------------------------ */

static void num_add(int L, const double *a, const double *b, double *out)
{
    if (L == 2) {
        dd_t x = { a[0], a[1] }, y = { b[0], b[1] };
        dd_t r = dd_add(x, y);
        out[0] = r.hi; out[1] = r.lo;
    } else {
        qd_t x, y, r;
        for (int i = 0; i < 4; ++i) { x.x[i] = a[i]; y.x[i] = b[i]; }
        r = qd_add(x, y);
        for (int i = 0; i < 4; ++i) out[i] = r.x[i];
    }
}

static void num_sub(int L, const double *a, const double *b, double *out)
{
    double nb[4];
    for (int i = 0; i < L; ++i) nb[i] = -b[i];
    num_add(L, a, nb, out);
}

/* acc <- acc + a * b (multiply, then add: one step of Eq. (1)). */
static void num_madd(int L, double *acc, const double *a, const double *b)
{
    if (L == 2) {
        dd_t x = { a[0], a[1] }, y = { b[0], b[1] }, c = { acc[0], acc[1] };
        dd_t r = dd_add(c, dd_mul(x, y));
        acc[0] = r.hi; acc[1] = r.lo;
    } else {
        qd_t x, y, c, r;
        for (int i = 0; i < 4; ++i) { x.x[i] = a[i]; y.x[i] = b[i]; c.x[i] = acc[i]; }
        r = qd_add(c, qd_mul(x, y));
        for (int i = 0; i < 4; ++i) acc[i] = r.x[i];
    }
}

/* ------------------------------------------------------------------ */
/* Exported element-wise operations (for the oracle's own tests)      */
/* ------------------------------------------------------------------ */

void orc_two_sum(int64_t n, const double *a, const double *b, double *s, double *e)
{
    for (int64_t i = 0; i < n; ++i) two_sum(a[i], b[i], &s[i], &e[i]);
}

void orc_fast_two_sum(int64_t n, const double *a, const double *b, double *s, double *e)
{
    for (int64_t i = 0; i < n; ++i) fast_two_sum(a[i], b[i], &s[i], &e[i]);
}

void orc_two_prod(int64_t n, int use_fma, const double *a, const double *b, double *p, double *e)
{
    for (int64_t i = 0; i < n; ++i) {
        if (use_fma) two_prod_fma(a[i], b[i], &p[i], &e[i]);
        else two_prod_dekker(a[i], b[i], &p[i], &e[i]);
    }
}

/* op: 0 add, 1 mul.  x, y, out: n elements, L interleaved limbs each. */
void orc_num_op(int L, int op, int64_t n, const double *x, const double *y, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *a = x + i * L, *b = y + i * L;
        double *o = out + i * L;
        if (op == 0) {
            num_add(L, a, b, o);
        } else {
            double acc[4] = { 0.0, 0.0, 0.0, 0.0 };
            num_madd(L, acc, a, b);
            for (int j = 0; j < L; ++j) o[j] = acc[j];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Simple algorithm, Eq. (1), on limb planes                          */
/* ------------------------------------------------------------------ */

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    return nthreads;
#else
    (void)nthreads;
    return 1;
#endif
}

/* C := A B with L-limb numbers stored as L separate row-major planes.
 * A: m x l (leading dimension lda), B: l x n (ldb), C: m x n (ldc). */
void orc_gemm_simple(int L, int64_t m, int64_t n, int64_t l,
                     const double *const *A, int64_t lda,
                     const double *const *B, int64_t ldb,
                     double *const *C, int64_t ldc, int nthreads)
{
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double acc[4] = { 0.0, 0.0, 0.0, 0.0 };
            for (int64_t k = 0; k < l; ++k) {
                double a[4], b[4];
                for (int q = 0; q < L; ++q) {
                    a[q] = A[q][i * lda + k];
                    b[q] = B[q][k * ldb + j];
                }
                num_madd(L, acc, a, b);
            }
            for (int q = 0; q < L; ++q) C[q][i * ldc + j] = acc[q];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Strassen, Eq. (3), and the Winograd variant                        */
/* Matrices inside the recursion are interleaved: element (i, j) of a */
/* matrix with leading dimension ld starts at p + (i*ld + j)*L.       */
/* ------------------------------------------------------------------ */

static void mat_gemm(int L, int64_t m, int64_t n, int64_t l,
                     const double *A, int64_t lda, const double *B, int64_t ldb,
                     double *C, int64_t ldc, int nt)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc[4] = { 0.0, 0.0, 0.0, 0.0 };
            for (int64_t k = 0; k < l; ++k)
                num_madd(L, acc, A + (i * lda + k) * L, B + (k * ldb + j) * L);
            for (int q = 0; q < L; ++q) C[(i * ldc + j) * L + q] = acc[q];
        }
}

/* out = x + sign * y, element-wise over an r x c block. */
static void mat_addsub(int L, int64_t r, int64_t c, const double *x, int64_t ldx,
                       const double *y, int64_t ldy, int sign, double *out, int64_t ldo)
{
    for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < c; ++j) {
            const double *a = x + (i * ldx + j) * L, *b = y + (i * ldy + j) * L;
            double *o = out + (i * ldo + j) * L;
            if (sign > 0) num_add(L, a, b, o);
            else num_sub(L, a, b, o);
        }
}

static double *mat_alloc(int L, int64_t r, int64_t c)
{
    double *p = (double *)calloc((size_t)(r * c * L), sizeof(double));
    return p;
}

static void strassen_rec(int L, int variant, int depth, int64_t m, int64_t n, int64_t l,
                         const double *A, int64_t lda, const double *B, int64_t ldb,
                         double *C, int64_t ldc, int nt)
{
    if (depth == 0 || (m % 2) || (n % 2) || (l % 2) || m < 2 || n < 2 || l < 2) {
        mat_gemm(L, m, n, l, A, lda, B, ldb, C, ldc, nt);
        return;
    }
    int64_t hm = m / 2, hn = n / 2, hl = l / 2;
    const double *A11 = A, *A12 = A + hl * L, *A21 = A + hm * lda * L, *A22 = A21 + hl * L;
    const double *B11 = B, *B12 = B + hn * L, *B21 = B + hl * ldb * L, *B22 = B21 + hn * L;
    double *C11 = C, *C12 = C + hn * L, *C21 = C + hm * ldc * L, *C22 = C21 + hn * L;
    double *P[8];
    for (int i = 1; i <= 7; ++i) P[i] = mat_alloc(L, hm, hn);
    double *SA = mat_alloc(L, hm, hl), *SB = mat_alloc(L, hl, hn);

    if (variant == 0) {
        /* Eq. (3), classic form. */
        mat_addsub(L, hm, hl, A11, lda, A22, lda, +1, SA, hl);
        mat_addsub(L, hl, hn, B11, ldb, B22, ldb, +1, SB, hn);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, SA, hl, SB, hn, P[1], hn, nt);
        mat_addsub(L, hm, hl, A21, lda, A22, lda, +1, SA, hl);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, SA, hl, B11, ldb, P[2], hn, nt);
        mat_addsub(L, hl, hn, B12, ldb, B22, ldb, -1, SB, hn);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, A11, lda, SB, hn, P[3], hn, nt);
        mat_addsub(L, hl, hn, B21, ldb, B11, ldb, -1, SB, hn);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, A22, lda, SB, hn, P[4], hn, nt);
        mat_addsub(L, hm, hl, A11, lda, A12, lda, +1, SA, hl);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, SA, hl, B22, ldb, P[5], hn, nt);
        mat_addsub(L, hm, hl, A21, lda, A11, lda, -1, SA, hl);
        mat_addsub(L, hl, hn, B11, ldb, B12, ldb, +1, SB, hn);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, SA, hl, SB, hn, P[6], hn, nt);
        mat_addsub(L, hm, hl, A12, lda, A22, lda, -1, SA, hl);
        mat_addsub(L, hl, hn, B21, ldb, B22, ldb, +1, SB, hn);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, SA, hl, SB, hn, P[7], hn, nt);
        /* C11 = P1 + P4 - P5 + P7, C12 = P3 + P5, C21 = P2 + P4,
         * C22 = P1 + P3 - P2 + P6, each summed left to right. */
        mat_addsub(L, hm, hn, P[1], hn, P[4], hn, +1, C11, ldc);
        mat_addsub(L, hm, hn, C11, ldc, P[5], hn, -1, C11, ldc);
        mat_addsub(L, hm, hn, C11, ldc, P[7], hn, +1, C11, ldc);
        mat_addsub(L, hm, hn, P[3], hn, P[5], hn, +1, C12, ldc);
        mat_addsub(L, hm, hn, P[2], hn, P[4], hn, +1, C21, ldc);
        mat_addsub(L, hm, hn, P[1], hn, P[3], hn, +1, C22, ldc);
        mat_addsub(L, hm, hn, C22, ldc, P[2], hn, -1, C22, ldc);
        mat_addsub(L, hm, hn, C22, ldc, P[6], hn, +1, C22, ldc);
    } else {
        /* Winograd variant: S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21,
         * S4 = A12 - S2; T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12,
         * T4 = T2 - B21; products A11 B11, A12 B21, S4 B22, A22 T4, S1 T1,
         * S2 T2, S3 T3. */
        double *S1 = mat_alloc(L, hm, hl), *S2 = mat_alloc(L, hm, hl);
        double *T1 = mat_alloc(L, hl, hn), *T2 = mat_alloc(L, hl, hn);
        mat_addsub(L, hm, hl, A21, lda, A22, lda, +1, S1, hl);
        mat_addsub(L, hm, hl, S1, hl, A11, lda, -1, S2, hl);
        mat_addsub(L, hl, hn, B12, ldb, B11, ldb, -1, T1, hn);
        mat_addsub(L, hl, hn, B22, ldb, T1, hn, -1, T2, hn);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, A11, lda, B11, ldb, P[1], hn, nt);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, A12, lda, B21, ldb, P[2], hn, nt);
        mat_addsub(L, hm, hl, A12, lda, S2, hl, -1, SA, hl);           /* S4 */
        strassen_rec(L, variant, depth - 1, hm, hn, hl, SA, hl, B22, ldb, P[3], hn, nt);
        mat_addsub(L, hl, hn, T2, hn, B21, ldb, -1, SB, hn);           /* T4 */
        strassen_rec(L, variant, depth - 1, hm, hn, hl, A22, lda, SB, hn, P[4], hn, nt);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, S1, hl, T1, hn, P[5], hn, nt);
        strassen_rec(L, variant, depth - 1, hm, hn, hl, S2, hl, T2, hn, P[6], hn, nt);
        mat_addsub(L, hm, hl, A11, lda, A21, lda, -1, SA, hl);         /* S3 */
        mat_addsub(L, hl, hn, B22, ldb, B12, ldb, -1, SB, hn);         /* T3 */
        strassen_rec(L, variant, depth - 1, hm, hn, hl, SA, hl, SB, hn, P[7], hn, nt);
        /* C11 = P1 + P2; U2 = P1 + P6; U3 = U2 + P7; U4 = U2 + P5;
         * C12 = U4 + P3; C21 = U3 - P4; C22 = U3 + P5. */
        double *U2 = mat_alloc(L, hm, hn), *U3 = mat_alloc(L, hm, hn), *U4 = mat_alloc(L, hm, hn);
        mat_addsub(L, hm, hn, P[1], hn, P[2], hn, +1, C11, ldc);
        mat_addsub(L, hm, hn, P[1], hn, P[6], hn, +1, U2, hn);
        mat_addsub(L, hm, hn, U2, hn, P[7], hn, +1, U3, hn);
        mat_addsub(L, hm, hn, U2, hn, P[5], hn, +1, U4, hn);
        mat_addsub(L, hm, hn, U4, hn, P[3], hn, +1, C12, ldc);
        mat_addsub(L, hm, hn, U3, hn, P[4], hn, -1, C21, ldc);
        mat_addsub(L, hm, hn, U3, hn, P[5], hn, +1, C22, ldc);
        free(S1); free(S2); free(T1); free(T2); free(U2); free(U3); free(U4);
    }
    for (int i = 1; i <= 7; ++i) free(P[i]);
    free(SA);
    free(SB);
}

/* Strassen C := A B on limb planes.  variant 0 = Eq. (3), 1 = Winograd.
 * Each dimension is zero-padded up to a multiple of 2^depth (zeros add
 * nothing, so the padded product restricted to the m x n corner is AB). */
int orc_gemm_strassen(int L, int variant, int depth, int64_t m, int64_t n, int64_t l,
                      const double *const *A, int64_t lda,
                      const double *const *B, int64_t ldb,
                      double *const *C, int64_t ldc, int nthreads)
{
    int nt = set_threads(nthreads);
    int64_t q = (int64_t)1 << depth;
    int64_t M = (m + q - 1) / q * q, N = (n + q - 1) / q * q, K = (l + q - 1) / q * q;
    double *Ai = mat_alloc(L, M, K), *Bi = mat_alloc(L, K, N), *Ci = mat_alloc(L, M, N);
    if (!Ai || !Bi || !Ci) { free(Ai); free(Bi); free(Ci); return -1; }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = 0; k < l; ++k)
            for (int p = 0; p < L; ++p) Ai[(i * K + k) * L + p] = A[p][i * lda + k];
    for (int64_t k = 0; k < l; ++k)
        for (int64_t j = 0; j < n; ++j)
            for (int p = 0; p < L; ++p) Bi[(k * N + j) * L + p] = B[p][k * ldb + j];
    strassen_rec(L, variant, depth, M, N, K, Ai, K, Bi, N, Ci, N, nt);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            for (int p = 0; p < L; ++p) C[p][i * ldc + j] = Ci[(i * N + j) * L + p];
    free(Ai); free(Bi); free(Ci);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Exact product: a fixed-point super-accumulator                     */
/* ------------------------------------------------------------------ */
/* value = sum_i w[i] * 2^(32 i + SA_EMIN); each word holds a 32-bit digit
 * but is an int64 so that many additions can be absorbed before carries
 * are propagated.  Range 2^-2240 .. 2^2112 covers every exact limb
 * product of inputs below 2^900 in magnitude (and above 2^-1000 when
 * nonzero). */
#define SA_EMIN (-2240)
#define SA_NW 136

typedef struct { int64_t w[SA_NW]; int pending; } superacc_t;

static void sa_clear(superacc_t *a) { memset(a, 0, sizeof(*a)); }

static void sa_carry(superacc_t *a)
{
    for (int i = 0; i < SA_NW - 1; ++i) {
        int64_t c = a->w[i] >> 32;          /* floor division by 2^32 */
        a->w[i] -= c * ((int64_t)1 << 32);
        a->w[i + 1] += c;
    }
    a->pending = 0;
}

static void sa_add(superacc_t *a, double x)
{
    if (x == 0.0) return;
    int e;
    double fr = frexp(x, &e);                   /* x = fr * 2^e, 0.5 <= |fr| < 1 */
    int64_t M = (int64_t)ldexp(fr, 53);         /* exact 53-bit integer */
    int pos = e - 53 - SA_EMIN;                 /* bit position of M's unit */
    int word = pos >> 5, off = pos & 31;
    uint64_t mag = (uint64_t)(M < 0 ? -M : M);
    unsigned __int128 v = (unsigned __int128)mag << off;
    int64_t d0 = (int64_t)(uint64_t)(v & 0xffffffffu);
    int64_t d1 = (int64_t)(uint64_t)((v >> 32) & 0xffffffffu);
    int64_t d2 = (int64_t)(uint64_t)(v >> 64);
    if (M < 0) { d0 = -d0; d1 = -d1; d2 = -d2; }
    a->w[word] += d0;
    a->w[word + 1] += d1;
    a->w[word + 2] += d2;
    if (++a->pending >= (1 << 24)) sa_carry(a);
}

/* Round the accumulated value to the nearest double (ties to even). */
static double sa_round(superacc_t *a)
{
    sa_carry(a);
    int neg = a->w[SA_NW - 1] < 0;
    uint64_t mag[SA_NW];
    if (neg) {
        /* two's-complement style negation of the digit vector */
        int64_t t[SA_NW];
        for (int i = 0; i < SA_NW; ++i) t[i] = -a->w[i];
        for (int i = 0; i < SA_NW - 1; ++i) {
            int64_t c = t[i] >> 32;
            t[i] -= c * ((int64_t)1 << 32);
            t[i + 1] += c;
        }
        for (int i = 0; i < SA_NW; ++i) mag[i] = (uint64_t)t[i];
    } else {
        for (int i = 0; i < SA_NW; ++i) mag[i] = (uint64_t)a->w[i];
    }
    int top = -1;
    for (int i = SA_NW - 1; i >= 0; --i)
        if (mag[i]) { top = i; break; }
    if (top < 0) return 0.0;
    uint64_t w2 = mag[top], w1 = top >= 1 ? mag[top - 1] : 0, w0 = top >= 2 ? mag[top - 2] : 0;
    int sticky = 0;
    for (int i = 0; i < top - 2; ++i)
        if (mag[i]) { sticky = 1; break; }
    unsigned __int128 X = ((unsigned __int128)w2 << 64) | ((unsigned __int128)w1 << 32) | w0;
    int bits = 0;
    for (unsigned __int128 t = X; t; t >>= 1) ++bits;
    int shift = bits - 53;            /* >= 12 because w2 >= 1 */
    uint64_t mant = (uint64_t)(X >> shift);
    unsigned __int128 rem = X & (((unsigned __int128)1 << shift) - 1);
    unsigned __int128 half = (unsigned __int128)1 << (shift - 1);
    if (rem > half || (rem == half && (sticky || (mant & 1)))) mant += 1;
    double r = ldexp((double)mant, shift + 32 * (top - 2) + SA_EMIN);
    return neg ? -r : r;
}

/* Exact C := A B: A has La limbs, B has Lb limbs (1, 2 or 4 planes), the
 * output is rounded limb by limb to nearest into Lc planes, so that
 * limb k is the double nearest to (exact - limbs 0..k-1). */
int orc_gemm_exact(int La, int Lb, int Lc, int64_t m, int64_t n, int64_t l,
                   const double *const *A, int64_t lda,
                   const double *const *B, int64_t ldb,
                   double *const *C, int64_t ldc, int nthreads)
{
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t i = 0; i < m; ++i) {
        superacc_t *acc = (superacc_t *)malloc(sizeof(superacc_t));
        for (int64_t j = 0; j < n; ++j) {
            sa_clear(acc);
            for (int64_t k = 0; k < l; ++k)
                for (int p = 0; p < La; ++p) {
                    double a = A[p][i * lda + k];
                    if (a == 0.0) continue;
                    for (int q = 0; q < Lb; ++q) {
                        double pr, er;
                        two_prod_fma(a, B[q][k * ldb + j], &pr, &er);
                        sa_add(acc, pr);
                        sa_add(acc, er);
                    }
                }
            for (int p = 0; p < Lc; ++p) {
                double r = sa_round(acc);
                C[p][i * ldc + j] = r;
                sa_add(acc, -r);
            }
        }
        free(acc);
    }
    return 0;
}

/* Exact sum-of-magnitudes product (|A| |B|), rounded to nearest double,
 * used for the componentwise error bounds. */
int orc_absprod_exact(int La, int Lb, int64_t m, int64_t n, int64_t l,
                      const double *const *A, int64_t lda,
                      const double *const *B, int64_t ldb,
                      double *C, int64_t ldc, int nthreads)
{
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t i = 0; i < m; ++i) {
        superacc_t *acc = (superacc_t *)malloc(sizeof(superacc_t));
        for (int64_t j = 0; j < n; ++j) {
            sa_clear(acc);
            for (int64_t k = 0; k < l; ++k) {
                /* |a| as a multi-limb value: the sign of the sum of limbs is
                 * the sign of the leading limb (limbs are non-overlapping). */
                double sa = A[0][i * lda + k] < 0 ? -1.0 : 1.0;
                double sb = B[0][k * ldb + j] < 0 ? -1.0 : 1.0;
                for (int p = 0; p < La; ++p)
                    for (int q = 0; q < Lb; ++q) {
                        double pr, er;
                        two_prod_fma(sa * A[p][i * lda + k], sb * B[q][k * ldb + j], &pr, &er);
                        sa_add(acc, pr);
                        sa_add(acc, er);
                    }
            }
            C[i * ldc + j] = sa_round(acc);
        }
        free(acc);
    }
    return 0;
}

/* Round the exact sum of limb planes X (L limbs) minus Y (L limbs) to the
 * nearest double, element-wise: the exact error of a result. */
void orc_exact_diff(int Lx, int Ly, int64_t n, const double *const *X, const double *const *Y, double *out)
{
    superacc_t *acc = (superacc_t *)malloc(sizeof(superacc_t));
    for (int64_t i = 0; i < n; ++i) {
        sa_clear(acc);
        for (int p = 0; p < Lx; ++p) sa_add(acc, X[p][i]);
        for (int p = 0; p < Ly; ++p) sa_add(acc, -Y[p][i]);
        out[i] = sa_round(acc);
    }
    free(acc);
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
