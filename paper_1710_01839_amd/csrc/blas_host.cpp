// Host side of the BLAS-style surface: C := alpha op(A) op(B) + beta C in
// DD / QD, and complex DD through a real embedding.  Argument checks, operand
// packing, the product (any algorithm of mpg_gemm_common) and the scaling
// epilogue, all on the context's stream.
#include <algorithm>

#include "blas_internal.hpp"
#include "capi_internal.hpp"

using namespace mpg;

namespace {

constexpr int kSlotPackA = 4, kSlotPackB = 5, kSlotProduct = 6;

bool all_zero(const double* x, int limbs) {
  for (int q = 0; q < limbs; ++q)
    if (x[q] != 0.0) return false;
  return true;
}

bool is_one(const double* x, int limbs) {
  if (x[0] != 1.0) return false;
  for (int q = 1; q < limbs; ++q)
    if (x[q] != 0.0) return false;
  return true;
}

bool valid_op(mpg_op t) { return t == MPG_OP_N || t == MPG_OP_T || t == MPG_OP_C; }

// Stored shape of an operand whose op() is rows x cols.
void stored_shape(mpg_op t, int64_t rows, int64_t cols, int64_t* sr, int64_t* sc) {
  *sr = t == MPG_OP_N ? rows : cols;
  *sc = t == MPG_OP_N ? cols : rows;
}

// Common checks of both forms.  planes: limb planes per matrix (2 or 4).
int check_form(mpg_ctx* c, int planes, mpg_op ta, mpg_op tb, int64_t m, int64_t n, int64_t k,
               const double* alpha, const double* const* A, int64_t lda, const double* const* B,
               int64_t ldb, const double* beta, double* const* C, int64_t ldc, bool use_t,
               int64_t max_dim) {
  if (!valid_op(ta) || !valid_op(tb)) return mpg_fail(c, MPG_ERR_ARG, "invalid op value");
  if (!alpha || !beta) return mpg_fail(c, MPG_ERR_ARG, "NULL alpha or beta");
  if (!A || !B || !C) return mpg_fail(c, MPG_ERR_ARG, "NULL limb array");
  if (m < 0 || n < 0 || k < 0) return mpg_fail(c, MPG_ERR_ARG, "negative dimension");
  if (m > max_dim || n > max_dim || k > max_dim) return mpg_fail(c, MPG_ERR_ARG, "dimension too large");
  if (m == 0 || n == 0) return MPG_OK;
  if (ldc < std::max<int64_t>(1, n)) return mpg_fail(c, MPG_ERR_ARG, "ldc < n");
  for (int q = 0; q < planes; ++q)
    if (!C[q]) return mpg_fail(c, MPG_ERR_ARG, "C plane %d is NULL", q);
  const size_t sc = mpg_span_bytes(m, n, ldc);
  for (int q = 0; q < planes; ++q)
    for (int r = q + 1; r < planes; ++r)
      if (mpg_overlaps(C[q], sc, C[r], sc))
        return mpg_fail(c, MPG_ERR_ALIAS, "C planes %d and %d overlap", q, r);
  if (!use_t) return MPG_OK;
  int64_t ar, ac, br, bc;
  stored_shape(ta, m, k, &ar, &ac);
  stored_shape(tb, k, n, &br, &bc);
  if (lda < std::max<int64_t>(1, ac)) return mpg_fail(c, MPG_ERR_ARG, "lda below the stored width of A");
  if (ldb < std::max<int64_t>(1, bc)) return mpg_fail(c, MPG_ERR_ARG, "ldb below the stored width of B");
  const size_t sa = mpg_span_bytes(ar, ac, lda), sb = mpg_span_bytes(br, bc, ldb);
  for (int q = 0; q < planes; ++q) {
    if (!A[q]) return mpg_fail(c, MPG_ERR_ARG, "A plane %d is NULL", q);
    if (!B[q]) return mpg_fail(c, MPG_ERR_ARG, "B plane %d is NULL", q);
  }
  for (int q = 0; q < planes; ++q)
    for (int r = 0; r < planes; ++r)
      if (mpg_overlaps(C[q], sc, A[r], sa) || mpg_overlaps(C[q], sc, B[r], sb))
        return mpg_fail(c, MPG_ERR_ALIAS, "C plane %d overlaps an input", q);
  return MPG_OK;
}

int pack(mpg_ctx* c, const PackArgs& p) {
  return mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_pack(p, c->stream); }, "operand pack");
}

// Packs op(X) (rows x cols) of `limbs` planes into a workspace slot; returns
// the packed planes (leading dimension cols).
int pack_op(mpg_ctx* c, int slot, int limbs, mpg_op t, int64_t rows, int64_t cols,
            const double* const* X, int64_t ldx, const double** out) {
  void* w = nullptr;
  int st = mpg_workspace(c, slot, (size_t)limbs * rows * cols * sizeof(double), &w);
  if (st != MPG_OK) return st;
  PackArgs p{};
  for (int q = 0; q < limbs; ++q) {
    double* dst = (double*)w + (size_t)q * rows * cols;
    p.job[q] = PackJob{X[q], dst, rows, cols, ldx, cols, 1, 1.0};
    out[q] = dst;
  }
  p.count = limbs;
  return pack(c, p);
}

}  // namespace

extern "C" int mpg_rgemm(mpg_ctx* c, int precision, mpg_op transa, mpg_op transb, int64_t m,
                         int64_t n, int64_t k, const double* alpha, const double* const* A,
                         int64_t lda, const double* const* B, int64_t ldb, const double* beta,
                         double* const* C, int64_t ldc, mpg_algo algo, const mpg_tile* tile) {
  if (!c) return MPG_ERR_ARG;
  if (precision != 2 && precision != 4) return mpg_fail(c, MPG_ERR_ARG, "precision must be 2 or 4");
  const int L = precision;
  const bool use_t = alpha && !all_zero(alpha, L) && k > 0;
  int st = check_form(c, L, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, use_t,
                      (int64_t)1 << 31);
  if (st != MPG_OK || m == 0 || n == 0) return st;
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  const bool use_c = !all_zero(beta, L);
  AxpbyArgs e{};
  e.ldc = ldc;
  e.m = m;
  e.n = n;
  for (int q = 0; q < L; ++q) {
    e.C[q] = C[q];
    e.alpha[q] = alpha[q];
    e.beta[q] = beta[q];
  }
  e.use_c = use_c;
  if (use_t) {
    const double* opA[4] = {A[0], A[1], L > 2 ? A[2] : nullptr, L > 2 ? A[3] : nullptr};
    const double* opB[4] = {B[0], B[1], L > 2 ? B[2] : nullptr, L > 2 ? B[3] : nullptr};
    int64_t ldA = lda, ldB = ldb;
    if (transa != MPG_OP_N) {
      if ((st = pack_op(c, kSlotPackA, L, transa, m, k, A, lda, opA)) != MPG_OK) return st;
      ldA = k;
    }
    if (transb != MPG_OP_N) {
      if ((st = pack_op(c, kSlotPackB, L, transb, k, n, B, ldb, opB)) != MPG_OK) return st;
      ldB = n;
    }
    if (is_one(alpha, L) && !use_c)
      return mpg_gemm_common(c, L, m, n, k, opA, ldA, opB, ldB, C, ldc, algo, tile);
    void* w = nullptr;
    if ((st = mpg_workspace(c, kSlotProduct, (size_t)L * m * n * sizeof(double), &w)) != MPG_OK)
      return st;
    double* T[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int q = 0; q < L; ++q) T[q] = (double*)w + (size_t)q * m * n;
    if ((st = mpg_gemm_common(c, L, m, n, k, opA, ldA, opB, ldB, T, n, algo, tile)) != MPG_OK)
      return st;
    for (int q = 0; q < L; ++q) e.T[q] = T[q];
    e.ldt = n;
  }
  e.use_t = use_t;
  return mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_axpby(L, e, c->stream); },
                    "alpha/beta epilogue");
}

extern "C" int mpg_zgemm_dd(mpg_ctx* c, mpg_op transa, mpg_op transb, int64_t m, int64_t n,
                            int64_t k, const double alpha[4], const double* const A[4],
                            int64_t lda, const double* const B[4], int64_t ldb,
                            const double beta[4], double* const C[4], int64_t ldc, mpg_algo algo,
                            const mpg_tile* tile) {
  if (!c) return MPG_ERR_ARG;
  const bool use_p = alpha && !all_zero(alpha, 4) && k > 0;
  int st = check_form(c, 4, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, use_p,
                      (int64_t)1 << 30);
  if (st != MPG_OK || m == 0 || n == 0) return st;
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  ZAxpbyArgs e{};
  e.ldc = ldc;
  e.m = m;
  e.n = n;
  for (int q = 0; q < 4; ++q) {
    e.C[q] = C[q];
    e.alpha[q] = alpha[q];
    e.beta[q] = beta[q];
  }
  e.use_c = !all_zero(beta, 4);
  e.use_p = use_p;
  if (use_p) {
    const int64_t K2 = 2 * k, N2 = 2 * n;
    void *wa = nullptr, *wb = nullptr, *wp = nullptr;
    if ((st = mpg_workspace(c, kSlotPackA, (size_t)2 * m * K2 * sizeof(double), &wa)) != MPG_OK ||
        (st = mpg_workspace(c, kSlotPackB, (size_t)2 * K2 * N2 * sizeof(double), &wb)) != MPG_OK ||
        (st = mpg_workspace(c, kSlotProduct, (size_t)2 * m * N2 * sizeof(double), &wp)) != MPG_OK)
      return st;
    const double* Ap[2] = {(double*)wa, (double*)wa + (size_t)m * K2};
    const double* Bp[2] = {(double*)wb, (double*)wb + (size_t)K2 * N2};
    double* Pp[2] = {(double*)wp, (double*)wp + (size_t)m * N2};
    const int ta = transa != MPG_OP_N, tb = transb != MPG_OP_N;
    const double sa = transa == MPG_OP_C ? -1.0 : 1.0, sb = transb == MPG_OP_C ? -1.0 : 1.0;
    // A' = [Re op(A) | Im op(A)]: m x 2k
    PackArgs pa{};
    for (int q = 0; q < 2; ++q) {
      double* d = const_cast<double*>(Ap[q]);
      pa.job[2 * q] = PackJob{A[q], d, m, k, lda, K2, ta, 1.0};
      pa.job[2 * q + 1] = PackJob{A[2 + q], d + k, m, k, lda, K2, ta, sa};
    }
    pa.count = 4;
    if ((st = pack(c, pa)) != MPG_OK) return st;
    // B' = [[Re op(B), Im op(B)], [-Im op(B), Re op(B)]]: 2k x 2n
    PackArgs pb{};
    for (int q = 0; q < 2; ++q) {
      double* d = const_cast<double*>(Bp[q]);
      pb.job[4 * q + 0] = PackJob{B[q], d, k, n, ldb, N2, tb, 1.0};
      pb.job[4 * q + 1] = PackJob{B[2 + q], d + n, k, n, ldb, N2, tb, sb};
      pb.job[4 * q + 2] = PackJob{B[2 + q], d + (size_t)k * N2, k, n, ldb, N2, tb, -sb};
      pb.job[4 * q + 3] = PackJob{B[q], d + (size_t)k * N2 + n, k, n, ldb, N2, tb, 1.0};
    }
    pb.count = 8;
    if ((st = pack(c, pb)) != MPG_OK) return st;
    if ((st = mpg_gemm_common(c, 2, m, N2, K2, Ap, K2, Bp, N2, Pp, N2, algo, tile)) != MPG_OK)
      return st;
    e.P[0] = Pp[0];
    e.P[1] = Pp[1];
    e.ldp = N2;
  }
  return mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_zaxpby(e, c->stream); },
                    "complex alpha/beta epilogue");
}
