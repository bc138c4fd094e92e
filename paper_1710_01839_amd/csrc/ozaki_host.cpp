// Host side of the split-precision (INT8 MFMA) double-double product.
#include <climits>
#include <cmath>
#include <cstring>

#include "capi_internal.hpp"
#include "blas_internal.hpp"
#include "crt_internal.hpp"
#include "internal.hpp"
#include "ozaki_internal.hpp"

using namespace mpg;

namespace {

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

__global__ void zero_int_kernel(int* p) { *p = 0; }

// Reads back the slice count the exponent scan found (the stream is
// synchronised).
int read_need(mpg_ctx* c, const int* counter, int* S) {
  int h = 0;
  hipError_t r = hipMemcpyAsync(&h, counter, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "slice-count read-back");
  *S = h;
  return MPG_OK;
}

int check_fp64_args(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A, int64_t lda,
                    const double* B, int64_t ldb) {
  if (m < 0 || n < 0 || l < 0) return mpg_fail(c, MPG_ERR_ARG, "negative dimension");
  if (l > 0 && (m > 0 && n > 0)) {
    if (!A || !B) return mpg_fail(c, MPG_ERR_ARG, "NULL input");
    if (lda < l) return mpg_fail(c, MPG_ERR_ARG, "lda < l");
    if (ldb < n) return mpg_fail(c, MPG_ERR_ARG, "ldb < n");
  }
  return MPG_OK;
}

// Exponents of A rows and B columns in the small workspace slot; with
// `with_need` the same pass also finds the exact slice count (in *counter).
int exponents(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A, const double* A_lo,
              int64_t lda, const double* B, const double* B_lo, int64_t ldb, bool with_need, int** e,
              int** f, int** counter) {
  void* small = nullptr;
  const int64_t mp = round_up(std::max<int64_t>(m, 1), 64), np = round_up(std::max<int64_t>(n, 1), 64);
  int st = mpg_workspace(c, 1, (size_t)(mp + 2 * np + 64) * sizeof(int), &small);
  if (st != MPG_OK) return st;
  *e = (int*)small;
  *f = *e + mp;
  int* low = *f + np;
  *counter = low + np;
  return mpg_launch(c, MPG_KCLASS_AUX, [&] {
    if (with_need) {
      hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, c->stream, *counter);
      hipError_t r = hipGetLastError();
      if (r != hipSuccess) return r;
    }
    int* need = with_need ? *counter : nullptr;
    hipError_t r = launch_ozaki_scan(A, A_lo, m, l, lda, 0, *e, nullptr, need, c->stream);
    if (r != hipSuccess) return r;
    return launch_ozaki_scan(B, B_lo, l, n, ldb, 1, *f, low, need, c->stream);
  }, "exponent scan");
}

}  // namespace

extern "C" int mpg_ozaki_slices_exact(mpg_ctx* c, int64_t m, int64_t n, int64_t l,
                                      const double* A, int64_t lda, const double* B, int64_t ldb,
                                      int* slices) {
  if (!c || !slices) return MPG_ERR_ARG;
  int st = check_fp64_args(c, m, n, l, A, lda, B, ldb);
  if (st != MPG_OK) return st;
  *slices = 0;
  if (m == 0 || n == 0 || l == 0) return MPG_OK;
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  int *e, *f, *counter;
  if ((st = exponents(c, m, n, l, A, nullptr, lda, B, nullptr, ldb, true, &e, &f, &counter)) != MPG_OK)
    return st;
  return read_need(c, counter, slices);
}

extern "C" int mpg_ozaki_split(mpg_ctx* c, int side, int64_t rows, int64_t cols, const double* X,
                               int64_t ldx, int slices, int8_t* out, int64_t ld_out,
                               int64_t plane, int32_t* exps) {
  if (!c) return MPG_ERR_ARG;
  if (side != 0 && side != 1) return mpg_fail(c, MPG_ERR_ARG, "side must be 0 (rows) or 1 (columns)");
  if (rows < 0 || cols < 0 || ldx < cols || slices < 1 || slices > ozaki_max_slices())
    return mpg_fail(c, MPG_ERR_ARG, "bad split arguments");
  if (rows == 0 || cols == 0) return MPG_OK;
  if (!X || !out || !exps) return mpg_fail(c, MPG_ERR_ARG, "NULL pointer");
  const int64_t lines = side == 0 ? rows : cols, len = side == 0 ? cols : rows;
  const int64_t lines_p = round_up(lines, 64), len_p = round_up(len, 64);
  if (ld_out < len_p || ld_out % 8 || plane < lines_p * ld_out || plane % 8 || (uintptr_t)out % 8)
    return mpg_fail(c, MPG_ERR_ARG, "digit planes: need ld_out >= %lld and plane >= %lld, both multiples "
                    "of 8, and out 8-byte aligned", (long long)len_p, (long long)(lines_p * ld_out));
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  return mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipError_t r = launch_ozaki_scan(X, nullptr, rows, cols, ldx, side, exps, nullptr, nullptr, c->stream);
    if (r != hipSuccess) return r;
    if (side == 0)
      return launch_ozaki_split_rows(X, nullptr, rows, cols, ldx, exps, slices, out, ld_out, plane,
                                     lines_p, len_p, c->stream);
    return launch_ozaki_split_cols(X, nullptr, rows, cols, ldx, exps, slices, out, ld_out, plane,
                                   lines_p, len_p, c->stream);
  }, "digit split");
}

namespace {

// One residue-form product after the scales: residue planes of the rows of
// A (+ A_lo) and of BT (+ BT_lo, B transposed: n x l, leading dimension l),
// one INT8 product per modulus and the reconstruction of the exact integer
// product, written to C as a double-double (limbs 2) or added to C as a
// quad-double (limbs 4).
// With a device-side plan, S and N are the largest the plan may hold
// (buffers and the reconstruction's word count are sized for them) and the
// kernels take the plan's own counts.
int crt_product(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A, const double* A_lo,
                int64_t lda, const int* e, const double* B, const double* B_lo, int64_t ldb, const int* f,
                int S, double* const* C, int limbs, int64_t ldc, const CrtPlan* plan = nullptr) {
  const int N = crt_moduli_for_bits(crt_product_bits(S, l));
  if (N == 0 || crt_words(N) == 0)
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "product of %d slices at l = %lld is too wide for the moduli",
                    S, (long long)l);
  c->last_slices = plan ? 0 : S;
  c->last_moduli = plan ? 0 : N;
  // planes padded to the residue products' tile (the rows kernel writes
  // zeros into the padding)
  const int64_t lp = round_up(l, crt_k_multiple()), mp = round_up(m, crt_tile_rows()),
                np = round_up(n, crt_tile_cols()), n4 = round_up(n, 4);
  const int64_t planeA = mp * lp, planeB = np * lp;
  const size_t cb = (sizeof(CrtResidueConsts) + 255) / 256 * 256;
  void *res = nullptr, *out = nullptr;
  int st;
  if ((st = mpg_workspace(c, 7, (size_t)N * (size_t)(planeA + planeB) + cb, &res)) != MPG_OK ||
      (st = mpg_workspace(c, 8, (size_t)N * (size_t)(m * n4) + 256 + sizeof(CrtTable), &out)) != MPG_OK)
    return st;
  int8_t* Ares = (int8_t*)res;
  int8_t* Bres = Ares + (size_t)N * planeA;
  CrtResidueConsts* consts = (CrtResidueConsts*)(Bres + (size_t)N * planeB);
  uint8_t* R = (uint8_t*)out;
  CrtTable* table = (CrtTable*)((char*)out + ((size_t)N * (size_t)(m * n4) + 255) / 256 * 256);
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipError_t r = launch_crt_table(N, table, c->stream, plan);
    if (r != hipSuccess) return r;
    r = launch_crt_residue_consts(N, S, consts, c->stream, plan);
    if (r != hipSuccess) return r;
    r = launch_crt_rows(A, A_lo, m, l, lda, e, S, N, Ares, mp, lp, consts, c->stream, plan);
    if (r != hipSuccess) return r;
    return launch_crt_cols(B, B_lo, n, l, ldb, f, S, N, Bres, np, lp, consts, c->stream, plan);
  }, "residue planes");
  if (st != MPG_OK) return st;
  CrtGemmArgs g{};
  g.m = m;
  g.n = n;
  g.l_pad = lp;
  g.A = Ares;
  g.B = Bres;
  g.planeA = planeA;
  g.planeB = planeB;
  g.R = R;
  g.ldr = n4;
  g.planeR = m * n4;
  g.N = N;
  g.plan = plan;
  g.product = -1;
  for (int j = 0; j < N; ++j) g.mods[j] = kCrtModuli[j];
  st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_crt_gemm(g, c->stream); },
                  "INT8 MFMA residue products");
  if (st != MPG_OK) return st;
  return mpg_launch(c, MPG_KCLASS_AUX, [&] {
    return launch_crt_reconstruct(R, n4, m * n4, N, table, e, f, S, m, n, C, limbs, ldc, c->stream, plan);
  }, "residue reconstruction");
}

// The double-double residue form after the scales.
int crt_tail(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A, const double* A_lo,
             int64_t lda, const double* B, const double* B_lo, int64_t ldb, double* C_hi,
             double* C_lo, int64_t ldc, int S, const int* e, const int* f) {
  const bool dd = B_lo != nullptr;
  double* Cp[4] = {C_hi, C_lo, nullptr, nullptr};
  return crt_product(c, m, n, l, A, A_lo, lda, e, B, dd ? B_lo : nullptr, ldb, f, S, Cp, 2, ldc);
}

__global__ void zero_ints_kernel(int* p, int count) {
  if ((int)threadIdx.x < count) p[threadIdx.x] = 0;
}

// C := A B through the INT8 path; A_lo / B_lo (both or neither) make the
// inputs double-double, each element split as one exact value.
int ozaki_product(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A, const double* A_lo,
                  int64_t lda, const double* B, const double* B_lo, int64_t ldb, double* C_hi,
                  double* C_lo, int64_t ldc, int slices, int pairs_mode) {
  if (!c) return MPG_ERR_ARG;
  int st = check_fp64_args(c, m, n, l, A, lda, B, ldb);
  if (st != MPG_OK) return st;
  const bool dd = A_lo || B_lo;
  if (dd && l > 0 && m > 0 && n > 0 && (!A_lo || !B_lo))
    return mpg_fail(c, MPG_ERR_ARG, "NULL lo limb");
  if (m == 0 || n == 0) return MPG_OK;
  if (!C_hi || !C_lo || ldc < n) return mpg_fail(c, MPG_ERR_ARG, "bad C");
  if (pairs_mode < 0 || pairs_mode > 2) return mpg_fail(c, MPG_ERR_ARG, "pairs_mode must be 0, 1 or 2");
  if (slices < 0 || slices > ozaki_max_slices())
    return mpg_fail(c, MPG_ERR_ARG, "slices must be 0 (exact) .. %d", ozaki_max_slices());
  {
    const size_t sa = mpg_span_bytes(m, l, lda), sb = mpg_span_bytes(l, n, ldb),
                 sc = mpg_span_bytes(m, n, ldc);
    auto ov = [](const void* x, size_t a, const void* y, size_t b) {
      return x && y && a && b && (const char*)x < (const char*)y + b && (const char*)y < (const char*)x + a;
    };
    if (ov(C_hi, sc, A, sa) || ov(C_hi, sc, B, sb) || ov(C_lo, sc, A, sa) || ov(C_lo, sc, B, sb) ||
        ov(C_hi, sc, C_lo, sc) || ov(C_hi, sc, A_lo, sa) || ov(C_hi, sc, B_lo, sb) ||
        ov(C_lo, sc, A_lo, sa) || ov(C_lo, sc, B_lo, sb))
      return mpg_fail(c, MPG_ERR_ALIAS, "C overlaps an input or its other limb");
  }
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  if (l == 0) {
    double* Cp[4] = {C_hi, C_lo, nullptr, nullptr};
    return mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_zero(Cp, 2, m, n, ldc, c->stream); },
                      "zero C");
  }
  const int64_t lp = round_up(l, 64), mp = round_up(m, 64), np = round_up(n, 64);
  int *e, *f, *counter;
  if ((st = exponents(c, m, n, l, A, A_lo, lda, B, B_lo, ldb, slices == 0, &e, &f, &counter)) != MPG_OK)
    return st;
  int S = slices;
  if (S == 0) {
    if ((st = read_need(c, counter, &S)) != MPG_OK) return st;
    S = std::max(S, 1);
    if (S > ozaki_max_slices())
      return mpg_fail(c, MPG_ERR_UNSUPPORTED, "exact slicing needs %d slices (max %d)", S,
                      ozaki_max_slices());
  }
  if (pairs_mode == 2) {
    if (S > kCrtMaxSlices)
      return mpg_fail(c, MPG_ERR_UNSUPPORTED, "the residue form holds at most %d slices (%d asked)",
                      kCrtMaxSlices, S);
    return crt_tail(c, m, n, l, A, A_lo, lda, B, B_lo, ldb, C_hi, C_lo, ldc, S, e, f);
  }
  // INT32 headroom of the general kernel (above ozaki_chunked_max_slices()
  // slices): SB pairs share a diagonal accumulator over the whole of K; the
  // other kernels flush their sums every 2^31 / (S 2^20) K steps
  if (S > ozaki_chunked_max_slices() &&
      (double)ozaki_block_slices() * (double)lp * 128.0 * 128.0 >= 2147483647.0)
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "l = %lld too large for exact INT32 sums with %d slices",
                    (long long)l, S);
  c->last_slices = S;
  c->last_moduli = 0;
  void* big = nullptr;
  const int64_t planeA = mp * lp, planeB = np * lp;
  if ((st = mpg_workspace(c, 0, (size_t)S * (size_t)(planeA + planeB), &big)) != MPG_OK) return st;
  int8_t* Asl = (int8_t*)big;
  int8_t* Bsl = Asl + (size_t)S * planeA;
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipError_t r = launch_ozaki_split_rows(A, A_lo, m, l, lda, e, S, Asl, lp, planeA, mp, lp, c->stream);
    if (r != hipSuccess) return r;
    return launch_ozaki_split_cols(B, B_lo, l, n, ldb, f, S, Bsl, lp, planeB, np, lp, c->stream);
  }, "digit split");
  if (st != MPG_OK) return st;
  OzakiGemmArgs g{};
  g.m = m;
  g.n = n;
  g.l_pad = lp;
  g.S = S;
  g.triangle = pairs_mode;
  g.A = Asl;
  g.B = Bsl;
  g.planeA = planeA;
  g.planeB = planeB;
  g.e = e;
  g.f = f;
  g.C_hi = C_hi;
  g.C_lo = C_lo;
  g.ldc = ldc;
  return mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_ozaki_gemm(g, c->stream); },
                    "INT8 MFMA product");
}

}  // namespace

// MPG_AUTO with a tabled residue form of the exact slice count, without a
// host read-back: the exponent scan's count becomes a device-side plan
// (slices, moduli, whether at most kCrtMaxSlices slices suffice); the
// residue-form kernels are launched for the most moduli any count may need
// and take the plan's counts, and the block kernel of the default tile is
// launched after them and runs only when the plan rules the residue form out.
// Same results as the explicit call (or the block kernel), bit for bit; the
// stream is never synchronised and nothing is allocated once the workspace
// has grown to the shape (so the calls can be captured in a HIP graph after
// one eager call).
int mpg_dd_crt_auto(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A, const double* A_lo,
                    int64_t lda, const double* B, const double* B_lo, int64_t ldb, double* C_hi, double* C_lo,
                    int64_t ldc, bool* used) {
  *used = false;
  const int Smax = kCrtMaxSlices;
  const int Nmax = crt_moduli_for_bits(crt_product_bits(Smax, l));
  if (Nmax == 0 || crt_words(Nmax) == 0) return MPG_OK;  // the caller runs the block kernel
  CrtModuliTable tab{};
  for (int S = 1; S <= Smax; ++S) {
    const int N = crt_moduli_for_bits(crt_product_bits(S, l));
    tab.N[S] = N > 0 && crt_words(N) > 0 ? N : 0;
    tab.W[S] = crt_words(tab.N[S]);
  }
  tab.W[0] = crt_words(1);
  int st;
  int *e, *f, *counter;
  if ((st = exponents(c, m, n, l, A, A_lo, lda, B, B_lo, ldb, true, &e, &f, &counter)) != MPG_OK) return st;
  CrtPlan* plan = reinterpret_cast<CrtPlan*>(counter + 16);  // inside the small slot's 64-int tail
  if ((st = mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_crt_plan(counter, tab, plan, c->stream); },
                       "residue-form plan")) != MPG_OK)
    return st;
  double* Cp[4] = {C_hi, C_lo, nullptr, nullptr};
  if ((st = crt_product(c, m, n, l, A, A_lo, lda, e, B, B_lo, ldb, f, Smax, Cp, 2, ldc, plan)) != MPG_OK)
    return st;
  // the fallback, run only when the plan says the residue form does not fit
  int variant = 0;
  if ((st = mpg_resolve_variant(c, 2, nullptr, &variant)) != MPG_OK) return st;
  GemmBatch g{};
  g.m = m;
  g.n = n;
  g.l = l;
  g.A[0] = A;
  g.A[1] = A_lo;
  g.B[0] = B;
  g.B[1] = B_lo;
  g.C[0] = C_hi;
  g.C[1] = C_lo;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.count = 1;
  g.skip = &plan->ok;
  if ((st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_dd_block(variant, g, c->stream); },
                       "block kernel (fallback)")) != MPG_OK)
    return st;
  *used = true;
  return MPG_OK;
}

extern "C" int mpgemm_ozaki_dd(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A,
                               int64_t lda, const double* B, int64_t ldb, double* C_hi,
                               double* C_lo, int64_t ldc, int slices, int pairs_mode) {
  return ozaki_product(c, m, n, l, A, nullptr, lda, B, nullptr, ldb, C_hi, C_lo, ldc, slices,
                       pairs_mode);
}

extern "C" int mpgemm_dd_ozaki(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A_hi,
                               const double* A_lo, int64_t lda, const double* B_hi,
                               const double* B_lo, int64_t ldb, double* C_hi, double* C_lo,
                               int64_t ldc, int slices, int pairs_mode) {
  if (c && l > 0 && m > 0 && n > 0 && (!A_lo || !B_lo)) return mpg_fail(c, MPG_ERR_ARG, "NULL lo limb");
  return ozaki_product(c, m, n, l, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc, slices,
                       pairs_mode);
}

// Quad-double C := A B through the residue form: each operand is split
// exactly into its leading and trailing double-double parts (limbs 0 + 1 and
// 2 + 3), A = A_H + A_L, B = B_H + B_L; C = A_H B_H + A_H B_L + A_L B_H, each
// product exact (one slice count for all three: the largest exact count of
// the parts taking part, at most 20, so each part's residue planes serve
// both of its products) and added into C in quad-double; A_L B_L (below
// 2^-210 of |A||B| for canonical operands) is left out.
int mpg_qd_crt(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* const* A, int64_t lda,
               const double* const* B, int64_t ldb, double* const* C, int64_t ldc) {
  const int64_t mp = round_up(std::max<int64_t>(m, 1), 64), np = round_up(std::max<int64_t>(n, 1), 64);
  void* small = nullptr;
  int st = mpg_workspace(c, 1, (size_t)(2 * mp + 3 * np + 64) * sizeof(int), &small);
  if (st != MPG_OK) return st;
  int* eH = (int*)small;
  int* eL = eH + mp;
  int* fH = eL + mp;
  int* fL = fH + np;
  int* low = fL + np;
  int* cnt = low + np;  // digits needed by A_H, A_L, B_H, B_L
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, c->stream, cnt, 4);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    if ((r = launch_ozaki_scan(A[0], A[1], m, l, lda, 0, eH, nullptr, cnt + 0, c->stream)) != hipSuccess) return r;
    if ((r = launch_ozaki_scan(A[2], A[3], m, l, lda, 0, eL, nullptr, cnt + 1, c->stream)) != hipSuccess) return r;
    if ((r = launch_ozaki_scan(B[0], B[1], l, n, ldb, 1, fH, low, cnt + 2, c->stream)) != hipSuccess) return r;
    return launch_ozaki_scan(B[2], B[3], l, n, ldb, 1, fL, low, cnt + 3, c->stream);
  }, "exponent scans");
  if (st != MPG_OK) return st;
  int need[4] = {0, 0, 0, 0};
  {
    hipError_t r = hipMemcpyAsync(need, cnt, sizeof(need), hipMemcpyDeviceToHost, c->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
    if (r != hipSuccess) return mpg_hip_fail(c, r, "slice-count read-back");
  }
  struct Part {
    int a, b;  // 0: leading part, 1: trailing part
  };
  const Part parts[3] = {{0, 0}, {0, 1}, {1, 0}};
  int S[3];
  for (int k = 0; k < 3; ++k) {
    S[k] = std::max(need[parts[k].a], need[2 + parts[k].b]);
    const bool zero = need[parts[k].a] == 0 || need[2 + parts[k].b] == 0;  // an all-zero part
    if (zero) S[k] = 0;
    if (S[k] > kCrtMaxSlices)
      return mpg_fail(c, MPG_ERR_UNSUPPORTED,
                      "an exact split of the quad-double operands needs %d slices per part (max %d)", S[k],
                      kCrtMaxSlices);
  }
  if ((st = mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_zero(C, 4, m, n, ldc, c->stream); },
                       "zero C")) != MPG_OK)
    return st;
  // one slice count for the three products, so each part's residue planes
  // are formed once and serve both products it takes part in
  int Sc = 0;
  for (int k = 0; k < 3; ++k) Sc = std::max(Sc, S[k]);
  if (Sc == 0) {
    c->last_slices = 0;
    c->last_moduli = 0;
    return MPG_OK;
  }
  const int N = crt_moduli_for_bits(crt_product_bits(Sc, l));
  if (N == 0 || crt_words(N) == 0)
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "product of %d slices at l = %lld is too wide for the moduli",
                    Sc, (long long)l);
  const int64_t lp = round_up(l, crt_k_multiple()), mpad = round_up(m, crt_tile_rows()),
                npad = round_up(n, crt_tile_cols()), n4 = round_up(n, 4);
  const int64_t planeA = mpad * lp, planeB = npad * lp;
  const size_t cb = (sizeof(CrtResidueConsts) + 255) / 256 * 256;
  void *res = nullptr, *out = nullptr;
  if ((st = mpg_workspace(c, 7, (size_t)N * (size_t)(2 * planeA + 2 * planeB) + cb, &res)) != MPG_OK ||
      (st = mpg_workspace(c, 8, (size_t)N * (size_t)(m * n4) + 256 + sizeof(CrtTable), &out)) != MPG_OK)
    return st;
  int8_t* Ares[2] = {(int8_t*)res, (int8_t*)res + (size_t)N * planeA};
  int8_t* Bres[2] = {Ares[1] + (size_t)N * planeA, Ares[1] + (size_t)N * (planeA + planeB)};
  CrtResidueConsts* consts = (CrtResidueConsts*)(Bres[1] + (size_t)N * planeB);
  uint8_t* R = (uint8_t*)out;
  CrtTable* table = (CrtTable*)((char*)out + ((size_t)N * (size_t)(m * n4) + 255) / 256 * 256);
  // parts that take part in a product (a zero part takes part in none)
  bool useA[2] = {false, false}, useB[2] = {false, false};
  for (int k = 0; k < 3; ++k)
    if (S[k] > 0) {
      useA[parts[k].a] = true;
      useB[parts[k].b] = true;
    }
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipError_t r = launch_crt_table(N, table, c->stream);
    if (r != hipSuccess) return r;
    if ((r = launch_crt_residue_consts(N, Sc, consts, c->stream)) != hipSuccess) return r;
    for (int pa = 0; pa < 2; ++pa)
      if (useA[pa] && (r = launch_crt_rows(A[2 * pa], A[2 * pa + 1], m, l, lda, pa ? eL : eH, Sc, N, Ares[pa],
                                           mpad, lp, consts, c->stream)) != hipSuccess)
        return r;
    for (int pb = 0; pb < 2; ++pb)
      if (useB[pb] && (r = launch_crt_cols(B[2 * pb], B[2 * pb + 1], n, l, ldb, pb ? fL : fH, Sc, N, Bres[pb],
                                           npad, lp, consts, c->stream)) != hipSuccess)
        return r;
    return hipSuccess;
  }, "residue planes");
  if (st != MPG_OK) return st;
  for (int k = 0; k < 3; ++k) {
    if (S[k] == 0) continue;
    const int pa = parts[k].a, pb = parts[k].b;
    CrtGemmArgs g{};
    g.m = m;
    g.n = n;
    g.l_pad = lp;
    g.A = Ares[pa];
    g.B = Bres[pb];
    g.planeA = planeA;
    g.planeB = planeB;
    g.R = R;
    g.ldr = n4;
    g.planeR = m * n4;
    g.N = N;
    g.product = -1;
    for (int j = 0; j < N; ++j) g.mods[j] = kCrtModuli[j];
    if ((st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_crt_gemm(g, c->stream); },
                         "INT8 MFMA residue products")) != MPG_OK)
      return st;
    if ((st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
           return launch_crt_reconstruct(R, n4, m * n4, N, table, pa ? eL : eH, pb ? fL : fH, Sc, m, n, C, 4,
                                         ldc, c->stream);
         }, "residue reconstruction")) != MPG_OK)
      return st;
  }
  const int slices = Sc;
  int moduli = 0;
  for (int k = 0; k < 3; ++k) moduli += S[k] > 0 ? N : 0;
  c->last_slices = slices;
  c->last_moduli = moduli;
  return MPG_OK;
}

// MPG_AUTO's quad-double residue form without a read-back: the four parts'
// slice counts become a device-side plan (one slice count, the products
// with an all-zero part and the parts no product takes), the residue-form
// kernels are launched for the most moduli 20 slices need and take the
// plan's counts and gates, and the quad-double block kernel launched after
// them runs only when more than 20 slices are needed (C is zeroed first, so
// either path leaves the product in C).
int mpg_qd_crt_auto(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* const* A, int64_t lda,
                    const double* const* B, int64_t ldb, double* const* C, int64_t ldc, bool* used) {
  *used = false;
  const int Smax = kCrtMaxSlices;
  const int Nmax = crt_moduli_for_bits(crt_product_bits(Smax, l));
  if (Nmax == 0 || crt_words(Nmax) == 0) return MPG_OK;  // the caller runs the block kernel
  CrtModuliTable tab{};
  for (int S = 1; S <= Smax; ++S) {
    const int N = crt_moduli_for_bits(crt_product_bits(S, l));
    tab.N[S] = N > 0 && crt_words(N) > 0 ? N : 0;
    tab.W[S] = crt_words(tab.N[S]);
  }
  tab.W[0] = crt_words(1);
  const int64_t mp = round_up(std::max<int64_t>(m, 1), 64), np = round_up(std::max<int64_t>(n, 1), 64);
  void* small = nullptr;
  int st = mpg_workspace(c, 1, (size_t)(2 * mp + 3 * np + 64) * sizeof(int), &small);
  if (st != MPG_OK) return st;
  int* eH = (int*)small;
  int* eL = eH + mp;
  int* fH = eL + mp;
  int* fL = fH + np;
  int* low = fL + np;
  int* cnt = low + np;  // digits needed by A_H, A_L, B_H, B_L
  CrtPlan* plan = reinterpret_cast<CrtPlan*>(cnt + 16);  // inside the slot's 64-int tail
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, c->stream, cnt, 4);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    if ((r = launch_ozaki_scan(A[0], A[1], m, l, lda, 0, eH, nullptr, cnt + 0, c->stream)) != hipSuccess) return r;
    if ((r = launch_ozaki_scan(A[2], A[3], m, l, lda, 0, eL, nullptr, cnt + 1, c->stream)) != hipSuccess) return r;
    if ((r = launch_ozaki_scan(B[0], B[1], l, n, ldb, 1, fH, low, cnt + 2, c->stream)) != hipSuccess) return r;
    if ((r = launch_ozaki_scan(B[2], B[3], l, n, ldb, 1, fL, low, cnt + 3, c->stream)) != hipSuccess) return r;
    if ((r = launch_crt_plan_qd(cnt, tab, plan, c->stream)) != hipSuccess) return r;
    return launch_zero(C, 4, m, n, ldc, c->stream);
  }, "exponent scans and residue-form plan");
  if (st != MPG_OK) return st;
  const int N = Nmax;
  const int64_t lp = round_up(l, crt_k_multiple()), mpad = round_up(m, crt_tile_rows()),
                npad = round_up(n, crt_tile_cols()), n4 = round_up(n, 4);
  const int64_t planeA = mpad * lp, planeB = npad * lp;
  const size_t cb = (sizeof(CrtResidueConsts) + 255) / 256 * 256;
  void *res = nullptr, *out = nullptr;
  if ((st = mpg_workspace(c, 7, (size_t)N * (size_t)(2 * planeA + 2 * planeB) + cb, &res)) != MPG_OK ||
      (st = mpg_workspace(c, 8, (size_t)N * (size_t)(m * n4) + 256 + sizeof(CrtTable), &out)) != MPG_OK)
    return st;
  int8_t* Ares[2] = {(int8_t*)res, (int8_t*)res + (size_t)N * planeA};
  int8_t* Bres[2] = {Ares[1] + (size_t)N * planeA, Ares[1] + (size_t)N * (planeA + planeB)};
  CrtResidueConsts* consts = (CrtResidueConsts*)(Bres[1] + (size_t)N * planeB);
  uint8_t* R = (uint8_t*)out;
  CrtTable* table = (CrtTable*)((char*)out + ((size_t)N * (size_t)(m * n4) + 255) / 256 * 256);
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipError_t r = launch_crt_table(N, table, c->stream, plan);
    if (r != hipSuccess) return r;
    if ((r = launch_crt_residue_consts(N, Smax, consts, c->stream, plan)) != hipSuccess) return r;
    for (int pa = 0; pa < 2; ++pa)
      if ((r = launch_crt_rows(A[2 * pa], A[2 * pa + 1], m, l, lda, pa ? eL : eH, Smax, N, Ares[pa], mpad, lp,
                               consts, c->stream, plan, pa)) != hipSuccess)
        return r;
    for (int pb = 0; pb < 2; ++pb)
      if ((r = launch_crt_cols(B[2 * pb], B[2 * pb + 1], n, l, ldb, pb ? fL : fH, Smax, N, Bres[pb], npad, lp,
                               consts, c->stream, plan, 2 + pb)) != hipSuccess)
        return r;
    return hipSuccess;
  }, "residue planes");
  if (st != MPG_OK) return st;
  const int pa_of[3] = {0, 0, 1}, pb_of[3] = {0, 1, 0};
  for (int k = 0; k < 3; ++k) {
    const int pa = pa_of[k], pb = pb_of[k];
    CrtGemmArgs g{};
    g.m = m;
    g.n = n;
    g.l_pad = lp;
    g.A = Ares[pa];
    g.B = Bres[pb];
    g.planeA = planeA;
    g.planeB = planeB;
    g.R = R;
    g.ldr = n4;
    g.planeR = m * n4;
    g.N = N;
    g.plan = plan;
    g.product = k;
    for (int j = 0; j < N; ++j) g.mods[j] = kCrtModuli[j];
    if ((st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_crt_gemm(g, c->stream); },
                         "INT8 MFMA residue products")) != MPG_OK)
      return st;
    if ((st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
           return launch_crt_reconstruct(R, n4, m * n4, N, table, pa ? eL : eH, pb ? fL : fH, Smax, m, n, C, 4,
                                         ldc, c->stream, plan, k);
         }, "residue reconstruction")) != MPG_OK)
      return st;
  }
  // the fallback, run only when the plan says the residue form does not fit
  int variant = 0;
  if ((st = mpg_resolve_variant(c, 4, nullptr, &variant)) != MPG_OK) return st;
  GemmBatch g{};
  g.m = m;
  g.n = n;
  g.l = l;
  for (int q = 0; q < 4; ++q) {
    g.A[q] = A[q];
    g.B[q] = B[q];
    g.C[q] = C[q];
  }
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.count = 1;
  g.skip = &plan->ok;
  if ((st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_qd_block(variant, g, c->stream); },
                       "block kernel (fallback)")) != MPG_OK)
    return st;
  c->last_slices = 0;
  c->last_moduli = 0;
  *used = true;
  return MPG_OK;
}

extern "C" int mpg_ozaki_last_slices(const mpg_ctx* c) { return c ? c->last_slices : 0; }

extern "C" int mpg_ozaki_last_moduli(const mpg_ctx* c) { return c ? c->last_moduli : 0; }

extern "C" int mpg_crt_moduli_for(int slices, int64_t l) {
  if (slices < 1 || slices > kCrtMaxSlices || l < 1) return 0;
  const int N = crt_moduli_for_bits(crt_product_bits(slices, l));
  return N > 0 && crt_words(N) > 0 ? N : 0;
}

// Bound on |x y - (kept digit products)|, in units of 2^(e + f), for
// |x| < 2^e, |y| < 2^f cut into S radix-256 digits: both remainders are
// below 2^(e or f + 2 - 8S) and the kept parts (truncations) below 2^e,
// 2^f, which gives 2^(3 - 8S) with all pairs; the triangle s + t <= S + 1
// also drops, on each diagonal g = S+2 .. 2S, 2S - g + 1 products of at
// most 128^2 2^(4 - 8g).
double mpg::ozaki_unit_bound(int S, int pairs_mode) {
  double b = std::ldexp(1.0, 3 - 8 * S);
  if (pairs_mode == 1)
    for (int g = S + 2; g <= 2 * S; ++g)
      b += (double)(2 * S - g + 1) * (128.0 * 128.0) * std::ldexp(1.0, 4 - 8 * g);
  return b;
}

int mpg::ozaki_chunks(int S, int64_t l) {
  const int64_t steps = (l + 63) / 64;
  const int64_t kchunk = std::max<int64_t>(1, (int64_t)(2147483647.0 / ((double)S * 64.0 * 128.0 * 128.0)));
  return S > ozaki_chunked_max_slices() ? 1 : (int)((steps + kchunk - 1) / kchunk);
}

extern "C" int mpg_ozaki_slices_for_bits(int bits, int pairs_mode) {
  if (bits < 1 || (pairs_mode != 0 && pairs_mode != 1)) return 0;
  for (int S = 1; S <= ozaki_max_slices(); ++S)
    if (ozaki_unit_bound(S, pairs_mode) <= std::ldexp(1.0, -bits)) return S;
  return 0;
}

extern "C" int mpg_int8_mfma_rate(mpg_ctx* c, double* tops) {
  if (!c || !tops) return MPG_ERR_ARG;
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  void* small = nullptr;
  if ((st = mpg_workspace(c, 1, 256, &small)) != MPG_OK) return st;
  const int blocks = 4 * c->num_cu, steps = 2000;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t r = hipEventCreate(&a);
  if (r == hipSuccess) r = hipEventCreate(&b);
  if (r == hipSuccess) r = launch_mfma_rate(blocks, steps, (int*)small, c->stream);  // warm-up
  float best = 0.f;
  for (int rep = 0; rep < 3 && r == hipSuccess; ++rep) {
    r = hipEventRecord(a, c->stream);
    if (r == hipSuccess) r = launch_mfma_rate(blocks, steps, (int*)small, c->stream);
    if (r == hipSuccess) r = hipEventRecord(b, c->stream);
    if (r == hipSuccess) r = hipEventSynchronize(b);
    float ms = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, a, b);
    if (r == hipSuccess && (best == 0.f || ms < best)) best = ms;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "INT8 MFMA rate");
  // 16 x 16 x 64 multiply-adds = 32768 operations per MFMA
  *tops = (double)blocks * 8 * steps * 32 * 32768.0 / (best * 1e-3) / 1e12;
  return MPG_OK;
}
