// Internal interfaces between the host driver (capi.cpp) and the kernel
// translation units.  Not installed; the public surface is include/mpgemm.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

// A batch of equal-shape problems C_p := A_p B_p, p = 0..count-1, with
// A_p = A + p * sA (per limb plane), etc.  Limb planes are given as arrays
// of up to 4 pointers (DD uses 2, QD 4).  Rows/cols beyond (m, n, l) are
// never touched.
struct GemmBatch {
  int64_t m, n, l;
  const double* A[4];
  int64_t lda, sA;
  const double* B[4];
  int64_t ldb, sB;
  double* C[4];
  int64_t ldc, sC;
  int count;
  // when set, a kernel whose *skip is nonzero at run time does nothing (the
  // fallback of a product decided on the device)
  const int* skip;
};

// Block-kernel tile variant description.
struct TileVariant {
  int bm, bn, bk, tm, tn, threads;
};

// ---- DD (dd_gemm.hip) ----
int dd_num_variants();
int dd_default_variant();  // index used when a tile leaves every field zero
const TileVariant& dd_variant(int v);
int dd_variant_resident(int v);  // workgroups per CU
hipError_t launch_dd_simple(const GemmBatch& g, hipStream_t s);
hipError_t launch_dd_block(int variant, const GemmBatch& g, hipStream_t s);

// Winograd operand formation for one recursion level.  `parents` matrices
// of 2h x 2w (stored with leading dimension ld_par, parent p at base +
// p * s_par, only rows < vr and cols < vc valid, the rest read as zero) give
// 7 children each (h x w, leading dimension w, child 7p + c at base + (7p +
// c) * s_ch).  side 0 = A operands, side 1 = B operands.
struct FormArgs {
  int side;
  int parents;
  int64_t h, w;
  const double* par[4];
  int64_t ld_par, s_par, vr, vc;
  double* ch[4];
  int64_t s_ch;
};
hipError_t launch_dd_winograd_form(const FormArgs& a, hipStream_t s);

// Winograd assembly: 7 children products (h x w each, leading dimension w,
// child 7p + c at base + (7p + c) * s_ch) of parent p give the parent's
// 2h x 2w product (leading dimension ld_par, at base + p * s_par), of which
// only rows < vr and cols < vc are written.
struct AssembleArgs {
  int parents;
  int64_t h, w;
  const double* ch[4];
  int64_t s_ch;
  double* par[4];
  int64_t ld_par, s_par, vr, vc;
};
hipError_t launch_dd_winograd_assemble(const AssembleArgs& a, hipStream_t s);

// ---- QD (qd_gemm.hip) ----
int qd_num_variants();
const TileVariant& qd_variant(int v);
int qd_variant_resident(int v);
hipError_t launch_qd_simple(const GemmBatch& g, hipStream_t s);
hipError_t launch_qd_block(int variant, const GemmBatch& g, hipStream_t s);
hipError_t launch_qd_winograd_form(const FormArgs& a, hipStream_t s);
hipError_t launch_qd_winograd_assemble(const AssembleArgs& a, hipStream_t s);

// C := 0 on an m x n block (l == 0 case).
hipError_t launch_zero(double* const* C, int limbs, int64_t m, int64_t n, int64_t ldc,
                       hipStream_t s);

}  // namespace mpg
