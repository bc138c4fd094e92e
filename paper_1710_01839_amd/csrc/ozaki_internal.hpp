// Internal interface of the split-precision (INT8 MFMA) path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace mpg {

struct OzakiGemmArgs {
  int64_t m, n, l_pad;      // real output size, padded K (multiple of 64)
  int S;                    // digit planes per operand
  int triangle;             // 1: keep pairs with s + t <= S + 1 only
  const int8_t* A;          // [S][m_pad][l_pad]
  const int8_t* B;          // [S][n_pad][l_pad] (columns of B, K contiguous)
  int64_t planeA, planeB;   // bytes per plane
  const int* e;             // row exponents of A (m)
  const int* f;             // column exponents of B (n)
  double* C_hi;
  double* C_lo;
  int64_t ldc;
};

// blocks x 512 threads of back-to-back INT8 MFMAs (32 per wavefront and
// step, `steps` steps); sink: one device int, written only in theory.
hipError_t launch_mfma_rate(int blocks, int steps, int* sink, hipStream_t s);

int ozaki_max_slices();
// Slices per pair block of the general kernel, and the largest slice count
// served by the kernels that split K into INT32-safe chunks.
int ozaki_block_slices();
int ozaki_chunked_max_slices();
// A-priori truncation bound per unit of 2^(e_i + f_j) per product term
// (S slices; pairs_mode 0 all pairs, 1 the triangle), and the number of
// INT32 chunks K is cut into (1 for the general kernel).
double ozaki_unit_bound(int S, int pairs_mode);
int ozaki_chunks(int S, int64_t l);
// Exponents e of the rows (by_col 0) or columns (by_col 1) of X (R x K):
// 1 + max ilogb, 0 for an all-zero line.  When `need` is given it is raised
// to the largest number of radix-256 digits any line needs to hold its
// elements exactly after scaling by 2^-(e + 2) (columns then use `low`, K
// ints of scratch); with Xlo (double-double input) the lo limbs' lowest
// set bits count too, the scale comes from X.  One pass over X (and Xlo).
hipError_t launch_ozaki_scan(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                             int by_col, int* e, int* low, int* need, hipStream_t s);
// Digit planes of the rows (columns) of X, or of X + Xlo split as one
// exact value when Xlo is given (double-double input).
hipError_t launch_ozaki_split_rows(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                                   const int* e, int S, int8_t* out, int64_t ld_out, int64_t plane,
                                   int64_t Rp, int64_t Kp, hipStream_t s);
hipError_t launch_ozaki_split_cols(const double* X, const double* Xlo, int64_t K, int64_t C, int64_t ld,
                                   const int* f, int S, int8_t* out, int64_t ld_out, int64_t plane,
                                   int64_t Cp, int64_t Kp, hipStream_t s);
hipError_t launch_ozaki_gemm(const OzakiGemmArgs& a, hipStream_t s);

}  // namespace mpg
