// Internal interface of the BLAS-style surface kernels (blas.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

// One copy of a rows x cols destination block:
//   dst[r * ldd + c] = sign * (trans ? src[c * lds + r] : src[r * lds + c]).
// sign is +1 or -1 (exact).
struct PackJob {
  const double* src;
  double* dst;
  int64_t rows, cols, lds, ldd;
  int trans;
  double sign;
};

constexpr int kMaxPackJobs = 8;

struct PackArgs {
  PackJob job[kMaxPackJobs];
  int count;
};

// C := alpha T + beta C, element-wise over m x n, limb planes of L limbs.
struct AxpbyArgs {
  const double* T[4];
  int64_t ldt;
  double* C[4];
  int64_t ldc;
  int64_t m, n;
  double alpha[4], beta[4];
  int use_t, use_c;
};

// Complex DD form: P = [Re | Im] (2 planes, ldp >= 2n), C four planes
// (re hi, re lo, im hi, im lo).
struct ZAxpbyArgs {
  const double* P[2];
  int64_t ldp;
  double* C[4];
  int64_t ldc;
  int64_t m, n;
  double alpha[4], beta[4];
  int use_p, use_c;
};

hipError_t launch_pack(const PackArgs& a, hipStream_t s);
hipError_t launch_axpby(int limbs, const AxpbyArgs& a, hipStream_t s);
hipError_t launch_zaxpby(const ZAxpbyArgs& a, hipStream_t s);

}  // namespace mpg
