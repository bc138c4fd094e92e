// Internal interface of the split-K reduction (splitk.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

// Partials of P chunk products, limb plane q of partial p at
// W[q] + p * m * n (row-major m x n, leading dimension n); the sum of the
// partials of every entry goes to C (leading dimension ldc).
struct SplitKReduceArgs {
  const double* W[4];
  double* C[4];
  int64_t m, n, ldc, P;
};

// Lanes of a wavefront that share one entry's partials (4 or 16).
int splitk_lanes_per_entry(int64_t m, int64_t n, int64_t P);
// limbs 2 (DD) or 4 (QD).
hipError_t launch_splitk_reduce(int limbs, const SplitKReduceArgs& a, hipStream_t s);

}  // namespace mpg
