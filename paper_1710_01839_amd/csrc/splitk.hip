// Split-K for skinny products: the K range of Eq. (1) / Eq. (2) is cut into
// P consecutive chunks, each chunk's partial product is formed by the block
// kernel (P problems of one grouped launch), and this kernel adds the
// partials of every entry in a fixed order.  Eq. (1) and Eq. (2) fix no
// order of summation, so any fixed order is admissible; this one is the
// same on every run (no atomics), which makes the result deterministic.
//
// Reduction of one entry: Q lanes of a wavefront share the entry; lane r
// adds the partials p = r, r + Q, r + 2Q, ... in increasing p with the
// accurate multi-limb sum, then log2(Q) butterfly steps over __shfl_xor add
// the lanes' sums pairwise, the lane with the lower index always first, so
// both lanes of a pair hold the same bits and the order is a fixed tree.
#include "mp_arith.hpp"
#include "splitk_internal.hpp"

namespace mpg {
namespace {

template <class Arith, int Q>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(SplitKReduceArgs a) {
  constexpr int L = Arith::L;
  constexpr int E = 64 / Q;  // entries per wavefront
  const int lane = threadIdx.x % 64;
  const int r = lane / E;
  const int64_t entry = ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * E + lane % E;
  const int64_t mn = a.m * a.n;
  const bool live = entry < mn;
  double s[L];
#pragma unroll
  for (int q = 0; q < L; ++q) s[q] = 0.0;
  if (live) {
    for (int64_t p = r; p < a.P; p += Q) {
      double x[L];
#pragma unroll
      for (int q = 0; q < L; ++q) x[q] = a.W[q][p * mn + entry];
      Arith::add(s, x, s);
    }
  }
  // butterfly over the Q lanes of the entry (lanes r and r ^ bit): the lane
  // without `bit` is the left operand in both lanes
#pragma unroll
  for (int bit = 1; bit < Q; bit <<= 1) {
    double o[L], left[L], right[L];
#pragma unroll
    for (int q = 0; q < L; ++q) o[q] = __shfl_xor(s[q], bit * E, 64);
    const bool upper = (r & bit) != 0;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      left[q] = upper ? o[q] : s[q];
      right[q] = upper ? s[q] : o[q];
    }
    Arith::add(left, right, s);
  }
  if (live && r == 0) {
    const int64_t i = entry / a.n, j = entry - i * a.n;
#pragma unroll
    for (int q = 0; q < L; ++q) a.C[q][i * a.ldc + j] = s[q];
  }
}

template <class Arith, int Q>
hipError_t launch_q(const SplitKReduceArgs& a, hipStream_t s) {
  constexpr int E = 64 / Q;
  const int64_t waves = (a.m * a.n + E - 1) / E;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((splitk_reduce_kernel<Arith, Q>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int splitk_lanes_per_entry(int64_t m, int64_t n, int64_t P) {
  // few entries: many lanes per entry; many entries: whole 128-byte lines of
  // consecutive entries per partial
  if (P >= 64 && m * n <= 4096) return 16;
  return 4;
}

hipError_t launch_splitk_reduce(int limbs, const SplitKReduceArgs& a, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0) return hipSuccess;
  if (a.P < 1 || (limbs != 2 && limbs != 4)) return hipErrorInvalidValue;
  const int Q = splitk_lanes_per_entry(a.m, a.n, a.P);
  if (limbs == 2) return Q == 16 ? launch_q<DDArith, 16>(a, s) : launch_q<DDArith, 4>(a, s);
  return Q == 16 ? launch_q<QDArith, 16>(a, s) : launch_q<QDArith, 4>(a, s);
}

}  // namespace mpg
