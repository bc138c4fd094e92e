// Double-double GEMM kernel instances (simple, block variants, Winograd
// operand formation / assembly).
#include "gemm_direct.hpp"
#include "gemm_kernels.hpp"

namespace mpg {
namespace {

using kern::variant_entry;
using kern::VariantEntry;

// Built DD tile variants (BM, BN, BK, TM, TN, threads).  The default (tile
// fields all zero) is the direct kernel, kDefaultVariant.  BK must be a
// multiple of the 8-step renormalisation period.
const VariantEntry kVariants[] = {
    variant_entry<DDArith, 64, 64, 16, 4, 4>(),
    variant_entry<DDArith, 32, 32, 16, 2, 2>(),
    variant_entry<DDArith, 128, 64, 8, 8, 4, 1>(),
    variant_entry<DDArith, 64, 128, 8, 4, 8, 1>(),
    variant_entry<DDArith, 128, 128, 8, 8, 8, 1>(),
    variant_entry<DDArith, 64, 64, 8, 4, 4>(),
    variant_entry<DDArith, 32, 64, 16, 2, 4>(),
    kern::direct_entry<DDArith, 2, 4>(),  // 64x64x8, 2x4, 512 threads, load unit to LDS
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kDefaultVariant = 7;

__global__ __launch_bounds__(256) void zero_kernel(double* C0, double* C1, double* C2, double* C3,
                                                   int limbs, int64_t m, int64_t n, int64_t ldc) {
  const int64_t total = m * n;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int64_t off = (idx / n) * ldc + idx % n;
    C0[off] = 0.0;
    if (limbs > 1) C1[off] = 0.0;
    if (limbs > 2) C2[off] = 0.0;
    if (limbs > 3) C3[off] = 0.0;
  }
}

}  // namespace

int dd_num_variants() { return kNumVariants; }
int dd_default_variant() { return kDefaultVariant; }
const TileVariant& dd_variant(int v) { return kVariants[v].v; }
int dd_variant_resident(int v) { return kern::resident_blocks(kVariants[v]); }

hipError_t launch_dd_simple(const GemmBatch& g, hipStream_t s) {
  return kern::launch_simple<DDArith>(g, s);
}

hipError_t launch_dd_block(int variant, const GemmBatch& g, hipStream_t s) {
  if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
  return kVariants[variant].fn(g, s);
}

hipError_t launch_dd_winograd_form(const FormArgs& a, hipStream_t s) {
  return kern::launch_form<DDArith>(a, s);
}

hipError_t launch_dd_winograd_assemble(const AssembleArgs& a, hipStream_t s) {
  return kern::launch_assemble<DDArith>(a, s);
}

hipError_t launch_zero(double* const* C, int limbs, int64_t m, int64_t n, int64_t ldc,
                       hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t blocks = (m * n + 255) / 256;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0,
                     s, C[0], limbs > 1 ? C[1] : C[0], limbs > 2 ? C[2] : C[0],
                     limbs > 3 ? C[3] : C[0], limbs, m, n, ldc);
  return hipGetLastError();
}

}  // namespace mpg
