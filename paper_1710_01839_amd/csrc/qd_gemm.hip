// Quad-double GEMM kernel instances (simple, block variants, Winograd
// operand formation / assembly).
#include "gemm_kernels.hpp"

namespace mpg {
namespace {

using kern::variant_entry;
using kern::VariantEntry;

// Built QD tile variants (BM, BN, BK, TM, TN, threads).  Index 0 is the
// default.
const VariantEntry kVariants[] = {
    variant_entry<QDArith, 32, 32, 8, 2, 2>(),
    variant_entry<QDArith, 64, 32, 8, 4, 2>(),
    variant_entry<QDArith, 64, 64, 8, 4, 4, 1>(),
    variant_entry<QDArith, 32, 64, 8, 2, 4>(),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int qd_num_variants() { return kNumVariants; }
const TileVariant& qd_variant(int v) { return kVariants[v].v; }
int qd_variant_resident(int v) { return kern::resident_blocks(kVariants[v]); }

hipError_t launch_qd_simple(const GemmBatch& g, hipStream_t s) {
  return kern::launch_simple<QDArith>(g, s);
}

hipError_t launch_qd_block(int variant, const GemmBatch& g, hipStream_t s) {
  if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
  return kVariants[variant].fn(g, s);
}

hipError_t launch_qd_winograd_form(const FormArgs& a, hipStream_t s) {
  return kern::launch_form<QDArith>(a, s);
}

hipError_t launch_qd_winograd_assemble(const AssembleArgs& a, hipStream_t s) {
  return kern::launch_assemble<QDArith>(a, s);
}

}  // namespace mpg
