// Internal interface of the residue (Chinese remainder) form of the split
// product: the integer images of the operands (the sums of their S radix-256
// digits) are multiplied modulo N small pairwise coprime moduli on INT8 MFMA,
// and the exact integer product is rebuilt from the N residues.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

// Pairwise coprime moduli, taken greedily from 256 downwards (largest first,
// so the first N carry the most bits).  Residues in [-p/2, p/2) fit a signed
// byte.  Their product is about 2^341.9.
constexpr int kCrtMaxModuli = 49;
constexpr int kCrtModuli[kCrtMaxModuli] = {
    256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193, 191,
    181, 179, 173, 167, 163, 157, 151, 149, 139, 137, 131, 127, 113, 109, 107, 103, 101,
    97,  89,  83,  79,  73,  71,  67,  61,  59,  53,  47,  43,  41,  37,  29};
// 32-bit words of the reconstruction (N 255 P < 2^(32 W) with room for the
// per-word sums); the largest supported product is 12 words.
constexpr int kCrtMaxWords = 12;
// Integer images hold at most this many digits (160 bits: four 40-bit words).
constexpr int kCrtMaxSlices = 20;

// Reconstruction table, built on the device for N moduli:
//   T[j] = (P / p_j) * ((P / p_j)^-1 mod p_j) (so X = sum_j r_j T[j] mod P),
//   P = prod p_j, half = P / 2 (P is even: 256 is the first modulus),
//   Pd = P rounded to a double.
//   frag: the T[j] in signed radix-256 digits d_jb in [-128, 127]
//   (T[j] = sum_b d_jb 256^b, positions below 4 kCrtMaxWords kept) in the
//   lane order of the A operand of v_mfma_i32_16x16x64_i8, rows = digit
//   positions, k = moduli: frag[g][l][k] = d_{16 (l / 16) + k, 16 g + l % 16}
//   (0 for moduli j >= N);
//   K0 = 128 sum_j T[j] in words (the offset that turns sums over r_j - 128
//   back into sums over r_j).
constexpr int kCrtFragGroups = 4 * kCrtMaxWords / 16;
struct CrtTable {
  uint32_t T[kCrtMaxModuli][kCrtMaxWords];
  uint32_t P[kCrtMaxWords];
  uint32_t half[kCrtMaxWords];
  double Pd;
  int N;
  uint32_t K0[kCrtMaxWords];
  alignas(16) int8_t frag[kCrtFragGroups][64][16];
};

// Slice and moduli counts of a residue-form product decided on the device
// (from the exponent scan's exact slice count), so that the host need not
// read them back: every kernel given a plan takes S and N from it, and
// none does anything when ok is 0 (more than kCrtMaxSlices slices).  For
// the quad-double form (three products of double-double parts) skip[k]
// marks a product with an all-zero part and unused[p] a part (A_H, A_L, B_H,
// B_L) no remaining product takes; a kernel given its index does nothing
// then.  W is crt_words(N): the reconstruction is launched once per built
// word count up to that of the most moduli, and only the launch of the
// plan's W works.
struct CrtPlan {
  int S, N, ok;
  int skip[3];
  int unused[4];
  int W;
};
// Moduli for 1..kCrtMaxSlices slices at one l (index S; 0: does not fit)
// and their reconstruction word counts (W[0]: that of one modulus).
struct CrtModuliTable {
  int N[kCrtMaxSlices + 1];
  int W[kCrtMaxSlices + 1];
};
hipError_t launch_crt_plan(const int* need, const CrtModuliTable& t, CrtPlan* plan, hipStream_t s);
// The quad-double plan from the four parts' exact slice counts
// (need[0..3]: A_H, A_L, B_H, B_L; 0 = an all-zero part).
hipError_t launch_crt_plan_qd(const int* need, const CrtModuliTable& t, CrtPlan* plan, hipStream_t s);

// One INT8 product per modulus: residue planes z of A ([N] planes of
// m_pad x l_pad) and of B ([N] planes of n_pad x l_pad, the columns of B as
// rows), in the tiled layout of crt_plane_offset, padded as crt_tile_rows(),
// crt_tile_cols() and crt_k_multiple() ask; output residues in [0, p_z) as
// bytes, R[z * planeR + r * ldr + c].
// K may run over several segments (a sum of products A_s B_s of equal
// shape, one INT32 accumulation): segment s reads the planes at A + segA[s],
// B + segB[s] (byte offsets; nseg 0 or 1 with zero offsets is one product).
constexpr int kCrtMaxSegments = 16;
struct CrtGemmArgs {
  int64_t m, n, l_pad;
  const int8_t* A;
  const int8_t* B;
  int64_t planeA, planeB;
  uint8_t* R;
  int64_t ldr, planeR;
  int N;
  int mods[kCrtMaxModuli];
  int nseg;
  int64_t segA[kCrtMaxSegments], segB[kCrtMaxSegments];
  const CrtPlan* plan;  // when set: moduli z >= plan->N do nothing
  int product;          // >= 0: nothing when plan->skip[product] is set
};

// Bits the integer product can need: |(A' B')_ij| < l 2^(16 S - 4), and the
// symmetric range needs P > 2 max |X|.
int crt_product_bits(int S, int64_t l);
// Fewest leading moduli whose product exceeds 2^bits (0 if none).
int crt_moduli_for_bits(int bits);
// 32-bit words the reconstruction of N moduli uses (0 if unsupported).
int crt_words(int N);

// Byte offset of element (r, k) in a residue plane of Kp columns: planes are
// stored in 1 KiB blocks of 16 rows x 64 k (block (r / 16, k / 64), row-major
// inside), so the 16 x 64 operand block of one K step is one contiguous
// kibibyte (whole cache lines) for the product kernel's LDS loads.
__host__ __device__ __forceinline__ int64_t crt_plane_offset(int64_t r, int64_t k, int64_t Kp) {
  return ((r >> 4) * (Kp >> 6) + (k >> 6)) * 1024 + (r & 15) * 64 + (k & 63);
}

// The MFMA digit sums of an output, four consecutive radix-256 positions
// 4wd .. 4wd + 3 (|x| < 2^20 each), as two int32 sums of 16-bit halves:
// x0 + 2^8 x1 and x2 + 2^8 x3 (each below 2^29 in magnitude), so that the
// word sum V_wd = sum_i x_i 2^(8i) is half0 + 2^16 half1 with no 64-bit
// arithmetic; packed low half first.
__device__ __forceinline__ uint64_t crt_half_sums(int x0, int x1, int x2, int x3) {
  const uint32_t h0 = (uint32_t)(x0 + (x1 << 8)), h1 = (uint32_t)(x2 + (x3 << 8));
  return (uint64_t)h0 | ((uint64_t)h1 << 32);
}

// The W 32-bit words of sum_h vh[h] 2^(16h) + K0 (2W half sums vh from
// crt_half_sums, K0 the table's constant) by a signed carry pass over 16-bit
// steps in int32: each step holds |vh| < 2^29, a 16-bit piece of K0 and a
// carry below 2^14.  The value is below 2^(32W), so the positions from 32W
// up cancel against the last carry, which is dropped.
template <int W>
__device__ __forceinline__ void crt_carry_halves(const int32_t* vh, const CrtTable& t, uint64_t (&acc)[W]) {
  int32_t carry = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint32_t k0 = t.K0[w];
    const int32_t s0 = vh[2 * w] + (int32_t)(k0 & 0xFFFFu) + carry;
    carry = s0 >> 16;
    const int32_t s1 = vh[2 * w + 1] + (int32_t)(k0 >> 16) + carry;
    carry = s1 >> 16;
    acc[w] = ((uint32_t)s0 & 0xFFFFu) | ((uint32_t)s1 << 16);
  }
}

// Reduces X' = sum_j r_j T_j (per 32-bit word in 64-bit accumulators, W
// words; X' < N 256 P < 2^(32 W)) to the centred CRT value: returns its sign
// and writes its magnitude words to y.  Branch-free, by borrow chains:
//   q: the quotient estimate, X' summed in doubles times rP = 1 / Pd
//      (rounded), scaled by 1 - 2^-45 so that it never exceeds
//      floor(X' / P) (the estimate's relative error is below 2^-48: W + 1
//      roundings in the sum and Pd, two more in 1 / Pd and the product) and
//      is at most one below it (X' / P < 2^14);
//   Y = X' - q P lies in [0, 2 P): P is subtracted where that leaves no
//      borrow;
//   Y >= P / 2 (no borrow in Y - P / 2) stands for Y - P: magnitude P - Y.
template <int W>
__device__ __forceinline__ bool crt_magnitude(const uint64_t (&acc)[W], const CrtTable& t, double rP,
                                              uint32_t (&y)[W]) {
  uint32_t x[W];
  uint64_t carry = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint64_t s = acc[w] + carry;
    x[w] = (uint32_t)s;
    carry = s >> 32;
  }
  double xd = 0.0;
#pragma unroll
  for (int w = W - 1; w >= 0; --w) xd += ldexp((double)x[w], 32 * w);
  const uint32_t q = (uint32_t)floor(xd * rP * (1.0 - 0x1p-45));
  uint32_t mc = 0;
  unsigned b = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint64_t qp = (uint64_t)q * t.P[w] + mc;
    mc = (uint32_t)(qp >> 32);
    y[w] = __builtin_subc(x[w], (uint32_t)qp, b, &b);
  }
  uint32_t z[W];
  b = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) z[w] = __builtin_subc(y[w], t.P[w], b, &b);
  const bool ge = b == 0;
#pragma unroll
  for (int w = 0; w < W; ++w) y[w] = ge ? z[w] : y[w];
  b = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) (void)__builtin_subc(y[w], t.half[w], b, &b);
  const bool neg = b == 0;
  b = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) z[w] = __builtin_subc(t.P[w], y[w], b, &b);
#pragma unroll
  for (int w = 0; w < W; ++w) y[w] = neg ? z[w] : y[w];
  return neg;
}

// plan (nullable): N from the plan (nothing when it is not ok).
hipError_t launch_crt_table(int N, CrtTable* t, hipStream_t s, const CrtPlan* plan = nullptr);

// Integer images are folded into words of five digits (40 bits, exact
// doubles), most significant word first: word k holds digits 5k .. 5k + 4
// (digit 0 the leading one), Horner-folded, so with S digits its weight is
// 256^max(S - 5k - 5, 0); kCrtImageWords of them hold 20 digits.  The
// residue constants of one slice count S: c[z][k] = that weight mod p_z
// (0 for words past the last digit) and inv[z] = 1 / p_z rounded to double.
constexpr int kCrtDigitsPerWord = 5;
constexpr int kCrtImageWords = kCrtMaxSlices / kCrtDigitsPerWord;
struct CrtResidueConsts {
  double c[kCrtMaxModuli][kCrtImageWords];
  double inv[kCrtMaxModuli];
};
// plan (nullable): S from the plan (nothing when it is not ok).
hipError_t launch_crt_residue_consts(int N, int S, CrtResidueConsts* rc, hipStream_t s,
                                     const CrtPlan* plan = nullptr);

// Residues of 8 elements' images (sum_w words[w][q] c[w], the first NW
// words nonzero, |word| < 2^41 + 2, c < 256: the sum stays below 2^51, so
// it, the rounded quotient's product and the remainder are exact in FP64)
// modulo p, packed as signed bytes (element q in byte q); inv is 1/p rounded.  The computed quotient acc inv is within 1/(2p) of the
// exact one (two roundings of relative 2^-53 on a value below 2^51 / p), so
// the remainder of its nearest integer lies in [-(p+1)/2, (p+1)/2]: for the
// odd moduli up to 253 that is inside [-127, 127] and already a signed
// byte.  With CENTRE (p = 256, 255) one correction each way brings it into
// [-p/2, p/2).  Any representative serves the products, which reduce modulo
// p at the end.
template <int NW, bool CENTRE>
__device__ __forceinline__ uint64_t crt_residues8(const double (&words)[kCrtImageWords][8],
                                                  const double* c, int p, double inv) {
  const double pd = (double)p;
  uint32_t v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) acc = __builtin_fma(words[w][q], c[w], acc);
    double r = __builtin_fma(-rint(acc * inv), pd, acc);
    if (CENTRE) {
      if (2.0 * r >= pd) r -= pd;
      if (2.0 * r < -pd) r += pd;
    }
    v[q] = (uint32_t)(int)r;
  }
  // the low bytes (two's complement) four at a time: two byte pairs, then
  // the pairs (three byte permutes per four elements)
  uint32_t half[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t p01 = __builtin_amdgcn_perm(v[4 * h + 1], v[4 * h], 0x0c0c0400u);      // e0 e1 0 0
    const uint32_t p23 = __builtin_amdgcn_perm(v[4 * h + 3], v[4 * h + 2], 0x0c0c0400u);  // e2 e3 0 0
    half[h] = __builtin_amdgcn_perm(p23, p01, 0x05040100u);                                // e0 e1 e2 e3
  }
  return (uint64_t)half[0] | (uint64_t)half[1] << 32;
}

// Residue planes straight from the operand rows: for each row r of X (R x K,
// X + Xlo as one exact value when Xlo is given) and its scale e[r], the S
// truncated radix-256 digits of x 2^-(e + 2) are folded into the image
// A' = trunc(x 2^(8S - 2 - e)) and reduced modulo the N leading moduli:
// plane z of out (Rp Kp bytes), element (r, k) at crt_plane_offset(r, k, Kp)
// (r < Rp, k < Kp, zeros in the padding).
// plan (nullable): S and N from the plan (nothing when it is not ok; the
// planes must hold the N given here, at least the plan's).
// part >= 0 (with a plan): nothing when plan->unused[part] is set.
hipError_t launch_crt_rows(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                           const int* e, int S, int N, int8_t* out, int64_t Rp, int64_t Kp,
                           const CrtResidueConsts* rc, hipStream_t s, const CrtPlan* plan = nullptr,
                           int part = -1);
// The same for the columns of X (K x R row-major, leading dimension ld):
// plane row r is column r of X (B's columns, read in place).
hipError_t launch_crt_cols(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                           const int* e, int S, int N, int8_t* out, int64_t Rp, int64_t Kp,
                           const CrtResidueConsts* rc, hipStream_t s, const CrtPlan* plan = nullptr,
                           int part = -1);

// Workgroup tile of the residue products: A's planes need rows padded to
// crt_tile_rows(), B's to crt_tile_cols(), K to crt_k_multiple().
int crt_tile_rows();
int crt_tile_cols();
int crt_k_multiple();
hipError_t launch_crt_gemm(const CrtGemmArgs& a, hipStream_t s);
// V_ij = X_ij 2^(e_i + f_j + 4 - 16 S), X the CRT value of the N residues:
// limbs 2: C (hi, lo) := V rounded to double-double; limbs 4: C (four
// limbs) := C + V in quad-double.
// plan (nullable): N and S from the plan (nothing when it is not ok; the
// word count is that of the N given here, at least the plan's).
// product >= 0 (with a plan): nothing when plan->skip[product] is set.
hipError_t launch_crt_reconstruct(const uint8_t* R, int64_t ldr, int64_t planeR, int N,
                                  const CrtTable* t, const int* e, const int* f, int S, int64_t m,
                                  int64_t n, double* const* C, int limbs, int64_t ldc, hipStream_t s,
                                  const CrtPlan* plan = nullptr, int product = -1);

}  // namespace mpg
