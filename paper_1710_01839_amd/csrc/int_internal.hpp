// Internal interface of the long-integer product (intgemm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crt_internal.hpp"

namespace mpg {

// Largest operand size: 64 words (2048 bits, 16 chunks of 128 bits).
constexpr int kIntMaxWords = 4 * kCrtMaxSegments;
// Chunk widths built: 3, 4 and 5 words (96, 128, 160 bits).
constexpr int kIntMaxChunkWords = 5;
// Largest number of leaf-diagonal terms of one diagonal of the product, and
// of chunks summed into one Karatsuba operand.
constexpr int kIntMaxTerms = 64;
constexpr int kIntMaxSumInputs = 8;

// Residue planes of every chunk (chunk_words words) of X's entries (R x K
// logical, word planes `pstride` elements apart, leading dimension ld; with
// cols the logical (r, k) entry is X[k][r]): plane c N + z (Rp Kp bytes
// each) of out, element (r, k) at crt_plane_offset(r, k, Kp), zeros in the
// padding (Rp a multiple of 32, Kp of 64).
struct IntResidueArgs {
  const uint32_t* X;
  int words;
  int64_t pstride, ld;
  int64_t R, K, Rp, Kp;
  int chunks, N;
  int8_t* out;
  int chunk_words;
};

// Residue planes of a chunk sum: chunk `out` := chunks in[0 .. nin) added,
// for every modulus (chunk c's planes at base + (c N + z) plane).
struct IntSumArgs {
  int8_t* base;
  int64_t plane;
  int N;
  int out;
  int nin;
  int in[kIntMaxSumInputs];
};

// C (words_c word planes, pstride apart, leading dimension ldc) += the CRT
// value of sum_q term_sign[q] R_q times 2^(32 word_off), R_q the residue
// planes at R + term_off[q] (N planes, ldr, planeR).
struct IntAccumArgs {
  const uint8_t* R;
  int64_t ldr, planeR;
  int N;
  const CrtTable* t;
  uint32_t* C;
  int words_c, word_off;
  int64_t pstride, ldc, m, n;
  int nterms;
  int64_t term_off[kIntMaxTerms];
  int term_sign[kIntMaxTerms];
};

hipError_t launch_int_residues(const IntResidueArgs& a, bool cols, hipStream_t s);
hipError_t launch_int_sum(const IntSumArgs& a, hipStream_t s);
hipError_t launch_int_accumulate(const IntAccumArgs& a, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* C, int words, int64_t pstride, int64_t m, int64_t n, int64_t ldc,
                           hipStream_t s);

}  // namespace mpg
