// Host side of the exact long-integer (fixed-point) matrix product.
#include <algorithm>

#include "capi_internal.hpp"
#include "crt_internal.hpp"
#include "int_internal.hpp"

using namespace mpg;

namespace {

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

int bit_length(int64_t v) {
  int b = 0;
  while (v > 0) {
    ++b;
    v >>= 1;
  }
  return b;
}

}  // namespace

extern "C" int mpg_int_words_needed(int words_a, int words_b, int64_t l) {
  if (words_a < 1 || words_b < 1 || l < 0) return 0;
  const int64_t bits = 32 * (int64_t)(words_a + words_b) - 2 + bit_length(std::max<int64_t>(l, 1)) + 1;
  return (int)((bits + 31) / 32);
}

extern "C" int mpg_int_gemm(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const uint32_t* A, int words_a,
                            int64_t lda, int64_t plane_a, const uint32_t* B, int words_b, int64_t ldb,
                            int64_t plane_b, uint32_t* C, int words_c, int64_t ldc, int64_t plane_c) {
  if (!c) return MPG_ERR_ARG;
  if (m < 0 || n < 0 || l < 0) return mpg_fail(c, MPG_ERR_ARG, "negative dimension");
  if (words_a < 1 || words_b < 1 || words_a > kIntMaxWords || words_b > kIntMaxWords)
    return mpg_fail(c, MPG_ERR_ARG, "operand words must be 1..%d", kIntMaxWords);
  if (m == 0 || n == 0) return MPG_OK;
  if (words_c < mpg_int_words_needed(words_a, words_b, l))
    return mpg_fail(c, MPG_ERR_ARG, "words_c = %d cannot hold every product (need %d)", words_c,
                    mpg_int_words_needed(words_a, words_b, l));
  if (!C || ldc < n || plane_c < (m - 1) * ldc + n) return mpg_fail(c, MPG_ERR_ARG, "bad C");
  if (l > 0 && (!A || !B || lda < l || ldb < n || plane_a < (m - 1) * lda + l || plane_b < (l - 1) * ldb + n))
    return mpg_fail(c, MPG_ERR_ARG, "bad A or B");
  {
    const size_t sa = ((size_t)(words_a - 1) * plane_a + (size_t)((m - 1) * lda + l)) * 4,
                 sb = ((size_t)(words_b - 1) * plane_b + (size_t)((l - 1) * ldb + n)) * 4,
                 sc = ((size_t)(words_c - 1) * plane_c + (size_t)((m - 1) * ldc + n)) * 4;
    if (l > 0 && (mpg_overlaps(C, sc, A, sa) || mpg_overlaps(C, sc, B, sb)))
      return mpg_fail(c, MPG_ERR_ALIAS, "C overlaps an input");
  }
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_zero_u32(C, words_c, plane_c, m, n, ldc, c->stream); },
                  "zero C");
  if (st != MPG_OK || l == 0) return st;

  const int ca = (words_a + 3) / 4, cb = (words_b + 3) / 4;
  // a diagonal sums at most min(ca, cb) chunk products, each below l 2^256
  const int bits = 256 + bit_length(l) + bit_length(std::min(ca, cb)) + 1;
  const int N = crt_moduli_for_bits(bits);
  if (N == 0 || crt_words(N) == 0)
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "l = %lld too large for the moduli", (long long)l);
  const int64_t lp = round_up(l, crt_k_multiple()), mp = round_up(m, crt_tile_rows()),
                np = round_up(n, crt_tile_cols()), n4 = round_up(n, 4);
  const int64_t planeA = mp * lp, planeB = np * lp;
  void *res = nullptr, *out = nullptr;
  if ((st = mpg_workspace(c, 7, (size_t)N * (size_t)(ca * planeA + cb * planeB), &res)) != MPG_OK ||
      (st = mpg_workspace(c, 8, (size_t)N * (size_t)(m * n4) + 256 + sizeof(CrtTable), &out)) != MPG_OK)
    return st;
  int8_t* Ares = (int8_t*)res;
  int8_t* Bres = Ares + (size_t)ca * N * planeA;
  uint8_t* R = (uint8_t*)out;
  CrtTable* table = (CrtTable*)((char*)out + ((size_t)N * (size_t)(m * n4) + 255) / 256 * 256);
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipError_t r = launch_crt_table(N, table, c->stream);
    if (r != hipSuccess) return r;
    IntResidueArgs ra{A, words_a, plane_a, lda, m, l, mp, lp, ca, N, Ares};
    if ((r = launch_int_residues(ra, false, c->stream)) != hipSuccess) return r;
    IntResidueArgs rb{B, words_b, plane_b, ldb, n, l, np, lp, cb, N, Bres};
    return launch_int_residues(rb, true, c->stream);
  }, "chunk residue planes");
  if (st != MPG_OK) return st;
  for (int g = 0; g <= ca + cb - 2; ++g) {
    CrtGemmArgs ga{};
    ga.m = m;
    ga.n = n;
    ga.l_pad = lp;
    ga.A = Ares;
    ga.B = Bres;
    ga.planeA = planeA;
    ga.planeB = planeB;
    ga.R = R;
    ga.ldr = n4;
    ga.planeR = m * n4;
    ga.N = N;
    for (int j = 0; j < N; ++j) ga.mods[j] = kCrtModuli[j];
    ga.nseg = 0;
    for (int cc = std::max(0, g - cb + 1); cc <= std::min(g, ca - 1); ++cc) {
      ga.segA[ga.nseg] = (int64_t)cc * N * planeA;
      ga.segB[ga.nseg] = (int64_t)(g - cc) * N * planeB;
      ++ga.nseg;
    }
    if ((st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_crt_gemm(ga, c->stream); },
                         "INT8 MFMA chunk products")) != MPG_OK)
      return st;
    IntAccumArgs aa{R, n4, m * n4, N, table, C, words_c, 4 * g, plane_c, ldc, m, n};
    if ((st = mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_int_accumulate(aa, c->stream); },
                         "diagonal reconstruction")) != MPG_OK)
      return st;
  }
  c->last_moduli = N;
  return MPG_OK;
}
