// Host side of the exact long-integer (fixed-point) matrix product.
#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

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

// ---------------------------------------------------------------------------
// Plan of one product: chunk width, Karatsuba depth over the chunk
// polynomials, the chunk sums to form, the leaf products and, for every
// diagonal of the full product, its signed leaf diagonals.
// ---------------------------------------------------------------------------

namespace {

struct Leaf {
  std::vector<int> u, v;  // coefficient chunk indices (-1: zero)
};

struct IntPlan {
  int cw = 4, depth = 0;
  int ca = 0, cb = 0, C = 0, L = 0;
  int N = 0;
  // chunk sums beyond the operands' own chunks: side 0 (A), 1 (B); entry k
  // becomes chunk index (own chunks + k)
  std::vector<std::vector<int>> sums[2];
  std::vector<Leaf> leaves;
  // leaf diagonals that have at least one nonzero pair, in order: (leaf, g)
  std::vector<std::pair<int, int>> leafdiags;
  // per diagonal G of the product: (leafdiag index, sign)
  std::vector<std::vector<std::pair<int, int>>> terms;
};

struct Contrib {
  int leaf, g, off, sign;
};

// Coefficient sets as sorted chunk lists; the map gives each multi-chunk set
// its chunk index.
struct SetTable {
  int own = 0;
  std::map<std::vector<int>, int> index;
  std::vector<std::vector<int>> sums;
  int get(const std::vector<int>& set) {
    if (set.empty()) return -1;
    if (set.size() == 1) return set[0];
    auto it = index.find(set);
    if (it != index.end()) return it->second;
    const int id = own + (int)sums.size();
    sums.push_back(set);
    index[set] = id;
    return id;
  }
};

std::vector<std::vector<int>> add_sets(const std::vector<std::vector<int>>& x, size_t lo, size_t hi, size_t h) {
  std::vector<std::vector<int>> out(h);
  for (size_t i = 0; i < h; ++i) {
    std::vector<int> s = x[lo + i];
    s.insert(s.end(), x[hi + i].begin(), x[hi + i].end());
    std::sort(s.begin(), s.end());
    out[i] = s;
  }
  return out;
}

// Karatsuba over coefficient-set polynomials u, v of equal length: returns
// the leaf diagonals and where they land (with sign) in u v.
std::vector<Contrib> karatsuba(const std::vector<std::vector<int>>& u, const std::vector<std::vector<int>>& v, int d,
                               SetTable (&st)[2], std::vector<Leaf>& leaves) {
  const size_t len = u.size();
  std::vector<Contrib> out;
  if (d == 0) {
    Leaf lf;
    for (size_t i = 0; i < len; ++i) {
      lf.u.push_back(st[0].get(u[i]));
      lf.v.push_back(st[1].get(v[i]));
    }
    const int id = (int)leaves.size();
    leaves.push_back(lf);
    for (int g = 0; g + 1 < 2 * (int)len; ++g) out.push_back({id, g, g, 1});
    return out;
  }
  const size_t h = len / 2;
  std::vector<std::vector<int>> u0(u.begin(), u.begin() + h), u1(u.begin() + h, u.end());
  std::vector<std::vector<int>> v0(v.begin(), v.begin() + h), v1(v.begin() + h, v.end());
  auto P0 = karatsuba(u0, v0, d - 1, st, leaves);
  auto P2 = karatsuba(u1, v1, d - 1, st, leaves);
  auto P1 = karatsuba(add_sets(u, 0, h, h), add_sets(v, 0, h, h), d - 1, st, leaves);
  const int H = (int)h;
  for (const auto& c : P0) {
    out.push_back({c.leaf, c.g, c.off, c.sign});
    out.push_back({c.leaf, c.g, c.off + H, -c.sign});
  }
  for (const auto& c : P2) {
    out.push_back({c.leaf, c.g, c.off + 2 * H, c.sign});
    out.push_back({c.leaf, c.g, c.off + H, -c.sign});
  }
  for (const auto& c : P1) out.push_back({c.leaf, c.g, c.off + H, c.sign});
  return out;
}

int bits_for(int cw, int ca, int cb, int64_t l) {
  // a diagonal sums at most min(ca, cb) chunk products, each below l 2^(64 cw)
  return 64 * cw + bit_length(l) + bit_length(std::min(ca, cb)) + 1;
}

// Builds the plan; returns MPG_OK or MPG_ERR_UNSUPPORTED with *why set.
int make_plan(int words_a, int words_b, int64_t l, int cw, int depth, IntPlan& P, const char** why) {
  P = IntPlan{};
  P.cw = cw;
  P.depth = depth;
  if (cw < 3 || cw > kIntMaxChunkWords || depth < 0 || depth > 3) {
    *why = "chunk width must be 3..5 words and the Karatsuba depth 0..3";
    return MPG_ERR_UNSUPPORTED;
  }
  P.ca = (words_a + cw - 1) / cw;
  P.cb = (words_b + cw - 1) / cw;
  P.N = crt_moduli_for_bits(bits_for(cw, P.ca, P.cb, l));
  if (P.N == 0 || crt_words(P.N) == 0) {
    *why = "the diagonal sums are too wide for the moduli (narrower chunks or a smaller l)";
    return MPG_ERR_UNSUPPORTED;
  }
  const int q = 1 << depth;
  P.C = (std::max(P.ca, P.cb) + q - 1) / q * q;
  P.L = P.C / q;
  if (P.L > kCrtMaxSegments) {
    *why = "more chunk pairs per diagonal than segments of one product (use a deeper split)";
    return MPG_ERR_UNSUPPORTED;
  }
  SetTable st[2];
  st[0].own = P.ca;
  st[1].own = P.cb;
  std::vector<std::vector<int>> u(P.C), v(P.C);
  for (int c = 0; c < P.C; ++c) {
    if (c < P.ca) u[c] = {c};
    if (c < P.cb) v[c] = {c};
  }
  const auto contribs = karatsuba(u, v, depth, st, P.leaves);
  for (int s2 = 0; s2 < 2; ++s2) {
    for (const auto& set : st[s2].sums)
      if ((int)set.size() > kIntMaxSumInputs) {
        *why = "Karatsuba sums of more than eight chunks";
        return MPG_ERR_UNSUPPORTED;
      }
    P.sums[s2] = st[s2].sums;
  }
  // leaf diagonals with a nonzero pair
  std::map<std::pair<int, int>, int> ld_index;
  for (int lf = 0; lf < (int)P.leaves.size(); ++lf)
    for (int g = 0; g + 1 < 2 * P.L; ++g) {
      bool any = false;
      for (int i = std::max(0, g - P.L + 1); i <= std::min(g, P.L - 1); ++i)
        if (P.leaves[lf].u[i] >= 0 && P.leaves[lf].v[g - i] >= 0) any = true;
      if (any) {
        ld_index[{lf, g}] = (int)P.leafdiags.size();
        P.leafdiags.push_back({lf, g});
      }
    }
  // diagonals of the product (those past ca + cb - 2 are zero and skipped)
  const int G = P.ca + P.cb - 1;
  std::vector<std::map<int, int>> acc(G);
  for (const auto& c : contribs) {
    if (c.off >= G) continue;
    auto it = ld_index.find({c.leaf, c.g});
    if (it == ld_index.end()) continue;
    acc[c.off][it->second] += c.sign;
  }
  P.terms.assign(G, {});
  for (int g = 0; g < G; ++g) {
    for (const auto& kv : acc[g])
      if (kv.second != 0) P.terms[g].push_back({kv.first, kv.second});
    if ((int)P.terms[g].size() > kIntMaxTerms) {
      *why = "too many leaf terms for one diagonal";
      return MPG_ERR_UNSUPPORTED;
    }
    for (const auto& t : P.terms[g])
      if (t.second < -1 || t.second > 1) {
        *why = "leaf term multiplicity above one";
        return MPG_ERR_UNSUPPORTED;
      }
  }
  return MPG_OK;
}

int check_int_args(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const uint32_t* A, int words_a, int64_t lda,
                   int64_t plane_a, const uint32_t* B, int words_b, int64_t ldb, int64_t plane_b, uint32_t* C,
                   int words_c, int64_t ldc, int64_t plane_c) {
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
  const size_t sa = ((size_t)(words_a - 1) * plane_a + (size_t)((m - 1) * lda + l)) * 4,
               sb = ((size_t)(words_b - 1) * plane_b + (size_t)((l - 1) * ldb + n)) * 4,
               sc = ((size_t)(words_c - 1) * plane_c + (size_t)((m - 1) * ldc + n)) * 4;
  if (l > 0 && (mpg_overlaps(C, sc, A, sa) || mpg_overlaps(C, sc, B, sb)))
    return mpg_fail(c, MPG_ERR_ALIAS, "C overlaps an input");
  return MPG_OK;
}

}  // namespace

// The product by a plan: residue planes of every chunk (and chunk sum), the
// INT8 products of the leaf diagonals, and the reconstruction of every
// diagonal of the product into C.
int mpg_int_run(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const uint32_t* A, int words_a, int64_t lda,
                int64_t plane_a, const uint32_t* B, int words_b, int64_t ldb, int64_t plane_b, uint32_t* C,
                int words_c, int64_t ldc, int64_t plane_c, int cw, int depth) {
  if (!c) return MPG_ERR_ARG;
  int st = check_int_args(c, m, n, l, A, words_a, lda, plane_a, B, words_b, ldb, plane_b, C, words_c, ldc, plane_c);
  if (st != MPG_OK || m == 0 || n == 0) return st;
  IntPlan P;
  const char* why = "";
  if (l > 0 && make_plan(words_a, words_b, l, cw, depth, P, &why) != MPG_OK)
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "long-integer product with %d-word chunks, Karatsuba depth %d: %s", cw,
                    depth, why);
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_zero_u32(C, words_c, plane_c, m, n, ldc, c->stream); },
                  "zero C");
  if (st != MPG_OK || l == 0) return st;
  const int N = P.N;
  const int64_t lp = round_up(l, crt_k_multiple()), mp = round_up(m, crt_tile_rows()),
                np = round_up(n, crt_tile_cols()), n4 = round_up(n, 4);
  const int64_t planeA = mp * lp, planeB = np * lp;
  const int chunksA = P.ca + (int)P.sums[0].size(), chunksB = P.cb + (int)P.sums[1].size();
  // one residue block per leaf diagonal, except that a plain product (no
  // split) reuses one block diagonal by diagonal
  const bool plain = P.depth == 0;
  const int64_t blocks = plain ? 1 : (int64_t)P.leafdiags.size();
  const size_t rblock = (size_t)N * (size_t)(m * n4);
  void *res = nullptr, *out = nullptr;
  if ((st = mpg_workspace(c, 7, (size_t)N * (size_t)(chunksA * planeA + chunksB * planeB), &res)) != MPG_OK ||
      (st = mpg_workspace(c, 8, (size_t)blocks * rblock + 256 + sizeof(CrtTable), &out)) != MPG_OK)
    return st;
  int8_t* Ares = (int8_t*)res;
  int8_t* Bres = Ares + (size_t)chunksA * N * planeA;
  uint8_t* R = (uint8_t*)out;
  CrtTable* table = (CrtTable*)((char*)out + ((size_t)blocks * rblock + 255) / 256 * 256);
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    hipError_t r = launch_crt_table(N, table, c->stream);
    if (r != hipSuccess) return r;
    IntResidueArgs ra{A, words_a, plane_a, lda, m, l, mp, lp, P.ca, N, Ares, P.cw};
    if ((r = launch_int_residues(ra, false, c->stream)) != hipSuccess) return r;
    IntResidueArgs rb{B, words_b, plane_b, ldb, n, l, np, lp, P.cb, N, Bres, P.cw};
    if ((r = launch_int_residues(rb, true, c->stream)) != hipSuccess) return r;
    for (int side = 0; side < 2; ++side)
      for (size_t k = 0; k < P.sums[side].size(); ++k) {
        IntSumArgs sa{};
        sa.base = side == 0 ? Ares : Bres;
        sa.plane = side == 0 ? planeA : planeB;
        sa.N = N;
        sa.out = (side == 0 ? P.ca : P.cb) + (int)k;
        sa.nin = (int)P.sums[side][k].size();
        for (int q = 0; q < sa.nin; ++q) sa.in[q] = P.sums[side][k][q];
        if ((r = launch_int_sum(sa, c->stream)) != hipSuccess) return r;
      }
    return hipSuccess;
  }, "chunk residue planes");
  if (st != MPG_OK) return st;
  auto product = [&](int ld, uint8_t* Rout) {
    const Leaf& lf = P.leaves[P.leafdiags[ld].first];
    const int g = P.leafdiags[ld].second;
    CrtGemmArgs ga{};
    ga.product = -1;
    ga.m = m;
    ga.n = n;
    ga.l_pad = lp;
    ga.A = Ares;
    ga.B = Bres;
    ga.planeA = planeA;
    ga.planeB = planeB;
    ga.R = Rout;
    ga.ldr = n4;
    ga.planeR = m * n4;
    ga.N = N;
    for (int j = 0; j < N; ++j) ga.mods[j] = kCrtModuli[j];
    ga.nseg = 0;
    for (int i = std::max(0, g - P.L + 1); i <= std::min(g, P.L - 1); ++i) {
      const int ia = lf.u[i], ib = lf.v[g - i];
      if (ia < 0 || ib < 0) continue;
      ga.segA[ga.nseg] = (int64_t)ia * N * planeA;
      ga.segB[ga.nseg] = (int64_t)ib * N * planeB;
      ++ga.nseg;
    }
    return mpg_launch(c, MPG_KCLASS_GEMM, [&] { return launch_crt_gemm(ga, c->stream); },
                      "INT8 MFMA chunk products");
  };
  auto accumulate = [&](int G, const std::vector<std::pair<int, int>>& terms, const uint8_t* Rbase) {
    IntAccumArgs aa{};
    aa.R = Rbase;
    aa.ldr = n4;
    aa.planeR = m * n4;
    aa.N = N;
    aa.t = table;
    aa.C = C;
    aa.words_c = words_c;
    aa.word_off = P.cw * G;
    aa.pstride = plane_c;
    aa.ldc = ldc;
    aa.m = m;
    aa.n = n;
    aa.nterms = (int)terms.size();
    for (int q = 0; q < aa.nterms; ++q) {
      aa.term_off[q] = plain ? 0 : (int64_t)terms[q].first * (int64_t)rblock;
      aa.term_sign[q] = terms[q].second;
    }
    return mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_int_accumulate(aa, c->stream); },
                      "diagonal reconstruction");
  };
  if (plain) {
    // diagonal by diagonal through one residue block
    for (int G = 0; G < (int)P.terms.size(); ++G) {
      if (P.terms[G].empty()) continue;
      if ((st = product(P.terms[G][0].first, R)) != MPG_OK) return st;
      if ((st = accumulate(G, P.terms[G], R)) != MPG_OK) return st;
    }
  } else {
    for (int ld = 0; ld < (int)P.leafdiags.size(); ++ld)
      if ((st = product(ld, R + (size_t)ld * rblock)) != MPG_OK) return st;
    for (int G = 0; G < (int)P.terms.size(); ++G)
      if (!P.terms[G].empty() && (st = accumulate(G, P.terms[G], R)) != MPG_OK) return st;
  }
  c->last_moduli = N;
  return MPG_OK;
}

// INT8 products per product of this plan (chunk pairs over all leaf
// diagonals times moduli), host only.
int64_t mpg_int_plan_products(int words_a, int words_b, int64_t l, int cw, int depth) {
  IntPlan P;
  const char* why = "";
  if (make_plan(words_a, words_b, l, cw, depth, P, &why) != MPG_OK) return 0;
  int64_t pairs = 0;
  for (const auto& ld : P.leafdiags) {
    const Leaf& lf = P.leaves[ld.first];
    for (int i = std::max(0, ld.second - P.L + 1); i <= std::min(ld.second, P.L - 1); ++i)
      if (lf.u[i] >= 0 && lf.v[ld.second - i] >= 0) ++pairs;
  }
  return pairs * P.N;
}

// Moduli of a plan (0 if it does not fit), host only.
int mpg_int_plan_moduli(int words_a, int words_b, int64_t l, int cw, int depth) {
  IntPlan P;
  const char* why = "";
  return make_plan(words_a, words_b, l, cw, depth, P, &why) == MPG_OK ? P.N : 0;
}

extern "C" int mpg_int_gemm_ex(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const uint32_t* A, int words_a,
                               int64_t lda, int64_t plane_a, const uint32_t* B, int words_b, int64_t ldb,
                               int64_t plane_b, uint32_t* C, int words_c, int64_t ldc, int64_t plane_c,
                               const mpg_int_algo* algo) {
  if (!c) return MPG_ERR_ARG;
  int cw = 4, depth = 0;
  mpg_int_algo t{};
  if (algo) {
    cw = algo->chunk_words;
    depth = algo->karatsuba_depth;
  } else if (mpg_int_table_lookup(c, m, n, l, words_a, words_b, &t)) {
    cw = t.chunk_words;
    depth = t.karatsuba_depth;
  }
  return mpg_int_run(c, m, n, l, A, words_a, lda, plane_a, B, words_b, ldb, plane_b, C, words_c, ldc, plane_c, cw,
                     depth);
}

extern "C" int mpg_int_gemm(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const uint32_t* A, int words_a,
                            int64_t lda, int64_t plane_a, const uint32_t* B, int words_b, int64_t ldb,
                            int64_t plane_b, uint32_t* C, int words_c, int64_t ldc, int64_t plane_c) {
  return mpg_int_gemm_ex(c, m, n, l, A, words_a, lda, plane_a, B, words_b, ldb, plane_b, C, words_c, ldc, plane_c,
                         nullptr);
}
