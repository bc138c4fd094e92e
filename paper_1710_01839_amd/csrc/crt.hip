// Residue (Chinese remainder) form of the split product: the reconstruction
// table, the residue weights of the image words and the rebuild of the
// exact integer product from its residues.
#include <cmath>

#include "crt_internal.hpp"
#include "mp_arith.hpp"

namespace mpg {
namespace {

// ---------------------------------------------------------------------
// Table: one thread per modulus j forms M_j = prod_{i != j} p_i in 32-bit
// words, y_j = M_j^-1 mod p_j (extended Euclid on M_j mod p_j) and
// T_j = M_j y_j (< P, no reduction needed).  Thread 0 also writes P, P / 2
// and P as a double.
// ---------------------------------------------------------------------
__device__ int inverse_mod(int a, int p) {
  int r0 = p, r1 = a, t0 = 0, t1 = 1;
  while (r1 != 0) {
    const int q = r0 / r1;
    int tmp = r0 - q * r1;
    r0 = r1;
    r1 = tmp;
    tmp = t0 - q * t1;
    t0 = t1;
    t1 = tmp;
  }
  return t0 < 0 ? t0 + p : t0;  // r0 == 1 for coprime a, p
}

__device__ void mul_small(uint32_t (&x)[kCrtMaxWords], uint32_t k) {
  uint64_t carry = 0;
#pragma unroll
  for (int w = 0; w < kCrtMaxWords; ++w) {
    const uint64_t t = (uint64_t)x[w] * k + carry;
    x[w] = (uint32_t)t;
    carry = t >> 32;
  }
}

__global__ __launch_bounds__(64) void crt_table_kernel(int N, CrtTable* t, const CrtPlan* plan) {
  if (plan) {
    if (!plan->ok) return;
    N = plan->N;
  }
  const int j = threadIdx.x;
  __shared__ uint32_t Ms[64][kCrtMaxWords];
  __shared__ uint64_t colsum[kCrtMaxWords];
  uint32_t M[kCrtMaxWords] = {1};
  if (j < N) {
    const int pj = kCrtModuli[j];
    int mmod = 1;
    for (int i = 0; i < N; ++i)
      if (i != j) {
        mul_small(M, (uint32_t)kCrtModuli[i]);
        mmod = (int)((int64_t)mmod * (kCrtModuli[i] % pj) % pj);
      }
    mul_small(M, (uint32_t)inverse_mod(mmod, pj));
  } else {
    M[0] = 0;
  }
  for (int w = 0; w < kCrtMaxWords; ++w) {
    if (j < N) t->T[j][w] = M[w];
    Ms[j][w] = M[w];
  }
  // signed radix-256 digits of T[j] into the MFMA fragment table (zeros for
  // the moduli past N, up to the 64 the K range of one product holds)
  {
    int carry = 0;
    for (int b = 0; b < 4 * kCrtMaxWords; ++b) {
      const int v = carry + (int)((M[b / 4] >> (8 * (b % 4))) & 0xffu);
      carry = v >= 128 ? 1 : 0;
      t->frag[b / 16][16 * (j / 16) + b % 16][j % 16] = (int8_t)(v - 256 * carry);
    }
  }
  __syncthreads();
  // K0 = 128 sum_j T[j]: per-word sums (below 2^45) by one thread per word,
  // then one carry pass
  if (j < kCrtMaxWords) {
    uint64_t sw = 0;
    for (int i = 0; i < N; ++i) sw += Ms[i][j];
    colsum[j] = sw << 7;
  }
  __syncthreads();
  if (j == 0) {
    uint64_t c = 0;
    for (int w = 0; w < kCrtMaxWords; ++w) {
      const uint64_t sw = colsum[w] + c;
      t->K0[w] = (uint32_t)sw;
      c = sw >> 32;
    }
  }
  if (j == 0) {
    uint32_t P[kCrtMaxWords] = {1};
    for (int i = 0; i < N; ++i) mul_small(P, (uint32_t)kCrtModuli[i]);
    double pd = 0.0;
    for (int w = kCrtMaxWords - 1; w >= 0; --w) {
      t->P[w] = P[w];
      // P is even: halving shifts each word right, taking the next word's
      // lowest bit
      const uint32_t up = w + 1 < kCrtMaxWords ? P[w + 1] : 0u;
      t->half[w] = (P[w] >> 1) | (up << 31);
      pd += ldexp((double)P[w], 32 * w);
    }
    t->Pd = pd;
    t->N = N;
  }
}

// ---------------------------------------------------------------------
// Reconstruction of one output:
//   1. X' = sum_j r_j T_j < N 255 P < 2^(32 W) in W 32-bit words (formed by
//      INT8 MFMAs over the T_j's digits, see the kernel below);
//   2. q = floor(X' / P) from doubles (X' / P < 2^14, relative error far
//      below 2^-14; X' times the rounded 1 / P), then Y = X' - q P by words; a negative Y or Y >= P is
//      corrected by one addition or subtraction of P;
//   3. centre: Y >= P / 2 stands for Y - P (negative, magnitude P - Y);
//   4. the words of the magnitude, each scaled exactly by
//      2^(32 w + e_i + f_j + 4 - 16 S), are summed into a double-double
//      (all of them, from the top) or added to a quad-double result (the
//      top eight words; the dropped ones are below 2^-192 of the top one).
// ---------------------------------------------------------------------
// The signed value (magnitude words y, sign neg) times 2^scale as a
// double-double: every word from the top, each scaled exactly, summed by
// Fast2Sum (once hi is nonzero it is at least the leading word's value,
// above any later word, so each error term is exact).  No word is chosen
// at run time: a per-lane top word would need selects over all W words for
// each word taken.  From the fifth word on they lie below 2^-96 of the
// leading one.
template <int W>
__device__ __forceinline__ void crt_to_dd(const uint32_t (&y)[W], bool neg, int scale, double& hi,
                                          double& lo) {
  hi = 0.0;
  lo = 0.0;
#pragma unroll
  for (int w = W - 1; w >= 0; --w) {
    const double v = ldexp((double)y[w], 32 * w + scale);
    const double s = hi + v;
    lo += v - (s - hi);
    hi = s;
  }
  dd_renorm(hi, lo);
  if (neg) {
    hi = -hi;
    lo = -lo;
  }
}

// The same as a quad-double: the top eight words (256 bits), each added
// from the top into a four-term expansion by a TwoSum chain, renormalised.
template <int W>
__device__ __forceinline__ void crt_to_qd(const uint32_t (&y)[W], bool neg, int scale, double (&s)[4]) {
  int top = -1;
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (y[w] != 0) top = w;
  s[0] = s[1] = s[2] = s[3] = 0.0;
  if (top < 0) return;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int w = top - k;
    if (w >= 0) {
      double e = ldexp((double)y[w], 32 * w + scale);
      two_sum(s[0], e, s[0], e);
      two_sum(s[1], e, s[1], e);
      two_sum(s[2], e, s[2], e);
      s[3] += e;
    }
  }
  qd_finish(s);
  if (neg)
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = -s[q];
}

struct RecArgs {
  const uint8_t* R;
  int64_t ldr, planeR;
  int N;
  const CrtTable* t;
  const int* e;
  const int* f;
  int base;  // 4 - 16 S
  int64_t m, n;
  double* C[4];
  int64_t ldc;
  const CrtPlan* plan;  // when set: N and S from it
  int product;          // >= 0: nothing when plan->skip[product] is set
};

typedef int v4i_t __attribute__((ext_vector_type(4)));

// QD = false: C (hi, lo) := the value; QD = true: C (four limbs) += it.
// A workgroup takes 256 consecutive columns of a row at a time:
//   1. the residues of its 256 outputs for every modulus go into LDS as
//      signed bytes u_j = r_j - 128, one row of moduli per output (a thread
//      loads four moduli x four columns and transposes the 4 x 4 bytes);
//   2. X_b = sum_j u_j d_jb for every digit position b of the T[j] is one
//      INT8 MFMA per 16 positions and 16 outputs (|X_b| <= 49 128^2 < 2^20,
//      exact in INT32), and the four positions of word w combine into
//      V_w = sum_i X_{4w+i} 2^(8i) (exact in 64 bits);
//   3. a thread per output adds K0 = 128 sum_j T[j] (sum_j r_j T[j] =
//      sum_w V_w 2^(32 w) + K0) with a signed carry pass: the value is below
//      2^(32 W), so the W low words hold it and the positions from 4W up
//      cancel against the last carry; then as before (quotient by P,
//      centring, double-double or quad-double).
template <int W, bool QD>
__global__ __launch_bounds__(256, 4) void crt_reconstruct_kernel(RecArgs a) {
  constexpr int G = (4 * W + 15) / 16;  // MFMAs (groups of 16 digit positions) per 16 outputs
  constexpr int LS = 68;                // bytes per output in the residue tile (17 dwords: no bank conflicts)
  static_assert(G <= kCrtFragGroups, "digit groups");
  // the residue tile and the word sums share one buffer: every tile read
  // is done (a barrier) before the first word sum is written
  constexpr int SMEM = 256 * LS > 256 * W * 8 ? 256 * LS : 256 * W * 8;
  __shared__ __attribute__((aligned(16))) uint8_t smem[SMEM];
  uint8_t* const tile = smem;
  uint64_t* const vs = reinterpret_cast<uint64_t*>(smem);  // per output: W pairs of half sums
  if (a.plan) {
    if (!a.plan->ok || a.plan->W != W || (a.product >= 0 && a.plan->skip[a.product])) return;
    a.N = a.plan->N;
    a.base = 4 - 16 * a.plan->S;
  }
  const CrtTable& t = *a.t;
  const double rP = 1.0 / t.Pd;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  v4i_t fa[G];
#pragma unroll
  for (int g = 0; g < G; ++g) fa[g] = *reinterpret_cast<const v4i_t*>(&t.frag[g][lane][0]);
  const int nzg = (a.N + 3) / 4;
  const int c = threadIdx.x % 64, zq = threadIdx.x / 64;
  const int64_t jt = j0 + threadIdx.x;  // its output in step 3
  const int fjt = jt < a.n ? a.f[jt] : 0;
  // all of a thread's loads for a row (up to four groups of four moduli) go
  // out together, and those of its next row while this one is computed.
  // The address is a uniform base (row, plane, column block) plus a 32-bit
  // lane offset; lanes past the row's end (the last column block; ldr and
  // j0 are multiples of 4) read its last four columns instead, whose values
  // reach only outputs that are not stored.  Moduli past N read nothing.
  const uint32_t lane_off = (uint32_t)(4 * c < a.ldr - j0 - 4 ? 4 * c : a.ldr - j0 - 4);
  uint32_t d[4][4];
  auto load_row = [&](int64_t i) {
    const uint8_t* row = a.R + i * a.ldr + j0;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int zg = zq + 4 * it;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int z = 4 * zg + q;
        d[it][q] = z < a.N ? *reinterpret_cast<const uint32_t*>(row + (int64_t)z * a.planeR + lane_off) : 0u;
      }
    }
  };
  if (blockIdx.y < a.m) load_row(blockIdx.y);
  for (int64_t i = blockIdx.y; i < a.m; i += gridDim.y) {
    // 4 x 4 byte transpose (element q of word b: byte b of d[q]) by byte
    // permutes: pairs of rows interleaved, then pairs of those
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int zg = zq + 4 * it;
      if (zg >= nzg) break;
      const uint32_t d0 = d[it][0] ^ 0x80808080u, d1 = d[it][1] ^ 0x80808080u;
      const uint32_t d2 = d[it][2] ^ 0x80808080u, d3 = d[it][3] ^ 0x80808080u;
      const uint32_t lo01 = __builtin_amdgcn_perm(d1, d0, 0x05010400u);  // d0.0 d1.0 d0.1 d1.1
      const uint32_t hi01 = __builtin_amdgcn_perm(d1, d0, 0x07030602u);  // d0.2 d1.2 d0.3 d1.3
      const uint32_t lo23 = __builtin_amdgcn_perm(d3, d2, 0x05010400u);
      const uint32_t hi23 = __builtin_amdgcn_perm(d3, d2, 0x07030602u);
      const uint32_t x[4] = {__builtin_amdgcn_perm(lo23, lo01, 0x05040100u),
                             __builtin_amdgcn_perm(lo23, lo01, 0x07060302u),
                             __builtin_amdgcn_perm(hi23, hi01, 0x05040100u),
                             __builtin_amdgcn_perm(hi23, hi01, 0x07060302u)};
#pragma unroll
      for (int b = 0; b < 4; ++b) *reinterpret_cast<uint32_t*>(tile + (4 * c + b) * LS + 4 * zg) = x[b];
    }
    __syncthreads();
    if (i + gridDim.y < a.m) load_row(i + gridDim.y);
    v4i_t fb[4];
#pragma unroll
    for (int og = 0; og < 4; ++og) {
      const int o = 64 * wave + 16 * og + lane % 16;
      const uint32_t* src = reinterpret_cast<const uint32_t*>(tile + o * LS + 16 * (lane / 16));
#pragma unroll
      for (int q = 0; q < 4; ++q) fb[og][q] = (int)src[q];
    }
    __syncthreads();  // the tile is read; its bytes take the word sums
#pragma unroll
    for (int og = 0; og < 4; ++og) {
      const int o = 64 * wave + 16 * og + lane % 16;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const v4i_t x = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[g], fb[og], v4i_t{0, 0, 0, 0}, 0, 0, 0);
        const int wd = 4 * g + lane / 16;  // lane holds positions 4 wd .. 4 wd + 3 of output o
        if (wd < W) vs[o * W + wd] = crt_half_sums(x[0], x[1], x[2], x[3]);
      }
    }
    __syncthreads();
    if (jt < a.n) {
      uint64_t acc[W];
      crt_carry_halves<W>(reinterpret_cast<const int32_t*>(vs + threadIdx.x * W), t, acc);
      uint32_t y[W];
      const bool neg = crt_magnitude<W>(acc, t, rP, y);
      const int64_t o = i * a.ldc + jt;
      if constexpr (!QD) {
        double hi, lo;
        crt_to_dd<W>(y, neg, a.e[i] + fjt + a.base, hi, lo);
        a.C[0][o] = hi;
        a.C[1][o] = lo;
      } else {
        double v[4], cq[4] = {a.C[0][o], a.C[1][o], a.C[2][o], a.C[3][o]}, r[4];
        crt_to_qd<W>(y, neg, a.e[i] + fjt + a.base, v);
        qd_add(cq, v, r);
#pragma unroll
        for (int q = 0; q < 4; ++q) a.C[q][o] = r[q];
      }
    }
    __syncthreads();  // the tile and the word sums are refilled for the next row
  }
}

__global__ void crt_plan_kernel(const int* need, CrtModuliTable t, CrtPlan* plan) {
  if (threadIdx.x != 0) return;
  const int S = max(*need, 1);
  const int N = S <= kCrtMaxSlices ? t.N[S] : 0;
  plan->S = S;
  plan->N = N;
  plan->W = N > 0 ? t.W[S] : 0;
  plan->ok = N > 0 ? 1 : 0;
  for (int k = 0; k < 3; ++k) plan->skip[k] = 0;
  for (int p = 0; p < 4; ++p) plan->unused[p] = 0;
}

// Products of the quad-double form: k = 0: A_H B_H, 1: A_H B_L, 2: A_L B_H;
// one slice count, the largest exact count of the parts taking part.
__global__ void crt_plan_qd_kernel(const int* need, CrtModuliTable t, CrtPlan* plan) {
  if (threadIdx.x != 0) return;
  const int pa[3] = {0, 0, 1}, pb[3] = {2, 3, 2};
  int S = 0;
  int used[4] = {0, 0, 0, 0};
  for (int k = 0; k < 3; ++k) {
    const bool zero = need[pa[k]] == 0 || need[pb[k]] == 0;
    plan->skip[k] = zero ? 1 : 0;
    if (!zero) {
      S = max(S, max(need[pa[k]], need[pb[k]]));
      used[pa[k]] = used[pb[k]] = 1;
    }
  }
  for (int p = 0; p < 4; ++p) plan->unused[p] = used[p] ? 0 : 1;
  // nothing to multiply (C stays zero) counts as a plan that fits
  const int N = S == 0 ? 1 : S <= kCrtMaxSlices ? t.N[S] : 0;
  plan->S = max(S, 1);
  plan->N = N;
  plan->W = N == 0 ? 0 : S == 0 ? t.W[0] : t.W[S];
  plan->ok = N > 0 ? 1 : 0;
}

__global__ void residue_consts_kernel(int N, int S, CrtResidueConsts* rc, const CrtPlan* plan) {
  if (plan) {
    if (!plan->ok) return;
    N = plan->N;
    S = plan->S;
  }
  const int z = threadIdx.x;
  if (z >= N) return;
  const int p = kCrtModuli[z];
  for (int k = 0; k < kCrtImageWords; ++k) {
    // 256^max(S - 5k - 5, 0) mod p; words past the last digit weigh nothing
    int c = 0;
    if (kCrtDigitsPerWord * k < S) {
      c = 1 % p;
      for (int b = 0; b < 8 * max(S - kCrtDigitsPerWord * (k + 1), 0); ++b) c = (2 * c) % p;
    }
    rc->c[z][k] = (double)c;
  }
  rc->inv[z] = 1.0 / (double)p;
}

}  // namespace

int crt_product_bits(int S, int64_t l) {
  int lb = 0;
  while (lb < 62 && ((int64_t)1 << lb) < l) ++lb;  // bit length of l - 1 for l >= 1
  return 16 * S - 4 + lb + 1;
}

int crt_moduli_for_bits(int bits) {
  // product of the leading moduli in 32-bit words, compared with 2^bits
  uint32_t P[kCrtMaxWords + 1] = {1};
  for (int j = 0; j < kCrtMaxModuli; ++j) {
    uint64_t carry = 0;
    for (int w = 0; w <= kCrtMaxWords; ++w) {
      const uint64_t t = (uint64_t)P[w] * (uint32_t)kCrtModuli[j] + carry;
      P[w] = (uint32_t)t;
      carry = t >> 32;
    }
    int top = 0;
    for (int w = kCrtMaxWords; w >= 0; --w)
      if (P[w]) {
        top = 32 * w + 32 - __builtin_clz(P[w]);
        break;
      }
    // P > 2^bits: a longer bit length, or the same length bits + 1 and P
    // not a power of two (only the first modulus, 256, is one)
    if (top > bits + 1 || (top == bits + 1 && j > 0))
      return j + 1;
  }
  return 0;
}

int crt_words(int N) {
  if (N < 1 || N > kCrtMaxModuli) return 0;
  // bit length of N 255 P
  uint32_t P[kCrtMaxWords + 1] = {1};
  auto mul = [&](uint32_t k) {
    uint64_t carry = 0;
    for (int w = 0; w <= kCrtMaxWords; ++w) {
      const uint64_t t = (uint64_t)P[w] * k + carry;
      P[w] = (uint32_t)t;
      carry = t >> 32;
    }
  };
  for (int j = 0; j < N; ++j) mul((uint32_t)kCrtModuli[j]);
  mul((uint32_t)(255 * N));
  int bits = 0;
  for (int w = kCrtMaxWords; w >= 0; --w)
    if (P[w]) {
      bits = 32 * w + 32 - __builtin_clz(P[w]);
      break;
    }
  int W = (bits + 31) / 32;
  W = W < 4 ? 4 : (W + 1) / 2 * 2;  // built: 4, 6, 8, 10, 12
  return W <= kCrtMaxWords ? W : 0;
}

hipError_t launch_crt_table(int N, CrtTable* t, hipStream_t s, const CrtPlan* plan) {
  if (N < 1 || N > kCrtMaxModuli) return hipErrorInvalidValue;
  hipLaunchKernelGGL(crt_table_kernel, dim3(1), dim3(64), 0, s, N, t, plan);
  return hipGetLastError();
}

hipError_t launch_crt_plan(const int* need, const CrtModuliTable& t, CrtPlan* plan, hipStream_t s) {
  hipLaunchKernelGGL(crt_plan_kernel, dim3(1), dim3(64), 0, s, need, t, plan);
  return hipGetLastError();
}

hipError_t launch_crt_plan_qd(const int* need, const CrtModuliTable& t, CrtPlan* plan, hipStream_t s) {
  hipLaunchKernelGGL(crt_plan_qd_kernel, dim3(1), dim3(64), 0, s, need, t, plan);
  return hipGetLastError();
}

hipError_t launch_crt_residue_consts(int N, int S, CrtResidueConsts* rc, hipStream_t s,
                                     const CrtPlan* plan) {
  if (N < 1 || N > kCrtMaxModuli || S < 1 || S > kCrtMaxSlices) return hipErrorInvalidValue;
  hipLaunchKernelGGL(residue_consts_kernel, dim3(1), dim3(64), 0, s, N, S, rc, plan);
  return hipGetLastError();
}

hipError_t launch_crt_reconstruct(const uint8_t* R, int64_t ldr, int64_t planeR, int N,
                                  const CrtTable* t, const int* e, const int* f, int S, int64_t m,
                                  int64_t n, double* const* C, int limbs, int64_t ldc, hipStream_t s,
                                  const CrtPlan* plan, int product) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (ldr % 4 || ldr < n || (limbs != 2 && limbs != 4)) return hipErrorInvalidValue;
  RecArgs a{R, ldr, planeR, N, t, e, f, 4 - 16 * S, m, n, {C[0], C[1], nullptr, nullptr}, ldc, plan, product};
  if (limbs == 4) {
    a.C[2] = C[2];
    a.C[3] = C[3];
  }
  const int64_t gx = (n + 255) / 256;
  if (gx > 0x7fffffff) return hipErrorInvalidValue;
  // about 4096 workgroups, each walking several rows (its next row's loads
  // overlap the current row's arithmetic)
  const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(m, 65535), (4096 + gx - 1) / gx));
  const dim3 grid((unsigned)gx, (unsigned)gy);
#define MPG_CRT_REC(WW)                                                                        \
  case WW:                                                                                     \
    if (limbs == 2)                                                                            \
      hipLaunchKernelGGL((crt_reconstruct_kernel<WW, false>), grid, dim3(256), 0, s, a);       \
    else                                                                                       \
      hipLaunchKernelGGL((crt_reconstruct_kernel<WW, true>), grid, dim3(256), 0, s, a);        \
    break;
  const int Wmax = crt_words(N);
  if (Wmax == 0) return hipErrorInvalidValue;
  // with a plan: one launch per built word count up to Wmax (the plan's N
  // is at most N, so its W is one of them); all but the plan's return at
  // once
  for (int W = plan ? 4 : Wmax; W <= Wmax; W += 2) {
    switch (W) {
      MPG_CRT_REC(4)
      MPG_CRT_REC(6)
      MPG_CRT_REC(8)
      MPG_CRT_REC(10)
      MPG_CRT_REC(12)
      default:
        return hipErrorInvalidValue;
    }
    const hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
  }
#undef MPG_CRT_REC
  return hipSuccess;
}

}  // namespace mpg
