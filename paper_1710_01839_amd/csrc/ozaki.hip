// Split-precision double-double product on INT8 MFMA (gfx950).
//
// FP64 inputs are scaled per row of A (2^-(e_i + 2)) and per column of B
// (2^-(f_j + 2)) into (-1/4, 1/4) and cut into S exact radix-256 digit
// planes of signed bytes (digits by truncation toward zero, then a carry
// from the least significant digit up that brings every digit into
// [-128, 127]).  Products of digit planes run on v_mfma_i32_16x16x64_i8
// with exact INT32 sums; the sums of one diagonal g = s + t of the (s, t)
// pair grid share the weight 2^(e_i + f_j + 4 - 8g) and are added, scaled
// exactly, into double-double accumulators.
#include <climits>

#include "mp_arith.hpp"
#include "ozaki_internal.hpp"
#include "crt_internal.hpp"

namespace mpg {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// The hardware deals workgroups round-robin over the 8 XCDs; remap the
// linear id so consecutive logical tiles run on one XCD.
__device__ __forceinline__ int xcd_remap(int w, int total) {
  constexpr int X = 8;
  const int q = total / X, r = total % X;
  const int xcd = w % X, local = w / X;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// ---------------------------------------------------------------------
// exponent scans
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void fill_int_kernel(int* p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

// Exponents of the leading bit (ilogb) and of the lowest set bit of a
// finite x != 0, read from its bit pattern (subnormals included).
__device__ __forceinline__ void bit_range(double x, int& top, int& low) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x) & 0x7FFFFFFFFFFFFFFFull;
  const int be = (int)(b >> 52);
  const unsigned long long mant = b & 0x000FFFFFFFFFFFFFull;
  if (be != 0) {
    top = be - 1023;
    low = top - 52 + __builtin_ctzll(mant | 0x0010000000000000ull);
  } else {
    top = 63 - __builtin_clzll(mant) - 1074;
    low = __builtin_ctzll(mant) - 1074;
  }
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// Radix-256 digits that hold every element of a line exactly once it is
// scaled by 2^-(e + 2): ceil((e + 2 - lowest set bit) / 8).
__device__ __forceinline__ int line_digits(int e, int low) {
  const int d = e + 2 - low;
  return d > 0 ? (d + 7) / 8 : 0;
}

// Rows of X (R x K): one workgroup per row writes e[r] = 1 + max ilogb over
// the row (max |x| < 2^e; 0 for an all-zero row) and, when `need` is given,
// raises *need to the row's digit count.  One pass over X.
// With Xlo (need only) the lowest set bit of the lo limbs counts too; the
// scale comes from X alone.
__global__ __launch_bounds__(256) void row_scan_kernel(const double* X, const double* Xlo, int64_t K,
                                                       int64_t ld, int* e, int* need) {
  __shared__ int s_top[4], s_low[4];
  const int64_t r = blockIdx.x;
  int top = INT_MIN, low = INT_MAX;
  // pass 0 reads X (scale and lowest bit), pass 1 Xlo (lowest bit); eight
  // loads of a thread are issued before any is used (clamped indices, the
  // values past K masked to zero)
  constexpr int V = 8;
  for (int pass = 0; pass < (Xlo ? 2 : 1); ++pass) {
    const double* row = (pass ? Xlo : X) + r * ld;
    for (int64_t k0 = threadIdx.x; k0 < K; k0 += V * 256) {
      double v[V];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int64_t k = k0 + 256 * j;
        v[j] = row[k < K ? k : K - 1];
      }
#pragma unroll
      for (int j = 0; j < V; ++j) {
        if (k0 + 256 * j < K && v[j] != 0.0) {
          int t, lo;
          bit_range(v[j], t, lo);
          if (pass == 0) top = max(top, t);
          low = min(low, lo);
        }
      }
    }
  }
  top = wave_max_int(top);
  low = wave_min_int(low);
  if ((threadIdx.x & 63) == 0) {
    s_top[threadIdx.x >> 6] = top;
    s_low[threadIdx.x >> 6] = low;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      top = max(top, s_top[w]);
      low = min(low, s_low[w]);
    }
    const int er = top == INT_MIN ? 0 : top + 1;
    e[r] = er;
    if (need && top != INT_MIN) {
      const int d = line_digits(er, low);
      if (d > 0) atomicMax(need, d);
    }
  }
}

// Columns of X (R x K): a workgroup covers 64 columns (each row's 64
// doubles are one coalesced read) and 64 rows, 4 threads per column; the
// per-workgroup maxima / minima go to top[c] / low[c] (initialised to
// INT_MIN / INT_MAX) with one atomic each.
constexpr int kColScanRows = 64;
__global__ __launch_bounds__(256) void col_scan_kernel(const double* X, const double* Xlo, int64_t R,
                                                       int64_t K, int64_t ld, int* top, int* low) {
  __shared__ int s_t[4][64], s_l[4][64];
  const int tc = threadIdx.x & 63, tg = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + tc;
  const int64_t r0 = (int64_t)blockIdx.y * kColScanRows;
  int t = INT_MIN, lo = INT_MAX;
  // pass 0 reads X (scale and lowest bit), pass 1 Xlo (lowest bit); the
  // thread's rows are loaded eight at a time before any is used (clamped
  // row indices, rows past R masked)
  if (c < K) {
    for (int pass = 0; pass < (Xlo ? 2 : 1); ++pass) {
      const double* col = (pass ? Xlo : X) + c;
      for (int i0 = tg; i0 < kColScanRows; i0 += 8 * 4) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t r = r0 + i0 + 4 * j;
          v[j] = col[(r < R ? r : R - 1) * ld];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (r0 + i0 + 4 * j < R && v[j] != 0.0) {
            int a, b;
            bit_range(v[j], a, b);
            if (pass == 0) t = max(t, a);
            lo = min(lo, b);
          }
        }
      }
    }
  }
  s_t[tg][tc] = t;
  s_l[tg][tc] = lo;
  __syncthreads();
  if (tg == 0 && c < K) {
#pragma unroll
    for (int g = 1; g < 4; ++g) {
      t = max(t, s_t[g][tc]);
      lo = min(lo, s_l[g][tc]);
    }
    if (t != INT_MIN) {
      atomicMax(&top[c], t);
      if (low) atomicMin(&low[c], lo);
    }
  }
}

// top[c] -> e[c] = top + 1 in place (0 for an all-zero column); raises
// *need (when given) to the columns' digit count, one atomic per wave.
__global__ __launch_bounds__(256) void col_finish_kernel(int* top_e, const int* low, int64_t K,
                                                         int* need) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int d = 0;
  if (c < K) {
    const int t = top_e[c];
    const int er = t == INT_MIN ? 0 : t + 1;
    top_e[c] = er;
    if (need && t != INT_MIN) d = line_digits(er, low[c]);
  }
  d = wave_max_int(d);
  if (need && (threadIdx.x & 63) == 0 && d > 0) atomicMax(need, d);
}

// ---------------------------------------------------------------------
// digit slicing
// ---------------------------------------------------------------------
// One digit of the remainder r = (y, yl): t = trunc(256 r) toward zero, in
// [-255, 255], and r becomes 256 r - t (same sign as the element, |r| < 1).
// FP64: multiplying by 256 and removing the integer part are exact.  DD: r
// is a renormalised pair, so 256 r is one too; its truncation is that of
// the leading part unless the leading part is an integer and the trailing
// part pulls toward zero (then one less in magnitude); the new remainder
// is renormalised by an exact TwoSum.
template <bool DD>
__device__ __forceinline__ double digit_value(double& y, double& yl) {
  const double sh = y * 256.0;
  if (!DD) {
    const double t = trunc(sh);
    y = sh - t;
    return t;
  }
  const double sl = yl * 256.0;
  double t = trunc(sh);
  if (t == sh && sh != 0.0 && sl != 0.0 && ((sl < 0.0) != (sh < 0.0))) t -= sh > 0.0 ? 1.0 : -1.0;
  two_sum(sh - t, sl, y, yl);
  return t;
}
template <bool DD>
__device__ __forceinline__ int digit_step(double& y, double& yl) {
  return (int)digit_value<DD>(y, yl);
}

// The carry that turns truncated digits into signed bytes, on one 8-byte
// word of a plane (8 elements): `word` holds the digits t mod 256 (their
// signs are the elements', bit q of `neg`), `c` the carries from the plane
// below (in: carries into this plane; out: carries into the plane above).
// The top plane (top = true) takes the carry and keeps no new one.
__device__ __forceinline__ unsigned long long carry_word(unsigned long long word, unsigned neg, int (&c)[8],
                                                         bool top) {
  unsigned long long o = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int b = (int)((word >> (8 * q)) & 0xFF);
    int u = ((neg >> q) & 1) && b != 0 ? b - 256 : b;
    u += c[q];
    if (!top) {
      c[q] = (u >= 128) - (u < -128);
      u -= 256 * c[q];
    }
    o |= (unsigned long long)(uint8_t)(int8_t)u << (8 * q);
  }
  return o;
}

// Rows of X (R x K) -> planes out[s][r][k] (r < Rp, k < Kp, zero padded).
// Each thread handles 8 consecutive k of one row: it writes the truncated
// digits of each plane (8 bytes per plane, top plane first), then reads
// its words back from the lowest plane up and applies the carry.  With DD
// the value is X + Xlo, split as one exact value.
template <bool DD>
__global__ __launch_bounds__(256) void split_rows_kernel(const double* X, const double* Xlo, int64_t R,
                                                         int64_t K, int64_t ld, const int* e, int S,
                                                         int8_t* out, int64_t ld_out,
                                                         int64_t plane, int64_t Rp, int64_t Kp) {
  const int64_t per_row = Kp / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= Rp * per_row) return;
  const int64_t r = idx / per_row, k0 = (idx % per_row) * 8;
  double y[8], yl[8];
  const int er = r < R ? e[r] : 0;
  unsigned neg = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t k = k0 + q;
    const bool ok = r < R && k < K;
    y[q] = ldexp(ok ? X[r * ld + k] : 0.0, -(er + 2));
    yl[q] = 0.0;
    if (DD) two_sum(y[q], ldexp(ok ? Xlo[r * ld + k] : 0.0, -(er + 2)), y[q], yl[q]);
    neg |= (unsigned)(y[q] < 0.0) << q;
  }
  unsigned long long* w = reinterpret_cast<unsigned long long*>(out + r * ld_out + k0);
  for (int s = 0; s < S; ++s) {
    unsigned long long word = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      word |= (unsigned long long)(uint8_t)digit_step<DD>(y[q], yl[q]) << (8 * q);
    w[s * plane / 8] = word;
  }
  int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = S - 1; s >= 0; --s) w[s * plane / 8] = carry_word(w[s * plane / 8], neg, c, s == 0);
}

// Residues of the 8 images in `words` (the first NW words nonzero) modulo
// the N leading moduli, one 8-byte store per plane (planes `plane` bytes
// apart).  The first two moduli (256, 255) need their residues centred to
// fit a signed byte; the odd ones after them do not.  The odd moduli go in
// groups of four whose constants are read together, so one wait on the
// uniform loads serves four moduli.
template <int NW>
__device__ __forceinline__ void crt_store_residues(const double (&words)[kCrtImageWords][8],
                                                   const CrtResidueConsts* __restrict__ rc, int N,
                                                   int8_t* __restrict__ out, int64_t plane) {
  for (int z = 0; z < min(N, 2); ++z)
    *reinterpret_cast<uint64_t*>(out + (int64_t)z * plane) =
        crt_residues8<NW, true>(words, rc->c[z], kCrtModuli[z], rc->inv[z]);
  constexpr int G = 4;
  for (int z = 2; z < N; z += G) {
    double c[G][NW], inv[G];
    int p[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int zj = min(z + j, N - 1);
#pragma unroll
      for (int w = 0; w < NW; ++w) c[j][w] = rc->c[zj][w];
      inv[j] = rc->inv[zj];
      p[j] = kCrtModuli[zj];
    }
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (z + j < N)  // uniform
        *reinterpret_cast<uint64_t*>(out + (int64_t)(z + j) * plane) =
            crt_residues8<NW, false>(words, c[j], p[j], inv[j]);
  }
}

// Residue planes of the residue form straight from the operand: one thread
// per 8 consecutive k of a row, as in split_rows_kernel, but the image (the
// truncated digits before any carry: the carry does not change their
// weighted sum) is cut into 40-bit words of five digits in registers and
// only the residues are written, one byte per element and modulus.
//
// COLS: the rows of the plane are the columns of X (X is K x R, element
// (r, k) at X[k ld + r]), read in place instead of through a transposed
// copy: for each k a wavefront's lanes read 64 contiguous bytes of a row of
// X.
constexpr int kCrtRowsTiledModuli = 24;
template <bool DD, bool COLS>
__global__ __launch_bounds__(256) void crt_rows_kernel(const double* X, const double* Xlo, int64_t R,
                                                       int64_t K, int64_t ld, const int* e, int S, int N,
                                                       int8_t* __restrict__ out, int64_t Rp, int64_t Kp,
                                                       const CrtResidueConsts* __restrict__ rc,
                                                       const CrtPlan* plan, int part) {
  if (plan) {
    if (!plan->ok || (part >= 0 && plan->unused[part])) return;
    S = plan->S;
    N = plan->N;
  }
  const int64_t per_row = Kp / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= Rp * per_row) return;
  int64_t r, k0;
  // a wavefront takes 8 rows x 64 k of the plane (Rp % 16 == 0 and
  // Kp % 64 == 0: whole groups), so its 8-byte stores of one plane fill 512
  // contiguous bytes, half of a 16 x 64 block.  Rows of X with few moduli
  // (few stores per load) keep one row x 512 k per wavefront, whose loads
  // span fewer rows: the 8 x 64 form was 12% faster with 44 moduli and 39%
  // slower with 16.
  const int64_t t = idx / 64, lane = idx % 64, row_groups = Rp / 8;
  if (!COLS && N < kCrtRowsTiledModuli) {
    r = idx / per_row;
    k0 = (idx % per_row) * 8;
  } else if (!COLS) {
    // lanes 8i .. 8i + 7: one row, 64 consecutive k
    r = (t % row_groups) * 8 + lane / 8;
    k0 = ((t / row_groups) * 8 + lane % 8) * 8;
  } else {
    // lanes i, i + 8, ..: 8 consecutive columns of X, one 64-byte segment of
    // a row of X for each k
    r = (t % row_groups) * 8 + lane % 8;
    k0 = ((t / row_groups) * 8 + lane / 8) * 8;
  }
  // y: the scaled leading part; yl: the scaled trailing part (DD), each cut
  // into digits on its own (a pair is not renormalised)
  double y[8], yl[8];
  unsigned neg = 0;  // bit q: the element hi + lo is negative (the sign of its rounded sum)
  const int er = r < R ? e[r] : 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t k = k0 + q;
    const bool ok = r < R && k < K;
    const int64_t at = COLS ? k * ld + r : r * ld + k;
    const double hi = ok ? X[at] : 0.0;
    y[q] = ldexp(hi, -(er + 2));
    yl[q] = 0.0;
    if (DD) {
      const double lo = ok ? Xlo[at] : 0.0;
      yl[q] = ldexp(lo, -(er + 2));
      neg |= (unsigned)(hi + lo < 0.0) << q;
    }
  }
  // word k holds digits 5k .. 5k + n - 1 (n = min(5, S - 5k)) folded by
  // Horner's rule, which is trunc(y 2^(8n)) of the remainder left by the
  // words before it: truncations toward zero of a same-signed remainder
  // compose, and scaling by 2^(8n), the integer part and the new remainder
  // are all exact, so a word costs one step instead of n digit steps.
  // DD: the two parts are cut on their own (|word| < 2^41; canonical pairs,
  // |lo| <= ulp(hi) / 2, keep both parts below 1 after the row scale), so the
  // words hold trunc(hi 2^s) + trunc(lo 2^s), s = 8S - 2 - e.
  double words[kCrtImageWords][8];
#pragma unroll
  for (int k = 0; k < kCrtImageWords; ++k) {
    const int n = min(kCrtDigitsPerWord, S - kCrtDigitsPerWord * k);
    const double scale = n > 0 ? __builtin_amdgcn_ldexp(1.0, 8 * n) : 0.0;  // uniform
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (n > 0) {  // uniform
        const double a = y[q] * scale;
        const double t = trunc(a);
        y[q] = a - t;
        words[k][q] = t;
        if (DD) {
          const double al = yl[q] * scale;
          const double tl = trunc(al);
          yl[q] = al - tl;
          words[k][q] += tl;
        }
      } else {
        words[k][q] = 0.0;
      }
    }
  }
  // DD: with I = trunc(hi 2^s) + trunc(lo 2^s) (the words) and the two
  // remainders rh, rl (|rh|, |rl| < 1), (hi + lo) 2^s = I + F, F = rh + rl,
  // so trunc((hi + lo) 2^s) = I + delta, delta = floor(F) when hi + lo >= 0
  // and ceil(F) when it is negative (|delta| <= 2), decided on the exact
  // sum f + g = F
  // delta goes into the word of the last digit, whose weight is 1 (|word|
  // stays below 2^41 + 2); the word is chosen by a uniform branch
  if (DD) {
    const int klast = (S - 1) / kCrtDigitsPerWord;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double f, g;
      two_sum(y[q], yl[q], f, g);
      const bool nq = (neg >> q) & 1;
      double t = nq ? ceil(f) : floor(f);
      if (t == f) t += nq ? (g > 0.0 ? 1.0 : 0.0) : (g < 0.0 ? -1.0 : 0.0);
#pragma unroll
      for (int k = 0; k < kCrtImageWords; ++k)
        if (k == klast) words[k][q] += t;
    }
  }
  // images of up to 10 (15) digits fill two (three) words: uniform branch
  int8_t* const o = out + crt_plane_offset(r, k0, Kp);
  if (S <= 2 * kCrtDigitsPerWord)
    crt_store_residues<2>(words, rc, N, o, Rp * Kp);
  else if (S <= 3 * kCrtDigitsPerWord)
    crt_store_residues<3>(words, rc, N, o, Rp * Kp);
  else
    crt_store_residues<kCrtImageWords>(words, rc, N, o, Rp * Kp);
}

// Columns of X (K x C, row-major) -> planes out[s][c][k] (transposed, c < Cp,
// k < Kp, zero padded).  A 32 (k) x 64 (c) tile is read coalesced along c
// (each thread keeps 8 remainders in registers); for each digit plane the
// digits pass through LDS and are written back as 8-byte runs along k; the
// thread that wrote a run applies the carry to it afterwards, lowest plane
// first (the elements' signs pass through LDS once).  DD as in
// split_rows_kernel.
constexpr int kColTileK = 32;
constexpr int kMaxSlices = 40;
template <bool DD>
__global__ __launch_bounds__(256) void split_cols_kernel(const double* X, const double* Xlo, int64_t K,
                                                         int64_t C, int64_t ld, const int* f, int S,
                                                         int8_t* out, int64_t ld_out,
                                                         int64_t plane, int64_t Cp, int64_t Kp) {
  __shared__ uint8_t dig[64][kColTileK + 8];
  __shared__ uint8_t negs[64][kColTileK + 8];
  const int64_t c0 = (int64_t)blockIdx.x * 64, k0 = (int64_t)blockIdx.y * kColTileK;
  const int tc = threadIdx.x % 64, tk = threadIdx.x / 64;  // 64 columns x 4
  const int64_t c = c0 + tc;
  const int fc = c < C ? f[c] : 0;
  double y[kColTileK / 4], yl[kColTileK / 4];
#pragma unroll
  for (int q = 0; q < kColTileK / 4; ++q) {
    const int64_t k = k0 + tk + 4 * q;
    const bool ok = c < C && k < K;
    y[q] = ldexp(ok ? X[k * ld + c] : 0.0, -(fc + 2));
    yl[q] = 0.0;
    if (DD) two_sum(y[q], ldexp(ok ? Xlo[k * ld + c] : 0.0, -(fc + 2)), y[q], yl[q]);
    negs[tc][tk + 4 * q] = y[q] < 0.0;
  }
  const int wc = threadIdx.x / 4, wk = (threadIdx.x % 4) * 8;
  const int64_t cc = c0 + wc;
  unsigned long long* w = reinterpret_cast<unsigned long long*>(out + cc * ld_out + k0 + wk);
  for (int s = 0; s < S; ++s) {
#pragma unroll
    for (int q = 0; q < kColTileK / 4; ++q) dig[tc][tk + 4 * q] = (uint8_t)digit_step<DD>(y[q], yl[q]);
    __syncthreads();
    unsigned long long word = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) word |= (unsigned long long)dig[wc][wk + q] << (8 * q);
    if (cc < Cp) w[s * plane / 8] = word;
    __syncthreads();
  }
  if (cc < Cp) {
    unsigned neg = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) neg |= (unsigned)negs[wc][wk + q] << q;
    int cy[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = S - 1; s >= 0; --s) w[s * plane / 8] = carry_word(w[s * plane / 8], neg, cy, s == 0);
  }
}

// ---------------------------------------------------------------------
// INT8 MFMA product with diagonal grouping, general form (used above
// kOzBandMaxS slices).
//
// Workgroup: 256 threads, C tile 64 x 64; wave w owns the 32 x 32 sub-tile
// (32 (w / 2), 32 (w % 2)) as 2 x 2 blocks of 16 x 16 MFMA outputs.  The
// (s, t) pair grid is walked in SB x SB blocks, from the smallest weights
// to the largest; for one block the K loop stages SB digit planes of A and
// SB of B (64 rows x 64 k bytes each, rows padded to 80 bytes so the
// 16-byte fragment reads of 8 lanes hit distinct banks) in LDS,
// double-buffered, and every kept pair adds into the INT32 accumulator of
// its diagonal (2 SB - 1 live diagonals).  At the end of the block each
// diagonal sum is converted to FP64 (exact), scaled by 2^(e_i + f_j + 4 - 8g)
// (exact) and added to the entry's double-double accumulator.
//
// MFMA operand layout (16 x 16 x 64, i8): lane l supplies row (l % 16) of
// A and column (l % 16) of B with the 16 bytes k = 16 (l / 16) .. +15 of
// the 64-wide K step (any fixed k order is exact as long as A and B use the
// same one); lane l receives D[4 (l / 16) + i][l % 16], i = 0..3.
// ---------------------------------------------------------------------
constexpr int kOzTile = 64;
constexpr int kOzK = 64;
constexpr int kOzRow = 80;  // padded LDS row in bytes

template <int SB>
__global__ __launch_bounds__(256, 1) void ozaki_mfma_kernel(OzakiGemmArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t sA[2][SB][kOzTile * kOzRow];
  __shared__ __attribute__((aligned(16))) int8_t sB[2][SB][kOzTile * kOzRow];

  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wr = wave / 2, wc = wave % 2;
  const int tiles_n = (int)((a.n + kOzTile - 1) / kOzTile);
  const int64_t m0 = (int64_t)(blockIdx.x / tiles_n) * kOzTile;
  const int64_t n0 = (int64_t)(blockIdx.x % tiles_n) * kOzTile;

  // per-lane output coordinates and their scale exponents
  int erow[2][4], fcol[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = m0 + 32 * wr + 16 * rb + 4 * (lane / 16) + i;
      erow[rb][i] = r < a.m ? a.e[r] : 0;
    }
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int64_t c = n0 + 32 * wc + 16 * cb + lane % 16;
    fcol[cb] = c < a.n ? a.f[c] : 0;
  }

  double hi[2][2][4], lo[2][2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) hi[rb][cb][i] = lo[rb][cb][i] = 0.0;

  // staging: thread -> (row = tid / 4, 16-byte chunk = tid % 4) of a 64 x 64 tile
  const int ld_row = tid / 4, ld_chunk = (tid % 4) * 16;
  const int nblk = (a.S + SB - 1) / SB;
  const int numK = (int)(a.l_pad / kOzK);

  // blocks of the pair grid in order of decreasing s0 + t0 (smallest weights first)
  for (int diag = 2 * (nblk - 1); diag >= 0; --diag) {
    for (int bs = 0; bs < nblk; ++bs) {
      const int bt = diag - bs;
      if (bt < 0 || bt >= nblk) continue;
      const int s0 = bs * SB, t0 = bt * SB;  // 0-based first slice of the block
      // any kept pair in this block?  (1-based s + t <= S + 1 for the triangle)
      if (a.triangle && (s0 + 1) + (t0 + 1) > a.S + 1) continue;
      const int ns = min(SB, a.S - s0), nt = min(SB, a.S - t0);

      v4i acc[2 * SB - 1][2][2];
#pragma unroll
      for (int g = 0; g < 2 * SB - 1; ++g)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) acc[g][rb][cb] = v4i{0, 0, 0, 0};

      uint4 ra[SB], rb_[SB];
      auto load = [&](int kt) {
        const int64_t k = (int64_t)kt * kOzK + ld_chunk;
#pragma unroll
        for (int q = 0; q < SB; ++q) {
          const int sq = q < ns ? s0 + q : s0;   // clamp: a valid plane, never used
          const int tq = q < nt ? t0 + q : t0;
          ra[q] = *reinterpret_cast<const uint4*>(a.A + sq * a.planeA + (m0 + ld_row) * a.l_pad + k);
          rb_[q] = *reinterpret_cast<const uint4*>(a.B + tq * a.planeB + (n0 + ld_row) * a.l_pad + k);
        }
      };
      auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < SB; ++q) {
          *reinterpret_cast<uint4*>(&sA[buf][q][ld_row * kOzRow + ld_chunk]) = ra[q];
          *reinterpret_cast<uint4*>(&sB[buf][q][ld_row * kOzRow + ld_chunk]) = rb_[q];
        }
      };

      load(0);
      store(0);
      __syncthreads();
      for (int kt = 0; kt < numK; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < numK) load(kt + 1);
        v4i fa[SB][2], fb[SB][2];
#pragma unroll
        for (int q = 0; q < SB; ++q)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int ra_row = 32 * wr + 16 * h + lane % 16;
            const int rb_row = 32 * wc + 16 * h + lane % 16;
            fa[q][h] = *reinterpret_cast<const v4i*>(&sA[cur][q][ra_row * kOzRow + 16 * (lane / 16)]);
            fb[q][h] = *reinterpret_cast<const v4i*>(&sB[cur][q][rb_row * kOzRow + 16 * (lane / 16)]);
          }
#pragma unroll
        for (int ds = 0; ds < SB; ++ds)
#pragma unroll
          for (int dt = 0; dt < SB; ++dt) {
            const bool keep = ds < ns && dt < nt &&
                              (!a.triangle || (s0 + ds + 1) + (t0 + dt + 1) <= a.S + 1);
            if (keep) {
#pragma unroll
              for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                  acc[ds + dt][rb][cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                      fa[ds][rb], fb[dt][cb], acc[ds + dt][rb][cb], 0, 0, 0);
            }
          }
        if (kt + 1 < numK) store(cur ^ 1);
        __syncthreads();
      }

      // flush the diagonals, smallest weight (largest g) first
#pragma unroll
      for (int gl = 2 * SB - 2; gl >= 0; --gl) {
        const int g = (s0 + 1) + (t0 + 1) + gl;  // 1-based s + t
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int v = acc[gl][rb][cb][i];
              if (v == 0) continue;
              const double x = ldexp((double)v, erow[rb][i] + fcol[cb] + 4 - 8 * g);
              double s, err;
              two_sum(hi[rb][cb][i], x, s, err);
              hi[rb][cb][i] = s;
              lo[rb][cb][i] = lo[rb][cb][i] + err;
            }
      }
    }
  }

#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = m0 + 32 * wr + 16 * rb + 4 * (lane / 16) + i;
        const int64_t c = n0 + 32 * wc + 16 * cb + lane % 16;
        if (r < a.m && c < a.n) {
          double h = hi[rb][cb][i], l = lo[rb][cb][i];
          dd_renorm(h, l);
          a.C_hi[r * a.ldc + c] = h;
          a.C_lo[r * a.ldc + c] = l;
        }
      }
}

// ---------------------------------------------------------------------
// INT8 MFMA product, LDS-staged form (slices <= kOzLdsMaxS).
//
// A wave that loads both operands itself moves every fragment from L2 once
// per wave, and the L2 -> CU path (about 15 bytes per clock and CU) then
// bounds it.
// Here the load unit moves the workgroup's digit blocks of one K step
// straight into LDS (buffer loads to LDS, 16 bytes per lane, no registers),
// double-buffered, and the four wavefronts read their fragments from LDS,
// so each block crosses from L2 once per workgroup.  A block is 16 rows (or
// columns) x 64 k of one slice, stored in MFMA lane order: lane l's 16 bytes
// (row l % 16, k chunk l / 16) at byte 16 l, so both the load and the
// fragment read are one contiguous 1 KiB per wavefront.
// Workgroup tile 64 x 64 over NW wavefronts: 2 x 2 waves of 2 x 2 blocks
// (NW = 4, one wave per SIMD) or 2 x 4 waves of 2 x 1 blocks (NW = 8: two
// waves per SIMD, so one issues MFMAs while the other waits for LDS reads or
// the barrier); the double-double accumulators wait in C between K chunks.
// ---------------------------------------------------------------------
constexpr int kOzLdsMaxS = 8;

template <int S, int NW>
struct OzLdsShape {
  static constexpr int BM = 64;
  static constexpr int BN = 64;
  static constexpr int WAVES_M = 2, WAVES_N = NW / 2;
  static constexpr int WM = BM / 16 / WAVES_M, WN = BN / 16 / WAVES_N;  // 16 x 16 blocks per wave
  static constexpr int NBA = BM / 16, NBB = BN / 16;   // blocks per slice and operand
  static constexpr int BLOCKS = S * (NBA + NBB);       // 1 KiB blocks per K step
};

// wavefronts per workgroup of the LDS-staged kernel
template <int S>
constexpr int oz_lds_waves() {
  return 8;
}

using lds_ptr = __attribute__((address_space(3))) void*;

// Moves one 1 KiB digit block into LDS: lane l's 16 bytes at base + voff
// land at dst + 16 l (base and dst uniform).  The buffer form of the LDS
// load is used, not the flat/global one: with a flat load pending the
// compiler cannot order LDS reads and makes every fragment read wait for
// all outstanding ones (lgkmcnt(0)), which removes the read-ahead.  The
// buffer builtins exist only for the device; the host pass sees an empty
// body.
__device__ __forceinline__ void oz_dma(const int8_t* base, uint32_t voff, int8_t* dst) {
#if defined(__HIP_DEVICE_COMPILE__)
  // raw buffer over `base`: num_records only has to exceed every offset used
  const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(base), (short)0, 0x7ffffff0,
                                                    0x00020000);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)dst, 16, (int)voff, 0, 0, 0);
#endif
}

// Moves step `kn`'s digit blocks of the workgroup tile into `dst`: block
// `blk` (A: slice blk / NBA, rows 16 (blk % NBA) ..; then B likewise) is one
// LDS load per wavefront, wavefronts taking blocks round-robin.
template <int S, int NW>
__device__ __forceinline__ void oz_lds_issue(int8_t* __restrict__ dst, const OzakiGemmArgs& a,
                                             int64_t m0, int64_t n0, int kn, uint32_t lane_off,
                                             int wave) {
  using Sh = OzLdsShape<S, NW>;
  constexpr int NBA = Sh::NBA, NBB = Sh::NBB, NBLK = Sh::BLOCKS;
#pragma unroll
  for (int i = 0; i < (NBLK + NW - 1) / NW; ++i) {
    const int blk = wave + NW * i;
    if (blk < NBLK) {
      const int8_t* src;
      if (blk < S * NBA) {
        const int s = blk / NBA, b = blk % NBA;
        src = a.A + s * a.planeA + (m0 + 16 * b) * a.l_pad;
      } else {
        const int t = (blk - S * NBA) / NBB, b = (blk - S * NBA) % NBB;
        src = a.B + t * a.planeB + (n0 + 16 * b) * a.l_pad;
      }
      oz_dma(src, lane_off + (uint32_t)kn * 64, dst + blk * 1024);
    }
  }
}

// One K step: start moving step `kn`'s blocks into `nxt` (when `more`),
// then the MFMAs on the fragments in `cur`.  The two buffers are distinct
// restrict pointers, so the compiler knows the fragment reads need not wait
// for the loads into the other buffer.
template <int S, bool TRI, int NW>
__device__ __forceinline__ void oz_lds_step(int8_t* __restrict__ nxt, const int8_t* __restrict__ cur,
                                            const OzakiGemmArgs& a, int64_t m0, int64_t n0, int kn,
                                            bool more, uint32_t lane_off, int lane, int wave,
                                            v4i (&acc)[2 * S - 1][OzLdsShape<S, NW>::WM][OzLdsShape<S, NW>::WN]) {
  using Sh = OzLdsShape<S, NW>;
  constexpr int WM = Sh::WM, WN = Sh::WN, NBA = Sh::NBA, NBB = Sh::NBB;
  if (more) oz_lds_issue<S, NW>(nxt, a, m0, n0, kn, lane_off, wave);
  const int wr = wave / Sh::WAVES_N, wc = wave % Sh::WAVES_N;
  // fragment reads in order of first use: A slice 0, the B slices, then
  // each A slice one slice ahead of the MFMAs that use it
  v4i fa[2][WM];
  auto read_a = [&](int s2, v4i (&f)[WM]) {
#pragma unroll
    for (int bi = 0; bi < WM; ++bi)
      f[bi] = *reinterpret_cast<const v4i*>(cur + (s2 * NBA + wr * WM + bi) * 1024 + 16 * lane);
  };
  read_a(0, fa[0]);
  v4i fb[S][WN];
#pragma unroll
  for (int t = 0; t < S; ++t)
#pragma unroll
    for (int bj = 0; bj < WN; ++bj)
      fb[t][bj] = *reinterpret_cast<const v4i*>(cur + (S * NBA + t * NBB + wc * WN + bj) * 1024 + 16 * lane);
#pragma unroll
  for (int s2 = 0; s2 < S; ++s2) {
    if (s2 + 1 < S) read_a(s2 + 1, fa[(s2 + 1) & 1]);
#pragma unroll
    for (int t = 0; t < S; ++t)
      if (!TRI || s2 + t <= S - 1)
#pragma unroll
        for (int bi = 0; bi < WM; ++bi)
#pragma unroll
          for (int bj = 0; bj < WN; ++bj)
            acc[s2 + t][bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[s2 & 1][bi], fb[t][bj],
                                                                        acc[s2 + t][bi][bj], 0, 0, 0);
    // keeps the reads of later slices from being hoisted (registers)
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int S, bool TRI, int NW>
__global__ __launch_bounds__(64 * NW, 1) void ozaki_lds_kernel(OzakiGemmArgs a, int tiles_m,
                                                               int tiles_n, int kchunk) {
  using Sh = OzLdsShape<S, NW>;
  constexpr int G = 2 * S - 1;
  constexpr int BM = Sh::BM, BN = Sh::BN, WM = Sh::WM, WN = Sh::WN, NBLK = Sh::BLOCKS;
  __shared__ __attribute__((aligned(16))) int8_t lds[2 * NBLK * 1024];
  // the wave index is uniform; saying so keeps block addresses in scalar
  // registers (a buffer resource must be)
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  int tm, tn;
  {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    constexpr int GR = 8;
    const int per_group = GR * tiles_n;
    const int group = w / per_group;
    const int first = group * GR;
    const int gsize = min(tiles_m - first, GR);
    const int in = w - group * per_group;
    tm = first + in % gsize;
    tn = in / gsize;
  }
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t r0 = m0 + 16 * WM * (wave / Sh::WAVES_N), c0 = n0 + 16 * WN * (wave % Sh::WAVES_N);
  // this lane's row / column inside a block and its 16-byte k chunk
  const uint32_t lane_off = (uint32_t)((lane % 16) * a.l_pad + 16 * (lane / 16));

  v4i acc[G][WM][WN];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int bi = 0; bi < WM; ++bi)
#pragma unroll
      for (int bj = 0; bj < WN; ++bj) acc[g][bi][bj] = v4i{0, 0, 0, 0};

  // exact diagonal sums -> double-double, smallest weights first.  The
  // double-double accumulators live in C itself between K chunks (each
  // lane owns its outputs), so they take no registers during the MFMAs.
  auto flush = [&](bool first, bool last) {
#pragma unroll
    for (int bi = 0; bi < WM; ++bi) {
#pragma unroll
      for (int bj = 0; bj < WN; ++bj) {
        const int64_t col = c0 + 16 * bj + lane % 16;
        const int fcol = col < a.n ? a.f[col] : 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t r = r0 + 16 * bi + 4 * (lane / 16) + i;
          const bool inside = r < a.m && col < a.n;
          const int erow = r < a.m ? a.e[r] : 0;
          double hi = 0.0, lo = 0.0;
          if (!first && inside) {
            hi = a.C_hi[r * a.ldc + col];
            lo = a.C_lo[r * a.ldc + col];
          }
#pragma unroll
          for (int g = G - 1; g >= 0; --g) {
            const double x = ldexp((double)acc[g][bi][bj][i], erow + fcol + 4 - 8 * (g + 2));
            double sum, err;
            two_sum(hi, x, sum, err);
            hi = sum;
            lo = lo + err;
          }
          if (last) dd_renorm(hi, lo);
          if (inside) {
            a.C_hi[r * a.ldc + col] = hi;
            a.C_lo[r * a.ldc + col] = lo;
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g][bi][bj] = v4i{0, 0, 0, 0};
      }
    }
  };

  const int numK = (int)(a.l_pad / 64);
  // step 0's blocks into buffer 0 (the issue half of a step, no MFMAs)
  if (numK > 0) oz_lds_issue<S, NW>(lds, a, m0, n0, 0, lane_off, wave);
  for (int kc = 0; kc < numK; kc += kchunk) {
    const int kend = min(numK, kc + kchunk);
    for (int kt = kc; kt < kend; ++kt) {
      int8_t* cur = lds + (kt & 1) * NBLK * 1024;
      int8_t* nxt = lds + ((kt & 1) ^ 1) * NBLK * 1024;
      // this thread's loads into `cur` are done; after the barrier
      // everyone's are, and nobody reads `nxt` any more
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      __syncthreads();
      oz_lds_step<S, TRI, NW>(nxt, cur, a, m0, n0, kt + 1, kt + 1 < numK, lane_off, lane, wave, acc);
    }
    flush(kc == 0, kend == numK);
  }
  if (numK == 0) flush(true, true);  // empty K: C := 0
}

// ---------------------------------------------------------------------
// INT8 MFMA product, band form (kOzLdsMaxS < slices <= kOzBandMaxS).
//
// With 2S - 1 diagonal accumulators live, a wavefront can own only one or
// two 16 x 16 blocks, and a workgroup's digit blocks of two K steps no
// longer fit LDS, so sharing operands between wavefronts has to come from
// elsewhere.  Here the four wavefronts of a workgroup stack vertically:
// wave w owns rows m0 + 16 w .. + 15 and the WN 16-column blocks of the
// workgroup's 16 WN columns.  Each wave loads its own A fragments straight
// into registers (no other wave uses those rows) and reloads each block of
// slices for the next K step right after its last use; only the
// workgroup's B blocks are moved into LDS by the load unit (double-buffered)
// and shared by all four waves.  Slices are processed four at a time so each
// B fragment read from LDS feeds 4 WN MFMAs.  Per K step a workgroup moves
// (4 + WN) S KiB for 4 WN S^2 MFMAs; a wave loading both operands itself
// would move 2S KiB for S^2.
// ---------------------------------------------------------------------
constexpr int kOzBandMaxS = 24;  // the band form takes kOzLdsMaxS + 1 .. kOzBandMaxS slices
// column blocks per wavefront: two while the 2S - 1 accumulators of both fit
template <int S>
constexpr int oz_band_wn() {
  return S <= 20 ? 2 : 1;
}

template <int S, int WN>
__device__ __forceinline__ void oz_band_issue(int8_t* __restrict__ dst, const OzakiGemmArgs& a,
                                              int64_t n0, int kn, uint32_t lane_off, int wave) {
  constexpr int NBLK = WN * S;  // B blocks per K step: slice t, column block bj
#pragma unroll
  for (int i = 0; i < (NBLK + 3) / 4; ++i) {
    const int blk = wave + 4 * i;
    if (blk < NBLK) {
      const int t = blk / WN, bj = blk % WN;
      oz_dma(a.B + t * a.planeB + (n0 + 16 * bj) * a.l_pad, lane_off + (uint32_t)kn * 64, dst + blk * 1024);
    }
  }
}

// One K step on the B blocks in `cur` and the A fragments in fa (slice s
// of this wave's rows, all resident); starts moving step kn's B blocks into
// `nxt` and reloads each block of A slices for step kn right after its last
// use (the last step re-reads its own, still valid, step).  The last block
// is the exception: reloaded at the end of a step, it would be waited for
// at the step boundary; instead each step loads its own last block at its
// start, a whole step before the MFMAs that use it.
template <int S, int WN, bool TRI>
__device__ __forceinline__ void oz_band_step(int8_t* __restrict__ nxt, const int8_t* __restrict__ cur,
                                             const OzakiGemmArgs& a, const int8_t* rowsA, int64_t n0,
                                             int kn, bool more, uint32_t lane_off, int lane, int wave,
                                             v4i (&fa)[S], v4i (&acc)[2 * S - 1][WN]) {
  constexpr int SB = 4;  // slices per block of the s loop
  constexpr int LAST = (S - 1) / SB * SB;  // first slice of the last block
  if (more) oz_band_issue<S, WN>(nxt, a, n0, kn, lane_off, wave);
  // the loads below must not move above the B loads
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s2 = LAST; s2 < S; ++s2)
    fa[s2] = *reinterpret_cast<const v4i*>(rowsA + s2 * a.planeA + (int64_t)(kn - 1) * 64 + lane_off);
  __builtin_amdgcn_sched_barrier(0);
  const int kr = more ? kn : kn - 1;
  auto read_b = [&](int t, v4i (&f)[WN]) {
#pragma unroll
    for (int bj = 0; bj < WN; ++bj)
      f[bj] = *reinterpret_cast<const v4i*>(cur + (WN * t + bj) * 1024 + 16 * lane);
  };
#pragma unroll
  for (int s0 = 0; s0 < S; s0 += SB) {
    // B fragments two slices ahead of their MFMAs (one slice's MFMAs,
    // 4 WN of them, can be shorter than an LDS read); the scheduling
    // barrier keeps later slices' reads from being hoisted (registers)
    v4i fb[3][WN];
    read_b(0, fb[0]);
    if (S > 1) read_b(1, fb[1]);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      if (t + 2 < S) read_b(t + 2, fb[(t + 2) % 3]);
#pragma unroll
      for (int s2 = s0; s2 < s0 + SB && s2 < S; ++s2)
        if (!TRI || s2 + t <= S - 1)
#pragma unroll
          for (int bj = 0; bj < WN; ++bj)
            acc[s2 + t][bj] =
                __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[s2], fb[t % 3][bj], acc[s2 + t][bj], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (s0 != LAST) {
#pragma unroll
      for (int s2 = s0; s2 < s0 + SB; ++s2)
        fa[s2] = *reinterpret_cast<const v4i*>(rowsA + s2 * a.planeA + (int64_t)kr * 64 + lane_off);
    }
    // keeps the reloads of this block of slices after its MFMAs (registers)
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int S, int WN, bool TRI>
__global__ __launch_bounds__(256, 1) void ozaki_band_kernel(OzakiGemmArgs a, int tiles_m,
                                                            int tiles_n, int kchunk) {
  constexpr int G = 2 * S - 1, NBLK = WN * S;
  __shared__ __attribute__((aligned(16))) int8_t lds[2 * NBLK * 1024];
  // the wave index is uniform; saying so keeps block addresses in scalar
  // registers (a buffer resource must be)
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  int tm, tn;
  {
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    constexpr int GR = 8;
    const int per_group = GR * tiles_n;
    const int group = w / per_group;
    const int first = group * GR;
    const int gsize = min(tiles_m - first, GR);
    const int in = w - group * per_group;
    tm = first + in % gsize;
    tn = in / gsize;
  }
  const int64_t m0 = (int64_t)tm * 64, n0 = (int64_t)tn * 16 * WN;
  const int64_t r0 = m0 + 16 * wave, c0 = n0;
  const uint32_t lane_off = (uint32_t)((lane % 16) * a.l_pad + 16 * (lane / 16));
  const int8_t* rowsA = a.A + r0 * a.l_pad;  // this wave's 16 rows (uniform)

  v4i acc[G][WN];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int bj = 0; bj < WN; ++bj) acc[g][bj] = v4i{0, 0, 0, 0};

  // exact diagonal sums -> double-double (accumulators wait in C between K
  // chunks), smallest weights first
  auto flush = [&](bool first, bool last) {
    int erow[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = r0 + 4 * (lane / 16) + i;
      erow[i] = r < a.m ? a.e[r] : 0;
    }
#pragma unroll
    for (int bj = 0; bj < WN; ++bj) {
      const int64_t col = c0 + 16 * bj + lane % 16;
      const int fcol = col < a.n ? a.f[col] : 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + 4 * (lane / 16) + i;
        const bool inside = r < a.m && col < a.n;
        double hi = 0.0, lo = 0.0;
        if (!first && inside) {
          hi = a.C_hi[r * a.ldc + col];
          lo = a.C_lo[r * a.ldc + col];
        }
#pragma unroll
        for (int g = G - 1; g >= 0; --g) {
          const double x = ldexp((double)acc[g][bj][i], erow[i] + fcol + 4 - 8 * (g + 2));
          double sum, err;
          two_sum(hi, x, sum, err);
          hi = sum;
          lo = lo + err;
        }
        if (last) dd_renorm(hi, lo);
        if (inside) {
          a.C_hi[r * a.ldc + col] = hi;
          a.C_lo[r * a.ldc + col] = lo;
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) acc[g][bj] = v4i{0, 0, 0, 0};
    }
  };

  const int numK = (int)(a.l_pad / 64);
  v4i fa[S];
  if (numK > 0) {
    oz_band_issue<S, WN>(lds, a, n0, 0, lane_off, wave);
    // step 0's A slices but the last block (each step loads that itself)
#pragma unroll
    for (int q = 0; q < (S - 1) / 4 * 4; ++q)
      fa[q] = *reinterpret_cast<const v4i*>(rowsA + q * a.planeA + lane_off);
  }
  for (int kc = 0; kc < numK; kc += kchunk) {
    const int kend = min(numK, kc + kchunk);
    for (int kt = kc; kt < kend; ++kt) {
      int8_t* cur = lds + (kt & 1) * NBLK * 1024;
      int8_t* nxt = lds + ((kt & 1) ^ 1) * NBLK * 1024;
      // this thread's loads are done (B blocks of this step, A fragments);
      // after the barrier everyone's are, and nobody reads `nxt` any more
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      __syncthreads();
      oz_band_step<S, WN, TRI>(nxt, cur, a, rowsA, n0, kt + 1, kt + 1 < numK, lane_off, lane, wave, fa, acc);
    }
    flush(kc == 0, kend == numK);
  }
  if (numK == 0) flush(true, true);  // empty K: C := 0
}

// ---------------------------------------------------------------------
// Residue form: one INT8 product per modulus.  Workgroup w (after the XCD
// remap) takes modulus z = w / tiles and tile w % tiles, so the workgroups
// of one XCD share one modulus' planes.  Every 2047 K steps the INT32 sums
// are reduced into [0, p_z) (exact integer arithmetic), and the final
// residues are stored as bytes.
// ---------------------------------------------------------------------
// v mod p in [0, p) for |v| < 2^31 and 29 <= p <= 256 (every modulus), in
// 32-bit arithmetic: v = hi 2^16 + lo folds to t = hi (2^16 mod p) + lo
// with |t| < 2^24, exact in FP32; the FP32 quotient t (1/p) is within 0.07
// of t / p (two roundings of relative 2^-24 on a quotient below 2^24 / 29),
// so its floor is off by at most one and t - q p lies in [-p, 2p); as
// unsigned numbers the one of r, r + p, r - p inside [0, p) is the smallest.
// (An FP64 quotient with two corrections cost 15% of the product kernel's
// time in the epilogue's 128 reductions per lane.)
__device__ __forceinline__ int crt_mod(int v, int p, int c16, float inv_pf) {
  const int t = (v >> 16) * c16 + (v & 0xffff);
  const int q = (int)floorf((float)t * inv_pf);
  const int r = t - q * p;
  return (int)min(min((unsigned)r, (unsigned)(r + p)), (unsigned)(r - p));
}

// Residue products on 256 x 256 workgroup tiles: with one digit pair per
// product, operand reuse has to come from the tile.  Eight wavefronts
// (4 x 2) each own a 64 x 128 block of outputs (4 x 8 MFMA blocks), so a
// K step reads 12 fragments from LDS for 32 MFMAs per wavefront (below the
// LDS rate the INT8 MFMA rate needs) and a workgroup moves 32 KiB per K
// step for 256 MFMAs.  Each K step of
// 64 is one LDS stage moved by the load unit as in the LDS-staged kernel;
// NBUF stages form a ring, loads run NBUF - 1 stages ahead of the MFMAs
// (a K step's compute is short next to the latency of an L2 miss).  Rows of
// A's and B's planes are padded to 256.
constexpr int kCrtWN = 8;  // 16-column MFMA blocks per wavefront
constexpr int kCrtBM = 256, kCrtBN = 32 * kCrtWN;
constexpr int kCrtNBA = kCrtBM / 16, kCrtNBB = kCrtBN / 16;

template <int NBUF>
__global__ __launch_bounds__(512, 1) void crt_tile_kernel(CrtGemmArgs c, int tiles_m, int tiles_n,
                                                          int kchunk) {
  constexpr int STEP_BLOCKS = kCrtNBA + kCrtNBB;  // 32 KiB per K step
  constexpr int STAGE = STEP_BLOCKS * 1024;
  constexpr int LOADS = STEP_BLOCKS / 8;          // LDS loads per wavefront per stage
  static_assert(LOADS * (NBUF - 2) <= 15, "vmcnt immediate");
  __shared__ __attribute__((aligned(16))) int8_t lds[NBUF * STAGE];
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int tiles = tiles_m * tiles_n;
  // With a device-side plan the grid holds the most moduli any plan may
  // use, and only its first plan->N x tiles workgroups work.  The remap is
  // taken over those: the hardware deals workgroup b to XCD b % 8, so a
  // prefix of the grid is spread evenly, and the idle workgroups at the end
  // return at once (a remap over the whole grid put the unused moduli's
  // tiles on whole XCDs, which then sat idle).
  int total = gridDim.x;
  if (c.plan) {
    if (c.product >= 0 && c.plan->skip[c.product]) return;
    total = min(c.plan->N, c.N) * tiles;  // 0 when the plan does not fit
    if ((int)blockIdx.x >= total) return;
  }
  int tm, tn, z;
  {
    const int w = xcd_remap(blockIdx.x, total);
    z = w / tiles;
    const int t = w - z * tiles;
    constexpr int GR = 8;
    const int per_group = GR * tiles_n;
    const int group = t / per_group;
    const int first = group * GR;
    const int gsize = min(tiles_m - first, GR);
    const int in = t - group * per_group;
    tm = first + in % gsize;
    tn = in / gsize;
  }
  const int p = c.mods[z];
  const int c16 = 65536 % p;
  const float inv_pf = 1.0f / (float)p;
  const int8_t* A = c.A + (int64_t)z * c.planeA;
  const int8_t* B = c.B + (int64_t)z * c.planeB;
  const int64_t lp = c.l_pad;
  const int64_t m0 = (int64_t)tm * kCrtBM, n0 = (int64_t)tn * kCrtBN;
  const int wr = wave / 2, wc = wave % 2;
  // within a 1 KiB block of the tiled plane layout: row lane % 16, k chunk lane / 16
  const uint32_t lane_off = (uint32_t)((lane % 16) * 64 + 16 * (lane / 16));

  // K steps per segment; the segments' products add up in one accumulation.
  // The loads are issued in step order by a running state: the segment's
  // per-load buffer resources (base of the load's row block) are made once
  // per segment, and the step within the segment is the scalar offset, so a
  // step's issue costs a few scalar instructions (no division by the step
  // count, no reload of the segment offsets).
  const int kps = (int)(lp / 64);
  __amdgpu_buffer_rsrc_t rs[LOADS];
  const auto set_segment = [&](int seg) {
    const int8_t* As = A + c.segA[seg];
    const int8_t* Bs = B + c.segB[seg];
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int b = wave + 8 * i;
      const int64_t rb = b < kCrtNBA ? m0 / 16 + b : n0 / 16 + (b - kCrtNBA);  // row block
      const int8_t* base = (b < kCrtNBA ? As : Bs) + rb * kps * 1024;
      // raw buffer: num_records only has to exceed every offset used
      rs[i] = __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(base), (short)0, 0x7ffffff0, 0x00020000);
    }
  };
  int next_seg = 0, next_kk = 0, next_slot = 0;
  set_segment(0);
  const auto issue_next = [&]() {
    int8_t* dst = lds + next_slot * STAGE;
#pragma unroll
    for (int i = 0; i < LOADS; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs[i], (lds_ptr)(dst + (wave + 8 * i) * 1024), 16, (int)lane_off,
                                               next_kk * 1024, 0, 0);
    next_slot = next_slot + 1 == NBUF ? 0 : next_slot + 1;
    if (++next_kk == kps) {
      next_kk = 0;
      if (++next_seg < c.nseg) set_segment(next_seg);
    }
  };

  v4i acc[4][kCrtWN];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < kCrtWN; ++bj) acc[bi][bj] = v4i{0, 0, 0, 0};

  const int numK = kps * c.nseg;
#pragma unroll
  for (int s = 0; s < NBUF - 1; ++s)
    if (s < numK) issue_next();
  int until_reduce = kchunk;
  for (int st = 0; st < numK; ++st) {
    // this wave's loads of step st are done once at most the later steps'
    // (up to NBUF - 2 of them) are outstanding; near the end fewer are
    const int later = min(NBUF - 2, numK - 1 - st);
    if (later >= NBUF - 2)
      __builtin_amdgcn_s_waitcnt(0x0F70 | (LOADS * (NBUF - 2)));
    else
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // everyone's loads of st have landed; slot (st - 1) is free.  A plain
    // barrier: __syncthreads() would add a fence that waits for every
    // outstanding load, including the steps still in flight; the memory
    // clobber keeps the compiler from moving LDS reads across it.
    asm volatile("s_barrier" ::: "memory");
    const int8_t* __restrict__ cur = lds + (st % NBUF) * STAGE;
    v4i fa[4], fb[kCrtWN];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
      fa[bi] = *reinterpret_cast<const v4i*>(cur + (4 * wr + bi) * 1024 + 16 * lane);
#pragma unroll
    for (int bj = 0; bj < kCrtWN; ++bj)
      fb[bj] = *reinterpret_cast<const v4i*>(cur + (kCrtNBA + kCrtWN * wc + bj) * 1024 + 16 * lane);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < kCrtWN; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[bi], fb[bj], acc[bi][bj], 0, 0, 0);
    // the next loads go out behind this step's MFMAs (into slot st - 1, free
    // since the barrier); issued ahead of them they held up the MFMA issue
    // while the load unit queued them (1-2% slower as measured)
    __builtin_amdgcn_sched_barrier(0);
    if (st + NBUF - 1 < numK) issue_next();
    __builtin_amdgcn_sched_barrier(0);
    if (--until_reduce == 0) {
      until_reduce = kchunk;
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < kCrtWN; ++bj)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[bi][bj][i] = crt_mod(acc[bi][bj][i], p, c16, inv_pf);
    }
  }
  uint8_t* R = c.R + (int64_t)z * c.planeR;
  const int64_t r0 = m0 + 64 * wr, c0 = n0 + 16 * kCrtWN * wc;
  if (r0 + 64 <= c.m && c0 + 16 * kCrtWN <= c.n) {
    // whole wavefront block inside C: one row pointer per (bi, i), the
    // columns as immediate offsets, no per-element tests
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uint8_t* rp = R + (r0 + 16 * bi + 4 * (lane / 16) + i) * c.ldr + c0 + lane % 16;
#pragma unroll
        for (int bj = 0; bj < kCrtWN; ++bj) rp[16 * bj] = (uint8_t)crt_mod(acc[bi][bj][i], p, c16, inv_pf);
      }
    return;
  }
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < kCrtWN; ++bj) {
      const int64_t col = c0 + 16 * bj + lane % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + 16 * bi + 4 * (lane / 16) + i;
        if (r < c.m && col < c.n) R[r * c.ldr + col] = (uint8_t)crt_mod(acc[bi][bj][i], p, c16, inv_pf);
      }
    }
}

// Sustained INT8 matrix-core rate: every wavefront issues back-to-back
// v_mfma_i32_16x16x64_i8 into 32 independent accumulators (no memory
// traffic), 8 wavefronts per workgroup, one workgroup per CU.  The sums are
// folded into one word that is stored only if it takes an impossible value,
// so the compiler keeps every product.
__global__ __launch_bounds__(512, 1) void mfma_rate_kernel(int steps, int* sink) {
  const int lane = threadIdx.x % 64;
  const v4i a = v4i{lane, lane + 1, lane + 2, lane + 3}, b = v4i{3 * lane, 1, 2, lane};
  v4i acc[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) acc[i] = v4i{0, 0, 0, 0};
  for (int st = 0; st < steps; ++st)
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[i], 0, 0, 0);
  int t = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) t += acc[i][0] + acc[i][3];
  if (t == 0x7fffffff) sink[0] = t;
}

struct OzKernels;

template <int S>
struct OzTable {
  static void fill(OzKernels& k);
};
template <>
struct OzTable<0> {
  static void fill(OzKernels&) {}
};

// Kernel per slice count: LDS-staged up to kOzLdsMaxS, band form up to
// kOzBandMaxS.
struct OzKernels {
  const void* all[kOzBandMaxS + 1] = {};
  const void* tri[kOzBandMaxS + 1] = {};
  int tile_m[kOzBandMaxS + 1] = {};  // workgroup tile rows / columns
  int tile_n[kOzBandMaxS + 1] = {};
  int threads[kOzBandMaxS + 1] = {};
  OzKernels() { OzTable<kOzBandMaxS>::fill(*this); }
};

template <int S>
void OzTable<S>::fill(OzKernels& k) {
  if constexpr (S <= kOzLdsMaxS) {
    constexpr int NW = oz_lds_waves<S>();
    k.all[S] = reinterpret_cast<const void*>(&ozaki_lds_kernel<S, false, NW>);
    k.tri[S] = reinterpret_cast<const void*>(&ozaki_lds_kernel<S, true, NW>);
    k.tile_m[S] = OzLdsShape<S, NW>::BM;
    k.tile_n[S] = OzLdsShape<S, NW>::BN;
    k.threads[S] = 64 * NW;
  } else {
    k.all[S] = reinterpret_cast<const void*>(&ozaki_band_kernel<S, oz_band_wn<S>(), false>);
    k.tri[S] = reinterpret_cast<const void*>(&ozaki_band_kernel<S, oz_band_wn<S>(), true>);
    k.tile_m[S] = 64;
    k.tile_n[S] = 16 * oz_band_wn<S>();
    k.threads[S] = 256;
  }
  OzTable<S - 1>::fill(k);
}

}  // namespace

hipError_t launch_mfma_rate(int blocks, int steps, int* sink, hipStream_t s) {
  if (blocks < 1 || steps < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mfma_rate_kernel, dim3((unsigned)blocks), dim3(512), 0, s, steps, sink);
  return hipGetLastError();
}

int ozaki_max_slices() { return kMaxSlices; }
int ozaki_block_slices() { return 4; }
int ozaki_chunked_max_slices() { return kOzBandMaxS; }

hipError_t launch_ozaki_scan(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                             int by_col, int* e, int* low, int* need, hipStream_t s) {
  if (!need) Xlo = nullptr;  // the lo limbs only matter for the digit count
  if (!by_col) {
    if (R <= 0) return hipSuccess;
    if (R > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(row_scan_kernel, dim3((unsigned)R), dim3(256), 0, s, X, Xlo, K, ld, e, need);
    return hipGetLastError();
  }
  if (K <= 0) return hipSuccess;
  if (need && !low) return hipErrorInvalidValue;
  const unsigned fb = (unsigned)std::min<int64_t>((K + 255) / 256, 65535);
  hipLaunchKernelGGL(fill_int_kernel, dim3(fb), dim3(256), 0, s, e, K, INT_MIN);
  if (need) hipLaunchKernelGGL(fill_int_kernel, dim3(fb), dim3(256), 0, s, low, K, INT_MAX);
  const int64_t gy = (R + kColScanRows - 1) / kColScanRows;
  if (R > 0) {
    if (gy > 65535 || (K + 63) / 64 > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(col_scan_kernel, dim3((unsigned)((K + 63) / 64), (unsigned)gy), dim3(256), 0, s,
                       X, Xlo, R, K, ld, e, need ? low : nullptr);
  }
  hipLaunchKernelGGL(col_finish_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, e, low, K,
                     need);
  return hipGetLastError();
}

hipError_t launch_ozaki_split_rows(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                                   const int* e, int S, int8_t* out, int64_t ld_out, int64_t plane,
                                   int64_t Rp, int64_t Kp, hipStream_t s) {
  const int64_t work = Rp * (Kp / 8);
  if (work <= 0 || S <= 0) return hipSuccess;
  const dim3 grid((unsigned)((work + 255) / 256));
  if (Xlo)
    hipLaunchKernelGGL(split_rows_kernel<true>, grid, dim3(256), 0, s, X, Xlo, R, K, ld, e, S, out,
                       ld_out, plane, Rp, Kp);
  else
    hipLaunchKernelGGL(split_rows_kernel<false>, grid, dim3(256), 0, s, X, Xlo, R, K, ld, e, S, out,
                       ld_out, plane, Rp, Kp);
  return hipGetLastError();
}

hipError_t launch_ozaki_split_cols(const double* X, const double* Xlo, int64_t K, int64_t C, int64_t ld,
                                   const int* f, int S, int8_t* out, int64_t ld_out, int64_t plane,
                                   int64_t Cp, int64_t Kp, hipStream_t s) {
  if (Cp <= 0 || Kp <= 0 || S <= 0) return hipSuccess;
  if (S > kMaxSlices) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(Cp / 64), (unsigned)(Kp / kColTileK));
  if (Xlo)
    hipLaunchKernelGGL(split_cols_kernel<true>, grid, dim3(256), 0, s, X, Xlo, K, C, ld, f, S, out,
                       ld_out, plane, Cp, Kp);
  else
    hipLaunchKernelGGL(split_cols_kernel<false>, grid, dim3(256), 0, s, X, Xlo, K, C, ld, f, S, out,
                       ld_out, plane, Cp, Kp);
  return hipGetLastError();
}

hipError_t launch_ozaki_gemm(const OzakiGemmArgs& a, hipStream_t s) {
  if (a.S >= 1 && a.S <= kOzBandMaxS) {
    // LDS-staged or band kernel on tiles of 16 to 64 rows / columns (digit
    // planes are padded to multiples of 64, so every tile reads inside them)
    static const OzKernels table;
    const int tm_rows = table.tile_m[a.S], tn_cols = table.tile_n[a.S];
    const int64_t tiles_m = (a.m + tm_rows - 1) / tm_rows, tiles_n = (a.n + tn_cols - 1) / tn_cols;
    // diagonal sums: at most S pairs of 64 k per K step, each |d d'| <= 128^2
    const double per_step = (double)a.S * 64.0 * 128.0 * 128.0;
    const int kchunk = std::max(1, (int)(2147483647.0 / per_step));
    OzakiGemmArgs args = a;
    int tm = (int)tiles_m, tn = (int)tiles_n;
    void* kargs[] = {(void*)&args, (void*)&tm, (void*)&tn, (void*)&kchunk};
    return hipLaunchKernel(a.triangle ? table.tri[a.S] : table.all[a.S],
                           dim3((unsigned)(tiles_m * tiles_n)), dim3(table.threads[a.S]), kargs, 0, s);
  }
  const int64_t tiles = ((a.m + kOzTile - 1) / kOzTile) * ((a.n + kOzTile - 1) / kOzTile);
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(ozaki_mfma_kernel<4>, dim3((unsigned)tiles), dim3(256), 0, s, a);
  return hipGetLastError();
}

namespace {
template <bool COLS>
hipError_t launch_crt_planes(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                             const int* e, int S, int N, int8_t* out, int64_t Rp, int64_t Kp,
                             const CrtResidueConsts* rc, hipStream_t s, const CrtPlan* plan, int part) {
  // the tiled plane layout (crt_plane_offset) needs whole 16-row x 64-k blocks
  if (S < 1 || S > kCrtMaxSlices || N < 1 || N > kCrtMaxModuli || Kp % 64 || Rp % 16)
    return hipErrorInvalidValue;
  const int64_t work = Rp * (Kp / 8);
  if (work <= 0) return hipSuccess;
  if ((work + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((work + 255) / 256));
  if (Xlo)
    hipLaunchKernelGGL((crt_rows_kernel<true, COLS>), grid, dim3(256), 0, s, X, Xlo, R, K, ld, e, S, N, out,
                       Rp, Kp, rc, plan, part);
  else
    hipLaunchKernelGGL((crt_rows_kernel<false, COLS>), grid, dim3(256), 0, s, X, Xlo, R, K, ld, e, S, N, out,
                       Rp, Kp, rc, plan, part);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_crt_rows(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                           const int* e, int S, int N, int8_t* out, int64_t Rp, int64_t Kp,
                           const CrtResidueConsts* rc, hipStream_t s, const CrtPlan* plan, int part) {
  return launch_crt_planes<false>(X, Xlo, R, K, ld, e, S, N, out, Rp, Kp, rc, s, plan, part);
}

hipError_t launch_crt_cols(const double* X, const double* Xlo, int64_t R, int64_t K, int64_t ld,
                           const int* e, int S, int N, int8_t* out, int64_t Rp, int64_t Kp,
                           const CrtResidueConsts* rc, hipStream_t s, const CrtPlan* plan, int part) {
  return launch_crt_planes<true>(X, Xlo, R, K, ld, e, S, N, out, Rp, Kp, rc, s, plan, part);
}

int crt_tile_rows() { return kCrtBM; }
int crt_tile_cols() { return kCrtBN; }
int crt_k_multiple() { return 64; }

hipError_t launch_crt_gemm(const CrtGemmArgs& c, hipStream_t s) {
  const int64_t tiles_m = (c.m + kCrtBM - 1) / kCrtBM, tiles_n = (c.n + kCrtBN - 1) / kCrtBN;
  const int64_t total = tiles_m * tiles_n * c.N;
  if (total <= 0) return hipSuccess;
  if (total > 0x7fffffff || c.N > kCrtMaxModuli || c.l_pad % 64 || c.nseg > kCrtMaxSegments)
    return hipErrorInvalidValue;
  constexpr int NBUF = 4;
  // INT32 sums: |r r'| <= 128^2 per product, 64 per K step, plus the
  // reduced residue carried over (< 256): reduce every 2047 K steps
  const int kchunk = (int)((2147483647.0 - 256.0) / (64.0 * 128.0 * 128.0));
  CrtGemmArgs args = c;
  if (args.nseg < 1) args.nseg = 1;
  int tm = (int)tiles_m, tn = (int)tiles_n, kc = kchunk;
  void* kargs[] = {(void*)&args, (void*)&tm, (void*)&tn, (void*)&kc};
  return hipLaunchKernel(reinterpret_cast<const void*>(&crt_tile_kernel<NBUF>), dim3((unsigned)total),
                         dim3(512), kargs, 0, s);
}

}  // namespace mpg

