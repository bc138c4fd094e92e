// Exact product of long-integer matrices through the residue form: the
// fixed-point analog of the paper's arbitrary-precision runs.
//
// Entries are two's complement integers of `words` 32-bit words, stored as
// word planes (plane w: word w of every entry).  An entry is cut into chunks
// of CW words (96, 128 or 160 bits), x = sum_c U_c 2^(32 CW c) with U_c in
// [0, 2^(32 CW)) below the top chunk and the top chunk signed.  For each
// chunk the residues modulo the N leading moduli are formed directly from its
// words; chunk polynomials may first be combined by Karatsuba's splitting
// (residue planes of chunk sums); the products of the leaf polynomials run
// diagonal by diagonal as INT8 products over a K made of the chunk pairs
// (segments), and each diagonal of the full product, a signed combination of
// leaf diagonals, is rebuilt exactly and added at 2^(32 CW g) into the
// multiword result.
#include "crt_internal.hpp"
#include "int_internal.hpp"

namespace mpg {
namespace {

// 2^(32 j) mod p_z and 1 / p_z (rounded) for the N moduli, built by the
// first threads of a block.
struct WordWeights {
  double c[kCrtMaxModuli][kIntMaxChunkWords];
  double inv[kCrtMaxModuli];
};

__device__ void word_weights(WordWeights& w, int N) {
  for (int z = threadIdx.x; z < N; z += blockDim.x) {
    const uint64_t p = (uint64_t)kCrtModuli[z];
    uint64_t v = 1;
    for (int j = 0; j < kIntMaxChunkWords; ++j) {
      w.c[z][j] = (double)v;
      v = (v << 32) % p;
    }
    w.inv[z] = 1.0 / (double)p;
  }
}

// Chunk c of an entry (CW words from word CW c; words past the entry's own
// are its sign extension; the top chunk's last word is signed).
template <int CW>
__device__ __forceinline__ void chunk_words(const uint32_t* X, int64_t pstride, int64_t off, int words,
                                            int c, int chunks, bool ok, double (&v)[CW]) {
  const int64_t top_word = (int64_t)words - 1;
  uint32_t sign = 0;
  if (ok) sign = (int32_t)X[top_word * pstride + off] < 0 ? 0xFFFFFFFFu : 0u;
#pragma unroll
  for (int j = 0; j < CW; ++j) {
    const int w = CW * c + j;
    uint32_t u = 0;
    if (ok) u = w < words ? X[(int64_t)w * pstride + off] : sign;
    v[j] = (c == chunks - 1 && j == CW - 1) ? (double)(int32_t)u : (double)u;
  }
}

// Residue planes of all chunks: plane c N + z of out, element (r, k) at
// crt_plane_offset(r, k, Kp).  COLS:
// element (r, k) is X[w][k][r] (the columns of B); else X[w][r][k].
// Rows: a thread takes 8 consecutive k of one row.  Columns: a block takes
// 32 columns x 64 k, a thread 8 consecutive k of one column (reads of one k
// across the 32 columns are contiguous).
template <bool COLS, int CW>
__global__ __launch_bounds__(256) void int_residue_kernel(IntResidueArgs a) {
  __shared__ WordWeights ww;
  word_weights(ww, a.N);
  __syncthreads();
  int64_t r, k0;
  if (!COLS) {
    const int64_t per_row = a.Kp / 8;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.Rp * per_row) return;
    r = idx / per_row;
    k0 = (idx % per_row) * 8;
  } else {
    r = (int64_t)blockIdx.x * 32 + threadIdx.x % 32;
    k0 = (int64_t)blockIdx.y * 64 + 8 * (threadIdx.x / 32);
    if (r >= a.Rp || k0 >= a.Kp) return;
  }
  const int64_t plane = a.Rp * a.Kp;
  for (int c = 0; c < a.chunks; ++c) {
    // the chunk's CW words of 8 elements
    double v[CW][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t k = k0 + q;
      const bool ok = r < a.R && k < a.K;
      const int64_t off = ok ? (COLS ? k * a.ld + r : r * a.ld + k) : 0;
      double t[CW];
      chunk_words<CW>(a.X, a.pstride, off, a.words, c, a.chunks, ok, t);
#pragma unroll
      for (int j = 0; j < CW; ++j) v[j][q] = t[j];
    }
    for (int z = 0; z < a.N; ++z) {
      const double pd = (double)kCrtModuli[z], inv = ww.inv[z];
      // the remainder of the rounded quotient lies in [-(p+1)/2, (p+1)/2]
      // (the quotient is within 1/(2p) of the exact one): a signed byte for
      // every odd modulus up to 253; only 256 and 255 are centred
      const bool centre = z < 2;  // uniform
      uint64_t packed = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        double acc = 0.0;  // |acc| < CW 2^32 256 <= 2^43: exact
#pragma unroll
        for (int j = 0; j < CW; ++j) acc = __builtin_fma(v[j][q], ww.c[z][j], acc);
        double res = __builtin_fma(-rint(acc * inv), pd, acc);
        if (centre) {
          if (2.0 * res >= pd) res -= pd;
          if (2.0 * res < -pd) res += pd;
        }
        packed |= (uint64_t)(uint8_t)(int8_t)(int)res << (8 * q);
      }
      *reinterpret_cast<uint64_t*>(a.out + ((int64_t)c * a.N + z) * plane + crt_plane_offset(r, k0, a.Kp)) =
          packed;
    }
  }
}

// Rebuilds each entry's diagonal sum Y (W words) and adds it, signed, into
// C's words from `word_off` up (carries and borrows run to the top word).
// The residues of Y modulo p_z are the signed sum of the terms' residues
// (each in [0, p_z)), brought back into [0, p_z): the sum is below
// 64 x 256 in magnitude, so its FP32 quotient by p_z is within 2^-8 of the
// exact one and one correction each way suffices.
//
// X' = sum_z r_z T_z is formed on INT8 MFMA as in the residue form's
// reconstruction: a workgroup stages the residues of 256 outputs of a row
// as signed bytes r_z - 128 in LDS (four moduli x four columns per thread,
// transposed in registers), one MFMA per 16 digit positions of the T_z
// (signed radix-256 digits from the table) and 16 outputs gives the
// position sums, each word's four positions combine into a 64-bit sum, and
// a thread per output adds 128 sum_z T_z with a signed carry pass (X' is
// below 2^(32 W)); a workgroup walks several rows.
typedef int v4i_t __attribute__((ext_vector_type(4)));

template <int W>
__global__ __launch_bounds__(256) void int_accumulate_kernel(IntAccumArgs a) {
  constexpr int G = (4 * W + 15) / 16;
  constexpr int LS = 68;  // bytes per output in the residue tile (17 dwords: no bank conflicts)
  static_assert(G <= kCrtFragGroups, "digit groups");
  constexpr int SMEM = 256 * LS > 256 * W * 8 ? 256 * LS : 256 * W * 8;
  __shared__ __attribute__((aligned(16))) uint8_t smem[SMEM];
  uint8_t* const tile = smem;
  uint64_t* const vs = reinterpret_cast<uint64_t*>(smem);  // per output: W pairs of half sums
  const CrtTable& t = *a.t;
  const double rP = 1.0 / t.Pd;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  v4i_t fa[G];
#pragma unroll
  for (int g = 0; g < G; ++g) fa[g] = *reinterpret_cast<const v4i_t*>(&t.frag[g][lane][0]);
  const int nzg = (a.N + 3) / 4;
  const int c = threadIdx.x % 64, zq = threadIdx.x / 64;
  const int64_t jc = j0 + 4 * c;        // this thread's four columns when staging
  const int64_t jt = j0 + threadIdx.x;  // its output in the tail
  const bool plain = a.nterms == 1 && a.term_sign[0] == 1;  // uniform
  // residues of four consecutive columns for modulus z (0 past the planes)
  auto residues4 = [&](const uint8_t* row, int z) -> uint32_t {
    if (z >= a.N || jc >= a.ldr) return 0u;
    if (plain) return *reinterpret_cast<const uint32_t*>(row + a.term_off[0] + (int64_t)z * a.planeR);
    const int p = kCrtModuli[z];
    const float inv_pf = 1.0f / (float)p;
    int sum[4] = {0, 0, 0, 0};
    for (int q = 0; q < a.nterms; ++q) {
      const uint32_t v = *reinterpret_cast<const uint32_t*>(row + a.term_off[q] + (int64_t)z * a.planeR);
#pragma unroll
      for (int b = 0; b < 4; ++b) sum[b] += a.term_sign[q] * (int)((v >> (8 * b)) & 0xffu);
    }
    uint32_t r4 = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int qq = (int)floorf((float)sum[b] * inv_pf);
      int r = sum[b] - qq * p;
      if (r < 0) r += p;
      if (r >= p) r -= p;
      r4 |= (uint32_t)r << (8 * b);
    }
    return r4;
  };
  for (int64_t i = blockIdx.y; i < a.m; i += gridDim.y) {
    const uint8_t* row = a.R + i * a.ldr + jc;
    uint32_t d[4][4];
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int q = 0; q < 4; ++q) d[it][q] = residues4(row, 4 * (zq + 4 * it) + q);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int zg = zq + 4 * it;
      if (zg >= nzg) break;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        uint32_t x = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) x |= ((d[it][q] >> (8 * b)) & 0xffu) << (8 * q);
        *reinterpret_cast<uint32_t*>(tile + (4 * c + b) * LS + 4 * zg) = x ^ 0x80808080u;
      }
    }
    __syncthreads();
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
        const int wd = 4 * g + lane / 16;
        if (wd < W) vs[o * W + wd] = crt_half_sums(x[0], x[1], x[2], x[3]);
      }
    }
    __syncthreads();
    if (jt < a.n) {
      uint64_t acc[W];
      crt_carry_halves<W>(reinterpret_cast<const int32_t*>(vs + threadIdx.x * W), t, acc);
      uint32_t y[W];
      const bool neg = crt_magnitude<W>(acc, t, rP, y);
      uint32_t* cw = a.C + i * a.ldc + jt;
      // C += (neg ? -Y : Y) at word_off, in two's complement over words_c words
      int64_t cy = 0;
      for (int w = a.word_off; w < a.words_c; ++w) {
        const int64_t yw = w - a.word_off < W ? (int64_t)y[w - a.word_off] : 0;
        if (yw == 0 && cy == 0 && w - a.word_off >= W) break;
        const int64_t cur = (int64_t)cw[(int64_t)w * a.pstride];
        const int64_t sres = neg ? cur - yw + cy : cur + yw + cy;
        cw[(int64_t)w * a.pstride] = (uint32_t)sres;
        cy = sres >> 32;  // -1, 0 or 1
      }
    }
    __syncthreads();  // the tile and the word sums are refilled for the next row
  }
}

// Residue planes of chunk sums: out (all N moduli) := the residues of the
// sum of the `nin` input chunks, each input's residue a signed byte of its
// class, the sum (|s| <= 8 128) brought into [-p/2, p/2] (256: -128 for
// 128, the same class); N planes of `plane` bytes per chunk.
__global__ __launch_bounds__(256) void int_sum_kernel(IntSumArgs a) {
  const int z = blockIdx.y;
  const int64_t e8 = (int64_t)blockIdx.x * 256 + threadIdx.x;  // 8 bytes per thread
  if (e8 * 8 >= a.plane) return;
  const int p = kCrtModuli[z];
  const float inv_pf = 1.0f / (float)p;
  int sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = 0; q < a.nin; ++q) {
    const uint64_t v = *reinterpret_cast<const uint64_t*>(a.base + ((int64_t)a.in[q] * a.N + z) * a.plane + 8 * e8);
#pragma unroll
    for (int b = 0; b < 8; ++b) sum[b] += (int)(int8_t)(uint8_t)(v >> (8 * b));
  }
  uint64_t packed = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int r = sum[b] - (int)rintf((float)sum[b] * inv_pf) * p;
    packed |= (uint64_t)(uint8_t)(int8_t)r << (8 * b);
  }
  *reinterpret_cast<uint64_t*>(a.base + ((int64_t)a.out * a.N + z) * a.plane + 8 * e8) = packed;
}

__global__ __launch_bounds__(256) void zero_u32_kernel(uint32_t* C, int words, int64_t pstride, int64_t m,
                                                       int64_t n, int64_t ldc) {
  const int64_t total = m * n;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int64_t off = (idx / n) * ldc + idx % n;
    for (int w = 0; w < words; ++w) C[(int64_t)w * pstride + off] = 0u;
  }
}

}  // namespace

hipError_t launch_int_residues(const IntResidueArgs& a, bool cols, hipStream_t s) {
  if (a.chunks < 1 || a.N < 1 || a.N > kCrtMaxModuli || a.Kp % 64 || a.Rp % 32) return hipErrorInvalidValue;
  if (a.chunk_words < 3 || a.chunk_words > kIntMaxChunkWords) return hipErrorInvalidValue;
  if (a.Rp <= 0 || a.Kp <= 0) return hipSuccess;
#define MPG_INT_RES(CW)                                                                                  \
  case CW:                                                                                               \
    if (!cols) {                                                                                         \
      const int64_t work = a.Rp * (a.Kp / 8);                                                            \
      hipLaunchKernelGGL((int_residue_kernel<false, CW>), dim3((unsigned)((work + 255) / 256)), dim3(256), \
                         0, s, a);                                                                       \
    } else {                                                                                             \
      if (a.Kp / 64 > 65535) return hipErrorInvalidValue;                                                \
      hipLaunchKernelGGL((int_residue_kernel<true, CW>), dim3((unsigned)(a.Rp / 32), (unsigned)(a.Kp / 64)), \
                         dim3(256), 0, s, a);                                                            \
    }                                                                                                    \
    break;
  switch (a.chunk_words) {
    MPG_INT_RES(3)
    MPG_INT_RES(4)
    MPG_INT_RES(5)
    default:
      return hipErrorInvalidValue;
  }
#undef MPG_INT_RES
  return hipGetLastError();
}

hipError_t launch_int_sum(const IntSumArgs& a, hipStream_t s) {
  if (a.nin < 1 || a.nin > kIntMaxSumInputs || a.N < 1 || a.N > kCrtMaxModuli || a.plane % 8)
    return hipErrorInvalidValue;
  if (a.plane <= 0) return hipSuccess;
  const int64_t blocks = (a.plane / 8 + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(int_sum_kernel, dim3((unsigned)blocks, (unsigned)a.N), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_int_accumulate(const IntAccumArgs& a, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0) return hipSuccess;
  if (a.ldr % 4 || a.ldr < a.n || a.nterms < 1 || a.nterms > kIntMaxTerms) return hipErrorInvalidValue;
  const int64_t gx = (a.n + 255) / 256;
  if (gx > 0x7fffffff) return hipErrorInvalidValue;
  // about 4096 workgroups, each walking several rows
  const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(a.m, 65535), (4096 + gx - 1) / gx));
  const dim3 grid((unsigned)gx, (unsigned)gy);
  switch (crt_words(a.N)) {
    case 4: hipLaunchKernelGGL(int_accumulate_kernel<4>, grid, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL(int_accumulate_kernel<6>, grid, dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL(int_accumulate_kernel<8>, grid, dim3(256), 0, s, a); break;
    case 10: hipLaunchKernelGGL(int_accumulate_kernel<10>, grid, dim3(256), 0, s, a); break;
    case 12: hipLaunchKernelGGL(int_accumulate_kernel<12>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* C, int words, int64_t pstride, int64_t m, int64_t n, int64_t ldc,
                           hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((m * n + 255) / 256, 65536);
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, words, pstride, m, n, ldc);
  return hipGetLastError();
}

}  // namespace mpg
