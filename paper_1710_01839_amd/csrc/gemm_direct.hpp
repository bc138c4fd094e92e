// Block algorithm, Eq. (2), for double-double operands whose tiles are moved
// from global memory into LDS by the load unit itself (buffer_load ... lds,
// 16 bytes per lane), so no registers are spent on staging.  The registers
// saved hold the next k's fragments instead, so the LDS reads overlap the
// arithmetic, and four wavefronts per SIMD still fit.
//
// Tile 64 x 64 x 8, TM x 4 accumulators per thread (TM = 2: 512 threads;
// TM = 4: 256 threads), LDS double buffered (32 KB per workgroup).  Every
// c_ij sees the operation sequence of the simple kernel (k ascending,
// renormalisation every 8 steps), so the results are bit-identical to the
// register-staged block kernels.
//
// Requirements (checked by the launcher, which otherwise runs the
// register-staged 64 x 64 x 8 kernel): l, n, lda, ldb and the per-problem
// strides even, every limb plane 16-byte aligned, lda < 2^21, ldb < 2^24.
// Out-of-range chunks (rows >= m, columns >= n, k >= l) are zero-filled by
// the buffer range check.
#pragma once
#include "gemm_kernels.hpp"

namespace mpg {
namespace kern {

constexpr int kDirectBK = 8;

template <int L>
struct alignas(16) DirectSmem {
  // A tile: 64 rows x 8 k per limb, stored as 16-byte chunks (two k); the
  // chunk slot of row r is XOR-swizzled by (r / TM) mod 4, so the four rows
  // one wavefront reads at once fall in different LDS banks.
  double A[2][L][64 * 8];
  // B tile: 8 k x 64 columns per limb, row-major.
  double B[2][L][8 * 64];
};

using lds_ptr = __attribute__((address_space(3))) void*;

// Per-thread description of the chunks it moves each step.
template <int L>
struct DirectLoads {
  const double* a_tile[L];  // row m0 of A, all limbs
  const double* b_tile[L];  // column n0 of B, all limbs
  int64_t ldb;
  int chunk;                // LDS chunk index (0..255) this thread fills
  bool do_a, do_b;          // which operands this thread moves
  int a_off, b_off;         // byte offsets of the chunk inside the tile
  int ac, bkr;              // its k-pair (A) and k row (B) inside the step
  bool a_row_ok, b_col_ok;
};

// Moves one step's tiles (all limbs) into the LDS buffers nA / nB.  The
// buffer-load builtins exist only for the device; the host pass of this
// header sees an empty body.
template <int L>
__device__ __forceinline__ void direct_issue(double* __restrict__ nA, double* __restrict__ nB,
                                             const DirectLoads<L>& d, int64_t k0, int64_t l) {
#if defined(__HIP_DEVICE_COMPILE__)
  constexpr int kInvalid = (int)0x80000000;
  // raw (unstrided) buffer over `base`: word 3 is the gfx9 data format for
  // 32-bit elements; num_records only has to exceed every valid byte offset,
  // invalid chunks use offset 0x80000000, which the hardware range check
  // turns into zeros without touching memory
  auto rsrc = [](const double* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, 0x7ffffff0,
                                             0x00020000);
  };
  const int dst = (d.chunk >> 6) * 128;
  if (d.do_a) {
    const int ao = d.a_row_ok && k0 + 2 * d.ac < l ? d.a_off : kInvalid;
#pragma unroll
    for (int q = 0; q < L; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc(d.a_tile[q] + k0), (lds_ptr)(nA + q * 512 + dst), 16,
                                               ao, 0, 0, 0);
  }
  if (d.do_b) {
    const int bo = d.b_col_ok && k0 + d.bkr < l ? d.b_off : kInvalid;
#pragma unroll
    for (int q = 0; q < L; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc(d.b_tile[q] + k0 * d.ldb), (lds_ptr)(nB + q * 512 + dst),
                                               16, bo, 0, 0, 0);
  }
#endif
}

// One k-step: start moving the next step's tiles into (nA, nB), then the
// eight multiply-add steps on (cA, cB).  The two buffer pairs are distinct
// restrict pointers, so the compiler knows the reads of the current tiles
// need not wait for the loads into the next ones.
template <class Arith, int TM>
__device__ __forceinline__ void direct_step(double* __restrict__ nA, double* __restrict__ nB,
                                            const double* __restrict__ cA, const double* __restrict__ cB,
                                            double (&acc)[TM][4][Arith::L], bool more,
                                            const DirectLoads<Arith::L>& d, int64_t k1, int64_t l,
                                            int tx, int ty) {
  constexpr int L = Arith::L, BK = kDirectBK, BN = 64, TN = 4;
  if (more) direct_issue<L>(nA, nB, d, k1, l);
  const int swz = ty & 3;
  auto read = [&](int k, double (&a)[TM][L], double (&b)[TN][L]) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int q = 0; q < L; ++q)
        a[i][q] = cA[q * 512 + (ty * TM + i) * BK + 2 * ((k >> 1) ^ swz) + (k & 1)];
#pragma unroll
    for (int j = 0; j < TN; j += 2)
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const double2 x = *reinterpret_cast<const double2*>(&cB[q * 512 + k * BN + tx * TN + j]);
        b[j][q] = x.x;
        b[j + 1][q] = x.y;
      }
  };
  // fragments of k + 1 are read while k is computed (software pipeline);
  // the scheduling barrier keeps each k's arithmetic in one piece so the two
  // fragment sets are the only extra registers
  double a[2][TM][L], b[2][TN][L];
  read(0, a[0], b[0]);
#pragma unroll
  for (int k = 0; k < BK; ++k) {
    if (k + 1 < BK) read(k + 1, a[(k + 1) & 1], b[(k + 1) & 1]);
#pragma unroll
    for (int i = 0; i < TM; ++i) Arith::template madd_row<TN>(acc[i], a[k & 1][i], b[k & 1]);
    __builtin_amdgcn_sched_barrier(0);
  }
  // BK equals the renormalisation period: one exact TwoSum per step
#pragma unroll
  for (int i = 0; i < TM; ++i) Arith::template renorm_row<TN>(acc[i]);
}

template <int TM>
constexpr int direct_threads() {
  return 16 * (64 / TM);
}

template <class Arith, int TM, int MINW>
__global__ __launch_bounds__(direct_threads<TM>(), MINW) void direct_kernel(GemmBatch g, int tiles_m,
                                                                            int tiles_n) {
  constexpr int L = Arith::L;
  constexpr int BM = 64, BN = 64, BK = kDirectBK, TN = 4, NT = direct_threads<TM>();
  static_assert(NT == 256 || NT == 512, "one or two chunks of 256 per operand");
  __shared__ DirectSmem<L> sm;
  if (g.skip && *g.skip) return;
  const int per_problem = tiles_m * tiles_n;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int p = w / per_problem;
  int tmi, tni;
  tile_coords(w - p * per_problem, tiles_m, tiles_n, tmi, tni);
  const int64_t m0 = (int64_t)tmi * BM, n0 = (int64_t)tni * BN;
  const int64_t m = g.m, n = g.n, l = g.l;

  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;

  // LDS chunk `chunk` of A is row ar, k-pair ac (slot swizzled by the
  // reading rows' (ar / TM) mod 4); of B, k row bkr, column pair bc
  DirectLoads<L> d;
  d.chunk = tid & 255;
  d.do_a = NT == 256 || tid < 256;
  d.do_b = NT == 256 || tid >= 256;
  const int ar = d.chunk >> 2;
  d.ac = (d.chunk & 3) ^ ((ar / TM) & 3);
  d.bkr = d.chunk >> 5;
  const int bc = d.chunk & 31;
  d.a_row_ok = m0 + ar < m;
  d.b_col_ok = n0 + 2 * bc < n;
  d.a_off = (int)(ar * g.lda * 8 + d.ac * 16);
  d.b_off = (int)(d.bkr * g.ldb * 8 + bc * 16);
  d.ldb = g.ldb;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    d.a_tile[q] = g.A[q] + p * g.sA + m0 * g.lda;
    d.b_tile[q] = g.B[q] + p * g.sB + n0;
  }

  double acc[TM][TN][L];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < L; ++q) acc[i][j][q] = 0.0;

  const int numK = (int)((l + BK - 1) / BK);
  if (numK > 0) direct_issue<L>(&sm.A[0][0][0], &sm.B[0][0][0], d, 0, l);
  for (int t = 0; t < numK; ++t) {
    const int cur = t & 1;
    // this thread's loads into `cur` are done; after the barrier everyone's
    // are, and nobody reads `cur ^ 1` any more
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    direct_step<Arith, TM>(&sm.A[cur ^ 1][0][0], &sm.B[cur ^ 1][0][0], &sm.A[cur][0][0],
                           &sm.B[cur][0][0], acc, t + 1 < numK, d, (int64_t)(t + 1) * BK, l, tx, ty);
  }

#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int64_t gi = m0 + ty * TM + i;
    if (gi >= m) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t gj = n0 + tx * TN + j;
      if (gj >= n) continue;
      Arith::finish(acc[i][j]);
#pragma unroll
      for (int q = 0; q < L; ++q) g.C[q][p * g.sC + gi * g.ldc + gj] = acc[i][j][q];
    }
  }
}

// True when the operands meet the alignment and size limits of the direct
// kernel (byte offsets inside one tile, 64 rows of A or 8 rows of B, fit in
// 31 bits).
inline bool direct_ok(const GemmBatch& g, int L) {
  auto even = [](int64_t x) { return (x & 1) == 0; };
  bool ok = even(g.l) && even(g.n) && even(g.lda) && even(g.ldb) &&
            (g.count <= 1 || (even(g.sA) && even(g.sB))) && g.lda < (int64_t(1) << 21) &&
            g.ldb < (int64_t(1) << 24);
  for (int q = 0; q < L; ++q)
    ok = ok && (reinterpret_cast<uintptr_t>(g.A[q]) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(g.B[q]) & 15) == 0;
  return ok;
}

template <class Arith, int TM, int MINW>
hipError_t launch_direct(const GemmBatch& g, hipStream_t s) {
  if (!direct_ok(g, Arith::L)) return launch_block<Arith, 64, 64, 8, 4, 4>(g, s);
  const int64_t tiles_m = (g.m + 63) / 64, tiles_n = (g.n + 63) / 64;
  const int64_t total = tiles_m * tiles_n * g.count;
  if (total <= 0) return hipSuccess;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((direct_kernel<Arith, TM, MINW>), dim3((unsigned)total),
                     dim3(direct_threads<TM>()), 0, s, g, (int)tiles_m, (int)tiles_n);
  return hipGetLastError();
}

template <class Arith, int TM, int MINW>
constexpr VariantEntry direct_entry() {
  return VariantEntry{{64, 64, kDirectBK, TM, 4, direct_threads<TM>()},
                      launch_direct<Arith, TM, MINW>,
                      reinterpret_cast<const void*>(&direct_kernel<Arith, TM, MINW>)};
}

}  // namespace kern
}  // namespace mpg
