// GEMM kernel templates shared by the DD and QD translation units:
// the simple algorithm (Eq. 1), the block algorithm (Eq. 2) as an
// LDS-staged register-blocked kernel, and the operand / assembly passes of
// Winograd's form of Strassen (Eq. 3).  `Arith` is DDArith or QDArith
// (mp_arith.hpp).
#pragma once
#include "internal.hpp"
#include "mp_arith.hpp"

namespace mpg {
namespace kern {

// The hardware deals workgroups round-robin over the 8 XCDs; remap the
// linear id so consecutive logical tiles run on one XCD and share its L2.
__device__ __forceinline__ int xcd_remap(int w, int total) {
  constexpr int X = 8;
  int q = total / X, r = total % X;
  int xcd = w % X, local = w / X;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Grouped tile order: 8 tile-rows are walked column by column so that the
// resident workgroups of an XCD reuse the same A row panels and B column
// panels from L2.
__device__ __forceinline__ void tile_coords(int t, int tiles_m, int tiles_n, int& tm, int& tn) {
  constexpr int G = 8;
  int per_group = G * tiles_n;
  int group = t / per_group;
  int first = group * G;
  int gsize = min(tiles_m - first, G);
  int in = t - group * per_group;
  tm = first + in % gsize;
  tn = in / gsize;
}

// ---------------------------------------------------------------------
// Simple algorithm, Eq. (1): one thread per c_ij, k in order.
// ---------------------------------------------------------------------
template <class Arith>
__global__ __launch_bounds__(256) void simple_kernel(GemmBatch g) {
  constexpr int L = Arith::L;
  const int p = blockIdx.z;
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (j >= g.n) return;
  for (int64_t i = (int64_t)blockIdx.y * 4 + threadIdx.y; i < g.m; i += (int64_t)gridDim.y * 4) {
    double acc[L];
#pragma unroll
    for (int q = 0; q < L; ++q) acc[q] = 0.0;
    for (int64_t k = 0; k < g.l; ++k) {
      double a[L], b[L];
#pragma unroll
      for (int q = 0; q < L; ++q) {
        a[q] = g.A[q][p * g.sA + i * g.lda + k];
        b[q] = g.B[q][p * g.sB + k * g.ldb + j];
      }
      Arith::madd(acc, a, b);
      if (Arith::kRenorm && (k % Arith::kRenorm) == Arith::kRenorm - 1) Arith::renorm(acc);
    }
    Arith::finish(acc);
#pragma unroll
    for (int q = 0; q < L; ++q) g.C[q][p * g.sC + i * g.ldc + j] = acc[q];
  }
}

template <class Arith>
hipError_t launch_simple(const GemmBatch& g, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || g.count <= 0) return hipSuccess;
  const int64_t gy = (g.m + 3) / 4;
  dim3 grid((unsigned)((g.n + 63) / 64), (unsigned)(gy < 65535 ? gy : 65535), (unsigned)g.count);
  hipLaunchKernelGGL(simple_kernel<Arith>, grid, dim3(64, 4), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Block algorithm, Eq. (2).  MINW is the minimum number of resident
// wavefronts per SIMD the register allocation must allow.  One workgroup computes a BM x BN tile of C
// and walks K in steps of BK.  Each step's A tile (BM x BK, row-major,
// rows padded by 2 doubles so that pairs of k stay 16-byte aligned and the
// rows of one wavefront fall in different LDS banks) and B tile (BK x BN)
// are staged in LDS for every limb plane, double-buffered: the next step's
// global loads are in flight while the current step is computed, and one
// barrier per step separates the two buffers.  Each thread owns a TM x TN
// block of accumulators in registers and performs the k-steps in order,
// so every c_ij sees exactly the operation sequence of the simple kernel
// (zero padding beyond l changes no accumulator).
// ---------------------------------------------------------------------
// LDS of one block-kernel workgroup (16-byte aligned: the k-pair reads are
// ds_read_b128).
template <int L, int BM, int BN, int BK>
struct alignas(16) BlockSmem {
  double A[2][L][BM * (BK + 2)];
  double B[2][L][BK * BN];
};

// One BM x BN output tile at (m0, n0) of the product C_p := A_p B_p whose
// limb planes start at Ap/Bp/Cp.  Called by every thread of the workgroup.
template <class Arith, int BM, int BN, int BK, int TM, int TN>
__device__ __forceinline__ void block_tile(BlockSmem<Arith::L, BM, BN, BK>& sm, int64_t m, int64_t n,
                                           int64_t l, const double* const* Ap, int64_t lda,
                                           const double* const* Bp, int64_t ldb,
                                           double* const* Cp, int64_t ldc, int64_t m0, int64_t n0) {
  constexpr int L = Arith::L;
  constexpr int NTX = BN / TN;
  constexpr int NTY = BM / TM;
  constexpr int NT = NTX * NTY;
  constexpr int LDS_A = BK + 2;
  constexpr int LA = BM * BK / NT;
  constexpr int LB = BK * BN / NT;
  static_assert(LA * NT == BM * BK && LB * NT == BK * BN, "tile not divisible by threads");
  static_assert(BK % 2 == 0 && TN % 2 == 0, "tile shape");
  static_assert(Arith::kRenorm == 0 || BK % Arith::kRenorm == 0, "renormalisation period");

  const int tid = threadIdx.x;
  const int tx = tid % NTX;
  const int ty = tid / NTX;

  double ra[L][LA], rb[L][LB];

  auto load_tile = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = tid + r * NT;
      const int row = e / BK, col = e % BK;
      const int64_t gi = m0 + row, gk = k0 + col;
      const bool ok = gi < m && gk < l;
      // always load (from element 0 when outside), then select: no branch,
      // so the loads stay in flight during the current step's arithmetic
      const int64_t off = ok ? gi * lda + gk : 0;
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const double v = Ap[q][off];
        ra[q][r] = ok ? v : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = tid + r * NT;
      const int row = e / BN, col = e % BN;
      const int64_t gk = k0 + row, gj = n0 + col;
      const bool ok = gk < l && gj < n;
      const int64_t off = ok ? gk * ldb + gj : 0;
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const double v = Bp[q][off];
        rb[q][r] = ok ? v : 0.0;
      }
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = tid + r * NT;
      const int row = e / BK, col = e % BK;
#pragma unroll
      for (int q = 0; q < L; ++q) sm.A[buf][q][row * LDS_A + col] = ra[q][r];
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = tid + r * NT;
#pragma unroll
      for (int q = 0; q < L; ++q) sm.B[buf][q][e] = rb[q][r];
    }
  };

  double acc[TM][TN][L];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < L; ++q) acc[i][j][q] = 0.0;

  const int numK = (int)((l + BK - 1) / BK);
  if (numK > 0) {
    load_tile(0);
    store_tile(0);
  }
  __syncthreads();

  for (int t = 0; t < numK; ++t) {
    const int cur = t & 1;
    if (t + 1 < numK) load_tile((int64_t)(t + 1) * BK);
    // One k-pair per iteration, not unrolled: a fully unrolled step lets the
    // compiler hoist the LDS reads of the whole tile and run out of
    // registers.  LDS latency is covered by the other resident wavefronts.
#pragma unroll 1
    for (int kp = 0; kp < BK; kp += 2) {
      double2 a2[TM][L];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int q = 0; q < L; ++q)
          a2[i][q] = *reinterpret_cast<const double2*>(&sm.A[cur][q][(ty * TM + i) * LDS_A + kp]);
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        double b[TN][L];
#pragma unroll
        for (int j = 0; j < TN; j += 2)
#pragma unroll
          for (int q = 0; q < L; ++q) {
            const double2 x =
                *reinterpret_cast<const double2*>(&sm.B[cur][q][(kp + kk) * BN + tx * TN + j]);
            b[j][q] = x.x;
            b[j + 1][q] = x.y;
          }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          double a[L];
#pragma unroll
          for (int q = 0; q < L; ++q) a[q] = kk ? a2[i][q].y : a2[i][q].x;
          Arith::template madd_row<TN>(acc[i], a, b);
        }
        if (Arith::kRenorm && ((kp + kk) % Arith::kRenorm) == Arith::kRenorm - 1) {
#pragma unroll
          for (int i = 0; i < TM; ++i) Arith::template renorm_row<TN>(acc[i]);
        }
      }
    }
    if (t + 1 < numK) store_tile(cur ^ 1);
    __syncthreads();
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
      for (int q = 0; q < L; ++q) Cp[q][gi * ldc + gj] = acc[i][j][q];
    }
  }
}

// Block algorithm, Eq. (2): one workgroup per output tile of one of
// g.count equal-shape problems.  MINW is the minimum number of resident
// wavefronts per SIMD the register allocation must allow.
template <class Arith, int BM, int BN, int BK, int TM, int TN, int MINW>
__global__ __launch_bounds__((BM / TM) * (BN / TN), MINW) void block_kernel(GemmBatch g, int tiles_m,
                                                                            int tiles_n) {
  constexpr int L = Arith::L;
  __shared__ BlockSmem<L, BM, BN, BK> sm;
  if (g.skip && *g.skip) return;
  const int per_problem = tiles_m * tiles_n;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int p = w / per_problem;
  int tm, tn;
  tile_coords(w - p * per_problem, tiles_m, tiles_n, tm, tn);
  const double* Ap[L];
  const double* Bp[L];
  double* Cp[L];
#pragma unroll
  for (int q = 0; q < L; ++q) {
    Ap[q] = g.A[q] + p * g.sA;
    Bp[q] = g.B[q] + p * g.sB;
    Cp[q] = g.C[q] + p * g.sC;
  }
  block_tile<Arith, BM, BN, BK, TM, TN>(sm, g.m, g.n, g.l, Ap, g.lda, Bp, g.ldb, Cp, g.ldc,
                                        (int64_t)tm * BM, (int64_t)tn * BN);
}

template <class Arith, int BM, int BN, int BK, int TM, int TN, int MINW = 2>
hipError_t launch_block(const GemmBatch& g, hipStream_t s) {
  const int64_t tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  const int64_t total = tiles_m * tiles_n * g.count;
  if (total <= 0) return hipSuccess;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  constexpr int NT = (BM / TM) * (BN / TN);
  hipLaunchKernelGGL((block_kernel<Arith, BM, BN, BK, TM, TN, MINW>), dim3((unsigned)total), dim3(NT), 0,
                     s, g, (int)tiles_m, (int)tiles_n);
  return hipGetLastError();
}

using LaunchFn = hipError_t (*)(const GemmBatch&, hipStream_t);
struct VariantEntry {
  TileVariant v;
  LaunchFn fn;
  const void* kernel;
};

template <class Arith, int BM, int BN, int BK, int TM, int TN, int MINW = 2>
constexpr VariantEntry variant_entry() {
  return VariantEntry{{BM, BN, BK, TM, TN, (BM / TM) * (BN / TN)},
                      launch_block<Arith, BM, BN, BK, TM, TN, MINW>,
                      reinterpret_cast<const void*>(&block_kernel<Arith, BM, BN, BK, TM, TN, MINW>)};
}

inline int resident_blocks(const VariantEntry& e) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, e.kernel, e.v.threads, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

// ---------------------------------------------------------------------
// Winograd operand formation and assembly (accurate multi-limb sums).
// ---------------------------------------------------------------------
template <class Arith>
__global__ __launch_bounds__(256) void form_kernel(FormArgs a) {
  constexpr int L = Arith::L;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y;
  if (idx >= a.h * a.w) return;
  const int64_t r = idx / a.w, c = idx % a.w;
  auto ld = [&](int64_t rr, int64_t cc, double (&v)[L]) {
    const bool ok = rr < a.vr && cc < a.vc;
#pragma unroll
    for (int q = 0; q < L; ++q) v[q] = ok ? a.par[q][p * a.s_par + rr * a.ld_par + cc] : 0.0;
  };
  auto sub = [&](const double (&x)[L], const double (&y)[L], double (&o)[L]) {
    double ny[L];
#pragma unroll
    for (int q = 0; q < L; ++q) ny[q] = -y[q];
    Arith::add(x, ny, o);
  };
  double x11[L], x12[L], x21[L], x22[L];
  ld(r, c, x11);
  ld(r, c + a.w, x12);
  ld(r + a.h, c, x21);
  ld(r + a.h, c + a.w, x22);
  double out[7][L];
  if (a.side == 0) {
    // S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2;
    // products A11 B11, A12 B21, S4 B22, A22 T4, S1 T1, S2 T2, S3 T3.
    double s1[L], s2[L], s3[L], s4[L];
    Arith::add(x21, x22, s1);
    sub(s1, x11, s2);
    sub(x11, x21, s3);
    sub(x12, s2, s4);
#pragma unroll
    for (int q = 0; q < L; ++q) {
      out[0][q] = x11[q]; out[1][q] = x12[q]; out[2][q] = s4[q]; out[3][q] = x22[q];
      out[4][q] = s1[q]; out[5][q] = s2[q]; out[6][q] = s3[q];
    }
  } else {
    // T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21.
    double t1[L], t2[L], t3[L], t4[L];
    sub(x12, x11, t1);
    sub(x22, t1, t2);
    sub(x22, x12, t3);
    sub(t2, x21, t4);
#pragma unroll
    for (int q = 0; q < L; ++q) {
      out[0][q] = x11[q]; out[1][q] = x21[q]; out[2][q] = x22[q]; out[3][q] = t4[q];
      out[4][q] = t1[q]; out[5][q] = t2[q]; out[6][q] = t3[q];
    }
  }
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    const int64_t off = (int64_t)(7 * p + o) * a.s_ch + idx;
#pragma unroll
    for (int q = 0; q < L; ++q) a.ch[q][off] = out[o][q];
  }
}

template <class Arith>
__global__ __launch_bounds__(256) void assemble_kernel(AssembleArgs a) {
  constexpr int L = Arith::L;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y;
  if (idx >= a.h * a.w) return;
  const int64_t r = idx / a.w, c = idx % a.w;
  double P[7][L];
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    const int64_t off = (int64_t)(7 * p + o) * a.s_ch + idx;
#pragma unroll
    for (int q = 0; q < L; ++q) P[o][q] = a.ch[q][off];
  }
  // C11 = P1 + P2; U2 = P1 + P6; U3 = U2 + P7; U4 = U2 + P5;
  // C12 = U4 + P3; C21 = U3 - P4; C22 = U3 + P5.
  double c11[L], u2[L], u3[L], u4[L], c12[L], c21[L], c22[L], n4[L];
  Arith::add(P[0], P[1], c11);
  Arith::add(P[0], P[5], u2);
  Arith::add(u2, P[6], u3);
  Arith::add(u2, P[4], u4);
  Arith::add(u4, P[2], c12);
#pragma unroll
  for (int q = 0; q < L; ++q) n4[q] = -P[3][q];
  Arith::add(u3, n4, c21);
  Arith::add(u3, P[4], c22);
  auto st = [&](int64_t rr, int64_t cc, const double (&v)[L]) {
    if (rr < a.vr && cc < a.vc) {
#pragma unroll
      for (int q = 0; q < L; ++q) a.par[q][p * a.s_par + rr * a.ld_par + cc] = v[q];
    }
  };
  st(r, c, c11);
  st(r, c + a.w, c12);
  st(r + a.h, c, c21);
  st(r + a.h, c + a.w, c22);
}

template <class Arith>
hipError_t launch_form(const FormArgs& a, hipStream_t s) {
  const int64_t n = a.h * a.w;
  if (n <= 0 || a.parents <= 0) return hipSuccess;
  hipLaunchKernelGGL(form_kernel<Arith>, dim3((unsigned)((n + 255) / 256), (unsigned)a.parents),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

template <class Arith>
hipError_t launch_assemble(const AssembleArgs& a, hipStream_t s) {
  const int64_t n = a.h * a.w;
  if (n <= 0 || a.parents <= 0) return hipSuccess;
  hipLaunchKernelGGL(assemble_kernel<Arith>, dim3((unsigned)((n + 255) / 256), (unsigned)a.parents),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace mpg
