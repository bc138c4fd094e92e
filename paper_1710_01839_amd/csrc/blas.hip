// Kernels of the BLAS-style surface C := alpha op(A) op(B) + beta C around
// the product kernels: operand packing (copy, transpose, sign) and the
// scaling epilogues.  All of them are O(n^2) and bound by HBM bandwidth.
//
// pack_kernel moves 64 x 64 tiles: a plain copy reads and writes rows
// directly; a transposing copy reads rows of the source into LDS (row pitch
// 65 doubles, so the column reads that follow touch distinct banks) and
// writes rows of the destination, both sides coalesced.
//
// The epilogues evaluate, per element, a short dot product of scalars and
// matrix entries with the accumulation step of the product kernels (DD:
// dd_madd and one renormalisation; QD: qd_madd and qd_finish), so their
// rounding error obeys the same componentwise bound per term.
#include "blas_internal.hpp"
#include "mp_arith.hpp"

namespace mpg {
namespace {

constexpr int kTile = 64;
constexpr int kRowsPerPass = 4;  // 256 threads = 64 columns x 4 rows

__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
  __shared__ double tile[kTile][kTile + 1];
  const PackJob& J = a.job[blockIdx.z];
  const int64_t c0 = (int64_t)blockIdx.x * kTile;
  if (c0 >= J.cols) return;  // uniform over the workgroup
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  for (int64_t r0 = (int64_t)blockIdx.y * kTile; r0 < J.rows; r0 += (int64_t)gridDim.y * kTile) {
    if (!J.trans) {
      for (int i = ty; i < kTile; i += kRowsPerPass) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < J.rows && c < J.cols) J.dst[r * J.ldd + c] = J.sign * J.src[r * J.lds + c];
      }
    } else {
      // destination (r, c) is source (c, r): stage source rows c0.. c0+63,
      // columns r0 .. r0+63
      for (int i = ty; i < kTile; i += kRowsPerPass) {
        const int64_t sr = c0 + i, sc = r0 + tx;
        if (sr < J.cols && sc < J.rows) tile[i][tx] = J.src[sr * J.lds + sc];
      }
      __syncthreads();
      for (int i = ty; i < kTile; i += kRowsPerPass) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < J.rows && c < J.cols) J.dst[r * J.ldd + c] = J.sign * tile[tx][i];
      }
      __syncthreads();
    }
  }
}

// C := alpha T + beta C (L limbs); T is skipped when use_t == 0 and C is not
// read when use_c == 0.
template <int L>
__global__ __launch_bounds__(256) void axpby_kernel(AxpbyArgs a) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  double al[L], be[L];
#pragma unroll
  for (int q = 0; q < L; ++q) {
    al[q] = a.alpha[q];
    be[q] = a.beta[q];
  }
  for (int64_t i = blockIdx.y; i < a.m; i += gridDim.y) {
    const int64_t ot = i * a.ldt + j, oc = i * a.ldc + j;
    double t[L], c[L];
#pragma unroll
    for (int q = 0; q < L; ++q) {
      t[q] = a.use_t ? a.T[q][ot] : 0.0;
      c[q] = a.use_c ? a.C[q][oc] : 0.0;
    }
    if constexpr (L == 2) {
      double hi = 0.0, lo = 0.0;
      if (a.use_t) dd_madd(hi, lo, al[0], al[1], t[0], t[1]);
      if (a.use_c) dd_madd(hi, lo, be[0], be[1], c[0], c[1]);
      dd_renorm(hi, lo);
      a.C[0][oc] = hi;
      a.C[1][oc] = lo;
    } else {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
      if (a.use_t) qd_madd(s, al, t);
      if (a.use_c) qd_madd(s, be, c);
      qd_finish(s);
#pragma unroll
      for (int q = 0; q < 4; ++q) a.C[q][oc] = s[q];
    }
  }
}

// Complex DD: P holds [Re | Im] of the product side by side (row i: real
// parts at columns 0..n-1, imaginary parts at n..2n-1), C is split into
// (re hi, re lo, im hi, im lo) planes; alpha and beta likewise.
//   Re C' = ar Pr - ai Pi + br Cr - bi Ci,  Im C' = ar Pi + ai Pr + br Ci + bi Cr.
__global__ __launch_bounds__(256) void zaxpby_kernel(ZAxpbyArgs a) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  const double arh = a.alpha[0], arl = a.alpha[1], aih = a.alpha[2], ail = a.alpha[3];
  const double brh = a.beta[0], brl = a.beta[1], bih = a.beta[2], bil = a.beta[3];
  for (int64_t i = blockIdx.y; i < a.m; i += gridDim.y) {
    const int64_t op = i * a.ldp + j, oc = i * a.ldc + j;
    double rh = 0.0, rl = 0.0, ih = 0.0, il = 0.0;
    if (a.use_p) {
      const double prh = a.P[0][op], prl = a.P[1][op];
      const double pih = a.P[0][op + a.n], pil = a.P[1][op + a.n];
      dd_madd(rh, rl, arh, arl, prh, prl);
      dd_madd(rh, rl, -aih, -ail, pih, pil);
      dd_madd(ih, il, arh, arl, pih, pil);
      dd_madd(ih, il, aih, ail, prh, prl);
    }
    if (a.use_c) {
      const double crh = a.C[0][oc], crl = a.C[1][oc], cih = a.C[2][oc], cil = a.C[3][oc];
      dd_madd(rh, rl, brh, brl, crh, crl);
      dd_madd(rh, rl, -bih, -bil, cih, cil);
      dd_madd(ih, il, brh, brl, cih, cil);
      dd_madd(ih, il, bih, bil, crh, crl);
    }
    dd_renorm(rh, rl);
    dd_renorm(ih, il);
    a.C[0][oc] = rh;
    a.C[1][oc] = rl;
    a.C[2][oc] = ih;
    a.C[3][oc] = il;
  }
}

dim3 elementwise_grid(int64_t m, int64_t n) {
  const int64_t gx = (n + 255) / 256;
  const int64_t gy = m < 65535 ? m : 65535;
  return dim3((unsigned)gx, (unsigned)gy);
}

}  // namespace

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  if (a.count <= 0 || a.count > kMaxPackJobs) return hipErrorInvalidValue;
  int64_t rows = 0, cols = 0;
  for (int k = 0; k < a.count; ++k) {
    rows = a.job[k].rows > rows ? a.job[k].rows : rows;
    cols = a.job[k].cols > cols ? a.job[k].cols : cols;
  }
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t gx = (cols + kTile - 1) / kTile, gy0 = (rows + kTile - 1) / kTile;
  const int64_t gy = gy0 < 65535 ? gy0 : 65535;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)gx, (unsigned)gy, (unsigned)a.count), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

hipError_t launch_axpby(int limbs, const AxpbyArgs& a, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0) return hipSuccess;
  if (limbs == 2)
    hipLaunchKernelGGL(axpby_kernel<2>, elementwise_grid(a.m, a.n), dim3(256), 0, s, a);
  else if (limbs == 4)
    hipLaunchKernelGGL(axpby_kernel<4>, elementwise_grid(a.m, a.n), dim3(256), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_zaxpby(const ZAxpbyArgs& a, hipStream_t s) {
  if (a.m <= 0 || a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zaxpby_kernel, elementwise_grid(a.m, a.n), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mpg
