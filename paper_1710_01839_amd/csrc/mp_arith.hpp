// Device-side error-free transforms and multi-limb accumulation steps for
// gfx950 (FP64 VALU).  Built with -ffp-contract=off: every FMA below is
// written explicitly, nothing else is fused or reassociated.
//
// Conventions: u = 2^-53 (unit roundoff of binary64, round to nearest).
#pragma once
#include <hip/hip_runtime.h>

namespace mpg {

// Knuth TwoSum: s = fl(a + b), s + e == a + b exactly (6 FP64 ops).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  double x = a + b;
  double bv = x - a;
  double av = x - bv;
  e = (a - av) + (b - bv);
  s = x;
}

// Dekker FastTwoSum, exact when exponent(a) >= exponent(b) (3 ops).
__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
  double x = a + b;
  e = b - (x - a);
  s = x;
}

// TwoProduct on the FMA unit: p = fl(a b), p + e == a b exactly (2 ops).
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

// ---------------------------------------------------------------------
// Double-double accumulation step (the inner operation of Eq. (1) and
// Eq. (2)):  (hi, lo) += (ah + al)(bh + bl), 10 FP64 ops.
//
// hi carries the running sum of the rounded head products fl(ah bh); the
// TwoSum of hi and the product is exact, and its error term is formed with
// the product's own TwoProduct error folded in: with bv = fl(s - hi),
//     hi + ah bh == s + (hi - av) + (ah bh - bv)      (exact identity)
// and fma(ah, bh, -bv) rounds (ah bh - bv) once.  The cross terms
// ah bl + al bh go straight into lo with two FMAs; al bl (< 2^-106 |ab|)
// is dropped.  lo is a plain FP64 sum of quantities of size u |partial sum|,
// so its own rounding errors are O(u^2) times the partial sums of |a||b|;
// renormalising (hi, lo) with an exact TwoSum every 8 steps keeps lo small
// enough that the componentwise error stays below 26 l 2^-106 (|A||B|)_ij,
// inside the 8 l 2^-104 = 32 l 2^-106 bound.
// ---------------------------------------------------------------------
__device__ __forceinline__ void dd_madd(double& hi, double& lo, double ah, double al,
                                        double bh, double bl) {
  double p = ah * bh;
  lo = __builtin_fma(ah, bl, lo);
  lo = __builtin_fma(al, bh, lo);
  double s = hi + p;
  double bv = s - hi;
  double av = s - bv;
  double da = hi - av;
  double db = __builtin_fma(ah, bh, -bv);
  lo = lo + (da + db);
  hi = s;
}

// Renormalisation period of dd_madd (steps between exact TwoSums).
constexpr int kDDRenorm = 8;

__device__ __forceinline__ void dd_renorm(double& hi, double& lo) {
  double s, e;
  two_sum(hi, lo, s, e);
  hi = s;
  lo = e;
}

// Accurate DD sum (two TwoSums, two FastTwoSum renormalisations), used for
// the O(n^2) Strassen operand and assembly additions.
__device__ __forceinline__ void dd_add(double ah, double al, double bh, double bl, double& rh,
                                       double& rl) {
  double s, e, t, f;
  two_sum(ah, bh, s, e);
  two_sum(al, bl, t, f);
  e = e + t;
  fast_two_sum(s, e, s, e);
  e = e + f;
  fast_two_sum(s, e, rh, rl);
}

}  // namespace mpg

namespace mpg {

// TwoSum with the rounded product x*y as second operand and the product's
// own rounding error folded into the error term (7 ops):
//   S + x y == s + err + d,  |d| <= u |x y - bv|.
__device__ __forceinline__ void two_sum_prod(double S, double x, double y, double& s, double& err) {
  double p = x * y;
  double t = S + p;
  double bv = t - S;
  double av = t - bv;
  double da = S - av;
  double db = __builtin_fma(x, y, -bv);
  err = da + db;
  s = t;
}

// ---------------------------------------------------------------------
// Quad-double accumulation step: (s0, s1, s2, s3) += a b, a and b four
// non-overlapping limbs.  Level k of the accumulator holds terms of size
// about 2^(-53k) of the partial sum.  At each level the new terms whose size
// scales with |a b| are first combined among themselves with exact TwoSums,
// the terms that scale with the partial sum S join afterwards, and exactly
// one TwoSum touches the level's accumulator, so only O(1) terms of size
// u^k S reach level k + 1 per step.  Level 3 is a plain FP64 sum (its
// rounding errors are O(u^4 S)); a bottom-up VecSum after every step keeps
// |s_{k+1}| <= about u |s_k|.  124 FP64 ops.
// ---------------------------------------------------------------------
__device__ __forceinline__ void qd_madd(double (&s)[4], const double (&a)[4], const double (&b)[4]) {
  double p00, e00, q0;
  two_prod(a[0], b[0], p00, e00);
  two_sum(s[0], p00, s[0], q0);
  // level 1
  double p01, e01, p10, e10, x1, y1, x2, y2, x3, y3, y4;
  two_prod(a[0], b[1], p01, e01);
  two_prod(a[1], b[0], p10, e10);
  two_sum(p01, p10, x1, y1);
  two_sum(x1, e00, x2, y2);
  two_sum(q0, x2, x3, y3);
  two_sum(s[1], x3, s[1], y4);
  // level 2
  double z1, w1, z2, w2, z3, w3, z4, w4, z5, w5, z6, w6, z7, w7, z8, w8, w9;
  two_sum(y1, y2, z1, w1);
  two_sum(e01, e10, z2, w2);
  two_sum(z1, z2, z3, w3);
  two_sum_prod(z3, a[0], b[2], z4, w4);
  two_sum_prod(z4, a[1], b[1], z5, w5);
  two_sum_prod(z5, a[2], b[0], z6, w6);
  two_sum(y3, y4, z7, w7);
  two_sum(z6, z7, z8, w8);
  two_sum(s[2], z8, s[2], w9);
  // level 3
  double t = w1 + w2;
  t = t + w3;
  t = t + w4;
  t = t + w5;
  t = t + w6;
  t = __builtin_fma(a[0], b[3], t);
  t = __builtin_fma(a[1], b[2], t);
  t = __builtin_fma(a[2], b[1], t);
  t = __builtin_fma(a[3], b[0], t);
  t = t + w7;
  t = t + w8;
  t = t + w9;
  s[3] = s[3] + t;
  // bottom-up VecSum
  two_sum(s[2], s[3], s[2], s[3]);
  two_sum(s[1], s[2], s[1], s[2]);
  two_sum(s[0], s[1], s[0], s[1]);
}

// Final QD normalisation: a second bottom-up VecSum and a top-down pass.
__device__ __forceinline__ void qd_finish(double (&s)[4]) {
  two_sum(s[2], s[3], s[2], s[3]);
  two_sum(s[1], s[2], s[1], s[2]);
  two_sum(s[0], s[1], s[0], s[1]);
  two_sum(s[1], s[2], s[1], s[2]);
  two_sum(s[2], s[3], s[2], s[3]);
}

// Accurate QD sum for the O(n^2) Strassen additions: the eight limbs are
// merged by exact TwoSums (a VecSum network) and renormalised.
__device__ __forceinline__ void qd_add(const double (&a)[4], const double (&b)[4], double (&r)[4]) {
  double x[8] = {a[0], b[0], a[1], b[1], a[2], b[2], a[3], b[3]};
  // three bottom-up VecSum passes: afterwards x[k] is of size about u^k
  // (|a| + |b|) for k < 3 and the tail x[3..7] about 8 u^3 (|a| + |b|)
#pragma unroll
  for (int pass = 0; pass < 3; ++pass)
#pragma unroll
    for (int i = 7; i > 0; --i) two_sum(x[i - 1], x[i], x[i - 1], x[i]);
  // fold the tail into limb 3 (plain sum: rounding errors O(u^4))
  double t = x[7];
  t = t + x[6];
  t = t + x[5];
  t = t + x[4];
  double s[4] = {x[0], x[1], x[2], x[3] + t};
  qd_finish(s);
  r[0] = s[0]; r[1] = s[1]; r[2] = s[2]; r[3] = s[3];
}

// ---------------------------------------------------------------------
// Arithmetic policies used by the GEMM kernel templates.
// ---------------------------------------------------------------------
struct DDArith {
  static constexpr int L = 2;
  static constexpr int kRenorm = kDDRenorm;  // exact TwoSum every 8 steps
  __device__ static __forceinline__ void madd(double (&c)[2], const double (&a)[2],
                                              const double (&b)[2]) {
    dd_madd(c[0], c[1], a[0], a[1], b[0], b[1]);
  }
  // N independent steps c[j] += a * b[j], written stage by stage across j so
  // that consecutive instructions belong to different accumulators (each
  // accumulator sees exactly the operations of dd_madd, in the same order).
  // One wavefront then has N-way instruction-level parallelism to cover the
  // FP64 pipeline latency instead of one dependent chain.
  template <int N>
  __device__ static __forceinline__ void madd_row(double (*c)[2], const double (&a)[2],
                                                  const double (*b)[2]) {
    if constexpr (N > 4) {  // groups of four keep the temporaries in registers
      madd_row<4>(c, a, b);
      madd_row<N - 4>(c + 4, a, b + 4);
      return;
    }
    double p[N], s[N], t[N];
#pragma unroll
    for (int j = 0; j < N; ++j) p[j] = a[0] * b[j][0];
#pragma unroll
    for (int j = 0; j < N; ++j) c[j][1] = __builtin_fma(a[0], b[j][1], c[j][1]);
#pragma unroll
    for (int j = 0; j < N; ++j) s[j] = c[j][0] + p[j];
#pragma unroll
    for (int j = 0; j < N; ++j) c[j][1] = __builtin_fma(a[1], b[j][0], c[j][1]);
#pragma unroll
    for (int j = 0; j < N; ++j) t[j] = s[j] - c[j][0];                        // bv
#pragma unroll
    for (int j = 0; j < N; ++j) p[j] = __builtin_fma(a[0], b[j][0], -t[j]);   // db
#pragma unroll
    for (int j = 0; j < N; ++j) t[j] = s[j] - t[j];                           // av
#pragma unroll
    for (int j = 0; j < N; ++j) t[j] = c[j][0] - t[j];                        // da
#pragma unroll
    for (int j = 0; j < N; ++j) t[j] = t[j] + p[j];                           // da + db
#pragma unroll
    for (int j = 0; j < N; ++j) c[j][1] = c[j][1] + t[j];
#pragma unroll
    for (int j = 0; j < N; ++j) c[j][0] = s[j];
  }
  __device__ static __forceinline__ void renorm(double (&c)[2]) { dd_renorm(c[0], c[1]); }
  // exact TwoSum of N accumulators, interleaved like madd_row
  template <int N>
  __device__ static __forceinline__ void renorm_row(double (*c)[2]) {
    double s[N], bv[N], t[N];
#pragma unroll
    for (int j = 0; j < N; ++j) s[j] = c[j][0] + c[j][1];
#pragma unroll
    for (int j = 0; j < N; ++j) bv[j] = s[j] - c[j][0];
#pragma unroll
    for (int j = 0; j < N; ++j) t[j] = s[j] - bv[j];
#pragma unroll
    for (int j = 0; j < N; ++j) t[j] = c[j][0] - t[j];
#pragma unroll
    for (int j = 0; j < N; ++j) bv[j] = c[j][1] - bv[j];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      c[j][0] = s[j];
      c[j][1] = t[j] + bv[j];
    }
  }
  __device__ static __forceinline__ void finish(double (&c)[2]) { dd_renorm(c[0], c[1]); }
  __device__ static __forceinline__ void add(const double (&a)[2], const double (&b)[2],
                                             double (&r)[2]) {
    dd_add(a[0], a[1], b[0], b[1], r[0], r[1]);
  }
};

struct QDArith {
  static constexpr int L = 4;
  static constexpr int kRenorm = 0;  // renormalised inside every step
  __device__ static __forceinline__ void madd(double (&c)[4], const double (&a)[4],
                                              const double (&b)[4]) {
    qd_madd(c, a, b);
  }
  template <int N>
  __device__ static __forceinline__ void madd_row(double (*c)[4], const double (&a)[4],
                                                  const double (*b)[4]) {
#pragma unroll
    for (int j = 0; j < N; ++j) qd_madd(c[j], a, b[j]);
  }
  __device__ static __forceinline__ void renorm(double (&)[4]) {}
  template <int N>
  __device__ static __forceinline__ void renorm_row(double (*)[4]) {}
  __device__ static __forceinline__ void finish(double (&c)[4]) { qd_finish(c); }
  __device__ static __forceinline__ void add(const double (&a)[4], const double (&b)[4],
                                             double (&r)[4]) {
    qd_add(a, b, r);
  }
};

}  // namespace mpg
