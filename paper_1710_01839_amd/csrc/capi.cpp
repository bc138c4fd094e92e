// C ABI of libmpgemm: context, argument validation, workspace, kernel
// timing and the host side of the algorithms (Strassen recursion driver).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpgemm.h"
#include "capi_internal.hpp"
#include "internal.hpp"
#include "splitk_internal.hpp"

using namespace mpg;

// ---------------------------------------------------------------------------
// context helpers
// ---------------------------------------------------------------------------

int mpg_fail(mpg_ctx* c, int status, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->last_error = buf;
  }
  return status;
}

int mpg_hip_fail(mpg_ctx* c, hipError_t e, const char* where) {
  return mpg_fail(c, MPG_ERR_HIP, "%s: %s (%s)", where, hipGetErrorName(e), hipGetErrorString(e));
}

int mpg_device_guard(mpg_ctx* c) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return mpg_hip_fail(c, e, "hipGetDevice");
  if (cur != c->device) {
    e = hipSetDevice(c->device);
    if (e != hipSuccess) return mpg_hip_fail(c, e, "hipSetDevice");
  }
  return MPG_OK;
}

int mpg_workspace(mpg_ctx* c, int slot, size_t bytes, void** out) {
  if (bytes == 0) {
    *out = nullptr;
    return MPG_OK;
  }
  if (bytes > c->ws_size[slot]) {
    if (c->ws[slot]) {
      hipError_t e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return mpg_hip_fail(c, e, "hipStreamSynchronize (workspace)");
      (void)hipFree(c->ws[slot]);
      c->ws[slot] = nullptr;
      c->ws_size[slot] = 0;
    }
    void* p = nullptr;
    const bool injected = c->fail_allocs > 0;
    if (injected) --c->fail_allocs;
    if (injected || hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return mpg_fail(c, MPG_ERR_NOMEM, "workspace allocation of %zu bytes failed", bytes);
    }
    c->ws[slot] = p;
    c->ws_size[slot] = bytes;
  }
  *out = c->ws[slot];
  return MPG_OK;
}

static hipEvent_t prof_event(mpg_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static int prof_resolve(mpg_ctx* c) {
  for (auto& r : c->prof_recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return mpg_hip_fail(c, e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return mpg_hip_fail(c, e, "hipEventElapsedTime");
    c->prof_ms[r.kclass] += ms;
    c->prof_n[r.kclass] += 1;
    c->event_pool.push_back(r.a);
    c->event_pool.push_back(r.b);
  }
  c->prof_recs.clear();
  return MPG_OK;
}

int mpg_launch(mpg_ctx* c, int kclass, const std::function<hipError_t()>& fn, const char* what) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c->prof) {
    a = prof_event(c);
    b = prof_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
  }
  hipError_t e;
  if (c->fail_launches > 0) {
    --c->fail_launches;
    e = hipErrorLaunchFailure;  // injected: nothing is launched
  } else {
    e = fn();
  }
  if (c->prof && a && b) {
    (void)hipEventRecord(b, c->stream);
    c->prof_recs.push_back({kclass, a, b});
    if (c->prof_recs.size() > 4096) {
      int st = prof_resolve(c);
      if (st != MPG_OK) return st;
    }
  }
  if (e != hipSuccess) return mpg_hip_fail(c, e, what);
  return MPG_OK;
}

bool mpg_overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b || abytes == 0 || bbytes == 0) return false;
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bbytes && y < x + abytes;
}

size_t mpg_span_bytes(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)((rows - 1) * ld + cols) * sizeof(double);
}

int mpg_check_gemm_args(mpg_ctx* c, int limbs, int64_t m, int64_t n, int64_t l,
                        const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
                        double* const* C, int64_t ldc) {
  if (m < 0 || n < 0 || l < 0) return mpg_fail(c, MPG_ERR_ARG, "negative dimension");
  if (m > (int64_t)1 << 31 || n > (int64_t)1 << 31 || l > (int64_t)1 << 31)
    return mpg_fail(c, MPG_ERR_ARG, "dimension too large");
  if (m == 0 || n == 0) return MPG_OK;
  if (ldc < std::max<int64_t>(1, n)) return mpg_fail(c, MPG_ERR_ARG, "ldc < n");
  for (int q = 0; q < limbs; ++q)
    if (!C[q]) return mpg_fail(c, MPG_ERR_ARG, "C limb %d is NULL", q);
  if (l == 0) return MPG_OK;
  if (lda < std::max<int64_t>(1, l)) return mpg_fail(c, MPG_ERR_ARG, "lda < l");
  if (ldb < std::max<int64_t>(1, n)) return mpg_fail(c, MPG_ERR_ARG, "ldb < n");
  for (int q = 0; q < limbs; ++q) {
    if (!A[q]) return mpg_fail(c, MPG_ERR_ARG, "A limb %d is NULL", q);
    if (!B[q]) return mpg_fail(c, MPG_ERR_ARG, "B limb %d is NULL", q);
  }
  const size_t sa = mpg_span_bytes(m, l, lda), sb = mpg_span_bytes(l, n, ldb),
               sc = mpg_span_bytes(m, n, ldc);
  for (int q = 0; q < limbs; ++q)
    for (int r = 0; r < limbs; ++r) {
      if (mpg_overlaps(C[q], sc, A[r], sa) || mpg_overlaps(C[q], sc, B[r], sb))
        return mpg_fail(c, MPG_ERR_ALIAS, "C limb %d overlaps an input", q);
      if (q < r && mpg_overlaps(C[q], sc, C[r], sc))
        return mpg_fail(c, MPG_ERR_ALIAS, "C limbs %d and %d overlap", q, r);
    }
  return MPG_OK;
}

// Resolve a tile request against the built variants of a precision.
int mpg_resolve_variant(mpg_ctx* c, int precision, const mpg_tile* t, int* variant) {
  *variant = precision == 2 ? dd_default_variant() : 0;
  if (!t || (t->bm == 0 && t->bn == 0 && t->bk == 0 && t->tm == 0 && t->tn == 0)) return MPG_OK;
  const int nv = mpg_num_variants(precision);
  for (int v = 0; v < nv; ++v) {
    mpg_tile x;
    mpg_variant(precision, v, &x);
    if ((t->bm == 0 || t->bm == x.bm) && (t->bn == 0 || t->bn == x.bn) &&
        (t->bk == 0 || t->bk == x.bk) && (t->tm == 0 || t->tm == x.tm) &&
        (t->tn == 0 || t->tn == x.tn)) {
      *variant = v;
      return MPG_OK;
    }
  }
  return mpg_fail(c, MPG_ERR_UNSUPPORTED, "no built %s block variant %dx%dx%d/%dx%d",
                  precision == 4 ? "QD" : "DD", t->bm, t->bn, t->bk, t->tm, t->tn);
}

// ---------------------------------------------------------------------------
// public: context
// ---------------------------------------------------------------------------

extern "C" int mpg_create(mpg_ctx** ctx, int device) {
  if (!ctx) return MPG_ERR_ARG;
  *ctx = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return MPG_ERR_HIP;
  if (device < 0 || device >= count) return MPG_ERR_ARG;
  mpg_ctx* c = new (std::nothrow) mpg_ctx();
  if (!c) return MPG_ERR_NOMEM;
  c->device = device;
  c->stream = nullptr;
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    delete c;
    return MPG_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
  mpg_noalloc_setup(device);
  *ctx = c;
  return MPG_OK;
}

extern "C" int mpg_destroy(mpg_ctx* c) {
  if (!c) return MPG_OK;
  (void)mpg_device_guard(c);
  (void)hipStreamSynchronize(c->stream);
  mpg_destroy_cached(c);
  for (int s = 0; s < mpg_ctx::kSlots; ++s)
    if (c->ws[s]) (void)hipFree(c->ws[s]);
  for (int k = 0; k < 2; ++k) {
    if (c->batch_pin[k]) (void)hipHostFree(c->batch_pin[k]);
    if (c->batch_done[k]) (void)hipEventDestroy(c->batch_done[k]);
  }
  for (auto& r : c->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  delete c;
  return MPG_OK;
}

extern "C" int mpg_set_stream(mpg_ctx* c, void* s) {
  if (!c) return MPG_ERR_ARG;
  c->stream = (hipStream_t)s;
  return MPG_OK;
}

extern "C" const char* mpg_status_string(int s) {
  switch (s) {
    case MPG_OK: return "MPG_OK";
    case MPG_ERR_ARG: return "MPG_ERR_ARG: invalid argument";
    case MPG_ERR_UNSUPPORTED: return "MPG_ERR_UNSUPPORTED: combination not built";
    case MPG_ERR_HIP: return "MPG_ERR_HIP: HIP runtime error";
    case MPG_ERR_NOMEM: return "MPG_ERR_NOMEM: allocation failed";
    case MPG_ERR_ALIAS: return "MPG_ERR_ALIAS: output overlaps an input";
    case MPG_ERR_STATE: return "MPG_ERR_STATE: object in the wrong state";
    default: return "unknown mpg status";
  }
}

extern "C" const char* mpg_last_error(const mpg_ctx* c) {
  return c ? c->last_error.c_str() : "no context";
}

extern "C" int mpg_num_variants(int precision) {
  if (precision == 2) return dd_num_variants();
  if (precision == 4) return qd_num_variants();
  return 0;
}

extern "C" int mpg_variant(int precision, int index, mpg_tile* t) {
  if (!t || index < 0 || index >= mpg_num_variants(precision)) return MPG_ERR_ARG;
  const TileVariant& v = precision == 2 ? dd_variant(index) : qd_variant(index);
  std::memset(t, 0, sizeof *t);
  t->bm = v.bm;
  t->bn = v.bn;
  t->bk = v.bk;
  t->tm = v.tm;
  t->tn = v.tn;
  return MPG_OK;
}

extern "C" int mpg_test_inject(mpg_ctx* c, int kind, int count) {
  if (!c || count < 0 || (kind != 1 && kind != 2)) return MPG_ERR_ARG;
  if (kind == 1)
    c->fail_allocs = count;
  else
    c->fail_launches = count;
  return MPG_OK;
}

extern "C" int mpg_variant_resident(mpg_ctx* c, int precision, int index, int* blocks) {
  if (!c || !blocks || index < 0 || index >= mpg_num_variants(precision)) return MPG_ERR_ARG;
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  *blocks = precision == 2 ? dd_variant_resident(index) : qd_variant_resident(index);
  return MPG_OK;
}

extern "C" int mpg_prof_enable(mpg_ctx* c, int on) {
  if (!c) return MPG_ERR_ARG;
  int st = prof_resolve(c);
  for (int k = 0; k < MPG_KCLASS_COUNT; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  c->prof = on != 0;
  return st;
}

extern "C" int mpg_prof_read(mpg_ctx* c, int kclass, double* total_ms, int64_t* launches) {
  if (!c || kclass < 0 || kclass >= MPG_KCLASS_COUNT) return MPG_ERR_ARG;
  int st = prof_resolve(c);
  if (st != MPG_OK) return st;
  if (total_ms) *total_ms = c->prof_ms[kclass];
  if (launches) *launches = c->prof_n[kclass];
  return MPG_OK;
}

// ---------------------------------------------------------------------------
// Strassen (Winograd form) driver, shared by DD and QD
// ---------------------------------------------------------------------------

static int64_t ipow7(int d) {
  int64_t r = 1;
  while (d-- > 0) r *= 7;
  return r;
}

int mpg_strassen(mpg_ctx* c, int limbs, int depth, int variant, int64_t m, int64_t n, int64_t l,
                 const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
                 double* const* C, int64_t ldc) {
  if (depth < 1 || depth > 3) return mpg_fail(c, MPG_ERR_ARG, "Strassen depth must be 1..3");
  const int64_t q = (int64_t)1 << depth;
  const int64_t M = (m + q - 1) / q * q, N = (n + q - 1) / q * q, K = (l + q - 1) / q * q;
  // workspace: per level j = 1..depth, A_j, B_j and P_j operand sets.
  struct Level {
    int64_t cnt, mr, kc, nc;  // count, rows of A_j / P_j, cols of A_j (= rows of B_j), cols of B_j
    size_t offA, offB, offP;
  };
  std::vector<Level> L(depth + 1);
  size_t elems = 0;
  for (int j = 1; j <= depth; ++j) {
    Level& v = L[j];
    v.cnt = ipow7(j);
    v.mr = M >> j;
    v.kc = K >> j;
    v.nc = N >> j;
    v.offA = elems;
    elems += (size_t)(v.cnt * v.mr * v.kc);
    v.offB = elems;
    elems += (size_t)(v.cnt * v.kc * v.nc);
    v.offP = elems;
    elems += (size_t)(v.cnt * v.mr * v.nc);
  }
  void* ws = nullptr;
  int st = mpg_workspace(c, 0, elems * limbs * sizeof(double), &ws);
  if (st != MPG_OK) return st;
  double* base = (double*)ws;
  auto plane = [&](size_t off, int q_) { return base + (size_t)q_ * elems + off; };

  auto form = limbs == 2 ? launch_dd_winograd_form : launch_qd_winograd_form;
  auto assemble = limbs == 2 ? launch_dd_winograd_assemble : launch_qd_winograd_assemble;

  // operand formation, top down
  for (int j = 1; j <= depth; ++j) {
    const Level& v = L[j];
    for (int side = 0; side < 2; ++side) {
      FormArgs f{};
      f.side = side;
      f.parents = (int)ipow7(j - 1);
      if (side == 0) {
        f.h = v.mr;
        f.w = v.kc;
      } else {
        f.h = v.kc;
        f.w = v.nc;
      }
      if (j == 1) {
        for (int q_ = 0; q_ < limbs; ++q_) f.par[q_] = side == 0 ? A[q_] : B[q_];
        f.ld_par = side == 0 ? lda : ldb;
        f.s_par = 0;
        f.vr = side == 0 ? m : l;
        f.vc = side == 0 ? l : n;
      } else {
        const Level& u = L[j - 1];
        for (int q_ = 0; q_ < limbs; ++q_) f.par[q_] = plane(side == 0 ? u.offA : u.offB, q_);
        f.ld_par = side == 0 ? u.kc : u.nc;
        f.s_par = side == 0 ? u.mr * u.kc : u.kc * u.nc;
        f.vr = side == 0 ? u.mr : u.kc;
        f.vc = side == 0 ? u.kc : u.nc;
      }
      for (int q_ = 0; q_ < limbs; ++q_) f.ch[q_] = plane(side == 0 ? v.offA : v.offB, q_);
      f.s_ch = f.h * f.w;
      st = mpg_launch(c, MPG_KCLASS_AUX, [&] { return form(f, c->stream); }, "Strassen operands");
      if (st != MPG_OK) return st;
    }
  }
  // all 7^depth leaf products in one grouped launch
  {
    const Level& v = L[depth];
    GemmBatch g{};
    g.m = v.mr;
    g.n = v.nc;
    g.l = v.kc;
    for (int q_ = 0; q_ < limbs; ++q_) {
      g.A[q_] = plane(v.offA, q_);
      g.B[q_] = plane(v.offB, q_);
      g.C[q_] = plane(v.offP, q_);
    }
    g.lda = v.kc;
    g.sA = v.mr * v.kc;
    g.ldb = v.nc;
    g.sB = v.kc * v.nc;
    g.ldc = v.nc;
    g.sC = v.mr * v.nc;
    g.count = (int)v.cnt;
    auto gemm = limbs == 2 ? launch_dd_block : launch_qd_block;
    st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return gemm(variant, g, c->stream); },
                    "Strassen leaf products");
    if (st != MPG_OK) return st;
  }
  // assembly, bottom up
  for (int j = depth; j >= 1; --j) {
    const Level& v = L[j];
    AssembleArgs a{};
    a.parents = (int)ipow7(j - 1);
    a.h = v.mr;
    a.w = v.nc;
    for (int q_ = 0; q_ < limbs; ++q_) a.ch[q_] = plane(v.offP, q_);
    a.s_ch = v.mr * v.nc;
    if (j == 1) {
      for (int q_ = 0; q_ < limbs; ++q_) a.par[q_] = C[q_];
      a.ld_par = ldc;
      a.s_par = 0;
      a.vr = m;
      a.vc = n;
    } else {
      const Level& u = L[j - 1];
      for (int q_ = 0; q_ < limbs; ++q_) a.par[q_] = plane(u.offP, q_);
      a.ld_par = u.nc;
      a.s_par = u.mr * u.nc;
      a.vr = u.mr;
      a.vc = u.nc;
    }
    st = mpg_launch(c, MPG_KCLASS_AUX, [&] { return assemble(a, c->stream); },
                    "Strassen assembly");
    if (st != MPG_OK) return st;
  }
  return MPG_OK;
}

// ---------------------------------------------------------------------------
// split-K driver (skinny shapes), shared by DD and QD
// ---------------------------------------------------------------------------

void mpg_splitk_plan(int64_t m, int64_t n, int64_t l, int bm, int bn, int bk, int resident, int num_cu,
                     int splits, int64_t* P, int64_t* Kc) {
  int64_t p = splits;
  if (p <= 0) {
    // enough chunks for two waves of resident workgroups, chunks of >= 256
    const int64_t tiles = ((m + bm - 1) / bm) * ((n + bn - 1) / bn);
    const int64_t target = 2 * (int64_t)std::max(num_cu, 1) * std::max(resident, 1);
    p = std::min((target + tiles - 1) / tiles, l / 256);
  }
  p = std::max<int64_t>(1, std::min(p, l));
  // chunk length: a multiple of the K step, so every chunk but the last is
  // whole K steps
  int64_t kc = (l + p - 1) / p;
  kc = (kc + bk - 1) / bk * bk;
  *Kc = kc;
  *P = (l + kc - 1) / kc;
}

int mpg_splitk(mpg_ctx* c, int limbs, int splits, int variant, int64_t m, int64_t n, int64_t l,
               const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
               double* const* C, int64_t ldc) {
  if (splits < 0) return mpg_fail(c, MPG_ERR_ARG, "splits must be >= 0");
  const TileVariant& tv = limbs == 2 ? dd_variant(variant) : qd_variant(variant);
  const int resident = limbs == 2 ? dd_variant_resident(variant) : qd_variant_resident(variant);
  int64_t P = 1, Kc = l;
  mpg_splitk_plan(m, n, l, tv.bm, tv.bn, tv.bk, resident, c->num_cu, splits, &P, &Kc);
  auto gemm = limbs == 2 ? launch_dd_block : launch_qd_block;
  GemmBatch g{};
  g.m = m;
  g.n = n;
  g.count = 1;
  if (P <= 1) {  // one chunk: the block kernel straight into C
    g.l = l;
    for (int q = 0; q < limbs; ++q) {
      g.A[q] = A[q];
      g.B[q] = B[q];
      g.C[q] = C[q];
    }
    g.lda = lda;
    g.ldb = ldb;
    g.ldc = ldc;
    return mpg_launch(c, MPG_KCLASS_GEMM, [&] { return gemm(variant, g, c->stream); }, "block kernel");
  }
  const size_t plane = (size_t)(m * n) * (size_t)P;
  void* ws = nullptr;
  int st = mpg_workspace(c, 9, plane * limbs * sizeof(double), &ws);
  if (st != MPG_OK) return st;
  double* W[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int q = 0; q < limbs; ++q) W[q] = (double*)ws + (size_t)q * plane;
  const int64_t full = l / Kc, tail = l - full * Kc;
  // the whole chunks as one grouped launch: problem p reads columns
  // [p Kc, (p + 1) Kc) of A and those rows of B, and writes partial p
  g.l = Kc;
  g.lda = lda;
  g.sA = Kc;
  g.ldb = ldb;
  g.sB = Kc * ldb;
  g.ldc = n;
  g.sC = m * n;
  g.count = (int)full;
  for (int q = 0; q < limbs; ++q) {
    g.A[q] = A[q];
    g.B[q] = B[q];
    g.C[q] = W[q];
  }
  if (full > 0 &&
      (st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return gemm(variant, g, c->stream); }, "split-K chunks")) !=
          MPG_OK)
    return st;
  if (tail > 0) {  // the shorter last chunk
    g.l = tail;
    g.count = 1;
    for (int q = 0; q < limbs; ++q) {
      g.A[q] = A[q] + full * Kc;
      g.B[q] = B[q] + full * Kc * ldb;
      g.C[q] = W[q] + (size_t)full * (size_t)(m * n);
    }
    if ((st = mpg_launch(c, MPG_KCLASS_GEMM, [&] { return gemm(variant, g, c->stream); },
                         "split-K last chunk")) != MPG_OK)
      return st;
  }
  SplitKReduceArgs r{};
  for (int q = 0; q < limbs; ++q) {
    r.W[q] = W[q];
    r.C[q] = C[q];
  }
  r.m = m;
  r.n = n;
  r.ldc = ldc;
  r.P = P;
  return mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_splitk_reduce(limbs, r, c->stream); },
                    "split-K reduction");
}

// ---------------------------------------------------------------------------
// public: GEMM entry points
// ---------------------------------------------------------------------------

int mpg_gemm_common(mpg_ctx* c, int limbs, int64_t m, int64_t n, int64_t l,
                    const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
                    double* const* C, int64_t ldc, mpg_algo algo, const mpg_tile* tile) {
  int st = mpg_check_gemm_args(c, limbs, m, n, l, A, lda, B, ldb, C, ldc);
  if (st != MPG_OK || m == 0 || n == 0) return st;
  st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  if (l == 0)
    return mpg_launch(c, MPG_KCLASS_AUX, [&] { return launch_zero(C, limbs, m, n, ldc, c->stream); },
                      "zero C");
  mpg_tile chosen{};
  if (tile) chosen = *tile;
  bool from_table = false;
  if (algo == MPG_AUTO) {
    int a = MPG_BLOCK;
    mpg_tile t{};
    if (mpg_table_lookup(c, limbs, m, n, l, &a, &t)) {
      algo = (mpg_algo)a;
      chosen = t;
      from_table = true;
    } else {
      algo = MPG_BLOCK;
    }
  }
  if (from_table && algo == MPG_OZAKI_CRT && chosen.slices == 0) {
    // the tabled residue form with the exact slice count, decided on the
    // device (no read-back): see mpg_dd_crt_auto / mpg_qd_crt_auto
    bool used = false;
    st = limbs == 2 ? mpg_dd_crt_auto(c, m, n, l, A[0], A[1], lda, B[0], B[1], ldb, C[0], C[1], ldc, &used)
                    : mpg_qd_crt_auto(c, m, n, l, A, lda, B, ldb, C, ldc, &used);
    if (st != MPG_OK || used) return st;
    algo = MPG_BLOCK;
    chosen = mpg_tile{};
  }
  if (algo == MPG_OZAKI || algo == MPG_OZAKI_CRT) {
    if (algo == MPG_OZAKI && limbs != 2)
      return mpg_fail(c, MPG_ERR_UNSUPPORTED, "the digit form of the split product is DD only");
    st = algo == MPG_OZAKI_CRT && limbs == 4
             ? mpg_qd_crt(c, m, n, l, A, lda, B, ldb, C, ldc)
             : mpgemm_dd_ozaki(c, m, n, l, A[0], A[1], lda, B[0], B[1], ldb, C[0], C[1], ldc, chosen.slices,
                               algo == MPG_OZAKI_CRT ? 2 : 0);
    // a tuned split product that the data's exact slice count rules out
    // (nothing is written to C then) falls back to the block kernel of the
    // same precision, so MPG_AUTO runs on any canonical input
    if (st != MPG_ERR_UNSUPPORTED || !from_table) return st;
    c->last_error.clear();
    algo = MPG_BLOCK;
    chosen = mpg_tile{};
  }
  int variant = 0;
  st = mpg_resolve_variant(c, limbs, &chosen, &variant);
  if (st != MPG_OK) return st;
  GemmBatch g{};
  g.m = m;
  g.n = n;
  g.l = l;
  for (int q = 0; q < limbs; ++q) {
    g.A[q] = A[q];
    g.B[q] = B[q];
    g.C[q] = C[q];
  }
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.count = 1;
  switch (algo) {
    case MPG_SIMPLE:
      return mpg_launch(c, MPG_KCLASS_GEMM,
                        [&] { return limbs == 2 ? launch_dd_simple(g, c->stream)
                                                : launch_qd_simple(g, c->stream); },
                        "simple kernel");
    case MPG_BLOCK:
      return mpg_launch(c, MPG_KCLASS_GEMM,
                        [&] { return limbs == 2 ? launch_dd_block(variant, g, c->stream)
                                                : launch_qd_block(variant, g, c->stream); },
                        "block kernel");
    case MPG_STRASSEN:
      return mpg_strassen(c, limbs, chosen.depth > 0 ? chosen.depth : 1, variant, m, n, l, A, lda,
                          B, ldb, C, ldc);
    case MPG_SPLITK:
      return mpg_splitk(c, limbs, chosen.splits, variant, m, n, l, A, lda, B, ldb, C, ldc);
    default:
      return mpg_fail(c, MPG_ERR_UNSUPPORTED, "algorithm %d not available for this call",
                      (int)algo);
  }
}

extern "C" int mpgemm_dd(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A_hi,
                         const double* A_lo, int64_t lda, const double* B_hi, const double* B_lo,
                         int64_t ldb, double* C_hi, double* C_lo, int64_t ldc, mpg_algo algo,
                         const mpg_tile* tile) {
  if (!c) return MPG_ERR_ARG;
  const double* A[4] = {A_hi, A_lo, nullptr, nullptr};
  const double* B[4] = {B_hi, B_lo, nullptr, nullptr};
  double* C[4] = {C_hi, C_lo, nullptr, nullptr};
  return mpg_gemm_common(c, 2, m, n, l, A, lda, B, ldb, C, ldc, algo, tile);
}

extern "C" int mpgemm_qd(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* const A[4],
                         int64_t lda, const double* const B[4], int64_t ldb, double* const C[4],
                         int64_t ldc, mpg_algo algo, const mpg_tile* tile) {
  if (!c || !A || !B || !C) return c ? mpg_fail(c, MPG_ERR_ARG, "NULL limb array") : MPG_ERR_ARG;
  return mpg_gemm_common(c, 4, m, n, l, A, lda, B, ldb, C, ldc, algo, tile);
}
