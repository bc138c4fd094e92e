// Tuner: chooses the algorithm (simple / block / Strassen) and its tile and
// depth for a shape by measured run time, following the tuning program of
// Section 3: (1) predict the full-size block time of every tile from a
// partial product (a slab of A's rows against the full B) and keep the best
// tile, (2) time simple, block and Strassen at full size, (3) take the
// fastest.  For DD the split-precision INT8 product with the exact slice
// count (the same componentwise accuracy class as the block kernel) is one
// more candidate, timed in step (2) beside the others.  Also an exhaustive
// mode (every candidate timed) and a mode where the run-time MLP ranks all
// candidates and only the best few are timed.  Measurements are appended to
// a JSONL timing database.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "capi_internal.hpp"
#include "crt_internal.hpp"
#include "ozaki_internal.hpp"

using namespace mpg;

bool mpg_mlp_ready(mpg_ctx* c);
void mpg_mlp_free(mpg_ctx* c);

namespace {

struct Cand {
  int algo;
  mpg_tile tile;
};

std::vector<Cand> candidates(int prec, int64_t m, int64_t n, int64_t l) {
  std::vector<Cand> out;
  Cand s{};
  s.algo = MPG_SIMPLE;
  out.push_back(s);
  const int nv = mpg_num_variants(prec);
  for (int v = 0; v < nv; ++v) {
    Cand b{};
    b.algo = MPG_BLOCK;
    mpg_variant(prec, v, &b.tile);
    out.push_back(b);
  }
  const int64_t mn = std::min(m, std::min(n, l));
  const int maxd = prec == 2 ? 3 : 2;
  for (int d = 1; d <= maxd; ++d) {
    if (mn < (int64_t)64 << d) break;  // leaves of at least 64 per side
    for (int v = 0; v < nv; ++v) {
      Cand t{};
      t.algo = MPG_STRASSEN;
      mpg_variant(prec, v, &t.tile);
      t.tile.depth = d;
      out.push_back(t);
    }
  }
  // split-K for skinny shapes: fewer C tiles than two waves of workgroups
  // and a K of at least two 256-long chunks
  if (l >= 512 && ((m + 63) / 64) * ((n + 63) / 64) < 512) {
    const int vs_dd[2] = {dd_default_variant(), 1}, vs_qd[1] = {0};
    const int* vs = prec == 2 ? vs_dd : vs_qd;
    for (int k = 0; k < (prec == 2 ? 2 : 1); ++k) {
      Cand t{};
      t.algo = MPG_SPLITK;
      mpg_variant(prec, vs[k], &t.tile);
      t.tile.splits = 0;
      out.push_back(t);
    }
  }
  if (prec == 2) {
    Cand z{};
    z.algo = MPG_OZAKI;
    z.tile.slices = 0;  // exact digit expansions, every slice pair
    out.push_back(z);
    z.algo = MPG_OZAKI_CRT;  // the same exact product through residues
    out.push_back(z);
  } else {
    Cand z{};
    z.algo = MPG_OZAKI_CRT;  // three residue-form products of the double-double parts
    out.push_back(z);
  }
  return out;
}

// Timing buffers for one shape: canonical multi-limb values, limb 0 in
// (-1, 1), each lower limb a uniform fraction of half an ulp of the limb
// above on a fixed grid of 2^-52 of that half-ulp (the next bits of a
// random significand).  The FP64 kernels' run time does not depend on the
// values; the split-precision product's does (its exact slice count
// follows the lowest set bits), and such limbs give it the count that
// general DD data needs.
struct Scratch {
  int limbs = 0;
  int64_t m = 0, n = 0, l = 0;
  double* A[4] = {};
  double* B[4] = {};
  double* C[4] = {};
};

__global__ void fill_kernel(double* p, const double* above, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    double u = (double)(z >> 11) * 0x1.0p-52 - 1.0;  // [-1, 1), grid 2^-52
    if (u == -1.0) u = 0.0;                            // (-1, 1): canonical pairs
    if (!above) {
      p[i] = u;
    } else {
      // half an ulp of x = 2^(ilogb x - 53)
      const double x = above[i];
      p[i] = x == 0.0 ? 0.0 : ldexp(u, ilogb(x) - 53);
    }
  }
}

void free_scratch(Scratch& s) {
  for (int q = 0; q < 4; ++q) {
    if (s.A[q]) (void)hipFree(s.A[q]);
    if (s.B[q]) (void)hipFree(s.B[q]);
    if (s.C[q]) (void)hipFree(s.C[q]);
    s.A[q] = s.B[q] = s.C[q] = nullptr;
  }
}

int make_scratch(mpg_ctx* c, int limbs, int64_t m, int64_t n, int64_t l, Scratch& s) {
  s.limbs = limbs;
  s.m = m;
  s.n = n;
  s.l = l;
  hipError_t r = hipSuccess;
  for (int q = 0; q < limbs && r == hipSuccess; ++q) {
    r = hipMalloc(&s.A[q], (size_t)(m * l) * sizeof(double));
    if (r == hipSuccess) r = hipMalloc(&s.B[q], (size_t)(l * n) * sizeof(double));
    if (r == hipSuccess) r = hipMalloc(&s.C[q], (size_t)(m * n) * sizeof(double));
  }
  if (r != hipSuccess) {
    free_scratch(s);
    (void)hipGetLastError();
    return mpg_fail(c, MPG_ERR_NOMEM, "tuner buffers for %lldx%lldx%lld", (long long)m,
                    (long long)n, (long long)l);
  }
  for (int q = 0; q < limbs; ++q) {
    hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, c->stream, s.A[q],
                       (const double*)(q ? s.A[q - 1] : nullptr), m * l, (uint64_t)(11 + q));
    hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, c->stream, s.B[q],
                       (const double*)(q ? s.B[q - 1] : nullptr), l * n, (uint64_t)(23 + q));
  }
  r = hipStreamSynchronize(c->stream);
  if (r != hipSuccess) {
    free_scratch(s);
    return mpg_hip_fail(c, r, "tuner buffer fill");
  }
  return MPG_OK;
}

int run(mpg_ctx* c, Scratch& s, int64_t rows, const Cand& cd) {
  return mpg_gemm_common(c, s.limbs, rows, s.n, s.l, s.A, s.l, s.B, s.n, s.C, s.n,
                         (mpg_algo)cd.algo, &cd.tile);
}

// Median of `reps` event-timed calls of fn() after one warm-up call.
template <class F>
int time_median(mpg_ctx* c, int reps, F&& fn, double* ms) {
  int st = fn();
  if (st != MPG_OK) return st;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return mpg_fail(c, MPG_ERR_HIP, "hipEventCreate");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return mpg_fail(c, MPG_ERR_HIP, "hipEventCreate");
  }
  std::vector<double> t;
  for (int r = 0; r < reps && st == MPG_OK; ++r) {
    (void)hipEventRecord(a, c->stream);
    st = fn();
    (void)hipEventRecord(b, c->stream);
    if (st != MPG_OK) break;
    hipError_t e = hipEventSynchronize(b);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
    if (e != hipSuccess) st = mpg_hip_fail(c, e, "tuner timing");
    t.push_back(f);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != MPG_OK) return st;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return MPG_OK;
}

int time_rows(mpg_ctx* c, Scratch& s, int64_t rows, const Cand& cd, int reps, double* ms) {
  return time_median(c, reps, [&] { return run(c, s, rows, cd); }, ms);
}

void db_append(mpg_ctx* c, int prec, int64_t m, int64_t n, int64_t l, const Cand& cd, double ms,
               const char* kind) {
  if (c->db_path.empty()) return;
  FILE* f = std::fopen(c->db_path.c_str(), "a");
  if (!f) return;
  std::fprintf(f,
               "{\"prec\":%d,\"m\":%lld,\"n\":%lld,\"l\":%lld,\"algo\":%d,\"bm\":%d,\"bn\":%d,"
               "\"bk\":%d,\"tm\":%d,\"tn\":%d,\"depth\":%d,\"slices\":%d,\"splits\":%d,\"ms\":%.6f,"
               "\"kind\":\"%s\"}\n",
               prec, (long long)m, (long long)n, (long long)l, cd.algo, cd.tile.bm, cd.tile.bn,
               cd.tile.bk, cd.tile.tm, cd.tile.tn, cd.algo == MPG_STRASSEN ? cd.tile.depth : 0,
               cd.algo == MPG_OZAKI || cd.algo == MPG_OZAKI_CRT ? cd.tile.slices : 0,
               cd.algo == MPG_SPLITK ? cd.tile.splits : 0, ms, kind);
  std::fclose(f);
}

// Workgroups of a block variant resident per CU (occupancy of the built
// kernel).
int resident_per_cu(mpg_ctx* c, int prec, const mpg_tile& t) {
  int v = 0;
  if (mpg_resolve_variant(c, prec, &t, &v) != MPG_OK) return 1;
  return prec == 2 ? dd_variant_resident(v) : qd_variant_resident(v);
}

}  // namespace

extern "C" int mpg_num_candidates(int precision, int64_t m, int64_t n, int64_t l) {
  if ((precision != 2 && precision != 4) || m <= 0 || n <= 0 || l <= 0) return 0;
  return (int)candidates(precision, m, n, l).size();
}

extern "C" int mpg_candidate(int precision, int64_t m, int64_t n, int64_t l, int index, int* algo,
                             mpg_tile* tile) {
  if ((precision != 2 && precision != 4) || !algo || !tile) return MPG_ERR_ARG;
  auto cs = candidates(precision, m, n, l);
  if (index < 0 || index >= (int)cs.size()) return MPG_ERR_ARG;
  *algo = cs[index].algo;
  *tile = cs[index].tile;
  return MPG_OK;
}

extern "C" int mpg_tune_set_db(mpg_ctx* c, const char* path) {
  if (!c) return MPG_ERR_ARG;
  c->db_path = path ? path : "";
  return MPG_OK;
}

extern "C" int mpg_time_candidate(mpg_ctx* c, int precision, int64_t m, int64_t n, int64_t l,
                                  int algo, const mpg_tile* tile, int reps, double* ms) {
  if (!c || !ms || (precision != 2 && precision != 4) || m <= 0 || n <= 0 || l <= 0 || reps < 1)
    return c ? mpg_fail(c, MPG_ERR_ARG, "bad timing request") : MPG_ERR_ARG;
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  Scratch s;
  if ((st = make_scratch(c, precision, m, n, l, s)) != MPG_OK) return st;
  Cand cd{};
  cd.algo = algo;
  if (tile) cd.tile = *tile;
  st = time_rows(c, s, m, cd, reps, ms);
  if (st == MPG_OK) db_append(c, precision, m, n, l, cd, *ms, "trial");
  free_scratch(s);
  return st;
}

// Slabs of a prediction of the full-size block-algorithm time from partial
// products (Section 3): rows of A whose product with the full B is timed.
// rule 1 (as printed for CPUs): one slab of two block rows (2 bm rows), its
// time scaled linearly in rows (*scale = m / rows).  rule 0 (GPU): with
// W = num_cu x resident workgroups in flight, a wave is enough tile rows to
// give each of them one tile; the slabs are one wave (*rows) and two waves
// (*rows2) and the time is extrapolated linearly in waves to the full
// product's *scale = tiles / W waves, t1 + (t2 - t1)(waves - 1), which
// leaves out the fixed cost of a launch (start-up, the last tiles' tail)
// that a single scaled slab would multiply.  The count of waves is not
// rounded up: a last, partial wave runs fewer tiles per CU, and each of
// them faster (measured: time follows the tile count).  A product of at
// most two waves is timed whole (*rows = m, *rows2 = 0, *scale = 1).
static void slab_plan(int64_t m, int64_t n, const mpg_tile& t, int rule, int64_t num_cu, int64_t resident,
                      int64_t* rows, int64_t* rows2, double* scale) {
  const int64_t tiles_n = (n + t.bn - 1) / t.bn, tiles_m = (m + t.bm - 1) / t.bm;
  *rows2 = 0;
  if (rule == 1) {
    *rows = std::min<int64_t>(m, 2 * (int64_t)t.bm);
    *scale = (double)m / (double)*rows;
    return;
  }
  const int64_t W = std::max<int64_t>(1, num_cu * resident);
  const int64_t wave_rows = std::max<int64_t>(1, (W + tiles_n - 1) / tiles_n);  // tile rows per wave
  if (tiles_m * tiles_n <= 2 * W || 2 * wave_rows >= tiles_m) {
    *rows = m;
    *scale = 1.0;
    return;
  }
  *rows = wave_rows * t.bm;
  *rows2 = 2 * wave_rows * t.bm;
  // waves of the full product in units of the slabs' waves
  *scale = (double)(tiles_m * tiles_n) / (double)(wave_rows * tiles_n);
}

static int predict_block(mpg_ctx* c, Scratch& s, int prec, const mpg_tile& t, int rule,
                         double* pred, double* slab_ms) {
  Cand cd{};
  cd.algo = MPG_BLOCK;
  cd.tile = t;
  int64_t rows = 0, rows2 = 0;
  double scale = 1.0;
  slab_plan(s.m, s.n, t, rule, c->num_cu, resident_per_cu(c, prec, t), &rows, &rows2, &scale);
  double t1 = 0.0, t2 = 0.0;
  int st = time_rows(c, s, rows, cd, 5, &t1);
  if (st == MPG_OK && rows2 > 0) st = time_rows(c, s, rows2, cd, 5, &t2);
  if (st != MPG_OK) return st;
  *slab_ms = t1 + t2;
  *pred = rows2 > 0 ? t1 + (t2 - t1) * (scale - 1.0) : t1 * scale;
  return MPG_OK;
}

extern "C" int mpg_predict_slab(int precision, int64_t m, int64_t n, int64_t l, const mpg_tile* tile,
                                int rule, int num_cu, int resident, int64_t* rows, int64_t* rows2,
                                double* scale) {
  if (!rows || !rows2 || !scale || (precision != 2 && precision != 4) || m <= 0 || n <= 0 || l <= 0 ||
      (rule != 0 && rule != 1) || num_cu < 1 || resident < 1)
    return MPG_ERR_ARG;
  int v = 0;
  if (mpg_resolve_variant(nullptr, precision, tile, &v) != MPG_OK) return MPG_ERR_UNSUPPORTED;
  mpg_tile t;
  mpg_variant(precision, v, &t);
  slab_plan(m, n, t, rule, num_cu, resident, rows, rows2, scale);
  return MPG_OK;
}

extern "C" int mpg_predict_block(mpg_ctx* c, int precision, int64_t m, int64_t n, int64_t l,
                                 const mpg_tile* tile, int rule, double* predicted_ms,
                                 double* slab_ms) {
  if (!c || !predicted_ms || (precision != 2 && precision != 4) || m <= 0 || n <= 0 || l <= 0 ||
      (rule != 0 && rule != 1))
    return c ? mpg_fail(c, MPG_ERR_ARG, "bad prediction request") : MPG_ERR_ARG;
  int v = 0;
  int st = mpg_resolve_variant(c, precision, tile, &v);
  if (st != MPG_OK) return st;
  mpg_tile t;
  mpg_variant(precision, v, &t);
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  Scratch s;
  if ((st = make_scratch(c, precision, m, n, l, s)) != MPG_OK) return st;
  double sm = 0.0;
  st = predict_block(c, s, precision, t, rule, predicted_ms, &sm);
  if (slab_ms) *slab_ms = sm;
  free_scratch(s);
  return st;
}

extern "C" int mpg_tune(mpg_ctx* c, int precision, int64_t m, int64_t n, int64_t l, int mode,
                        int topk, int* best_algo, mpg_tile* best_tile, double* best_ms,
                        double* seconds, int* trials) {
  if (!c) return MPG_ERR_ARG;
  if ((precision != 2 && precision != 4) || m <= 0 || n <= 0 || l <= 0 || mode < 0 || mode > 2)
    return mpg_fail(c, MPG_ERR_ARG, "bad tuning request");
  if (mode == MPG_TUNE_MLP && !mpg_mlp_ready(c))
    return mpg_fail(c, MPG_ERR_STATE, "MLP mode needs a trained or loaded run-time model");
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  Scratch s;
  if ((st = make_scratch(c, precision, m, n, l, s)) != MPG_OK) return st;
  const auto t0 = std::chrono::steady_clock::now();
  const auto cands = candidates(precision, m, n, l);
  int ntrials = 0;
  Cand best{};
  double bms = INFINITY;
  // a candidate the shape does not admit (MPG_ERR_UNSUPPORTED, e.g. the
  // split product's K limit above 24 slices) or whose workspace does not fit
  // in memory (MPG_ERR_NOMEM) is skipped, not a failure
  auto trial = [&](const Cand& cd) -> int {
    double ms = 0.0;
    int r = time_rows(c, s, m, cd, 3, &ms);
    if (r == MPG_ERR_UNSUPPORTED || r == MPG_ERR_NOMEM) {
      c->last_error.clear();
      return MPG_OK;
    }
    if (r != MPG_OK) return r;
    ++ntrials;
    db_append(c, precision, m, n, l, cd, ms, "trial");
    if (ms < bms) {
      bms = ms;
      best = cd;
    }
    return MPG_OK;
  };
  if (mode == MPG_TUNE_EXHAUSTIVE) {
    for (const auto& cd : cands)
      if ((st = trial(cd)) != MPG_OK) break;
  } else if (mode == MPG_TUNE_PAPER) {
    // (1) predicted block time for every tile, keep the best tile
    double bp = INFINITY;
    mpg_tile bt{};
    for (const auto& cd : cands) {
      if (cd.algo != MPG_BLOCK) continue;
      double pred = 0.0, slab = 0.0;
      if ((st = predict_block(c, s, precision, cd.tile, 0, &pred, &slab)) != MPG_OK) break;
      db_append(c, precision, m, n, l, cd, pred, "predicted");
      if (pred < bp) {
        bp = pred;
        bt = cd.tile;
      }
    }
    // (2) simple, block with that tile, Strassen over it, split-K (skinny
    // shapes) and the split-precision products, at full size
    if (st == MPG_OK) {
      std::vector<Cand> finals;
      Cand x{};
      x.algo = MPG_SIMPLE;
      finals.push_back(x);
      x.algo = MPG_BLOCK;
      x.tile = bt;
      finals.push_back(x);
      for (const auto& cd : cands)
        if (cd.algo == MPG_STRASSEN && cd.tile.bm == bt.bm && cd.tile.bn == bt.bn &&
            cd.tile.bk == bt.bk && cd.tile.tm == bt.tm && cd.tile.tn == bt.tn)
          finals.push_back(cd);
      for (const auto& cd : cands)
        if (cd.algo == MPG_SPLITK || cd.algo == MPG_OZAKI || cd.algo == MPG_OZAKI_CRT) finals.push_back(cd);
      // (3) the fastest of them
      for (const auto& cd : finals)
        if ((st = trial(cd)) != MPG_OK) break;
    }
  } else {
    // the run-time model ranks every candidate, the best `topk` are timed
    std::vector<float> X(cands.size() * MPG_MLP_FEATURES), y(cands.size());
    for (size_t i = 0; i < cands.size(); ++i)
      mpg_mlp_features(precision, m, n, l, cands[i].algo, &cands[i].tile, 1,
                       &X[i * MPG_MLP_FEATURES]);
    st = mpg_mlp_predict(c, X.data(), (int)cands.size(), y.data());
    if (st == MPG_OK) {
      std::vector<size_t> idx(cands.size());
      for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return y[a] < y[b]; });
      // default: one timed candidate per 9 ranked, at least 2
      const int dflt = std::max(2, (int)((idx.size() + 8) / 9));  // 4 of 35 DD, 2 of 13 QD
      const int k = std::max(1, std::min<int>(topk > 0 ? topk : dflt, (int)idx.size()));
      for (int i = 0; i < k; ++i)
        if ((st = trial(cands[idx[i]])) != MPG_OK) break;
    }
  }
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  free_scratch(s);
  if (st != MPG_OK) return st;
  if (ntrials == 0) return mpg_fail(c, MPG_ERR_UNSUPPORTED, "no candidate ran for this shape");
  if (best_algo) *best_algo = best.algo;
  if (best_tile) *best_tile = best.tile;
  if (best_ms) *best_ms = bms;
  if (seconds) *seconds = secs;
  if (trials) *trials = ntrials;
  c->table[std::make_tuple(precision, m, n, l)] = std::make_pair(best.algo, best.tile);
  return MPG_OK;
}

extern "C" int mpg_tune_table_set(mpg_ctx* c, int precision, int64_t m, int64_t n, int64_t l,
                                  int algo, const mpg_tile* tile) {
  if (!c || (precision != 2 && precision != 4) || algo < MPG_SIMPLE || algo > MPG_SPLITK ||
      (algo == MPG_OZAKI && precision != 2))
    return MPG_ERR_ARG;
  mpg_tile t{};
  if (tile) t = *tile;
  c->table[std::make_tuple(precision, m, n, l)] = std::make_pair(algo, t);
  return MPG_OK;
}

// Train the run-time model on every "trial" row of a timing database
// (target: natural log of the milliseconds).
extern "C" int mpg_mlp_train_db(mpg_ctx* c, const char* path, int epochs, float lr,
                                float* final_loss, int* rows_used) {
  if (!c || !path) return MPG_ERR_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return mpg_fail(c, MPG_ERR_ARG, "cannot open %s", path);
  std::vector<float> X, y;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    int prec, algo, bm, bn, bk, tm, tn, depth, slices, splits;
    long long m, n, l;
    double ms;
    char kind[32];
    if (std::sscanf(line,
                    "{\"prec\":%d,\"m\":%lld,\"n\":%lld,\"l\":%lld,\"algo\":%d,\"bm\":%d,\"bn\":%d,"
                    "\"bk\":%d,\"tm\":%d,\"tn\":%d,\"depth\":%d,\"slices\":%d,\"splits\":%d,\"ms\":%lf,"
                    "\"kind\":\"%31[a-z]\"",
                    &prec, &m, &n, &l, &algo, &bm, &bn, &bk, &tm, &tn, &depth, &slices, &splits, &ms,
                    kind) != 15)
      continue;
    if (std::strcmp(kind, "trial") != 0 || !(ms > 0.0)) continue;
    mpg_tile t{bm, bn, bk, tm, tn, depth, slices, splits};
    float feat[MPG_MLP_FEATURES];
    if (mpg_mlp_features(prec, m, n, l, algo, &t, 1, feat) != MPG_OK) continue;
    X.insert(X.end(), feat, feat + MPG_MLP_FEATURES);
    y.push_back((float)std::log(ms));
  }
  std::fclose(f);
  if (y.empty()) return mpg_fail(c, MPG_ERR_ARG, "no timing rows in %s", path);
  std::vector<float> losses(epochs);
  int st = mpg_mlp_train(c, X.data(), y.data(), (int)y.size(), epochs, lr, losses.data());
  if (st != MPG_OK) return st;
  if (final_loss) *final_loss = losses.back();
  if (rows_used) *rows_used = (int)y.size();
  return MPG_OK;
}

extern "C" int mpg_ozaki_tune(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int bits,
                              const double* A, int64_t lda, const double* B, int64_t ldb,
                              int* slices, int* pairs_mode, double* ms) {
  if (!c) return MPG_ERR_ARG;
  if (m <= 0 || n <= 0 || l <= 0 || !slices || !pairs_mode || (!A) != (!B))
    return mpg_fail(c, MPG_ERR_ARG, "bad split-product tuning request");
  int s_all = mpg_ozaki_slices_for_bits(bits, 0), s_tri = mpg_ozaki_slices_for_bits(bits, 1);
  if (s_all == 0 || s_tri == 0)
    return mpg_fail(c, MPG_ERR_ARG, "no slice count reaches %d bits", bits);
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  if (A) {
    int se = 0;
    if ((st = mpg_ozaki_slices_exact(c, m, n, l, A, lda, B, ldb, &se)) != MPG_OK) return st;
    s_all = std::min(s_all, std::max(se, 1));
  }
  Scratch sc;
  if ((st = make_scratch(c, 2, m, n, l, sc)) != MPG_OK) return st;
  const int cand[2][2] = {{s_all, 0}, {s_tri, 1}};
  double best = INFINITY;
  for (const auto& cd : cand) {
    double t = 0.0;
    st = time_median(c, 3, [&] {
      return mpgemm_ozaki_dd(c, m, n, l, sc.A[0], l, sc.B[0], n, sc.C[0], sc.C[1], n, cd[0], cd[1]);
    }, &t);
    if (st != MPG_OK) break;
    Cand z{};
    z.algo = MPG_OZAKI;
    z.tile.slices = cd[0];
    db_append(c, 1, m, n, l, z, t, cd[1] ? "splittri" : "split");
    if (t < best) {
      best = t;
      *slices = cd[0];
      *pairs_mode = cd[1];
    }
  }
  free_scratch(sc);
  if (st == MPG_OK && ms) *ms = best;
  return st;
}

namespace {

// Normwise a-priori bound of a method for C := A B, per entry of C in units
// of l max|A| max|B|.  DD / QD simple and block: the componentwise bound
// 8 l u (|A||B|)_ij (u = 2^-104, 2^-208) with (|A||B|)_ij <= l max|A| max|B|;
// Winograd-Strassen of depth d on a square product padded to N: Higham's
// [18^d (N0^2 + 6 N0) - 6 N] 8 u max|A| max|B|, N0 = N / 2^d; QD inputs
// rounded to DD add 2^-105 (|A||B|).  The split product: the truncation
// bound times 2^(e_i + f_j) <= 4 max|a_i.| max|b_.j|, plus the
// double-double recombination of its T = (2S - 1) x chunks exactly scaled
// terms: every TwoSum into the high limb is exact, the error terms are
// below 2^-53 of the running sum, so their sum in the low limb rounds off
// at most T^2/2 2^-106 of the largest running sum; the running sums are
// below the sum of the terms' magnitudes, at most 16.2 l max|A| max|B|
// (signed-byte digits: sum_s |D_s| 256^-s <= 128/255, scales below
// 4 max|a|, 4 max|b|); and the final rounding adds 2^-106 |C|.  The
// residue form (pairs 2) computes the kept product (the same as with all
// pairs) exactly and rounds it once: the truncation bound plus 2^-104.
double method_bound(int in_limbs, int prec, int algo, const mpg_tile& t, int pairs, int64_t m,
                    int64_t l) {
  const double L = (double)l;
  // quad-double through the residue form: the three kept part products are
  // exact, each is rounded to quad-double and added (a few 2^-211 of the
  // magnitudes), and the dropped product of the trailing parts is below
  // 2^-210 l max|A| max|B| for canonical operands
  if (algo == MPG_OZAKI_CRT && prec == 4) return std::ldexp(1.0, -204);
  if (algo == MPG_OZAKI) {
    if (in_limbs > 2 || t.slices < 1) return INFINITY;
    const int S = t.slices;
    if (pairs == 2)
      return S <= kCrtMaxSlices && mpg_crt_moduli_for(S, l) > 0
                 ? 4.0 * ozaki_unit_bound(S, 0) + std::ldexp(1.0, -104)
                 : INFINITY;
    const double T = (double)(2 * S - 1) * ozaki_chunks(S, l);
    const double recomb = (4.1 * T * T + 2.0) * std::ldexp(1.0, -105);
    return 4.0 * ozaki_unit_bound(S, pairs) + recomb;
  }
  const double u8 = 8.0 * std::ldexp(1.0, prec == 2 ? -104 : -208);
  double b;
  if (algo == MPG_STRASSEN) {
    const int64_t q = (int64_t)1 << t.depth, N = (m + q - 1) / q * q;
    const double N0 = (double)(N / q);
    b = (std::pow(18.0, t.depth) * (N0 * N0 + 6.0 * N0) - 6.0 * (double)N) * u8 / L;
  } else {
    b = u8 * L;
  }
  if (prec == 2 && in_limbs == 4) b += std::ldexp(1.0, -105);
  return b;
}

}  // namespace

extern "C" double mpg_method_bound(int in_limbs, int precision, int algo, const mpg_tile* tile,
                                   int pairs_mode, int64_t m, int64_t n, int64_t l) {
  if ((in_limbs != 1 && in_limbs != 2 && in_limbs != 4) || (precision != 2 && precision != 4) ||
      m <= 0 || n <= 0 || l <= 0 || (algo == MPG_STRASSEN && (!tile || tile->depth < 1 || tile->depth > 3 ||
                                                              m != n || n != l)) ||
      (algo == MPG_OZAKI && (precision != 2 || !tile)) || (algo == MPG_OZAKI_CRT && precision == 2 && !tile) ||
      algo < MPG_SIMPLE || algo > MPG_SPLITK)
    return INFINITY;
  mpg_tile t{};
  if (tile) t = *tile;
  if (algo == MPG_OZAKI_CRT && precision == 4) return method_bound(in_limbs, 4, MPG_OZAKI_CRT, t, 0, m, l);
  if (algo == MPG_OZAKI_CRT) return method_bound(in_limbs, precision, MPG_OZAKI, t, 2, m, l);
  if (algo == MPG_OZAKI && (pairs_mode < 0 || pairs_mode > 2)) return INFINITY;
  return method_bound(in_limbs, precision, algo, t, pairs_mode, m, l);
}

extern "C" int mpg_select_method(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int in_limbs, int bits,
                                 int* precision, int* algo, mpg_tile* tile, int* pairs_mode,
                                 double* bound_bits, double* ms) {
  if (!c) return MPG_ERR_ARG;
  if (m <= 0 || n <= 0 || l <= 0 || (in_limbs != 1 && in_limbs != 2 && in_limbs != 4) || bits < 1 ||
      !precision || !algo || !tile || !pairs_mode)
    return mpg_fail(c, MPG_ERR_ARG, "bad method selection request");
  struct Choice {
    int prec, algo, pairs;
    mpg_tile tile;
  };
  const double target = std::ldexp(1.0, -bits);
  std::vector<Choice> feasible;
  auto consider = [&](int prec, int a, mpg_tile t, int pairs) {
    if (method_bound(in_limbs, prec, a, t, pairs, m, l) <= target) feasible.push_back({prec, a, pairs, t});
  };
  const bool square = m == n && n == l;
  consider(4, MPG_OZAKI_CRT, mpg_tile{}, 0);
  for (int prec : {2, 4}) {
    consider(prec, MPG_BLOCK, mpg_tile{}, 0);
    for (int d = 1; d <= (prec == 2 ? 3 : 2) && square && m >= (int64_t)64 << d; ++d) {
      mpg_tile t{};
      t.depth = d;
      consider(prec, MPG_STRASSEN, t, 0);
    }
  }
  for (int pairs : {0, 1, 2})
    for (int S = 1; S <= ozaki_max_slices(); ++S) {
      mpg_tile t{};
      t.slices = S;
      if (method_bound(in_limbs, 2, MPG_OZAKI, t, pairs, m, l) <= target) {
        consider(2, MPG_OZAKI, t, pairs);
        break;
      }
    }
  if (feasible.empty())
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "no method's bound reaches %d bits", bits);
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  Scratch s;
  if ((st = make_scratch(c, 4, m, n, l, s)) != MPG_OK) return st;
  double best = INFINITY;
  for (const Choice& ch : feasible) {
    double t = 0.0;
    st = time_median(c, 3, [&] {
      if (ch.algo == MPG_OZAKI)
        return in_limbs == 1
                   ? mpgemm_ozaki_dd(c, m, n, l, s.A[0], l, s.B[0], n, s.C[0], s.C[1], n, ch.tile.slices,
                                     ch.pairs)
                   : mpgemm_dd_ozaki(c, m, n, l, s.A[0], s.A[1], l, s.B[0], s.B[1], n, s.C[0], s.C[1], n,
                                     ch.tile.slices, ch.pairs);
      return mpg_gemm_common(c, ch.prec, m, n, l, s.A, l, s.B, n, s.C, n, (mpg_algo)ch.algo, &ch.tile);
    }, &t);
    if (st == MPG_ERR_UNSUPPORTED) {
      st = MPG_OK;
      continue;
    }
    if (st != MPG_OK) break;
    if (t < best) {
      best = t;
      *precision = ch.prec;
      *algo = ch.algo;
      *tile = ch.tile;
      *pairs_mode = ch.pairs;
      if (bound_bits) *bound_bits = -std::log2(method_bound(in_limbs, ch.prec, ch.algo, ch.tile, ch.pairs, m, l));
    }
  }
  free_scratch(s);
  if (st != MPG_OK) return st;
  if (!(best < INFINITY)) return mpg_fail(c, MPG_ERR_UNSUPPORTED, "no feasible method ran");
  if (ms) *ms = best;
  return MPG_OK;
}

bool mpg_table_lookup(mpg_ctx* c, int precision, int64_t m, int64_t n, int64_t l, int* algo,
                      mpg_tile* tile) {
  auto it = c->table.find(std::make_tuple(precision, m, n, l));
  if (it == c->table.end()) return false;
  *algo = it->second.first;
  *tile = it->second.second;
  return true;
}

void mpg_destroy_cached(mpg_ctx* c) { mpg_mlp_free(c); }

// ---------------------------------------------------------------------------
// Plans of the long-integer product: candidates, slab prediction (Section 3)
// and the three tuning modes
// ---------------------------------------------------------------------------

namespace {

constexpr int kIntDbAlgo = 16;  // DB rows of the long-integer product (precision 0)

std::vector<mpg_int_algo> int_candidates(int wa, int wb, int64_t l) {
  std::vector<mpg_int_algo> out;
  for (int cw : {4, 3, 5})
    for (int d = 0; d <= 2; ++d) {
      const int ca = (wa + cw - 1) / cw, cb = (wb + cw - 1) / cw;
      if (d > 0 && (1 << d) > std::max(ca, cb)) break;  // nothing left to split
      if (mpg_int_plan_products(wa, wb, l, cw, d) > 0) out.push_back(mpg_int_algo{cw, d});
    }
  return out;
}

__global__ void fill_words_kernel(uint32_t* p, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    p[i] = (uint32_t)(z ^ (z >> 31));
  }
}

struct IntScratch {
  int64_t m = 0, n = 0, l = 0;
  int wa = 0, wb = 0, wc = 0;
  uint32_t *A = nullptr, *B = nullptr, *C = nullptr;
};

void free_int_scratch(IntScratch& s) {
  if (s.A) (void)hipFree(s.A);
  if (s.B) (void)hipFree(s.B);
  if (s.C) (void)hipFree(s.C);
  s.A = s.B = s.C = nullptr;
}

int make_int_scratch(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int wa, int wb, IntScratch& s) {
  s.m = m;
  s.n = n;
  s.l = l;
  s.wa = wa;
  s.wb = wb;
  s.wc = mpg_int_words_needed(wa, wb, l);
  hipError_t r = hipMalloc(&s.A, (size_t)(wa * m * l) * 4);
  if (r == hipSuccess) r = hipMalloc(&s.B, (size_t)(wb * l * n) * 4);
  if (r == hipSuccess) r = hipMalloc(&s.C, (size_t)(s.wc * m * n) * 4);
  if (r != hipSuccess) {
    free_int_scratch(s);
    (void)hipGetLastError();
    return mpg_fail(c, MPG_ERR_NOMEM, "tuner buffers of the long-integer product");
  }
  hipLaunchKernelGGL(fill_words_kernel, dim3(1024), dim3(256), 0, c->stream, s.A, (int64_t)wa * m * l, 31ull);
  hipLaunchKernelGGL(fill_words_kernel, dim3(1024), dim3(256), 0, c->stream, s.B, (int64_t)wb * l * n, 37ull);
  r = hipStreamSynchronize(c->stream);
  if (r != hipSuccess) {
    free_int_scratch(s);
    return mpg_hip_fail(c, r, "tuner buffer fill");
  }
  return MPG_OK;
}

int run_int(mpg_ctx* c, IntScratch& s, int64_t rows, const mpg_int_algo& a) {
  return mpg_int_run(c, rows, s.n, s.l, s.A, s.wa, s.l, s.m * s.l, s.B, s.wb, s.n, s.l * s.n, s.C, s.wc, s.n,
                     s.m * s.n, a.chunk_words, a.karatsuba_depth);
}

void int_db_append(mpg_ctx* c, const IntScratch& s, const mpg_int_algo& a, double ms, const char* kind) {
  if (c->db_path.empty()) return;
  FILE* f = std::fopen(c->db_path.c_str(), "a");
  if (!f) return;
  std::fprintf(f,
               "{\"prec\":0,\"m\":%lld,\"n\":%lld,\"l\":%lld,\"algo\":%d,\"bm\":%d,\"bn\":%d,\"bk\":%d,\"tm\":0,"
               "\"tn\":0,\"depth\":%d,\"slices\":0,\"splits\":0,\"ms\":%.6f,\"kind\":\"%s\"}\n",
               (long long)s.m, (long long)s.n, (long long)s.l, kIntDbAlgo, s.wa, s.wb, a.chunk_words,
               a.karatsuba_depth, ms, kind);
  std::fclose(f);
}

// Section 3 for the long-integer product, in the GPU form: a wave is
// enough 256-row tile rows of the residue products for one workgroup on
// every CU (each launch has tile rows x column tiles x moduli workgroups);
// slabs of one and two waves, extrapolated linearly in tile rows (waves) to
// the product's, without rounding; at most two waves: the product itself.
int int_slab_plan(int64_t m, int64_t n, int64_t l, int wa, int wb, const mpg_int_algo& a, int num_cu, int64_t* r1,
                  int64_t* r2, double* scale) {
  const int N = mpg_int_plan_moduli(wa, wb, l, a.chunk_words, a.karatsuba_depth);
  const int64_t tr = crt_tile_rows(), tiles_n = (n + crt_tile_cols() - 1) / crt_tile_cols();
  const int64_t tiles_m = (m + tr - 1) / tr;
  const int64_t per_row = std::max<int64_t>(1, tiles_n * std::max(N, 1));   // workgroups per tile row
  const int64_t wave_rows = std::max<int64_t>(1, (num_cu + per_row - 1) / per_row);
  if (tiles_m <= 2 * wave_rows) {
    *r1 = m;
    *r2 = 0;
    *scale = 1.0;
    return MPG_OK;
  }
  *r1 = wave_rows * tr;
  *r2 = 2 * wave_rows * tr;
  *scale = (double)tiles_m / (double)wave_rows;
  return MPG_OK;
}

int int_predict(mpg_ctx* c, IntScratch& s, const mpg_int_algo& a, double* pred, double* slab_ms) {
  int64_t r1 = 0, r2 = 0;
  double scale = 1.0;
  int_slab_plan(s.m, s.n, s.l, s.wa, s.wb, a, c->num_cu, &r1, &r2, &scale);
  double t1 = 0.0, t2 = 0.0;
  int st = time_median(c, 3, [&] { return run_int(c, s, r1, a); }, &t1);
  if (st == MPG_OK && r2 > 0) st = time_median(c, 3, [&] { return run_int(c, s, r2, a); }, &t2);
  if (st != MPG_OK) return st;
  *slab_ms = t1 + t2;
  *pred = r2 > 0 ? t1 + (t2 - t1) * (scale - 1.0) : t1;
  return MPG_OK;
}

}  // namespace

bool mpg_int_table_lookup(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int words_a, int words_b,
                          mpg_int_algo* algo) {
  auto it = c->int_table.find(std::make_tuple(m, n, l, words_a, words_b));
  if (it == c->int_table.end()) return false;
  *algo = it->second;
  return true;
}

extern "C" int mpg_int_num_candidates(int words_a, int words_b, int64_t l) {
  if (words_a < 1 || words_b < 1 || l < 1) return 0;
  return (int)int_candidates(words_a, words_b, l).size();
}

extern "C" int mpg_int_candidate(int words_a, int words_b, int64_t l, int index, mpg_int_algo* algo) {
  if (!algo || words_a < 1 || words_b < 1 || l < 1) return MPG_ERR_ARG;
  const auto cs = int_candidates(words_a, words_b, l);
  if (index < 0 || index >= (int)cs.size()) return MPG_ERR_ARG;
  *algo = cs[index];
  return MPG_OK;
}

extern "C" int64_t mpg_int_products(int words_a, int words_b, int64_t l, const mpg_int_algo* algo) {
  if (!algo || words_a < 1 || words_b < 1 || l < 1) return 0;
  return mpg_int_plan_products(words_a, words_b, l, algo->chunk_words, algo->karatsuba_depth);
}

extern "C" int mpg_int_time(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int words_a, int words_b,
                            const mpg_int_algo* algo, int reps, double* ms) {
  if (!c || !algo || !ms || m <= 0 || n <= 0 || l <= 0 || words_a < 1 || words_b < 1 || reps < 1)
    return c ? mpg_fail(c, MPG_ERR_ARG, "bad timing request") : MPG_ERR_ARG;
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  IntScratch s;
  if ((st = make_int_scratch(c, m, n, l, words_a, words_b, s)) != MPG_OK) return st;
  st = time_median(c, reps, [&] { return run_int(c, s, m, *algo); }, ms);
  if (st == MPG_OK) int_db_append(c, s, *algo, *ms, "trial");
  free_int_scratch(s);
  return st;
}

extern "C" int mpg_int_predict(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int words_a, int words_b,
                               const mpg_int_algo* algo, double* predicted_ms, double* slab_ms) {
  if (!c || !algo || !predicted_ms || m <= 0 || n <= 0 || l <= 0 || words_a < 1 || words_b < 1)
    return c ? mpg_fail(c, MPG_ERR_ARG, "bad prediction request") : MPG_ERR_ARG;
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  IntScratch s;
  if ((st = make_int_scratch(c, m, n, l, words_a, words_b, s)) != MPG_OK) return st;
  double sm = 0.0;
  st = int_predict(c, s, *algo, predicted_ms, &sm);
  if (slab_ms) *slab_ms = sm;
  free_int_scratch(s);
  return st;
}

extern "C" int mpg_int_tune(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int words_a, int words_b, int mode,
                            int topk, mpg_int_algo* best_algo, double* best_ms, double* seconds, int* trials) {
  if (!c) return MPG_ERR_ARG;
  if (m <= 0 || n <= 0 || l <= 0 || words_a < 1 || words_b < 1 || mode < 0 || mode > 2)
    return mpg_fail(c, MPG_ERR_ARG, "bad tuning request");
  if (mode == MPG_TUNE_MLP && !mpg_mlp_ready(c))
    return mpg_fail(c, MPG_ERR_STATE, "MLP mode needs a trained or loaded run-time model");
  const auto cands = int_candidates(words_a, words_b, l);
  if (cands.empty()) return mpg_fail(c, MPG_ERR_UNSUPPORTED, "no plan fits this product");
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  IntScratch s;
  if ((st = make_int_scratch(c, m, n, l, words_a, words_b, s)) != MPG_OK) return st;
  const auto t0 = std::chrono::steady_clock::now();
  int ntrials = 0;
  mpg_int_algo best{};
  double bms = INFINITY;
  auto trial = [&](const mpg_int_algo& a) -> int {
    double ms = 0.0;
    int r = time_median(c, 3, [&] { return run_int(c, s, m, a); }, &ms);
    if (r == MPG_ERR_UNSUPPORTED || r == MPG_ERR_NOMEM) {
      c->last_error.clear();
      return MPG_OK;
    }
    if (r != MPG_OK) return r;
    ++ntrials;
    int_db_append(c, s, a, ms, "trial");
    if (ms < bms) {
      bms = ms;
      best = a;
    }
    return MPG_OK;
  };
  if (mode == MPG_TUNE_EXHAUSTIVE) {
    for (const auto& a : cands)
      if ((st = trial(a)) != MPG_OK) break;
  } else if (mode == MPG_TUNE_PAPER) {
    // (1) the predicted time of every plan; (2) the best predicted and the
    // default plan at full size; (3) the faster
    double bp = INFINITY;
    mpg_int_algo bpa = cands[0];
    for (const auto& a : cands) {
      double pred = 0.0, slab = 0.0;
      if ((st = int_predict(c, s, a, &pred, &slab)) != MPG_OK) break;
      int_db_append(c, s, a, pred, "predicted");
      if (pred < bp) {
        bp = pred;
        bpa = a;
      }
    }
    if (st == MPG_OK) st = trial(bpa);
    if (st == MPG_OK && (bpa.chunk_words != cands[0].chunk_words || bpa.karatsuba_depth != cands[0].karatsuba_depth))
      st = trial(cands[0]);
  } else {
    std::vector<float> X(cands.size() * MPG_MLP_FEATURES), y(cands.size());
    for (size_t i = 0; i < cands.size(); ++i) {
      mpg_tile t{words_a, words_b, cands[i].chunk_words, 0, 0, cands[i].karatsuba_depth, 0, 0};
      mpg_mlp_features(0, m, n, l, kIntDbAlgo, &t, 1, &X[i * MPG_MLP_FEATURES]);
    }
    st = mpg_mlp_predict(c, X.data(), (int)cands.size(), y.data());
    if (st == MPG_OK) {
      std::vector<size_t> idx(cands.size());
      for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return y[a] < y[b]; });
      const int dflt = std::max(2, (int)((idx.size() + 3) / 4));
      const int k = std::max(1, std::min<int>(topk > 0 ? topk : dflt, (int)idx.size()));
      for (int i = 0; i < k; ++i)
        if ((st = trial(cands[idx[i]])) != MPG_OK) break;
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  free_int_scratch(s);
  if (st != MPG_OK) return st;
  if (ntrials == 0) return mpg_fail(c, MPG_ERR_UNSUPPORTED, "no plan ran for this product");
  if (best_algo) *best_algo = best;
  if (best_ms) *best_ms = bms;
  if (seconds) *seconds = secs;
  if (trials) *trials = ntrials;
  c->int_table[std::make_tuple(m, n, l, words_a, words_b)] = best;
  return MPG_OK;
}
