// Host side of the run-time model: parameter state on the device, training
// (full-batch Adam on the GPU kernels), prediction, save / load, and the
// feature map of a (shape, precision, algorithm, tile) candidate.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "capi_internal.hpp"
#include "mlp_internal.hpp"

using namespace mpg;

struct mpg_mlp_state {
  int F = MPG_MLP_FEATURES;
  int P = 0;
  bool ready = false;  // parameters set or trained
  float* prm = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  int step = 0;
  // per-call scratch
  float* X = nullptr;
  float* t = nullptr;
  float* partial = nullptr;
  float* out = nullptr;
  float* losses = nullptr;
  int cap_rows = 0, cap_epochs = 0;
};

namespace {

void free_state(mpg_mlp_state* s) {
  for (float* p : {s->prm, s->m, s->v, s->grad, s->X, s->t, s->partial, s->out, s->losses})
    if (p) (void)hipFree(p);
  delete s;
}

int state(mpg_ctx* c, mpg_mlp_state** out) {
  if (!c->mlp) {
    mpg_mlp_state* s = new mpg_mlp_state();
    s->P = mlp_num_params(s->F);
    hipError_t r = hipMalloc(&s->prm, s->P * sizeof(float));
    if (r == hipSuccess) r = hipMalloc(&s->m, s->P * sizeof(float));
    if (r == hipSuccess) r = hipMalloc(&s->v, s->P * sizeof(float));
    if (r == hipSuccess) r = hipMalloc(&s->grad, (s->P + 1) * sizeof(float));
    if (r != hipSuccess) {
      free_state(s);
      return mpg_hip_fail(c, r, "MLP allocation");
    }
    c->mlp = s;
  }
  *out = c->mlp;
  return MPG_OK;
}

int reserve(mpg_ctx* c, mpg_mlp_state* s, int rows, int epochs) {
  if (rows > s->cap_rows) {
    for (float** p : {&s->X, &s->t, &s->partial, &s->out})
      if (*p) (void)hipFree(*p), *p = nullptr;
    hipError_t r = hipMalloc(&s->X, (size_t)rows * s->F * sizeof(float));
    if (r == hipSuccess) r = hipMalloc(&s->t, (size_t)rows * sizeof(float));
    if (r == hipSuccess)
      r = hipMalloc(&s->partial, (size_t)mlp_grad_chunks(rows) * (s->P + 1) * sizeof(float));
    if (r == hipSuccess) r = hipMalloc(&s->out, (size_t)rows * sizeof(float));
    if (r != hipSuccess) return mpg_hip_fail(c, r, "MLP scratch allocation");
    s->cap_rows = rows;
  }
  if (epochs > s->cap_epochs) {
    if (s->losses) (void)hipFree(s->losses);
    hipError_t r = hipMalloc(&s->losses, (size_t)epochs * sizeof(float));
    if (r != hipSuccess) return mpg_hip_fail(c, r, "MLP loss buffer");
    s->cap_epochs = epochs;
  }
  return MPG_OK;
}

// Deterministic He-uniform initialisation (splitmix64 stream), zero biases.
void default_init(std::vector<float>& p, int F) {
  const int H = kMlpHidden;
  uint64_t x = 0x1710018390000000ull;
  auto next = [&]() {
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;  // U(-1, 1)
  };
  p.assign(mlp_num_params(F), 0.f);
  size_t o = 0;
  const double l1 = std::sqrt(6.0 / F), l2 = std::sqrt(6.0 / H);
  for (int i = 0; i < H * F; ++i) p[o++] = (float)(l1 * next());
  o += H;
  for (int i = 0; i < H * H; ++i) p[o++] = (float)(l2 * next());
  o += H;
  for (int i = 0; i < H; ++i) p[o++] = (float)(l2 * next());
}

int upload_params(mpg_ctx* c, mpg_mlp_state* s, const float* host) {
  hipError_t r = hipMemcpy(s->prm, host, s->P * sizeof(float), hipMemcpyHostToDevice);
  if (r == hipSuccess) r = hipMemset(s->m, 0, s->P * sizeof(float));
  if (r == hipSuccess) r = hipMemset(s->v, 0, s->P * sizeof(float));
  if (r != hipSuccess) return mpg_hip_fail(c, r, "MLP parameter upload");
  s->step = 0;
  s->ready = true;
  return MPG_OK;
}

int upload_rows(mpg_ctx* c, mpg_mlp_state* s, const float* X, const float* t, int rows) {
  hipError_t r = hipMemcpyAsync(s->X, X, (size_t)rows * s->F * sizeof(float),
                                hipMemcpyHostToDevice, c->stream);
  if (r == hipSuccess && t)
    r = hipMemcpyAsync(s->t, t, (size_t)rows * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "MLP data upload");
  return MPG_OK;
}

}  // namespace

void mpg_mlp_free(mpg_ctx* c) {
  if (c->mlp) free_state(c->mlp);
  c->mlp = nullptr;
}

bool mpg_mlp_ready(mpg_ctx* c) { return c->mlp && c->mlp->ready; }

extern "C" int mpg_mlp_num_params(void) { return mlp_num_params(MPG_MLP_FEATURES); }

extern "C" int mpg_mlp_features(int precision, int64_t m, int64_t n, int64_t l, int algo,
                                const mpg_tile* tile, int batch, float* out) {
  if (!out || m <= 0 || n <= 0 || l <= 0 || batch <= 0) return MPG_ERR_ARG;
  mpg_tile t{};
  if (tile) t = *tile;
  auto lg = [](double v) { return v > 0 ? std::log2(v) : 0.0; };
  float f[MPG_MLP_FEATURES] = {};
  if (precision == 0) {  // long-integer product: operand words, chunk words, Karatsuba depth
    f[0] = (float)(lg((double)m) / 12.0);
    f[1] = (float)(lg((double)n) / 12.0);
    f[2] = (float)(lg((double)l) / 12.0);
    f[8] = (float)(lg(32.0 * t.bm) / 12.0);
    f[9] = (float)(lg(32.0 * t.bn) / 12.0);
    f[10] = (float)t.bk / 8.f;
    f[12] = (float)t.depth / 3.f;
    f[14] = 3.f;
    std::memcpy(out, f, sizeof f);
    return MPG_OK;
  }
  f[0] = (float)(lg((double)m) / 12.0);
  f[1] = (float)(lg((double)n) / 12.0);
  f[2] = (float)(lg((double)l) / 12.0);
  f[3] = precision == 2 ? 1.f : 0.f;
  f[4] = precision == 4 ? 1.f : 0.f;
  f[5] = algo == MPG_SIMPLE ? 1.f : 0.f;
  f[6] = algo == MPG_BLOCK || algo == MPG_SPLITK ? 1.f : 0.f;
  f[7] = algo == MPG_STRASSEN ? 1.f : 0.f;
  f[8] = (float)(lg((double)t.bm) / 8.0);
  f[9] = (float)(lg((double)t.bn) / 8.0);
  f[10] = (float)(lg((double)t.bk) / 5.0);
  f[11] = (float)(t.tm * t.tn) / 64.f;
  f[12] = (float)(algo == MPG_STRASSEN ? t.depth : 0) / 3.f;
  // split-K: its chunks are a batch of problems (the planned count with two
  // resident workgroups on 256 CUs when the tile leaves it to the shape)
  int64_t chunks = batch;
  if (algo == MPG_SPLITK) {
    int64_t P = 1, Kc = l;
    mpg_splitk_plan(m, n, l, t.bm > 0 ? t.bm : 64, t.bn > 0 ? t.bn : 64, t.bk > 0 ? t.bk : 8, 2, 256,
                    t.splits, &P, &Kc);
    chunks = P;
  }
  f[13] = (float)(lg((double)chunks) / 10.0);
  f[14] = algo == MPG_OZAKI ? 1.f : algo == MPG_OZAKI_CRT ? 2.f : 0.f;  // split product, residue form
  std::memcpy(out, f, sizeof f);
  return MPG_OK;
}

extern "C" int mpg_mlp_set_params(mpg_ctx* c, const float* params, int count) {
  if (!c || !params || count != mpg_mlp_num_params()) return c ? mpg_fail(c, MPG_ERR_ARG, "need %d parameters", mpg_mlp_num_params()) : MPG_ERR_ARG;
  mpg_mlp_state* s;
  int st = mpg_device_guard(c);
  if (st == MPG_OK) st = state(c, &s);
  if (st != MPG_OK) return st;
  hipError_t r = hipStreamSynchronize(c->stream);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "hipStreamSynchronize");
  return upload_params(c, s, params);
}

extern "C" int mpg_mlp_get_params(mpg_ctx* c, float* params, int count) {
  if (!c || !params || count != mpg_mlp_num_params()) return MPG_ERR_ARG;
  if (!mpg_mlp_ready(c)) return mpg_fail(c, MPG_ERR_STATE, "MLP has no parameters");
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  hipError_t r = hipMemcpyAsync(params, c->mlp->prm, count * sizeof(float), hipMemcpyDeviceToHost,
                                c->stream);
  if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
  return r == hipSuccess ? MPG_OK : mpg_hip_fail(c, r, "MLP parameter read");
}

extern "C" int mpg_mlp_grad(mpg_ctx* c, const float* X, const float* y, int rows, float* loss,
                            float* grad) {
  if (!c || !X || !y || rows <= 0) return MPG_ERR_ARG;
  if (!mpg_mlp_ready(c)) return mpg_fail(c, MPG_ERR_STATE, "MLP has no parameters");
  mpg_mlp_state* s = c->mlp;
  int st = mpg_device_guard(c);
  if (st == MPG_OK) st = reserve(c, s, rows, 1);
  if (st == MPG_OK) st = upload_rows(c, s, X, y, rows);
  if (st != MPG_OK) return st;
  st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
    return launch_mlp_grad(s->prm, s->X, s->t, rows, s->F, s->partial, s->grad, nullptr, 0, c->stream);
  }, "MLP gradient");
  if (st != MPG_OK) return st;
  std::vector<float> g(s->P + 1);
  hipError_t r = hipMemcpyAsync(g.data(), s->grad, g.size() * sizeof(float), hipMemcpyDeviceToHost,
                                c->stream);
  if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "MLP gradient read");
  if (grad) std::memcpy(grad, g.data(), s->P * sizeof(float));
  if (loss) *loss = g[s->P];
  return MPG_OK;
}

extern "C" int mpg_mlp_train(mpg_ctx* c, const float* X, const float* y, int rows, int epochs,
                             float lr, float* losses) {
  if (!c || !X || !y || rows <= 0 || epochs <= 0 || !(lr > 0.f)) return MPG_ERR_ARG;
  mpg_mlp_state* s;
  int st = mpg_device_guard(c);
  if (st == MPG_OK) st = state(c, &s);
  if (st != MPG_OK) return st;
  if (!s->ready) {
    std::vector<float> p;
    default_init(p, s->F);
    if ((st = upload_params(c, s, p.data())) != MPG_OK) return st;
  }
  if ((st = reserve(c, s, rows, epochs)) != MPG_OK) return st;
  if ((st = upload_rows(c, s, X, y, rows)) != MPG_OK) return st;
  for (int e = 0; e < epochs; ++e) {
    st = mpg_launch(c, MPG_KCLASS_AUX, [&] {
      hipError_t r = launch_mlp_grad(s->prm, s->X, s->t, rows, s->F, s->partial, s->grad,
                                     s->losses, e, c->stream);
      if (r != hipSuccess) return r;
      return launch_mlp_adam(s->prm, s->grad, s->m, s->v, s->P, lr, ++s->step, c->stream);
    }, "MLP training step");
    if (st != MPG_OK) return st;
  }
  if (losses) {
    hipError_t r = hipMemcpyAsync(losses, s->losses, (size_t)epochs * sizeof(float),
                                  hipMemcpyDeviceToHost, c->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
    if (r != hipSuccess) return mpg_hip_fail(c, r, "MLP loss read");
  }
  return MPG_OK;
}

extern "C" int mpg_mlp_predict(mpg_ctx* c, const float* X, int rows, float* out) {
  if (!c || !X || !out || rows < 0) return MPG_ERR_ARG;
  if (rows == 0) return MPG_OK;
  if (!mpg_mlp_ready(c)) return mpg_fail(c, MPG_ERR_STATE, "MLP has no parameters");
  mpg_mlp_state* s = c->mlp;
  int st = mpg_device_guard(c);
  if (st == MPG_OK) st = reserve(c, s, rows, 1);
  if (st == MPG_OK) st = upload_rows(c, s, X, nullptr, rows);
  if (st != MPG_OK) return st;
  st = mpg_launch(c, MPG_KCLASS_AUX,
                  [&] { return launch_mlp_forward(s->prm, s->X, rows, s->F, s->out, c->stream); },
                  "MLP forward");
  if (st != MPG_OK) return st;
  hipError_t r = hipMemcpyAsync(out, s->out, (size_t)rows * sizeof(float), hipMemcpyDeviceToHost,
                                c->stream);
  if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
  return r == hipSuccess ? MPG_OK : mpg_hip_fail(c, r, "MLP prediction read");
}

extern "C" int mpg_mlp_save(mpg_ctx* c, const char* path) {
  if (!c || !path) return MPG_ERR_ARG;
  std::vector<float> p(mpg_mlp_num_params());
  int st = mpg_mlp_get_params(c, p.data(), (int)p.size());
  if (st != MPG_OK) return st;
  FILE* f = std::fopen(path, "wb");
  if (!f) return mpg_fail(c, MPG_ERR_ARG, "cannot open %s", path);
  const int hdr[4] = {0x4d4c5031 /* "MLP1" */, MPG_MLP_FEATURES, kMlpHidden, (int)p.size()};
  const bool ok = std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
                  std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  std::fclose(f);
  return ok ? MPG_OK : mpg_fail(c, MPG_ERR_ARG, "write to %s failed", path);
}

extern "C" int mpg_mlp_load(mpg_ctx* c, const char* path) {
  if (!c || !path) return MPG_ERR_ARG;
  FILE* f = std::fopen(path, "rb");
  if (!f) return mpg_fail(c, MPG_ERR_ARG, "cannot open %s", path);
  int hdr[4];
  std::vector<float> p(mpg_mlp_num_params());
  bool ok = std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 0x4d4c5031 &&
            hdr[1] == MPG_MLP_FEATURES && hdr[2] == kMlpHidden && hdr[3] == (int)p.size() &&
            std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
  std::fclose(f);
  if (!ok) return mpg_fail(c, MPG_ERR_ARG, "%s is not a saved run-time model", path);
  return mpg_mlp_set_params(c, p.data(), (int)p.size());
}
