// Host side of batched uneven double-double products: descriptor
// construction, the persistent launch, and plans that capture that launch
// once in a HIP graph and replay it.
#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "batch_internal.hpp"
#include "capi_internal.hpp"

using namespace mpg;

struct mpg_batch_plan {
  mpg_ctx* ctx = nullptr;
  int count = 0;
  int variant = 0;
  int grid = 0;
  BatchProblem* d_desc = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Validate and lay out the problems in out[0 .. count] (header, then the
// descriptors): tiles of all problems end to end, problems ordered by
// decreasing l (cost per tile) so that the strided walk hands every workgroup
// a similar mix of long and short tiles.  Allocates nothing.
int fill_desc(mpg_ctx* c, int count, const mpg_dd_problem* P, int variant, BatchProblem* out) {
  if (count < 0 || (count > 0 && !P)) return mpg_fail(c, MPG_ERR_ARG, "bad problem list");
  int bm, bn;
  batch_variant_tile(variant, &bm, &bn);
  for (int i = 0; i < count; ++i) {
    const double* A[4] = {P[i].A_hi, P[i].A_lo, nullptr, nullptr};
    const double* B[4] = {P[i].B_hi, P[i].B_lo, nullptr, nullptr};
    double* C[4] = {P[i].C_hi, P[i].C_lo, nullptr, nullptr};
    int st = mpg_check_gemm_args(c, 2, P[i].m, P[i].n, P[i].l, A, P[i].lda, B, P[i].ldb, C, P[i].ldc);
    if (st != MPG_OK) return mpg_fail(c, st, "problem %d: %s", i, c->last_error.c_str());
  }
  out[0] = BatchProblem{};
  for (int k = 0; k < count; ++k) {
    const mpg_dd_problem& q = P[k];
    BatchProblem& d = out[k + 1];
    d = BatchProblem{};
    d.m = q.m;
    d.n = q.n;
    d.l = q.l;
    d.lda = q.lda;
    d.ldb = q.ldb;
    d.ldc = q.ldc;
    d.A[0] = q.A_hi;
    d.A[1] = q.A_lo;
    d.B[0] = q.B_hi;
    d.B[1] = q.B_lo;
    d.C[0] = q.C_hi;
    d.C[1] = q.C_lo;
    d.tile_start = k;  // the problem's index: keeps equal-l problems in call order
  }
  std::sort(out + 1, out + 1 + count, [](const BatchProblem& a, const BatchProblem& b) {
    return a.l != b.l ? a.l > b.l : a.tile_start < b.tile_start;
  });
  int64_t start = 0;
  for (int k = 1; k <= count; ++k) {
    BatchProblem& d = out[k];
    const int64_t tm = d.m > 0 && d.n > 0 ? (d.m + bm - 1) / bm : 0;
    d.tiles_n = d.m > 0 && d.n > 0 ? (d.n + bn - 1) / bn : 1;
    d.tile_start = start;
    start += tm * d.tiles_n;
  }
  // the tile queue is an int that every workgroup advances once past the end
  if (start > (int64_t)INT_MAX / 2)
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "%lld tiles: too many for one batch", (long long)start);
  out[0].tile_start = start;
  out[0].tiles_n = count;
  return MPG_OK;
}

int build_desc(mpg_ctx* c, int count, const mpg_dd_problem* P, int variant,
               std::vector<BatchProblem>& out) {
  out.assign((size_t)std::max(count, 0) + 1, BatchProblem{});
  return fill_desc(c, count, P, variant, out.data());
}

int batch_variant(mpg_ctx* c, const mpg_tile* tile, int* v) {
  if (!tile || (tile->bm == 0 && tile->bn == 0 && tile->bk == 0 && tile->tm == 0 && tile->tn == 0)) {
    *v = 1;  // 32 x 32 tiles: most problems of a batch are small
    return MPG_OK;
  }
  return mpg_resolve_variant(c, 2, tile, v);
}

int grid_for(mpg_ctx* c, int v, int64_t total) {
  const int64_t g = (int64_t)c->num_cu * batch_blocks_per_cu(v);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, total));
}

}  // namespace

extern "C" int mpgemm_dd_batched(mpg_ctx* c, int count, const mpg_dd_problem* problems,
                                 const mpg_tile* tile) {
  if (!c) return MPG_ERR_ARG;
  int v, st;
  if ((st = batch_variant(c, tile, &v)) != MPG_OK) return st;
  std::vector<BatchProblem> desc;
  if ((st = build_desc(c, count, problems, v, desc)) != MPG_OK) return st;
  if (count == 0 || desc[0].tile_start == 0) return MPG_OK;
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  // Descriptors alternate between two slots (pinned host staging + device
  // copy), so the host does not wait for the previous call: only for the
  // call before it, which used the same slot.
  const int k = c->batch_next;
  hipError_t r = hipSuccess;
  if (!c->batch_done[k]) r = hipEventCreateWithFlags(&c->batch_done[k], hipEventDisableTiming);
  else r = hipEventSynchronize(c->batch_done[k]);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "batch descriptor slot");
  const size_t bytes = batch_desc_bytes(count);
  if (bytes > c->batch_pin_size[k]) {
    if (c->batch_pin[k]) (void)hipHostFree(c->batch_pin[k]);
    c->batch_pin[k] = nullptr;
    c->batch_pin_size[k] = 0;
    if ((r = hipHostMalloc(&c->batch_pin[k], bytes, hipHostMallocDefault)) != hipSuccess) {
      c->batch_pin[k] = nullptr;
      (void)hipGetLastError();
      return mpg_fail(c, MPG_ERR_NOMEM, "pinned staging of %zu bytes failed", bytes);
    }
    c->batch_pin_size[k] = bytes;
  }
  void* d = nullptr;
  if ((st = mpg_workspace(c, 2 + k, bytes, &d)) != MPG_OK) return st;
  std::memcpy(c->batch_pin[k], desc.data(), desc.size() * sizeof(BatchProblem));
  r = hipMemcpyAsync(d, c->batch_pin[k], desc.size() * sizeof(BatchProblem), hipMemcpyHostToDevice,
                     c->stream);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "descriptor upload");
  const int grid = grid_for(c, v, desc[0].tile_start);
  st = mpg_launch(c, MPG_KCLASS_GEMM,
                  [&] { return launch_batch_persistent(v, (BatchProblem*)d, count, grid, c->stream); },
                  "persistent batch kernel");
  if (st != MPG_OK) return st;
  if ((r = hipEventRecord(c->batch_done[k], c->stream)) != hipSuccess)
    return mpg_hip_fail(c, r, "batch descriptor slot");
  c->batch_next = k ^ 1;
  return MPG_OK;
}

extern "C" int mpg_batch_plan_create(mpg_ctx* c, int count, const mpg_dd_problem* problems,
                                     const mpg_tile* tile, mpg_batch_plan** plan) {
  if (!c || !plan) return MPG_ERR_ARG;
  *plan = nullptr;
  int v, st;
  if ((st = batch_variant(c, tile, &v)) != MPG_OK) return st;
  std::vector<BatchProblem> desc;
  if ((st = build_desc(c, count, problems, v, desc)) != MPG_OK) return st;
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  mpg_batch_plan* p = new mpg_batch_plan();
  p->ctx = c;
  p->count = count;
  p->variant = v;
  // the grid is fixed at capture; size it for the largest total tile count
  // any later update may bring (the kernel reads the count at run time)
  p->grid = (int)((int64_t)c->num_cu * batch_blocks_per_cu(v));
  hipError_t r = hipMalloc(&p->d_desc, batch_desc_bytes(count));
  if (r == hipSuccess)
    r = hipMemcpy(p->d_desc, desc.data(), desc.size() * sizeof(BatchProblem), hipMemcpyHostToDevice);
  hipStream_t cs = nullptr;
  if (r == hipSuccess) r = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (r == hipSuccess) r = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (r == hipSuccess) {
    hipError_t lr = launch_batch_persistent(v, p->d_desc, count, p->grid, cs);
    r = hipStreamEndCapture(cs, &p->graph);
    if (lr != hipSuccess) r = lr;
  }
  if (r == hipSuccess) r = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (r != hipSuccess) {
    mpg_batch_plan_destroy(p);
    return mpg_hip_fail(c, r, "batch plan capture");
  }
  *plan = p;
  return MPG_OK;
}

extern "C" int mpg_batch_plan_update(mpg_batch_plan* p, const mpg_dd_problem* problems) {
  if (!p) return MPG_ERR_ARG;
  mpg_ctx* c = p->ctx;
  std::vector<BatchProblem> desc;
  int st = build_desc(c, p->count, problems, p->variant, desc);
  if (st != MPG_OK) return st;
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  hipError_t r = hipStreamSynchronize(c->stream);
  if (r == hipSuccess)
    r = hipMemcpy(p->d_desc, desc.data(), desc.size() * sizeof(BatchProblem), hipMemcpyHostToDevice);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "batch plan update");
  return MPG_OK;
}

extern "C" int mpg_batch_plan_launch(mpg_batch_plan* p, void* stream) {
  if (!p || !p->exec) return MPG_ERR_ARG;
  mpg_ctx* c = p->ctx;
  int st = mpg_device_guard(c);
  if (st != MPG_OK) return st;
  hipStream_t s = stream ? (hipStream_t)stream : c->stream;
  if (s == c->stream)
    return mpg_launch(c, MPG_KCLASS_GEMM, [&] { return hipGraphLaunch(p->exec, s); },
                      "batch graph launch");
  hipError_t r = hipGraphLaunch(p->exec, s);
  return r == hipSuccess ? MPG_OK : mpg_hip_fail(c, r, "batch graph launch");
}

extern "C" int mpg_batch_plan_destroy(mpg_batch_plan* p) {
  if (!p) return MPG_OK;
  if (p->ctx) {
    (void)mpg_device_guard(p->ctx);
    (void)hipStreamSynchronize(p->ctx->stream);
  }
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_desc) (void)hipFree(p->d_desc);
  delete p;
  return MPG_OK;
}

// ---------------------------------------------------------------------------
// The batched product without allocation: descriptors and tile queue in a
// fixed device array (one per GPU), staged through a fixed host array.
// ---------------------------------------------------------------------------

namespace {

constexpr int kNoAllocMaxProblems = 8192;
constexpr size_t kNoAllocScratchBytes = (size_t)1 << 20;
static_assert((kNoAllocMaxProblems + 1) * sizeof(BatchProblem) + sizeof(int) <= kNoAllocScratchBytes,
              "descriptors and queue of the largest batch fit the scratch array");
constexpr int kNoAllocMaxDevices = 16;

}  // namespace

// Device memory of the allocation-free entry point (each GPU holds its own
// copy until the process ends).  In host code this name stands for the array
// but is not its device address: the address comes from hipGetSymbolAddress,
// once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

struct NoAllocDevice {
  std::once_flag once;
  int status = MPG_ERR_STATE;      // MPG_OK once set up
  hipError_t err = hipSuccess;     // the failing HIP call's error, if any
  void* ptr = nullptr;             // device address of this GPU's scratch
  hipEvent_t uploaded = nullptr;   // after the last upload from `staging`
  bool pending = false;
  alignas(256) BatchProblem staging[kNoAllocMaxProblems + 1];
};
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

}  // namespace

// Set-up of the allocation-free batched product for the current device
// (called by mpg_create with that device current; the work runs once per
// device): the device address of its scratch array and the event that
// orders reuse of the host staging.
void mpg_noalloc_setup(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return;
  NoAllocDevice& d = g_noalloc[device];
  std::call_once(d.once, [&d] {
    void* p = nullptr;
    hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (r == hipSuccess) r = hipEventCreateWithFlags(&d.uploaded, hipEventDisableTiming);
    if (r != hipSuccess) {
      (void)hipGetLastError();
      d.err = r;
      d.status = MPG_ERR_HIP;
      return;
    }
    d.ptr = p;
    d.status = MPG_OK;
  });
}

extern "C" int mpgemm_dd_batched_noalloc(mpg_ctx* c, int count, const mpg_dd_problem* problems,
                                         const mpg_tile* tile) {
  if (!c) return MPG_ERR_ARG;
  if (count < 0 || count > kNoAllocMaxProblems)
    return mpg_fail(c, MPG_ERR_ARG, "%d problems: the allocation-free batch holds 0..%d", count,
                    kNoAllocMaxProblems);
  if (c->device < 0 || c->device >= kNoAllocMaxDevices)
    return mpg_fail(c, MPG_ERR_UNSUPPORTED, "device %d: the allocation-free batch serves devices 0..%d",
                    c->device, kNoAllocMaxDevices - 1);
  NoAllocDevice& d = g_noalloc[c->device];
  if (d.status != MPG_OK)
    return d.err != hipSuccess ? mpg_hip_fail(c, d.err, "scratch set-up")
                               : mpg_fail(c, MPG_ERR_STATE, "scratch not set up");
  int v, st;
  if ((st = batch_variant(c, tile, &v)) != MPG_OK) return st;
  if ((st = mpg_device_guard(c)) != MPG_OK) return st;
  // the host staging is reused: the previous call's upload must have read it
  hipError_t r = hipSuccess;
  if (d.pending) {
    if ((r = hipEventSynchronize(d.uploaded)) != hipSuccess) return mpg_hip_fail(c, r, "staging reuse");
    d.pending = false;
  }
  if ((st = fill_desc(c, count, problems, v, d.staging)) != MPG_OK) return st;
  const int64_t total = d.staging[0].tile_start;
  if (count == 0 || total == 0) return MPG_OK;
  BatchProblem* dev = static_cast<BatchProblem*>(d.ptr);
  r = hipMemcpyAsync(dev, d.staging, (size_t)(count + 1) * sizeof(BatchProblem), hipMemcpyHostToDevice,
                     c->stream);
  if (r == hipSuccess) r = hipEventRecord(d.uploaded, c->stream);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "descriptor upload");
  d.pending = true;
  // the queue counter behind the descriptors is zeroed by a fill kernel
  // before the persistent launch
  r = launch_batch_persistent(v, dev, count, grid_for(c, v, total), c->stream);
  if (r != hipSuccess) return mpg_hip_fail(c, r, "persistent batch kernel");
  return MPG_OK;
}
