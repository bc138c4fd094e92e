// Persistent kernel for a batch of uneven double-double products: a fixed
// grid draws tiles from one global tile index space (problem tiles laid end
// to end, problems by decreasing l, so the most expensive tiles go first)
// through an atomic queue, each tile computed by the block-algorithm tile
// routine of the single-problem kernel (bitwise identical results).  A
// workgroup leaves when it draws an index past the last tile.
#include "batch_internal.hpp"
#include "gemm_kernels.hpp"

namespace mpg {
namespace {

__global__ void queue_reset_kernel(int* next) {
  if (threadIdx.x == 0) *next = 0;
}

template <int BM, int BN, int BK, int TM, int TN, int MINW>
__global__ __launch_bounds__((BM / TM) * (BN / TN), MINW) void persistent_kernel(
    const BatchProblem* desc, int* next) {
  __shared__ kern::BlockSmem<2, BM, BN, BK> sm;
  __shared__ int s_w;
  const int64_t total = desc[0].tile_start;
  const int count = (int)desc[0].tiles_n;
  const BatchProblem* probs = desc + 1;
  for (;;) {
    if (threadIdx.x == 0) s_w = atomicAdd(next, 1);
    __syncthreads();
    const int64_t w = s_w;
    if (w >= total) break;
    // last problem whose first tile is <= w
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (probs[mid].tile_start <= w) lo = mid;
      else hi = mid - 1;
    }
    const BatchProblem& P = probs[lo];
    const int64_t t = w - P.tile_start;
    const int64_t tm = t / P.tiles_n, tn = t % P.tiles_n;
    kern::block_tile<DDArith, BM, BN, BK, TM, TN>(sm, P.m, P.n, P.l, P.A, P.lda, P.B, P.ldb, P.C,
                                                  P.ldc, tm * BM, tn * BN);
    __syncthreads();
  }
}

using Fn = const void*;
struct Entry {
  int bm, bn;
  Fn fn;
  int threads;
};

#define MPG_ENTRY(BM, BN, BK, TM, TN, W) \
  {BM, BN, reinterpret_cast<Fn>(&persistent_kernel<BM, BN, BK, TM, TN, W>), (BM / TM) * (BN / TN)}

// Same shapes and indices as the DD block variants.
const Entry kEntries[] = {
    MPG_ENTRY(64, 64, 16, 4, 4, 2),  MPG_ENTRY(32, 32, 16, 2, 2, 2),
    MPG_ENTRY(128, 64, 8, 8, 4, 1),  MPG_ENTRY(64, 128, 8, 4, 8, 1),
    MPG_ENTRY(128, 128, 8, 8, 8, 1), MPG_ENTRY(64, 64, 8, 4, 4, 2),
    MPG_ENTRY(32, 64, 16, 2, 4, 2),  MPG_ENTRY(64, 64, 8, 2, 4, 2),
};
constexpr int kN = sizeof(kEntries) / sizeof(kEntries[0]);

}  // namespace

int batch_num_variants() { return kN; }

void batch_variant_tile(int v, int* bm, int* bn) {
  *bm = kEntries[v].bm;
  *bn = kEntries[v].bn;
}

int batch_blocks_per_cu(int v) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kEntries[v].fn, kEntries[v].threads, 0) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

size_t batch_desc_bytes(int count) { return (size_t)(count + 1) * sizeof(BatchProblem) + sizeof(int); }

int* batch_queue(BatchProblem* d_desc, int count) { return reinterpret_cast<int*>(d_desc + count + 1); }

hipError_t launch_batch_persistent(int v, BatchProblem* d_desc, int count, int grid, hipStream_t s) {
  if (v < 0 || v >= kN) return hipErrorInvalidValue;
  int* next = batch_queue(d_desc, count);
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, s, next);
  hipError_t r = hipGetLastError();
  if (r != hipSuccess) return r;
  const BatchProblem* desc = d_desc;
  void* args[] = {(void*)&desc, (void*)&next};
  return hipLaunchKernel(kEntries[v].fn, dim3(grid), dim3(kEntries[v].threads), args, 0, s);
}

}  // namespace mpg
