// Internal interface of the batched persistent DD kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

// One problem of a batch, as read by the persistent kernel.  The array is
// preceded by a header element whose tile_start holds the total tile count
// and whose tiles_n holds the problem count, so a captured launch stays
// valid when the descriptors are rewritten.  The device copy is followed by
// one int: the tile queue the workgroups draw from (zeroed by a reset
// kernel before each persistent launch).
struct BatchProblem {
  int64_t m, n, l, lda, ldb, ldc;
  const double* A[2];
  const double* B[2];
  double* C[2];
  int64_t tile_start;  // first global tile index of this problem
  int64_t tiles_n;     // tiles along n
};

int batch_num_variants();
// Tile shape (BM, BN) of a variant (same indices as the DD block variants).
void batch_variant_tile(int v, int* bm, int* bn);
// Workgroups of variant v that fit on one CU.
int batch_blocks_per_cu(int v);
// Device bytes for `count` problems: header, descriptors, queue counter.
size_t batch_desc_bytes(int count);
// The queue counter inside a device descriptor copy of `count` problems.
int* batch_queue(BatchProblem* d_desc, int count);
// Zeroes the queue, then the persistent kernel (both on stream s).
hipError_t launch_batch_persistent(int v, BatchProblem* d_desc, int count, int grid, hipStream_t s);

}  // namespace mpg
