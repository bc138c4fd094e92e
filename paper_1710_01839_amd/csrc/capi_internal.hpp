// Host-side internals shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <functional>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mpgemm.h"
#include "internal.hpp"

struct mpg_mlp_state;  // mlp_host.cpp

struct mpg_ctx {
  int device = 0;
  int num_cu = 256;
  hipStream_t stream = nullptr;
  std::string last_error;

  // workspace slots (grow-only, freed with the context): 0 = large operand
  // workspace (Strassen blocks, digit planes), 1 = small (exponents, counters)
  // 2, 3 = batch descriptors (two calls in flight), 4, 5 = packed operands
  // of the BLAS-style calls, 6 = their product before scaling, 7 = residue
  // planes of the residue-form split product, 8 = its product residues and
  // reconstruction table, 9 = split-K partials
  static constexpr int kSlots = 10;
  void* ws[kSlots] = {};
  size_t ws_size[kSlots] = {};
  // batch descriptor uploads: pinned host staging per descriptor slot, and
  // an event after the launch that read it (the slot is free again once it
  // has completed)
  void* batch_pin[2] = {nullptr, nullptr};
  size_t batch_pin_size[2] = {0, 0};
  hipEvent_t batch_done[2] = {nullptr, nullptr};
  int batch_next = 0;
  // failure injection (mpg_test_inject): the next fail_allocs workspace
  // allocations and fail_launches kernel launches fail without a HIP call
  int fail_allocs = 0;
  int fail_launches = 0;

  // kernel timing
  bool prof = false;
  struct Rec {
    int kclass;
    hipEvent_t a, b;
  };
  std::vector<Rec> prof_recs;
  std::vector<hipEvent_t> event_pool;
  double prof_ms[MPG_KCLASS_COUNT] = {0.0, 0.0};
  int64_t prof_n[MPG_KCLASS_COUNT] = {0, 0};

  // tuning table: (precision, m, n, l) -> (algo, tile)
  std::map<std::tuple<int, int64_t, int64_t, int64_t>, std::pair<int, mpg_tile>> table;
  // long-integer product plans: (m, n, l, words_a, words_b) -> plan
  std::map<std::tuple<int64_t, int64_t, int64_t, int, int>, mpg_int_algo> int_table;

  // JSONL timing database of the tuner (empty: none)
  std::string db_path;

  // slice count used by the last split-precision product
  int last_slices = 0;
  int last_moduli = 0;  // moduli of the last residue-form product

  // learned time model (owned)
  mpg_mlp_state* mlp = nullptr;
};

int mpg_fail(mpg_ctx* c, int status, const char* fmt, ...);
int mpg_hip_fail(mpg_ctx* c, hipError_t e, const char* where);
int mpg_device_guard(mpg_ctx* c);
int mpg_workspace(mpg_ctx* c, int slot, size_t bytes, void** out);
int mpg_launch(mpg_ctx* c, int kclass, const std::function<hipError_t()>& fn, const char* what);
size_t mpg_span_bytes(int64_t rows, int64_t cols, int64_t ld);
bool mpg_overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);
int mpg_check_gemm_args(mpg_ctx* c, int limbs, int64_t m, int64_t n, int64_t l,
                        const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
                        double* const* C, int64_t ldc);
int mpg_resolve_variant(mpg_ctx* c, int precision, const mpg_tile* t, int* variant);
int mpg_strassen(mpg_ctx* c, int limbs, int depth, int variant, int64_t m, int64_t n, int64_t l,
                 const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
                 double* const* C, int64_t ldc);
// K chunks of a split-K product (splits 0: chosen from the shape and the
// variant's occupancy on num_cu CUs; at least 1, chunks of at least 256
// unless splits asks for shorter ones) and the chunk length.
void mpg_splitk_plan(int64_t m, int64_t n, int64_t l, int bm, int bn, int bk, int resident, int num_cu,
                     int splits, int64_t* P, int64_t* Kc);
int mpg_splitk(mpg_ctx* c, int limbs, int splits, int variant, int64_t m, int64_t n, int64_t l,
               const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
               double* const* C, int64_t ldc);
// MPG_AUTO's asynchronous double-double residue form (ozaki_host.cpp);
// *used false: the shape admits no residue form, run the block kernel.
int mpg_dd_crt_auto(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* A, const double* A_lo,
                    int64_t lda, const double* B, const double* B_lo, int64_t ldb, double* C_hi, double* C_lo,
                    int64_t ldc, bool* used);
// Quad-double product through the residue form (C := A B, four limbs).
int mpg_qd_crt(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* const* A, int64_t lda,
               const double* const* B, int64_t ldb, double* const* C, int64_t ldc);
// MPG_AUTO's asynchronous quad-double residue form; *used as for DD.
int mpg_qd_crt_auto(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const double* const* A, int64_t lda,
                    const double* const* B, int64_t ldb, double* const* C, int64_t ldc, bool* used);
int mpg_gemm_common(mpg_ctx* c, int limbs, int64_t m, int64_t n, int64_t l,
                    const double* const* A, int64_t lda, const double* const* B, int64_t ldb,
                    double* const* C, int64_t ldc, mpg_algo algo, const mpg_tile* tile);

// tuning table (tuner.cpp)
bool mpg_table_lookup(mpg_ctx* c, int precision, int64_t m, int64_t n, int64_t l, int* algo,
                      mpg_tile* tile);
// set-up of the allocation-free batched product on the current device
// (batch_host.cpp), once per device
void mpg_noalloc_setup(int device);
// long-integer product plans (intgemm_host.cpp / tuner.cpp)
bool mpg_int_table_lookup(mpg_ctx* c, int64_t m, int64_t n, int64_t l, int words_a, int words_b,
                          mpg_int_algo* algo);
int mpg_int_run(mpg_ctx* c, int64_t m, int64_t n, int64_t l, const uint32_t* A, int words_a, int64_t lda,
                int64_t plane_a, const uint32_t* B, int words_b, int64_t ldb, int64_t plane_b, uint32_t* C,
                int words_c, int64_t ldc, int64_t plane_c, int cw, int depth);
int64_t mpg_int_plan_products(int words_a, int words_b, int64_t l, int cw, int depth);
int mpg_int_plan_moduli(int words_a, int words_b, int64_t l, int cw, int depth);
// cached objects owned by the context (MLP state)
void mpg_destroy_cached(mpg_ctx* c);
