/*
 * mpgemm.h -- C ABI of the MI355X (gfx950) multiple-precision dense matrix
 * multiplication library libmpgemm.so.
 *
 * The library computes C := AB (Section 2 of Kouya, "Tuning Technique for
 * Multiple Precision Dense Matrix Multiplication using Prediction of
 * Computational Time", arXiv:1710.01839), A m x l, B l x n, C m x n, in
 * double-double (DD, two FP64 limbs) or quad-double (QD, four limbs)
 * arithmetic, by the simple algorithm (Eq. 1), the block algorithm (Eq. 2)
 * or Strassen's recursion (Eq. 3, Winograd's variant of it), and chooses
 * among them with the tuning procedure of Section 3.
 *
 * Conventions for every entry point:
 *   - Matrices are row-major limb planes: a DD matrix is two separate FP64
 *     arrays (hi, lo), a QD matrix four; element (i, j) of a plane with
 *     leading dimension ld is at offset i*ld + j.  lda >= l, ldb >= n,
 *     ldc >= n.  Inputs must be canonical (each limb at most half an ulp of
 *     the limb before it) and finite with magnitude below 2^900.
 *   - All matrix pointers are DEVICE pointers owned by the caller.  The
 *     library owns only its workspace (cached in the context) and the
 *     objects it creates.
 *   - Calls are asynchronous on the context's stream (mpg_set_stream); C is
 *     valid once that stream has completed the call.
 *   - C := AB overwrites C.  m == 0 or n == 0 is a no-op; l == 0 sets C = 0.
 *   - C must not overlap A or B (MPG_ERR_ALIAS).
 *   - Every call returns an mpg_status.  Argument errors are detected before
 *     anything is launched.  A HIP failure returns MPG_ERR_HIP and
 *     mpg_last_error() holds the HIP error name.
 *   - One context must not be used by two host threads at once.
 */
#ifndef MPGEMM_H
#define MPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpg_ctx mpg_ctx;

typedef enum {
  MPG_OK = 0,
  MPG_ERR_ARG = -1,         /* invalid argument (null pointer, bad size or ld) */
  MPG_ERR_UNSUPPORTED = -2, /* a tile / algorithm combination that is not built */
  MPG_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  MPG_ERR_NOMEM = -4,       /* workspace allocation failed */
  MPG_ERR_ALIAS = -5,       /* C overlaps A or B */
  MPG_ERR_STATE = -6        /* object in the wrong state (e.g. MLP not trained) */
} mpg_status;

typedef enum {
  MPG_AUTO = 0,     /* use the context's tuning table, else a default; a tabled split
                       product the data's exact slice count rules out falls back to
                       MPG_BLOCK of the same precision.  A tabled DD or QD residue
                       form (MPG_OZAKI_CRT, slices 0) stays asynchronous: the slice
                       and moduli counts (for QD also the part products with an
                       all-zero part) are decided on the device, the residue-form
                       kernels are launched for the most moduli 20 slices need and
                       take the device's counts, and the block kernel launched after
                       them runs only when more than 20 slices are needed; after one
                       eager call of a shape (which grows the workspace) the call
                       allocates nothing and can be captured in a HIP graph, whose
                       replays decide again from the data (mpg_ozaki_last_slices and
                       mpg_ozaki_last_moduli then read 0).  The tabled digit form
                       (MPG_OZAKI, slices 0) reads its count back (one stream
                       synchronisation). */
  MPG_SIMPLE = 1,   /* Eq. (1): one thread per c_ij, k in order */
  MPG_BLOCK = 2,    /* Eq. (2): LDS-staged tiles, register-blocked accumulators */
  MPG_STRASSEN = 3, /* Eq. (3), Winograd's form, `depth` levels over MPG_BLOCK */
  MPG_OZAKI = 4,    /* split-precision INT8 product (DD only: mpgemm_dd_ozaki with
                       tile->slices, all pairs) */
  MPG_OZAKI_CRT = 5, /* its residue form: DD through mpgemm_dd_ozaki with tile->slices,
                       pairs_mode 2; QD as three residue-form products of the
                       operands' double-double parts (mpgemm_qd) */
  MPG_SPLITK = 6    /* Eq. (2) with K cut into tile->splits consecutive chunks (0: as
                       many as fill the GPU twice with workgroups, chunks of at least
                       256), each chunk's product by MPG_BLOCK of the tile into
                       workspace, the partials of every entry added in a fixed order
                       (lanes of a wavefront sum interleaved partials in order, then a
                       butterfly across the lanes); for skinny shapes (few C tiles,
                       long K) */
} mpg_algo;

/* Tile / algorithm parameters.  Zero fields mean "library default" (DD:
 * 64 x 64 x 8 with 2 x 4 per thread, operands moved to LDS by the load unit
 * when n, l and the leading dimensions are even; QD: 32 x 32 x 8, 2 x 2).
 * (bm, bn, bk, tm, tn) must name one of the built block-kernel variants
 * (mpg_num_variants / mpg_variant), otherwise MPG_ERR_UNSUPPORTED.  The
 * paper's block size n_min corresponds to the C tile (bm x bn) and its
 * K-step bk. */
typedef struct {
  int bm, bn, bk; /* C tile of one workgroup and K step staged in LDS */
  int tm, tn;     /* per-thread register block */
  int depth;      /* Strassen recursion depth (MPG_STRASSEN), 1..3 */
  int slices;     /* Ozaki slice count (MPG_OZAKI) */
  int splits;     /* K chunks of MPG_SPLITK (0: chosen from the shape) */
} mpg_tile;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  The stream defaults to the
 * null stream.  *ctx receives the new context. */
int mpg_create(mpg_ctx** ctx, int device);
/* Free the context, its workspace and cached objects (synchronises its
 * stream first).  NULL is accepted. */
int mpg_destroy(mpg_ctx* ctx);
/* Set the stream (a hipStream_t passed as void*) used by later calls. */
int mpg_set_stream(mpg_ctx* ctx, void* hip_stream);
/* Static text of a status code. */
const char* mpg_status_string(int status);
/* Detail of the last error on this context ("" if none). */
const char* mpg_last_error(const mpg_ctx* ctx);

/* ---- block-kernel variants -------------------------------------------- */

/* Number of built block-kernel tile variants (DD: precision 2, QD: 4). */
int mpg_num_variants(int precision);
/* Fill *tile with variant `index` of the given precision. */
int mpg_variant(int precision, int index, mpg_tile* tile);
/* Workgroups of block variant `index` that the runtime's occupancy
 * calculator places on one CU of the context's device (the wave size of the
 * GPU form of the time prediction is this times the CU count). */
int mpg_variant_resident(mpg_ctx* ctx, int precision, int index, int* blocks);

/* ---- DD GEMM ---------------------------------------------------------- */

/* C := A B in double-double.  A = A_hi + A_lo (m x l), B = B_hi + B_lo
 * (l x n), C = C_hi + C_lo (m x n).  algo MPG_SIMPLE, MPG_BLOCK,
 * MPG_STRASSEN (tile->depth levels of Winograd's recursion over the block
 * kernel, odd or non-tile dimensions zero-padded in workspace), MPG_SPLITK
 * or MPG_AUTO.  tile may be NULL.  Error: componentwise |C - AB|_ij <=
 * 8 l 2^-104 (|A||B|)_ij for SIMPLE, BLOCK and SPLITK; STRASSEN obeys a
 * normwise bound that grows with depth.  SIMPLE and BLOCK give bitwise
 * identical results; SPLITK is deterministic (a fixed order for each
 * shape and chunk count) and exact wherever the block kernel is (integer
 * data). */
int mpgemm_dd(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l,
              const double* A_hi, const double* A_lo, int64_t lda,
              const double* B_hi, const double* B_lo, int64_t ldb,
              double* C_hi, double* C_lo, int64_t ldc,
              mpg_algo algo, const mpg_tile* tile);

/* ---- QD GEMM ---------------------------------------------------------- */

/* C := A B in quad-double.  A, B and C are arrays of four limb-plane
 * pointers (leading limb first), each plane row-major with the given
 * leading dimension.  algo MPG_SIMPLE, MPG_BLOCK, MPG_STRASSEN, MPG_SPLITK
 * or MPG_AUTO as for mpgemm_dd.  Error: componentwise |C - AB|_ij <=
 * 8 l 2^-208 (|A||B|)_ij for SIMPLE, BLOCK (bitwise identical to each
 * other) and SPLITK.
 * MPG_OZAKI_CRT: each operand is split exactly into its double-double parts
 * (limbs 0 + 1, limbs 2 + 3); A_H B_H, A_H B_L and A_L B_H are formed
 * exactly by the residue form (one slice count, the largest exact count of
 * the parts taking part, at most 20, else MPG_ERR_UNSUPPORTED; synchronises
 * the stream once for the counts)
 * and added in quad-double; A_L B_L is left out (below 2^-210 (|A||B|) for
 * canonical operands). */
int mpgemm_qd(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l,
              const double* const A[4], int64_t lda,
              const double* const B[4], int64_t ldb,
              double* const C[4], int64_t ldc,
              mpg_algo algo, const mpg_tile* tile);

/* ---- BLAS-style form: transposes, alpha / beta, complex DD ------------- */

/* op(X): X, its transpose, or its conjugate transpose (the transpose for
 * real matrices). */
typedef enum { MPG_OP_N = 0, MPG_OP_T = 1, MPG_OP_C = 2 } mpg_op;

/* C := alpha op(A) op(B) + beta C, the xGEMM form of the BLAS around the
 * product of Eq. (1), in DD (precision 2) or QD (precision 4).  op(A) is
 * m x k and op(B) is k x n: A is stored m x k (lda >= k) for MPG_OP_N and
 * k x m (lda >= m) otherwise; B is stored k x n (ldb >= n) or n x k
 * (ldb >= k).  A, B and C are arrays of `precision` limb-plane DEVICE
 * pointers (leading limb first); alpha and beta are HOST arrays of
 * `precision` limbs.  algo and tile choose the product as for mpgemm_dd /
 * mpgemm_qd (MPG_OZAKI with precision 2 only).
 *   - beta == 0: C is not read (NaN in C does not propagate).
 *   - alpha == 0 or k == 0: A and B are not read; C := beta C.
 *   - transposed operands are copied to workspace by an O(mk + kn) pack
 *     kernel; unless alpha == 1 and beta == 0 the product goes to workspace
 *     and an element-wise kernel forms alpha T + beta C.
 * Error (SIMPLE, BLOCK): |C' - (alpha op(A) op(B) + beta C)|_ij <=
 *   2^-104 [(8k + 16) |alpha| (|op(A)||op(B)|)_ij + 16 |beta| |C_ij|]
 * with 2^-208 for QD; other algorithms add their own product bound scaled
 * by |alpha|.  C must not overlap A or B (MPG_ERR_ALIAS). */
int mpg_rgemm(mpg_ctx* ctx, int precision, mpg_op transa, mpg_op transb,
              int64_t m, int64_t n, int64_t k, const double* alpha,
              const double* const* A, int64_t lda,
              const double* const* B, int64_t ldb, const double* beta,
              double* const* C, int64_t ldc, mpg_algo algo, const mpg_tile* tile);

/* Complex double-double C := alpha op(A) op(B) + beta C (op: MPG_OP_N,
 * MPG_OP_T, MPG_OP_C).  Each complex matrix is four limb-plane DEVICE
 * pointers {re hi, re lo, im hi, im lo} with one leading dimension; alpha and
 * beta are HOST arrays in the same order.  Storage shapes and leading
 * dimensions as for mpg_rgemm; m, n, k <= 2^30.
 * The four real products are formed in one real DD product of the embedding
 *   [Re op(A)  Im op(A)] . [[Re op(B), Im op(B)], [-Im op(B), Re op(B)]]
 * (m x 2k times 2k x 2n, packed in workspace, conjugation folded into the
 * pack), so each real and imaginary part accumulates its 2k terms in one DD
 * accumulator; algo and tile apply to that product (MPG_OZAKI allowed).
 * An element-wise kernel forms alpha P + beta C.  beta == 0: C not read;
 * alpha == 0 or k == 0: C := beta C.
 * Error (SIMPLE, BLOCK), both parts:
 *   2^-104 [(16k + 32)(|ar| + |ai|) ((|Ar| + |Ai|)(|Br| + |Bi|))_ij
 *           + 32 (|br| + |bi|)(|Cr| + |Ci|)_ij]. */
int mpg_zgemm_dd(mpg_ctx* ctx, mpg_op transa, mpg_op transb,
                 int64_t m, int64_t n, int64_t k, const double alpha[4],
                 const double* const A[4], int64_t lda,
                 const double* const B[4], int64_t ldb, const double beta[4],
                 double* const C[4], int64_t ldc, mpg_algo algo, const mpg_tile* tile);

/* ---- exact long-integer (fixed-point) products -------------------------- */

/* C := A B exactly for matrices of long integers: the fixed-point analog of
 * the paper's 128- to 2048-bit runs (a fixed-point number x 2^-f is its
 * integer x; the product carries 2^-(fa + fb)).  Entries are two's
 * complement integers of words_a / words_b 32-bit words (1..64: up to 2048
 * bits), stored as word planes: word w of entry (i, k) of A is
 * A[w * plane_a + i * lda + k] (DEVICE memory); likewise B (l x n) and C
 * (m x n, words_c planes).  words_c must be at least
 * mpg_int_words_needed(words_a, words_b, l), so every product fits and the
 * result is exact.  Through INT8 matrix cores: entries are cut into 128-bit
 * chunks; for each modulus of the residue form the chunk pairs of one
 * diagonal (chunk indices summing to g) are multiplied in one INT8 product
 * over a K made of the pairs; each diagonal's exact integer sum is rebuilt
 * by the Chinese remainder theorem and added at 2^(128 g) into C.  C must
 * not overlap A or B. */
int mpg_int_gemm(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l,
                 const uint32_t* A, int words_a, int64_t lda, int64_t plane_a,
                 const uint32_t* B, int words_b, int64_t ldb, int64_t plane_b,
                 uint32_t* C, int words_c, int64_t ldc, int64_t plane_c);
/* Words that hold every entry of a product of words_a- and words_b-word
 * operands with inner dimension l: ceil((32 (words_a + words_b) - 1 +
 * bit length of l) / 32) (0 for bad arguments).  Host only. */
int mpg_int_words_needed(int words_a, int words_b, int64_t l);

/* How the long-integer product is formed (all choices give the same exact
 * result):
 *   chunk_words      3, 4 or 5: entries are cut into chunks of 96, 128 or
 *                    160 bits; wider chunks mean fewer chunk pairs but more
 *                    moduli per product (the diagonal sums have
 *                    64 chunk_words + log2 l + log2 chunks + 1 bits, at most
 *                    the 342 bits of the 49 moduli);
 *   karatsuba_depth  0..3 levels of Karatsuba's splitting of the chunk
 *                    polynomials (x = 2^(32 chunk_words)): each level forms
 *                    the residues of the chunk sums of the two halves and
 *                    needs three half-length products instead of four; the
 *                    leaf products' diagonals are kept and each diagonal of
 *                    the product is rebuilt from its signed combination
 *                    (residues combined modulo each modulus first).
 * A plan that does not fit (chunks too wide for l, more than 16 chunk pairs
 * per diagonal, sums of more than eight chunks) gives MPG_ERR_UNSUPPORTED. */
typedef struct {
  int chunk_words;
  int karatsuba_depth;
} mpg_int_algo;

/* mpg_int_gemm with an explicit plan (algo) or, with algo NULL, the
 * context's tuning table for this shape and these word counts (filled by
 * mpg_int_tune), else 128-bit chunks without splitting.  mpg_int_gemm is
 * this call with algo NULL. */
int mpg_int_gemm_ex(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l,
                    const uint32_t* A, int words_a, int64_t lda, int64_t plane_a,
                    const uint32_t* B, int words_b, int64_t ldb, int64_t plane_b,
                    uint32_t* C, int words_c, int64_t ldc, int64_t plane_c,
                    const mpg_int_algo* algo);

/* Candidate plans of a product (every chunk width and Karatsuba depth 0..2
 * that fits), host only; and the INT8 products a plan runs (chunk pairs of
 * all leaf diagonals times moduli, each of m x n x l), 0 if it does not fit. */
int mpg_int_num_candidates(int words_a, int words_b, int64_t l);
int mpg_int_candidate(int words_a, int words_b, int64_t l, int index, mpg_int_algo* algo);
int64_t mpg_int_products(int words_a, int words_b, int64_t l, const mpg_int_algo* algo);

/* Median of `reps` timings (after a warm-up) of the plan on library buffers
 * of the shape (uniform random words); milliseconds. */
int mpg_int_time(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l, int words_a, int words_b,
                 const mpg_int_algo* algo, int reps, double* ms);

/* Section 3's prediction for the long-integer product, GPU form: the plan's
 * time on slabs of A's rows against the full B, one and two waves of the
 * residue products (a wave: enough 256-row tile rows that the tile rows x
 * column tiles x moduli workgroups of a product occupy every CU once),
 * extrapolated linearly in tile rows to m; a product of at most two waves is
 * timed whole.  Timed on library buffers (uniform random words; the time
 * does not depend on the values).  *slab_ms (nullable): the slabs' time. */
int mpg_int_predict(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l, int words_a, int words_b,
                    const mpg_int_algo* algo, double* predicted_ms, double* slab_ms);

/* Tunes the plan of one product (mode as mpg_tune: exhaustive; the paper's
 * procedure: predict every candidate from slabs, then time the best
 * predicted one and the default plan at full size and keep the faster; or
 * the run-time model ranks the candidates and the best topk (0: one per 4,
 * at least 2) are timed).  The winner enters the table used by
 * mpg_int_gemm.  Outputs nullable, as for mpg_tune. */
int mpg_int_tune(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l, int words_a, int words_b, int mode,
                 int topk, mpg_int_algo* best, double* best_ms, double* seconds, int* trials);

/* ---- batches of uneven DD products ------------------------------------ */

/* One problem C := A B of a batch (same conventions as mpgemm_dd). */
typedef struct {
  int64_t m, n, l, lda, ldb, ldc;
  const double *A_hi, *A_lo, *B_hi, *B_lo;
  double *C_hi, *C_lo;
} mpg_dd_problem;

typedef struct mpg_batch_plan mpg_batch_plan;

/* All problems in one persistent launch: a grid of (CUs x resident
 * workgroups) draws the tiles of every problem, laid end to end (problems
 * by decreasing l), from an atomic queue, with the block algorithm (Eq. 2)
 * of tile variant `tile` (NULL: 32 x 32 tiles); results are bitwise those
 * of mpgemm_dd(MPG_BLOCK) with that tile.  `problems` is a host array; the
 * descriptors are staged in pinned memory and uploaded on the context
 * stream in one of two alternating slots (the call waits only for the
 * context's batch before the previous one).  Asynchronous otherwise. */
int mpgemm_dd_batched(mpg_ctx* ctx, int count, const mpg_dd_problem* problems,
                      const mpg_tile* tile);

/* mpgemm_dd_batched for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * persistent launch and bitwise the same results, with the descriptors and
 * the tile queue in a fixed 1 MiB device array per GPU (set up once per
 * device by mpg_create) instead of context workspace and pinned staging.
 * Makes no hipMalloc, hipFree, hipHostMalloc or other allocating call.
 *   count      0..8192 problems (MPG_ERR_ARG beyond; devices 0..15).
 *   problems   host array, read during the call only; the descriptors pass
 *              through a fixed host staging array, so a call first waits
 *              for the previous call's upload from it to complete.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * descriptors; the queue counter is zeroed by a kernel before each launch.
 * Calls that overlap on one GPU (two streams, or two host threads) race on
 * the array and the staging: order them on one stream.  Errors as for
 * mpgemm_dd_batched. */
int mpgemm_dd_batched_noalloc(mpg_ctx* ctx, int count, const mpg_dd_problem* problems,
                              const mpg_tile* tile);

/* Capture that persistent launch once in a HIP graph.  The plan owns the
 * graph and a device copy of the descriptors; `problems` is only read
 * during the call. */
int mpg_batch_plan_create(mpg_ctx* ctx, int count, const mpg_dd_problem* problems,
                          const mpg_tile* tile, mpg_batch_plan** plan);
/* Replay the graph on `stream` (a hipStream_t; NULL = the context stream). */
int mpg_batch_plan_launch(mpg_batch_plan* plan, void* stream);
/* Rewrite the descriptors in place (same count; shapes and pointers may
 * change); the captured graph stays valid.  Waits for the context stream. */
int mpg_batch_plan_update(mpg_batch_plan* plan, const mpg_dd_problem* problems);
/* Free the plan (waits for the context stream).  NULL is accepted. */
int mpg_batch_plan_destroy(mpg_batch_plan* plan);

/* ---- split-precision (Ozaki) DD product on INT8 MFMA ------------------ */

/* C := A B to double-double accuracy from FP64 inputs A (m x l) and B
 * (l x n) through INT8 matrix cores (error-free splitting of Ozaki, Ogita,
 * Oishi and Rump; INT8 form of Ootomo, Ozaki and Yokota).  Each row of A is
 * scaled by 2^-(e_i + 2) and each column of B by 2^-(f_j + 2) into
 * (-1/4, 1/4) (e_i the smallest integer with max_k |a_ik| < 2^e_i) and cut
 * into `slices` radix-256 digit planes of signed bytes: digits by
 * truncation toward zero (exact), then a carry from the least significant
 * digit up brings each into [-128, 127].  The products of digit planes s
 * and t are exact INT32 sums, grouped by diagonal g = s + t, scaled by
 * 2^(e_i + f_j + 4 - 8g) and added in double-double.
 *   slices     1..40, or 0 = as many as make every digit expansion exact,
 *              ceil((e_i + 2 - lowest set bit) / 8) over all rows and
 *              columns (found by a device scan; synchronises the stream).
 *              With the exact count and pairs_mode 0 the only rounding is
 *              the double-double recombination, so the result meets the
 *              DD bound 8 l 2^-104 (|A||B|)_ij.
 *   pairs_mode 0: all slices^2 digit-plane pairs; 1: only s + t <= slices + 1;
 *              2: the residue (Chinese remainder) form: the integer images
 *              A'_ik = sum of the row's digits (|A'_ik| < 2^(8 slices - 2)),
 *              likewise B', are reduced modulo the N leading moduli of
 *              {256, 255, 253, 251, 247, 241, ...} (pairwise coprime, taken
 *              greedily from 256 down; residues are signed bytes), N chosen
 *              so that their product P exceeds 2 l 2^(16 slices - 4); one
 *              INT8 product per modulus (N products instead of slices^2),
 *              each reduced modulo its modulus; the exact integer product
 *              X = (A' B')_ij is rebuilt by the Chinese remainder theorem in
 *              32-bit words and C_ij = X 2^(e_i + f_j + 4 - 16 slices) is
 *              rounded to double-double once (no recombination error).
 *              slices <= 20; any l (sums reduced every 2047 K steps).
 * With fewer slices the truncation error is below
 * l 2^(e_i + f_j) 2^(3 - 8 slices) per entry (pairs_mode 0 and 2).
 * Up to 24 slices any l (the INT32 sums are flushed every 2048 / slices
 * K steps of 64); above 24 slices l <= 32704.  C_hi/C_lo must not overlap
 * A, B. */
int mpgemm_ozaki_dd(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l,
                    const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* C_hi, double* C_lo, int64_t ldc, int slices, int pairs_mode);

/* C := A B for double-double inputs (A_hi + A_lo, B_hi + B_lo) through the
 * same INT8 path.  Each element's two limbs are split together as one
 * exact value: the scaled remainder is kept as a renormalised pair and
 * each digit is the truncation toward zero of its exact value.  The scales
 * e_i, f_j come from the hi limbs; the exact slice count (slices = 0)
 * covers the lowest set bit of either limb, so the result is the exact
 * product of the limb sums up to the double-double recombination (inside
 * the DD bound 8 l 2^-104 (|A||B|)_ij).  Arguments, limits and errors as
 * for mpgemm_ozaki_dd; the lo limbs share the leading dimension of their
 * hi limbs.  mpgemm_dd with MPG_OZAKI calls this with tile->slices and
 * pairs_mode 0. */
int mpgemm_dd_ozaki(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l,
                    const double* A_hi, const double* A_lo, int64_t lda,
                    const double* B_hi, const double* B_lo, int64_t ldb,
                    double* C_hi, double* C_lo, int64_t ldc, int slices, int pairs_mode);

/* Moduli of the last pairs_mode 2 product on this context (0 if none). */
int mpg_ozaki_last_moduli(const mpg_ctx* ctx);
/* Moduli a pairs_mode 2 product of `slices` slices and inner dimension l
 * uses (0 if slices is outside 1..20 or the product is too wide).  Host
 * only. */
int mpg_crt_moduli_for(int slices, int64_t l);

/* The slice count that makes the digit planes of A's rows and B's columns
 * exact (the count slices = 0 would use).  Synchronises the stream. */
int mpg_ozaki_slices_exact(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l,
                           const double* A, int64_t lda, const double* B, int64_t ldb,
                           int* slices);

/* The splitting step alone.  side 0: rows of X (rows x cols) get exponents
 * exps[rows] and digit planes out[s][r][k]; side 1: columns of X get
 * exps[cols] and planes out[s][c][k] (transposed, K contiguous).  Lines are
 * padded to a multiple of 64 and K to a multiple of 64 with zero digits:
 * ld_out >= round64(K) and plane >= round64(lines) * ld_out bytes, both
 * multiples of 8, out 8-byte aligned.  out and exps are device buffers
 * owned by the caller. */
int mpg_ozaki_split(mpg_ctx* ctx, int side, int64_t rows, int64_t cols,
                    const double* X, int64_t ldx, int slices,
                    int8_t* out, int64_t ld_out, int64_t plane, int32_t* exps);

/* Sustained INT8 matrix-core rate of the device, in TOP/s (1 multiply-add =
 * 2 operations): back-to-back v_mfma_i32_16x16x64_i8 with no memory
 * traffic, four workgroups of 8 wavefronts per CU, the best of three
 * event-timed runs.  The ceiling the split products' kernels are compared
 * with beside the datasheet peak.  Synchronises the stream. */
int mpg_int8_mfma_rate(mpg_ctx* ctx, double* tops);

/* Slice count used by the context's last mpgemm_ozaki_dd / mpgemm_dd_ozaki call. */
int mpg_ozaki_last_slices(const mpg_ctx* ctx);

/* Fewest slices whose a-priori truncation bound meets a target of `bits`:
 * |C - AB|_ij <= l 2^(e_i + f_j) 2^-bits before the double-double rounding
 * of the recombination (e_i, f_j the row and column scales above).  The
 * bound per unit of l 2^(e_i + f_j) is 2^(3 - 8S) with all pairs
 * (pairs_mode 0) and that plus sum over g = S+2..2S of
 * (2S - g + 1) 128^2 2^(4 - 8g) with the triangle (pairs_mode 1).  Host
 * only.  Returns 0 for bits < 1, a bad pairs_mode, or a target that 40
 * slices do not reach. */
int mpg_ozaki_slices_for_bits(int bits, int pairs_mode);

/* Slice count and pair set of the split-precision product of FP64 inputs
 * for an accuracy target of `bits` (as for mpg_ozaki_slices_for_bits),
 * chosen by measured time.  Candidates: the fewest slices meeting the
 * target with all pairs, and with the triangle; when A and B (device, as
 * for mpgemm_ozaki_dd) are given, the exact slice count of that data with
 * all pairs replaces the first when it is smaller (its product is exact
 * before the recombination).  Each candidate is timed at full size (median
 * of 3 after a warm-up) on library buffers; the fastest is returned in
 * *slices, *pairs_mode, *ms (ms nullable).  Synchronises the stream. */
int mpg_ozaki_tune(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l, int bits,
                   const double* A, int64_t lda, const double* B, int64_t ldb,
                   int* slices, int* pairs_mode, double* ms);

/* ---- tuner (Section 3) ------------------------------------------------ */

typedef enum {
  MPG_TUNE_EXHAUSTIVE = 0, /* time every candidate at full size */
  MPG_TUNE_PAPER = 1,      /* the paper's procedure: (1) predict the block time of
                              every tile from a slab product, keep the best tile;
                              (2) time simple, block and Strassen over that tile,
                              the split-K candidates (skinny shapes) and the
                              split-product candidates (DD: MPG_OZAKI and
                              MPG_OZAKI_CRT; QD: MPG_OZAKI_CRT);
                              (3) take the fastest */
  MPG_TUNE_MLP = 2         /* the run-time model ranks every candidate; only the
                              best `topk` are timed, the fastest measured wins */
} mpg_tune_mode;

/* Candidates for a shape: MPG_SIMPLE, MPG_BLOCK with every built tile,
 * MPG_STRASSEN with every tile and depth 1..3 (DD) / 1..2 (QD) while the
 * leaves keep at least 64 per side, MPG_SPLITK (splits 0) with the default
 * and the 32 x 32 x 16 DD tiles (the default QD tile) when C has fewer than
 * 512 64 x 64 tiles and l >= 512, and last, for DD, MPG_OZAKI and
 * MPG_OZAKI_CRT with slices = 0 (exact slice count; all pairs, residue
 * form), for QD MPG_OZAKI_CRT.  precision: 2 (DD) or 4 (QD).
 * The tuner times them on its own buffers: limb 0 uniform in (-1, 1), each
 * lower limb a uniform fraction of half an ulp of the limb above (the next
 * 53 bits of a random significand). */
int mpg_num_candidates(int precision, int64_t m, int64_t n, int64_t l);
int mpg_candidate(int precision, int64_t m, int64_t n, int64_t l, int index,
                  int* algo, mpg_tile* tile);

/* Append every measurement to the JSONL file `path` (NULL: stop). */
int mpg_tune_set_db(mpg_ctx* ctx, const char* path);

/* Median of `reps` HIP-event timings (after one warm-up run) of one
 * candidate on library-owned buffers of the shape; milliseconds. */
int mpg_time_candidate(mpg_ctx* ctx, int precision, int64_t m, int64_t n, int64_t l,
                       int algo, const mpg_tile* tile, int reps, double* ms);

/* Section 3's prediction of the full-size block time from partial
 * products: time A[0:r, :] B and extrapolate.  rule 1: r = 2 bm (two block
 * rows) scaled by m / r, as printed for CPUs; rule 0 (GPU form): slabs of
 * one and of two waves of workgroups (a wave gives every resident
 * workgroup one tile), extrapolated linearly in waves to the full product;
 * a product of at most two waves is timed whole.  *slab_ms (nullable): the
 * time of the timed slabs (the prediction's cost). */
int mpg_predict_block(mpg_ctx* ctx, int precision, int64_t m, int64_t n, int64_t l,
                      const mpg_tile* tile, int rule, double* predicted_ms, double* slab_ms);
/* The slabs mpg_predict_block times, host only, for num_cu CUs with
 * `resident` workgroups each.  rule 1: *rows = min(m, 2 bm), *rows2 = 0,
 * *scale = m / rows (prediction t(rows) scale).  rule 0: *rows and *rows2
 * the rows of one and two waves (whole tile rows), *scale the full
 * product's tiles over the tiles of the one-wave slab, not rounded
 * (prediction t1 + (t2 - t1)(scale - 1)); at most two waves: *rows = m,
 * *rows2 = 0, *scale = 1.  tile as for mpgemm_dd (NULL: the default); an
 * unbuilt tile gives MPG_ERR_UNSUPPORTED. */
int mpg_predict_slab(int precision, int64_t m, int64_t n, int64_t l, const mpg_tile* tile, int rule,
                     int num_cu, int resident, int64_t* rows, int64_t* rows2, double* scale);

/* Tune one shape; the winner also enters the context's table used by
 * MPG_AUTO.  topk: candidates timed in MLP mode (0: one per 9 candidates,
 * at least 2: 4 of the 35 DD candidates, 2 of the 14 QD ones).  Outputs (each
 * nullable): winner, its median time, wall-clock seconds of the search
 * (trials, warm-ups, predictions and model inference), number of
 * full-size trials. */
int mpg_tune(mpg_ctx* ctx, int precision, int64_t m, int64_t n, int64_t l, int mode, int topk,
             int* best_algo, mpg_tile* best_tile, double* best_ms, double* seconds, int* trials);

/* Put a choice into the table used by MPG_AUTO directly (MPG_OZAKI: DD
 * only, tile->slices as for mpgemm_dd_ozaki). */
int mpg_tune_table_set(mpg_ctx* ctx, int precision, int64_t m, int64_t n, int64_t l,
                       int algo, const mpg_tile* tile);

/* ---- method choice by accuracy target ---------------------------------- */

/* Normwise a-priori bound of a method for C := A B, per entry of C, in units
 * of l max|A| max|B| (returns +inf for a combination that does not exist):
 *   DD / QD simple and block (precision 2 / 4): 8 l u, u = 2^-104 / 2^-208
 *     (the componentwise bound 8 l u (|A||B|)_ij with (|A||B|)_ij <=
 *     l max|A| max|B|); QD inputs (in_limbs 4) rounded to DD add 2^-105;
 *   Winograd-Strassen depth 1..3 (square m = n = l only, padded to N, a
 *     multiple of 2^depth): [18^d (N0^2 + 6 N0) - 6 N] 8 u / l, N0 = N / 2^d
 *     (Higham's bound for the Winograd recursion);
 *   MPG_OZAKI (precision 2, in_limbs 1 or 2; tile->slices, pairs_mode):
 *     4 x the truncation bound of mpg_ozaki_slices_for_bits (the row and
 *     column scales are below 2 max|a_i.| and 2 max|b_.j|) plus
 *     (4.1 T^2 + 2) 2^-105, T = (2S - 1) x chunks of K, for the
 *     double-double recombination; pairs_mode 2 (or algo MPG_OZAKI_CRT), the
 *     residue form (slices <= 20): the all-pairs truncation bound x 4 plus
 *     2^-104 for the single rounding of the exact kept product;
 *   MPG_OZAKI_CRT with precision 4 (quad-double through the residue form):
 *     2^-204 (exact part products, quad-double roundings and additions, the
 *     dropped product of the trailing parts).  Feasible only when each
 *     part's exact slice count is at most 20 (the call then fails with
 *     MPG_ERR_UNSUPPORTED otherwise).
 * Host only. */
double mpg_method_bound(int in_limbs, int precision, int algo, const mpg_tile* tile,
                        int pairs_mode, int64_t m, int64_t n, int64_t l);

/* Chooses how to compute C := A B for an accuracy target (the closing
 * proposal of the paper: pick the precision from the accuracy the user
 * needs): max_ij |C - AB|_ij <= 2^-bits l max|A| max|B|, for inputs of
 * in_limbs limbs (1 FP64, 2 DD, 4 QD).  Candidates: DD and QD block (default
 * tile), Winograd-Strassen depth 1..3 (DD) / 1..2 (QD) for square shapes,
 * and the split INT8 product (FP64 or DD inputs) with the fewest slices
 * whose bound meets the target, all pairs, triangle and the residue form
 * (*pairs_mode 0, 1, 2), and quad-double through the residue form.  Every candidate
 * whose mpg_method_bound is within the target is timed at full size on
 * library buffers (median of 3); the fastest is returned: *precision (2:
 * call mpgemm_dd, or mpgemm_ozaki_dd / mpgemm_dd_ozaki for MPG_OZAKI with
 * tile->slices and *pairs_mode; 4: mpgemm_qd), *algo, *tile, *pairs_mode,
 * and (nullable) the bits its bound guarantees and its time.  A target
 * that no candidate meets gives MPG_ERR_UNSUPPORTED. */
int mpg_select_method(mpg_ctx* ctx, int64_t m, int64_t n, int64_t l, int in_limbs, int bits,
                      int* precision, int* algo, mpg_tile* tile, int* pairs_mode,
                      double* bound_bits, double* ms);

/* ---- run-time model (MLP) -------------------------------------------- */

/* Features of one candidate (MPG_MLP_FEATURES floats): log2 m, n, l / 12;
 * DD and QD indicators; simple / block / Strassen indicators (split-K:
 * block); log2 bm / 8, log2 bn / 8, log2 bk / 5, tm tn / 64, Strassen
 * depth / 3, log2 batch / 10 (split-K: its chunk count); split product:
 * 1 digit form, 2 residue form, else 0.  The long-integer product
 * (precision 0; tile: bm, bn = operand words, bk = chunk words, depth =
 * Karatsuba depth): log2 of the operand bits / 12 in the bm and bn slots,
 * chunk words / 8 in the bk slot, the depth / 3, and 3 in the last.  Target
 * of the model: natural log of milliseconds. */
#define MPG_MLP_FEATURES 15
int mpg_mlp_features(int precision, int64_t m, int64_t n, int64_t l, int algo,
                     const mpg_tile* tile, int batch, float* out);

/* The model: MPG_MLP_FEATURES -> 64 -> 64 -> 1, ReLU, FP32, parameters in
 * one array W1 (64 x F), b1, W2 (64 x 64), b2, W3 (64), b3, row-major. */
int mpg_mlp_num_params(void);
/* Set / read the parameters (host arrays of mpg_mlp_num_params floats);
 * setting them resets the optimiser state. */
int mpg_mlp_set_params(mpg_ctx* ctx, const float* params, int count);
int mpg_mlp_get_params(mpg_ctx* ctx, float* params, int count);
/* Mean squared error of the model on (X rows x F, y) and its gradient
 * (host arrays), computed on the GPU. */
int mpg_mlp_grad(mpg_ctx* ctx, const float* X, const float* y, int rows, float* loss,
                 float* grad);
/* Full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8) for `epochs` steps on
 * the GPU; initialises the parameters (He-uniform, fixed seed) if none are
 * set.  losses (nullable, `epochs` floats): loss before each step. */
int mpg_mlp_train(mpg_ctx* ctx, const float* X, const float* y, int rows, int epochs,
                  float lr, float* losses);
/* Train on every trial row of a timing database written by the tuner. */
int mpg_mlp_train_db(mpg_ctx* ctx, const char* path, int epochs, float lr,
                     float* final_loss, int* rows_used);
/* Predicted log-milliseconds for `rows` feature rows. */
int mpg_mlp_predict(mpg_ctx* ctx, const float* X, int rows, float* out);
int mpg_mlp_save(mpg_ctx* ctx, const char* path);
int mpg_mlp_load(mpg_ctx* ctx, const char* path);

/* ---- kernel timing (HIP events on the context stream) ------------------ */

/* Kernel classes timed when profiling is on. */
typedef enum {
  MPG_KCLASS_GEMM = 0,    /* the multiply-add kernel of a call (simple/block/grouped) */
  MPG_KCLASS_AUX = 1,     /* O(n^2) kernels: Strassen operands/assembly, slicing, scans */
  MPG_KCLASS_COUNT = 2
} mpg_kclass;

/* Turn event timing of every launch on (1) or off (0); turning it on clears
 * the counters. */
int mpg_prof_enable(mpg_ctx* ctx, int on);
/* Synchronise the recorded events and return total milliseconds and number
 * of launches of kernel class `kclass` since profiling was enabled. */
int mpg_prof_read(mpg_ctx* ctx, int kclass, double* total_ms, int64_t* launches);

/* ---- failure injection (tests of the error paths) ---------------------- */

/* kind 1: the next `count` workspace allocations of this context fail
 * (MPG_ERR_NOMEM, no hipMalloc is made); kind 2: the next `count` kernel
 * launches of this context fail with hipErrorLaunchFailure (MPG_ERR_HIP,
 * nothing is launched; the call returns at that launch).  count 0 clears.
 * The tuner's own timing buffers are not workspace and are not affected. */
int mpg_test_inject(mpg_ctx* ctx, int kind, int count);

#ifdef __cplusplus
}
#endif

#endif /* MPGEMM_H */
