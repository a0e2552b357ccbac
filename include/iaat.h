/*
 * iaat.h -- C ABI of libiaat, input-aware adaptive tiling (IAAT) small GEMM
 * on MI355X (gfx950).
 *
 * Operation (the GEMM statement of Section I):
 *
 *     C = alpha * op(A) * op(B) + beta * C,
 *
 * with C an M x N matrix, op(A) M x K, op(B) K x N, every matrix stored
 * column-major (the default of the note under Table 1), and op(X) = X or X^T.
 * The layout names NN, NT, TN, TT give op(A) then op(B) (same note):
 *
 *     op(A)(i,p) = A[i + p*lda]  (A not transposed, A stored M x K)
 *                = A[p + i*lda]  (A transposed,     A stored K x M)
 *     op(B)(p,j) = B[p + j*ldb]  (B not transposed, B stored K x N)
 *                = B[j + p*ldb]  (B transposed,     B stored N x K)
 *
 * The small-GEMM domain is cbrt(MNK) <= 80, or <= 32 for TN (Section I and
 * the closing paragraph of Section VI).  Sizes outside it are still computed
 * correctly; they are simply not what the tile table is tuned for.
 *
 * How it is computed (Sections III-V): an install-time generator emits a
 * family of size-specialised tile kernels; a run-time tiler covers the M x N
 * of C with blocks that are each one of those kernels (the kernel executing
 * plan).  Operands are read in place: no pack copy, and the K reduction of
 * every block runs over the whole K.
 *
 * Conventions for every entry point
 *  - Pointers named A, B, C, probs_dev, status are DEVICE memory (HIP device
 *    or managed allocations on the context's device); pointers named
 *    *_host are host memory.  The library never frees caller memory and keeps
 *    no caller pointer past the call, except that work queued on a stream
 *    reads/writes the operands until that work completes.
 *  - Calls that take a stream only enqueue work on it (asynchronous); the
 *    caller keeps operands alive until the stream has passed that work.
 *  - Return value: IAAT_OK (0), or -i when argument i (1-based, counting
 *    the context) is invalid -- checked before any GPU work is queued, the
 *    LAPACK convention -- or one of the IAAT_ERR_* codes below.
 *    iaat_last_error() gives a message for the calling thread's last failure.
 *  - C must not overlap A or B.
 */
#ifndef IAAT_H
#define IAAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct iaat_ctx* iaat_ctx_t;
typedef struct iaat_vbplan* iaat_vbplan_t;
typedef void* iaat_stream_t; /* a hipStream_t; NULL means the null stream */

enum { IAAT_OP_N = 0, IAAT_OP_T = 1 };

/* Precision of A and B for the batched form (C, alpha, beta and the
 * accumulation are always FP32).  The reduced-precision modes extend the
 * paper's FP32/FP64 kernels (Table 1) to matrix-core input types; each
 * product of two such inputs is exact in FP32, so results differ from the
 * exact product of the dequantised inputs only by FP32 accumulation. */
enum {
    IAAT_PREC_F32 = 0,    /* A, B float */
    IAAT_PREC_BF16 = 1,   /* A, B bfloat16 (uint16 codes) */
    IAAT_PREC_F16 = 2,    /* A, B IEEE binary16 */
    IAAT_PREC_F8E4M3 = 3, /* A, B FP8 E4M3 (OCP, bias 7, max 448) of x * 2^e per matrix;
                             ab_scale = 2^-(eA + eB) undoes the scales */
    IAAT_PREC_BF16X3 = 4  /* A, B each a bfloat16 pair hi = bf16(x), lo = bf16(x - hi):
                             the lo matrix follows the hi matrix, ld * (stored columns)
                             elements after it; op(A)op(B) is taken as
                             lo*hi + hi*lo + hi*hi (split-bfloat16 compensation) */
};

#define IAAT_OK 0
#define IAAT_ERR_HIP (-100)         /* a HIP runtime call failed */
#define IAAT_ERR_NOMEM (-101)       /* a device or host allocation failed */
#define IAAT_ERR_TABLE (-102)       /* the tile table file is unreadable or mismatched */
#define IAAT_ERR_UNSUPPORTED (-103) /* valid request the library does not provide */

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`: loads the tile table (the
 * install-time artefact) from `tile_table_path`, or the built-in table when
 * it is NULL or empty, and uploads it to the device.  Sets *out.  The calling
 * thread's current device is restored on return.
 * Errors: -1 out is NULL; -2 no such device; IAAT_ERR_TABLE; IAAT_ERR_HIP;
 * IAAT_ERR_NOMEM. */
int iaat_create(iaat_ctx_t* out, int device, const char* tile_table_path);

/* Releases a context and its device memory.  Work it queued must have
 * completed.  NULL is accepted (no-op). */
int iaat_destroy(iaat_ctx_t ctx);

/* Message for the calling thread's most recent failed call ("" if none).
 * The string is owned by the library and valid until the next call on the
 * same thread. */
const char* iaat_last_error(void);

/* ------------------------------------------------------- one problem/call */

/* C = alpha*op(A)*op(B) + beta*C for one problem, enqueued on `stream` as
 * one kernel launch whose work-groups are the blocks of the tile plan for
 * (layout, M, N) (Section V: the kernel executing plan).
 *   ta, tb     IAAT_OP_N or IAAT_OP_T                        (args 2, 3)
 *   m, n, k    >= 0, each < 2^31                              (args 4, 5, 6)
 *   A, lda     lda >= max(1, ta==N ? m : k)                   (args 8, 9)
 *   B, ldb     ldb >= max(1, tb==N ? k : n)                   (args 10, 11)
 *   C, ldc     ldc >= max(1, m)                               (args 13, 14)
 * Quick returns: m == 0 or n == 0 does nothing.  alpha == 0 or k == 0 sets
 * C = beta*C without reading A or B (which may then be NULL).  beta == 0
 * never reads C, so NaN/Inf already in C do not propagate.  A and B may be
 * NULL only in those cases; C only when m == 0 or n == 0.
 * Does not allocate.  Re-entrant. */
int iaat_gemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
              float alpha, const float* A, int64_t lda, const float* B, int64_t ldb,
              float beta, float* C, int64_t ldc, iaat_stream_t stream);

/* ------------------------------------------------- many uneven problems */

/* One problem of a batch: 64 bytes, naturally aligned. */
typedef struct iaat_problem {
    const void* A;   /* device pointer; element type set by the batch precision */
    const void* B;   /* device pointer */
    float* C;        /* device pointer, FP32 */
    int32_t trans;   /* bit 0: op(A) = A^T; bit 1: op(B) = B^T; other bits 0 */
    int32_t m, n, k;
    int32_t lda, ldb, ldc;
    float alpha, beta;
    float ab_scale;  /* extra factor on op(A)op(B) (dequantisation); 1 for FP32 */
} iaat_problem;

/* Per-problem status codes written to `status` by the batched forms: 0, or
 * -i where i is the iaat_gemm argument number of the offending field
 * (-2 trans bit 0, -3 trans bit 1 / unknown bits, -4 m, -5 n, -6 k, -8 A,
 * -9 lda, -10 B, -11 ldb, -13 C, -14 ldc).  An invalid problem is skipped;
 * the others are computed. */

/* Computes every problem of a batch in one persistent kernel launch on
 * `stream`.  The descriptors are already in device
 * memory (`probs_dev`, count entries); validation, tile-plan lookup and the
 * work queue all run on the device, so the host does O(1) work.
 *   count >= 0 (arg 3); prec one of IAAT_PREC_* (arg 4); status: NULL or a
 *   device array of count int32 (arg 5).
 * Problems must not write overlapping C.  FP32 results are bitwise identical
 * to iaat_gemm on each problem (same tile plan, same block kernels).  With
 * a reduced-precision `prec`, A and B hold codes of that type (ld in
 * elements) and alpha * ab_scale multiplies op(A)op(B); those problems are
 * covered by 16 x 16 matrix-core tiles with FP32 accumulation (FP8 codes are
 * widened exactly to binary16 for the matrix cores, whose FP8 dot product
 * does not sum in full FP32 precision).
 * Does not allocate; keeps no state on the device between calls. */
int iaat_gemm_vbatched_device(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count,
                              int prec, int32_t* status, iaat_stream_t stream);

/* Same, with the descriptors in host memory: they are copied into a
 * context-owned pinned staging ring and then to the device on `stream`
 * before the launch.  The call returns once the descriptors are staged; it
 * may block while earlier batched calls of this context still use the
 * staging slot.  The staging area grows (allocates) when `count` exceeds
 * its capacity. */
int iaat_gemm_vbatched(iaat_ctx_t ctx, const iaat_problem* probs_host, int64_t count,
                       int prec, int32_t* status, iaat_stream_t stream);

/* One quantisation job: the A and B operands of one problem.  Each source is
 * a contiguous FP32 array of *_n elements (a whole stored matrix, ld times
 * stored columns); the destination receives *_n codes of the target type
 * (2 * *_n bfloat16 for IAAT_PREC_BF16X3: hi then lo).  All pointers are
 * device memory; a_n or b_n may be 0 (nothing done for that operand). */
typedef struct iaat_qjob {
    const float* a_src;
    const float* b_src;
    void* a_dst;
    void* b_dst;
    int64_t a_n, b_n;
    iaat_problem* prob; /* NULL, or a device descriptor whose ab_scale is set:
                           2^-(eA + eB) for FP8, 1 otherwise */
    float* scales;      /* NULL, or device float[2] receiving 2^eA, 2^eB (FP8; 1 otherwise) */
} iaat_qjob;

/* Quantises the operands of `count` problems (jobs_dev: device array) to
 * `prec` in one launch on `stream`, rounding to nearest even:
 *   BF16, F16   direct rounding of x (binary16 overflows to inf past 65504);
 *   F8E4M3      per matrix, e = the largest integer with absmax * 2^e <= 448
 *               (0 for an all-zero or non-finite absmax), codes of x * 2^e
 *               saturating at +-448, zero always encoded +0;
 *   BF16X3      hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in FP32).
 * Errors: -1 ctx, -2 prec (not a reduced-precision mode), -3 jobs_dev NULL
 * with count > 0, -4 count < 0. */
int iaat_quantize_batch(iaat_ctx_t ctx, int prec, const iaat_qjob* jobs_dev, int64_t count,
                        iaat_stream_t stream);

/* Graph-replayed batch: captures the batched launch for the descriptor
 * array `probs_dev` (count entries) into a HIP graph once; each
 * iaat_vbplan_launch replays it on `stream`.  The descriptor array is read
 * at every replay, so the caller may change its contents (pointers, sizes,
 * scalars) between replays; its address and `count` are fixed.
 * iaat_vbplan_create allocates and synchronises the device; launch does
 * neither.
 * create errors: -1 ctx, -2 probs_dev, -3 count, -4 prec, -6 out. */
int iaat_vbplan_create(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count, int prec,
                       int32_t* status, iaat_vbplan_t* out);
int iaat_vbplan_launch(iaat_vbplan_t plan, iaat_stream_t stream);
int iaat_vbplan_destroy(iaat_vbplan_t plan); /* NULL accepted */

/* ------------------------------------------------------ introspection */

/* One block of a tile plan: rows [i0, i0+rows) x cols [j0, j0+cols) of a
 * (sub)problem of at most 80 x 80, computed by generated kernel `kid`. */
typedef struct iaat_block {
    int32_t i0, j0, rows, cols, kid;
} iaat_block;

/* Writes the tile plan the context uses for a layout (0 NN, 1 TN, 2 NT,
 * 3 TT: bit 0 = A^T, bit 1 = B^T) and 1 <= m, n <= 80 into out[0..cap).
 * Returns the number of blocks (which may exceed cap), or -i. */
int iaat_plan_query(iaat_ctx_t ctx, int layout, int m, int n, iaat_block* out, int cap);

/* The built-in (untuned) plan the run-time tiler makes for (layout, m, n),
 * 1 <= m, n <= 80, without a context or a device; same output convention
 * as iaat_plan_query. */
int iaat_default_plan(int layout, int m, int n, iaat_block* out, int cap);

/* Number of generated kernels in the library's family, and the description
 * of kernel `kid`: family (0 MFMA tile grid, 1 row strip, 2 column strip,
 * 3 K-split reduction), its two size parameters, and its block extent. */
int iaat_family_size(void);
int iaat_family_info(int kid, int32_t* family, int32_t* p1, int32_t* p2,
                     int32_t* block_rows, int32_t* block_cols);

/* 1 if (layout, m, n, k) is in the small-GEMM domain (MNK <= 80^3, or
 * <= 32^3 for TN, evaluated in exact integers), else 0; -i for a bad
 * argument. */
int iaat_in_small_domain(int layout, int64_t m, int64_t n, int64_t k);

#ifdef __cplusplus
}
#endif
#endif /* IAAT_H */
