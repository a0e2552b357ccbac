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

/* Same-size repeated problems (the case the closing remark of Section VI
 * names as IAAT's best fit): `batch` problems of one shape and layout,
 * problem z at A + z*stride_a, B + z*stride_b, C + z*stride_c (strides in
 * elements).  The tile plan is looked up once and shared: one launch of
 * the strided kernel; or, when both sides of C are 40..80 and not both
 * multiples of 32 and the operands fit the staging buffer (where the staged
 * batched kernel of iaat_gemm_vbatched is faster), a descriptor-writing
 * launch and the staged kernel, with a stream-ordered descriptor buffer of
 * 64 bytes per problem (hipMallocAsync / hipFreeAsync on `stream`).
 * Argument numbers: ta 2, tb 3, m 4, n 5, k 6, A 8, lda 9, stride_a 10,
 * B 11, ldb 12, stride_b 13, C 15, ldc 16, stride_c 17, batch 18.  Strides
 * are >= 0; when batch > 1, stride_c >= ldc*n (outputs must not overlap).
 * Quick returns and NULL rules as iaat_gemm.  Allocates only that
 * descriptor buffer.  Results are bitwise those of iaat_gemm on each
 * problem. */
int iaat_gemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                              float alpha, const float* A, int64_t lda, int64_t stride_a,
                              const float* B, int64_t ldb, int64_t stride_b, float beta, float* C,
                              int64_t ldc, int64_t stride_c, int64_t batch, iaat_stream_t stream);

/* DGEMM (Table 1, row D): the same operation in FP64 (operands, scalars,
 * C and accumulation).  Input-aware like the FP32 path: the run-time
 * tiler's plan for (layout, M, N) from the same tile table, each plan block
 * (one wavefront) run by the family member for that block shape instantiated
 * for FP64 -- matrix-core grids on v_mfma_f64_16x16x4_f64, strips and
 * K-split blocks as FMA chains -- with operands read in place.  Argument
 * numbers, quick returns and NULL rules as iaat_gemm /
 * iaat_gemm_strided_batched.  Does not allocate. */
int iaat_dgemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
               int64_t ldc, iaat_stream_t stream);
int iaat_dgemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                               double alpha, const double* A, int64_t lda, int64_t stride_a,
                               const double* B, int64_t ldb, int64_t stride_b, double beta,
                               double* C, int64_t ldc, int64_t stride_c, int64_t batch,
                               iaat_stream_t stream);

/* CGEMM (Table 1, row C): complex single precision.  A, B, C hold
 * interleaved (re, im) FP32 pairs; lda, ldb, ldc and strides count complex
 * elements; alpha and beta point to host (re, im) pairs; op(X) = X or X^T
 * (no conjugation).  Same plan-driven execution as DGEMM; each complex
 * product is four real FP32 products (Eq. 2) on the matrix cores.  Argument numbers, quick returns (alpha =
 * 0 + 0i or K = 0: C = beta*C; beta = 0 + 0i: C not read) and NULL rules as
 * iaat_gemm / iaat_gemm_strided_batched (-7 / -14: alpha / beta NULL). */
int iaat_cgemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, const float* alpha,
               const void* A, int64_t lda, const void* B, int64_t ldb, const float* beta, void* C,
               int64_t ldc, iaat_stream_t stream);
int iaat_cgemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                               const float* alpha, const void* A, int64_t lda, int64_t stride_a,
                               const void* B, int64_t ldb, int64_t stride_b, const float* beta,
                               void* C, int64_t ldc, int64_t stride_c, int64_t batch,
                               iaat_stream_t stream);

/* ZGEMM (Table 1, row Z): complex double precision.  A, B, C hold
 * interleaved (re, im) FP64 pairs; lda, ldb, ldc and strides count complex
 * elements; alpha and beta point to host (re, im) FP64 pairs; op(X) = X or
 * X^T (no conjugation).  Each complex product is Eq. 2's four real products
 * on the FP64 matrix cores.  Argument numbers, quick returns and NULL
 * rules as iaat_cgemm / iaat_cgemm_strided_batched.  Does not allocate. */
int iaat_zgemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, const double* alpha,
               const void* A, int64_t lda, const void* B, int64_t ldb, const double* beta, void* C,
               int64_t ldc, iaat_stream_t stream);
int iaat_zgemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                               const double* alpha, const void* A, int64_t lda, int64_t stride_a,
                               const void* B, int64_t ldb, int64_t stride_b, const double* beta,
                               void* C, int64_t ldc, int64_t stride_c, int64_t batch,
                               iaat_stream_t stream);

/* Element types of the DGEMM / CGEMM / ZGEMM forms (Table 1, rows D, C, Z). */
enum {
    IAAT_DT_F64 = 1,  /* real FP64 */
    IAAT_DT_C64 = 2,  /* complex FP32: interleaved (re, im) float pairs */
    IAAT_DT_C128 = 3  /* complex FP64: interleaved (re, im) double pairs */
};

/* One problem of an uneven D/C/Z batch: 96 bytes, naturally aligned.
 * Leading dimensions count elements (complex elements for C64 / C128).
 * alpha and beta are (re, im); the imaginary parts are ignored for
 * IAAT_DT_F64, and for IAAT_DT_C64 both parts are rounded to FP32. */
typedef struct iaat_xproblem {
    const void* A;   /* device pointer */
    const void* B;   /* device pointer */
    void* C;         /* device pointer */
    int32_t trans;   /* bit 0: op(A) = A^T; bit 1: op(B) = B^T; other bits 0 */
    int32_t m, n, k;
    int32_t lda, ldb, ldc;
    int32_t reserved0;
    double alpha[2];
    double beta[2];
    int64_t reserved1;
} iaat_xproblem;

/* iaat_xgemm_vbatched runs `count` independent problems of element type
 * `dtype` (IAAT_DT_*) whose descriptors are in device memory
 * (Section V-B's input-aware execution applied per problem: each problem's
 * plan comes from the run-time tiler's table for its layout and M x N, the
 * same table the FP32 path uses, and every plan block runs on the family
 * member for that block shape and element type).  One wavefront per
 * problem.  status: NULL, or a device int32 array of `count` entries that
 * receives each problem's validation code (0, or the negative argument
 * number iaat_gemm would return: -3 trans, -4 m, ... -14 ldc) -- a problem
 * that fails validation is skipped.  Quick returns per problem as
 * iaat_cgemm.  Returns 0, -1 ctx NULL, -2 probs NULL with count > 0, -3
 * count < 0 or above 2^40, -4 dtype.  Does not allocate; the descriptors
 * and C regions must not overlap between problems. */
int iaat_xgemm_vbatched(iaat_ctx_t ctx, int dtype, const iaat_xproblem* probs_dev, int64_t count,
                        int32_t* status_dev, iaat_stream_t stream);

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

/* Computes every problem of a batch in one batched launch on `stream` (a
 * staging kernel whose work-groups each take windows of up to 16 problems, plus a
 * companion kernel for problems too large to stage).  The descriptors are
 * already in device memory (`probs_dev`, count entries); validation,
 * tile-plan lookup and batching all run on the device, so the host does
 * O(1) work.
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
 * create errors: -1 ctx, -2 probs_dev, -3 count, -4 prec, -6 out.
 * An FP32 plan hands windows of consecutive problems out to work-groups
 * dynamically from a counter the plan owns (cleared by a kernel at the start of each
 * replay), so replays of ONE plan must not overlap: launch them on one
 * stream, or wait between them.
 */
int iaat_vbplan_create(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count, int prec,
                       int32_t* status, iaat_vbplan_t* out);
int iaat_vbplan_launch(iaat_vbplan_t plan, iaat_stream_t stream);
int iaat_vbplan_destroy(iaat_vbplan_t plan); /* NULL accepted */

/* Graph-replayed batches from HOST descriptors (Section V-B's executing
 * plan, replayed): iaat_vbatched_plan reserves pinned host staging and a
 * device descriptor array for up to `capacity` problems of precision `prec`;
 * iaat_vbatched_run copies `count` <= capacity host descriptors into the
 * pinned staging (after the plan's previous run has read it) and replays a
 * HIP graph holding the host-to-device descriptor copy and the batched
 * launch, captured again only when `count` differs from the previous run.
 * Per-problem argument errors are not reported (use the device-descriptor
 * forms with a status array for that); invalid problems are skipped.  Runs
 * of one plan must be issued on one stream, or waited for in between.
 * plan errors: -1 ctx, -2 capacity (< 1 or > 2^31-1), -3 prec, -4 out;
 * run errors: -1 plan, -2 probs NULL with count > 0, -3 count out of
 * [0, capacity].  iaat_vbatched_free accepts NULL. */
typedef struct iaat_hplan* iaat_hplan_t;
int iaat_vbatched_plan(iaat_ctx_t ctx, int64_t capacity, int prec, iaat_hplan_t* out);
int iaat_vbatched_run(iaat_hplan_t plan, const iaat_problem* probs_host, int64_t count,
                      iaat_stream_t stream);
int iaat_vbatched_free(iaat_hplan_t plan);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP32
 * batched launch of iaat_vbplan_* (windows of problems handed out to
 * work-groups from a counter, which balances uneven batches) without a plan
 * object.  The counter lives in a fixed 256-byte array of device memory that
 * the library holds on each GPU until the process ends; its address is
 * taken once per device by iaat_create.  No call here allocates or frees
 * memory.  A kernel clears the counter at the start of every call, so the
 * array keeps nothing a later call relies on; but every call on one GPU
 * uses the same array, so calls that may run at the same time on one GPU
 * (different streams, contexts or threads) race and must be serialised by
 * the caller.  Results are bitwise those of iaat_gemm_vbatched_device and
 * iaat_vbplan_launch on the same descriptors.
 *   probs_dev: device array of count descriptors (FP32: ab_scale 1 or the
 *   factor on op(A)op(B)); count in [0, 2^31 - 1] (the counter's range);
 *   status: NULL or a device array of count int32 (as the batched forms).
 * Errors: -1 ctx, -2 probs_dev NULL with count > 0, -3 count outside
 * [0, 2^31 - 1], IAAT_ERR_HIP (launch, or no scratch address on the
 * context's device). */
int iaat_gemm_vbatched_noalloc(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count,
                               int32_t* status, iaat_stream_t stream);

/* ------------------------------------------------ ablation: traditional */

/* The traditional small-GEMM scheme that IAAT replaces (Section I; Fig. 2(a)
 * against Section V), for measuring what the pack step and boundary
 * handling cost on this GPU.  iaat_trad_create validates a batch (host
 * descriptors, FP32; -2 names the first invalid problem) and allocates a
 * workspace for its packed operands.  iaat_trad_pack copies every op(A) and
 * op(B) into zero-padded, tile-contiguous buffers (rows, columns and K
 * rounded up to 16); iaat_trad_compute then runs one uniform 16 x 16
 * matrix-core tile per wavefront over them, masking only the C store.
 * Pack must precede compute on the stream; the operands must not change in
 * between.  Results meet the same tolerance as the IAAT path (the order of
 * the K sum differs).  For the ablation only: iaat_gemm_vbatched* is the
 * path to use. */
typedef struct iaat_tradplan* iaat_tradplan_t;
int iaat_trad_create(iaat_ctx_t ctx, const iaat_problem* probs_host, int64_t count,
                     iaat_tradplan_t* out);
int iaat_trad_pack(iaat_tradplan_t plan, iaat_stream_t stream);
int iaat_trad_compute(iaat_tradplan_t plan, iaat_stream_t stream);
int64_t iaat_trad_workspace_bytes(iaat_tradplan_t plan);
int iaat_trad_destroy(iaat_tradplan_t plan); /* NULL accepted */

/* ---------------------------------------------------------------- serving */

/* A request loop over the batched form (continuous batching).  Requests
 * arrive at any time with a list of GEMMs whose A and B stay resident in
 * device memory; a scheduler thread admits them in arrival order while their
 * outputs fit in a server-owned device arena of `mem_cap_bytes` (admission
 * by memory), packs admitted requests into batched launches of at most
 * `max_batch_gemms` problems, and keeps up to two launches in flight on each
 * of `n_streams` streams, so requests that arrive while others run join the
 * next launch as soon as a launch slot and arena space free up.  Each GEMM's
 * result is exactly what the batched form computes for it alone (the tile
 * plan depends only on the problem, and the block kernels do not depend on
 * the batch). */
typedef struct iaat_server* iaat_server_t;

typedef struct iaat_serve_cfg {
    uint64_t mem_cap_bytes; /* output arena (admission cap), > 0 */
    int32_t n_streams;      /* 1..16 */
    int32_t max_batch_gemms;/* problems per launch, >= 1; also the largest request */
    int32_t prec;           /* IAAT_PREC_* of every served GEMM */
    int32_t reserved;
} iaat_serve_cfg;

enum { IAAT_REQ_QUEUED = 0, IAAT_REQ_ADMITTED = 1, IAAT_REQ_DONE = 3 };

typedef struct iaat_req_status {
    int32_t state;      /* IAAT_REQ_* */
    int32_t err;        /* 0, or the first non-zero per-problem status code */
    double t_arrival;   /* seconds on the server clock (iaat_serve_clock) */
    double t_launch;    /* admitted and launched */
    double t_done;      /* completion observed */
    float* out;         /* device address of the request's outputs while kept
                           (see iaat_serve_submit), else NULL */
} iaat_req_status;

typedef struct iaat_serve_stats {
    uint64_t submitted, done, failed, launches, gemms_done;
    double p50, p99, max_latency; /* seconds, t_done - t_arrival of done requests */
    double gflops;                /* 2MNK of done requests / (last t_done - first t_arrival) */
    uint64_t peak_admitted_bytes; /* most arena bytes held at once */
    int64_t peak_queue_depth;     /* most requests waiting for admission */
    double p99_submit_lag;        /* seconds a request was submitted after its t_arrival
                                     (load-generator lag, part of the latency) */
} iaat_serve_stats;

/* Starts a server on the context's device (allocates the arena, streams,
 * pinned staging; runs one tiny GEMM per launch slot, so first-use costs of
 * streams and kernels are paid before the server clock starts; starts the
 * scheduler thread).
 * Errors: -1 ctx; -2 cfg NULL or out of range; -3 out NULL; IAAT_ERR_NOMEM;
 * IAAT_ERR_HIP. */
int iaat_serve_start(iaat_ctx_t ctx, const iaat_serve_cfg* cfg, iaat_server_t* out);

/* Submits one request of `count` GEMMs (host descriptors, copied by the
 * call).  For each GEMM, A and B are device operands and C names the
 * INITIAL value C0 (device, ldc x n, read only when beta != 0; NULL allowed
 * when beta == 0): the result is written to the request's own output region
 * in the arena with the caller's ldc, GEMM i at float offset out_off(i) =
 * sum over earlier GEMMs of their C span ldc*(n-1)+m rounded up to 64
 * floats (when beta != 0 only that span of C0 is read).  `t_arrival` is the request's arrival on
 * the server clock (< 0: now); latencies are measured from it.  With
 * keep_output != 0 the output region stays allocated after completion until
 * iaat_serve_release; otherwise it is freed at completion.
 * Errors: -1 server; -2 gemms NULL or count < 1; -3 count > max_batch_gemms,
 * or the outputs exceed the arena; -4 a GEMM's arguments are invalid (its
 * number in iaat_last_error); -6 ticket NULL; IAAT_ERR_UNSUPPORTED after stop. */
int iaat_serve_submit(iaat_server_t srv, const iaat_problem* gemms_host, int64_t count,
                      double t_arrival, int keep_output, uint64_t* ticket);

/* Status of a request: returns 0 when done, 1 while queued or running, or
 * -2 for an unknown ticket; fills *st when st is not NULL. */
int iaat_serve_poll(iaat_server_t srv, uint64_t ticket, iaat_req_status* st);

/* Frees a kept output region (the request must be done). -2 unknown ticket
 * or not kept, -3 not done. */
int iaat_serve_release(iaat_server_t srv, uint64_t ticket);

/* Seconds since the server started (the clock of t_arrival / t_done). */
double iaat_serve_clock(iaat_server_t srv);

int iaat_serve_stats_get(iaat_server_t srv, iaat_serve_stats* out);

/* Open-loop replay of a request trace (a load generator running in a native
 * thread): request r arrives t_arrival[r] seconds after the call starts and
 * holds n_gemms[r] GEMMs, the pool entries pool_idx[first_r ..] (first_r =
 * sum of earlier n_gemms) of the host descriptor array `pool` (pool_size
 * entries, C = initial values).  Each request is submitted at its arrival
 * time (or at once when the replay is behind), then the call waits for all
 * of them; latency_out (NULL or n_req doubles) receives t_done - t_arrival
 * per request.  Returns 0, or the first submit error. */
int iaat_serve_replay(iaat_server_t srv, int64_t n_req, const double* t_arrival,
                      const int32_t* n_gemms, const int64_t* pool_idx, const iaat_problem* pool,
                      int64_t pool_size, double* latency_out);

/* Waits for every submitted request, stops the scheduler and frees the
 * server.  NULL accepted. */
int iaat_serve_stop(iaat_server_t srv);

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

/* Tile-table editing (the install-time autotuner's interface).
 * iaat_plan_set stages a plan for (layout, m, n): `blocks` (nblk <= 15
 * entries; i0, j0, kid are used, rows/cols ignored) must cover the m x n
 * exactly with kernels of the family -- the same check every loaded table
 * passes -- else -5 (-1 ctx, -2 layout, -3 m, -4 n, -6 nblk).  Staged plans
 * take effect at iaat_table_commit, which waits for the device to be idle
 * and uploads the table (no work of this context may be queued meanwhile).
 * iaat_table_save writes the table in use to `path` in the format
 * iaat_create loads. */
int iaat_plan_set(iaat_ctx_t ctx, int layout, int m, int n, const iaat_block* blocks, int nblk);
int iaat_table_commit(iaat_ctx_t ctx);
int iaat_table_save(iaat_ctx_t ctx, const char* path);

/* Number of generated kernels in the library's family, and the description
 * of kernel `kid`: family (0 MFMA tile grid, 1 row strip, 2 column strip,
 * 3 K-split reduction), its two size parameters, and its block extent. */
int iaat_family_size(void);
int iaat_family_info(int kid, int32_t* family, int32_t* p1, int32_t* p2,
                     int32_t* block_rows, int32_t* block_cols);

/* The install-time generator instantiates the family per (shape, layout,
 * data type) (Section IV, Algorithm 1; Table 1's S, D, C, Z rows).
 * iaat_family_dtypes writes up to `cap` data-type codes the family is built
 * for (0 FP32, then IAAT_DT_F64, IAAT_DT_C64, IAAT_DT_C128) and returns how
 * many there are.  The FP32 batched kernel runs members from LDS in units
 * (one or two tiles of a grid, up to four rows or columns of a strip, one
 * row of a K-split block): iaat_staged_unit_count and iaat_staged_unit_info
 * describe them (family and size parameters as iaat_family_info; -1 for a
 * unit id out of range). */
int iaat_family_dtypes(int32_t* codes, int cap);
int iaat_staged_unit_count(void);
int iaat_staged_unit_info(int unit, int32_t* family, int32_t* p1, int32_t* p2);

/* 1 if (layout, m, n, k) is in the small-GEMM domain (MNK <= 80^3, or
 * <= 32^3 for TN, evaluated in exact integers), else 0; -i for a bad
 * argument. */
int iaat_in_small_domain(int layout, int64_t m, int64_t n, int64_t k);

#ifdef __cplusplus
}
#endif
#endif /* IAAT_H */
