/*
 * Oracle (test infrastructure only): the plain FP64 GEMM the small-GEMM
 * path must reproduce.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library; the product path never does.
 *
 * What it computes (Section I, the GEMM statement; column-major storage and
 * the NN/NT/TN/TT naming from the note under Table 1):
 *
 *     C*[i,j] = alpha * sum_{p<K} opA(i,p) * opB(p,j)  +  beta * C0[i,j]
 *
 *     opA(i,p) = A[i + p*lda]  if A is not transposed (A stored M x K)
 *              = A[p + i*lda]  if A is transposed     (A stored K x M)
 *     opB(p,j) = B[p + j*ldb]  if B is not transposed (B stored K x N)
 *              = B[j + p*ldb]  if B is transposed     (B stored N x K)
 *
 * Readings where the paper is silent (its kernels compute C_c = A_c B_c + C_c
 * with no scalars, Section IV-B):
 *   - alpha == 0 or K == 0: the sum is not formed, A and B are not read.
 *   - beta == 0: C0 is not read (so NaN/Inf already in C0 do not propagate).
 *   - M == 0 or N == 0: nothing to do.
 * Every FP32 input is widened exactly to FP64; each product of two FP32
 * values is exact in FP64; the sum runs over p in increasing order.  No
 * blocking, no reordering, no threading inside one problem.
 */
#include <stdint.h>
#include <stddef.h>
#include <pthread.h>
#include <time.h>

static double op_a(int ta, const float* A, int64_t lda, int64_t i, int64_t p)
{
    return ta ? (double)A[p + i * lda] : (double)A[i + p * lda];
}

static double op_b(int tb, const float* B, int64_t ldb, int64_t p, int64_t j)
{
    return tb ? (double)B[j + p * ldb] : (double)B[p + j * ldb];
}

/* One problem.  out is M x N column-major with leading dimension ldo. */
void oracle_gemm_f64(int ta, int tb, int64_t m, int64_t n, int64_t k,
                     double alpha, const float* A, int64_t lda,
                     const float* B, int64_t ldb,
                     double beta, const float* C0, int64_t ldc,
                     double* out, int64_t ldo)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (alpha != 0.0 && k > 0) {
                for (int64_t p = 0; p < k; ++p)
                    s += op_a(ta, A, lda, i, p) * op_b(tb, B, ldb, p, j);
            }
            double r = alpha * s;
            if (beta != 0.0)
                r += beta * (double)C0[i + j * ldc];
            out[i + j * ldo] = r;
        }
    }
}

/* Same definition with FP64 operands: used for the dequantized-input parity
 * oracle of the reduced-precision modes, where A and B values are exact
 * multiples of small powers of two and are handed over already widened. */
void oracle_gemm_f64_d(int ta, int tb, int64_t m, int64_t n, int64_t k,
                       double alpha, const double* A, int64_t lda,
                       const double* B, int64_t ldb,
                       double beta, const float* C0, int64_t ldc,
                       double* out, int64_t ldo)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (alpha != 0.0 && k > 0) {
                for (int64_t p = 0; p < k; ++p) {
                    double a = ta ? A[p + i * lda] : A[i + p * lda];
                    double b = tb ? B[j + p * ldb] : B[p + j * ldb];
                    s += a * b;
                }
            }
            double r = alpha * s;
            if (beta != 0.0)
                r += beta * (double)C0[i + j * ldc];
            out[i + j * ldo] = r;
        }
    }
}

/* ---- batch driver: the same function over many problems, threads over
 * problems (never inside one).  Problems are described struct-of-arrays with
 * element offsets into one FP32 buffer; outputs go to an FP64 buffer at
 * out_off[i] with leading dimension m[i]. ---- */
typedef struct {
    int64_t count;
    const int32_t* trans;   /* bit0: A transposed, bit1: B transposed */
    const int32_t* m; const int32_t* n; const int32_t* k;
    const int32_t* lda; const int32_t* ldb; const int32_t* ldc;
    const float* alpha; const float* beta;
    const int64_t* a_off; const int64_t* b_off; const int64_t* c_off;
    const int64_t* out_off;
    const float* buf;
    double* out;
    int nthreads;
    int tid;
} batch_job;

static void* batch_worker(void* arg)
{
    const batch_job* jb = (const batch_job*)arg;
    for (int64_t q = jb->tid; q < jb->count; q += jb->nthreads) {
        oracle_gemm_f64(jb->trans[q] & 1, (jb->trans[q] >> 1) & 1,
                        jb->m[q], jb->n[q], jb->k[q],
                        (double)jb->alpha[q], jb->buf + jb->a_off[q], jb->lda[q],
                        jb->buf + jb->b_off[q], jb->ldb[q],
                        (double)jb->beta[q], jb->buf + jb->c_off[q], jb->ldc[q],
                        jb->out + jb->out_off[q], jb->m[q] > 0 ? jb->m[q] : 1);
    }
    return NULL;
}

/* Runs the batch on nthreads POSIX threads; returns wall seconds. */
/* DGEMM (Table 1, row D): the same definition with every operand, C0
 * included, in FP64.  C0 is not read when beta == 0; A and B are not read
 * when alpha == 0 or k == 0. */
void oracle_dgemm(int ta, int tb, int64_t m, int64_t n, int64_t k,
                  double alpha, const double* A, int64_t lda,
                  const double* B, int64_t ldb,
                  double beta, const double* C0, int64_t ldc,
                  double* out, int64_t ldo)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            if (alpha != 0.0 && k > 0) {
                for (int64_t p = 0; p < k; ++p) {
                    double a = ta ? A[p + i * lda] : A[i + p * lda];
                    double b = tb ? B[j + p * ldb] : B[p + j * ldb];
                    s += a * b;
                }
            }
            double r = alpha * s;
            if (beta != 0.0)
                r += beta * C0[i + j * ldc];
            out[i + j * ldo] = r;
        }
    }
}

/* CGEMM (Table 1, row C): complex operands stored as interleaved FP32
 * (re, im) pairs, widened exactly to FP64; complex alpha, beta; op(X) = X or
 * X^T (no conjugation).  out is interleaved FP64.  C0 is not read when
 * beta == 0; A and B are not read when alpha == 0 or k == 0. */
void oracle_cgemm(int ta, int tb, int64_t m, int64_t n, int64_t k,
                  double alpha_re, double alpha_im, const float* A, int64_t lda,
                  const float* B, int64_t ldb, double beta_re, double beta_im,
                  const float* C0, int64_t ldc, double* out, int64_t ldo)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double sr = 0.0, si = 0.0;
            if ((alpha_re != 0.0 || alpha_im != 0.0) && k > 0) {
                for (int64_t p = 0; p < k; ++p) {
                    int64_t ia = ta ? p + i * lda : i + p * lda;
                    int64_t ib = tb ? j + p * ldb : p + j * ldb;
                    double ar = A[2 * ia], ai = A[2 * ia + 1];
                    double br = B[2 * ib], bi = B[2 * ib + 1];
                    sr += ar * br - ai * bi;
                    si += ar * bi + ai * br;
                }
            }
            double rr = alpha_re * sr - alpha_im * si;
            double ri = alpha_re * si + alpha_im * sr;
            if (beta_re != 0.0 || beta_im != 0.0) {
                double cr = C0[2 * (i + j * ldc)], ci = C0[2 * (i + j * ldc) + 1];
                rr += beta_re * cr - beta_im * ci;
                ri += beta_re * ci + beta_im * cr;
            }
            out[2 * (i + j * ldo)] = rr;
            out[2 * (i + j * ldo) + 1] = ri;
        }
    }
}

/* ZGEMM (Table 1, row Z): complex operands stored as interleaved FP64
 * (re, im) pairs; complex alpha, beta; op(X) = X or X^T (no conjugation).
 * Each complex product expands as in Eq. 2 into four real products, the
 * real part (ar*br - ai*bi) and the imaginary part (ar*bi + ai*br), summed
 * over p in increasing order in FP64.  out is interleaved FP64.  C0 is not
 * read when beta == 0; A and B are not read when alpha == 0 or k == 0. */
void oracle_zgemm(int ta, int tb, int64_t m, int64_t n, int64_t k,
                  double alpha_re, double alpha_im, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double beta_re, double beta_im,
                  const double* C0, int64_t ldc, double* out, int64_t ldo)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            double sr = 0.0, si = 0.0;
            if ((alpha_re != 0.0 || alpha_im != 0.0) && k > 0) {
                for (int64_t p = 0; p < k; ++p) {
                    int64_t ia = ta ? p + i * lda : i + p * lda;
                    int64_t ib = tb ? j + p * ldb : p + j * ldb;
                    double ar = A[2 * ia], ai = A[2 * ia + 1];
                    double br = B[2 * ib], bi = B[2 * ib + 1];
                    sr += ar * br - ai * bi;
                    si += ar * bi + ai * br;
                }
            }
            double rr = alpha_re * sr - alpha_im * si;
            double ri = alpha_re * si + alpha_im * sr;
            if (beta_re != 0.0 || beta_im != 0.0) {
                double cr = C0[2 * (i + j * ldc)], ci = C0[2 * (i + j * ldc) + 1];
                rr += beta_re * cr - beta_im * ci;
                ri += beta_re * ci + beta_im * cr;
            }
            out[2 * (i + j * ldo)] = rr;
            out[2 * (i + j * ldo) + 1] = ri;
        }
    }
}

double oracle_gemm_batch(int64_t count, const int32_t* trans,
                         const int32_t* m, const int32_t* n, const int32_t* k,
                         const int32_t* lda, const int32_t* ldb, const int32_t* ldc,
                         const float* alpha, const float* beta,
                         const int64_t* a_off, const int64_t* b_off, const int64_t* c_off,
                         const int64_t* out_off, const float* buf, double* out,
                         int nthreads)
{
    enum { MAXT = 256 };
    if (nthreads < 1) nthreads = 1;
    if (nthreads > MAXT) nthreads = MAXT;
    batch_job jobs[MAXT];
    pthread_t th[MAXT];
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int t = 0; t < nthreads; ++t) {
        batch_job j = {count, trans, m, n, k, lda, ldb, ldc, alpha, beta,
                       a_off, b_off, c_off, out_off, buf, out, nthreads, t};
        jobs[t] = j;
        if (nthreads > 1)
            pthread_create(&th[t], NULL, batch_worker, &jobs[t]);
    }
    if (nthreads == 1)
        batch_worker(&jobs[0]);
    else
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}
