/*
 * lsh_dev.h -- batched complex dense building blocks of liblsh (gfx950), the
 * primitives the level merges of Algorithm 1 and the apply of Algorithm 2 are
 * made of (paper Sec. 4.1: the products S_a G_ab, the inverse of
 * [[I, S_a G_ab], [S_b G_ba, I]], the scattering matrices of eq. (smat)).
 * Exposed for unit parity tests and for callers that reuse them.
 *
 * All pointers are device pointers (caller-owned), matrices row-major,
 * interleaved complex; prec = LSH_FP64 (double2) or LSH_FP32 (float2).
 * stream: hipStream_t as void*.  Return codes as in lsh.h.
 */
#ifndef LSH_DEV_H
#define LSH_DEV_H
#include "lsh.h"
#ifdef __cplusplus
extern "C" {
#endif

/* C_b = alpha op(A_b) op(B_b) + beta D_b for b < batch, on the matrix cores.
 * op: 0 = N, 1 = T, 2 = conjugate transpose, 3 = conjugate.  op(A) is M x K
 * (A stored M x K for op 0/3, K x M otherwise), op(B) K x N likewise.
 * alpha, beta: host double[2] (re, im).  Strides (sA, sB, sD, sC) in
 * elements; 0 shares one operand across the batch.  D may equal C. */
int lsh_dev_gemm(int prec, int M, int N, int K, const double* alpha, const void* A, long lda, long sA, int opA,
                 const void* B, long ldb, long sB, int opB, const double* beta, const void* D, long ldd, long sD,
                 void* C, long ldc, long sC, int batch, void* stream);

/* As lsh_dev_gemm, with ws (device, ws_bytes) as scratch for the partial
 * products: an FP32 product with fewer than 256 output tiles of 64 x 64 and
 * K >= 64 splits K over workgroups (as the preconditioner's shared box
 * products do); otherwise, or without room in ws, it is lsh_dev_gemm.  ws
 * must not be in use by other work on the device until the call's work on
 * the stream has finished. */
int lsh_dev_gemm_split(int prec, int M, int N, int K, const double* alpha, const void* A, long lda, long sA,
                       int opA, const void* B, long ldb, long sB, int opB, const double* beta, const void* D,
                       long ldd, long sD, void* C, long ldc, long sC, int batch, void* ws, size_t ws_bytes,
                       void* stream);

/* In place: A_b <- A_b^{-1} (c x c, leading dimension lda >= c, stride sA)
 * by Gauss-Jordan elimination with partial pivoting.  info: device
 * int[batch], 0 or j+1 for a zero pivot at step j.  ws: device workspace of
 * at least lsh_dev_inverse_workspace(prec, c, batch) bytes (256-byte
 * aligned), in use until the call's work on the stream has finished.
 * Errors: LSH_ERR_WORKSPACE_TOO_SMALL. */
int lsh_dev_inverse_workspace(int prec, int c, int batch, size_t* bytes /* host */);
int lsh_dev_inverse(int prec, void* A, int c, long lda, long sA, int batch, int* info, void* ws, size_t ws_bytes,
                    void* stream);

/* As lsh_dev_inverse, with the scratch in a static device array of the
 * library (32 MiB, one per GPU, held until the process ends) instead of a
 * caller workspace: for callers that cannot allocate device memory (code
 * under graph capture, allocation-free serving loops).  Allocates nothing.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (other streams or host threads) race.  Errors:
 * LSH_ERR_WORKSPACE_TOO_SMALL when lsh_dev_inverse_workspace(prec, c,
 * batch) exceeds 32 MiB. */
int lsh_dev_inverse_static(int prec, void* A, int c, long lda, long sA, int batch, int* info, void* stream);

/* ---- GEMM autotuner (the level merges' products, Algorithm 1)
 * The batched complex GEMM has several variants per precision (workgroup
 * tile shape and LDS K depth); every variant of a precision adds the same
 * products in the same order, so the choice changes only the time.  A call
 * takes the variant recorded for its shape's bucket (half-octaves of M, N,
 * K and the batch: round(2 log2 x)), else a wave-quantisation model.
 * lsh_gemm_variants: count and ';'-separated names (host char[cap]).
 * lsh_gemm_tune: times every variant on M x K times K x N products (A per
 * problem, B shared, as in the level merges), reps launches each after one
 * warm-up, in a workspace of lsh_gemm_tune_workspace bytes; writes each
 * variant's mean ms (host double[count], may be NULL) and the fastest
 * (*best), and records it for the shape's bucket.  Synchronises the stream.
 * lsh_gemm_table_save / _load: the recorded choices as a text file (load
 * adds the file's entries; *entries = their count).
 * lsh_gemm_record(1) starts recording the (precision, M, N, K, batch) of
 * every product (precision 1 = FP32, 0 = FP64); lsh_gemm_recorded returns
 * the distinct shapes with the number of products of each (host int[6 * cap]:
 * precision, M, N, K, batch, count).
 * lsh_gemm_force_variant(v): this host thread's products use variant v
 * (-1: the table or model). */
int lsh_gemm_variants(int prec, int* count, char* names, int cap);
int lsh_gemm_tune_workspace(int prec, int M, int N, int K, int batch, size_t* bytes);
int lsh_gemm_tune(int prec, int M, int N, int K, int batch, int reps, void* ws, size_t ws_bytes, void* stream,
                  int* best, double* ms);
int lsh_gemm_table_save(const char* path);
int lsh_gemm_table_load(const char* path, int* entries);
int lsh_gemm_table_clear(void);
int lsh_gemm_record(int on);
int lsh_gemm_recorded(int* count, int* shapes, int cap);
int lsh_gemm_force_variant(int variant);

/* Levels of an FP32 factor whose merges use the Woodbury form with a merge
 * inverse of order r <= 90 (it fits in LDS) and that have at least
 * min_boxes boxes run as one persistent launch per level (the merge chain
 * and the scattering matrices of every box, in lsh_factor_create, lsh_build
 * and, over all instances, lsh_batch_factor); the other levels use separate
 * launches (the same bits either way).  lsh_fused_levels sets min_boxes
 * for later factors: 0 never fuses (the default: on MI355X the separate
 * launches are faster), 1 fuses every such level, -1 restores the
 * default. */
int lsh_fused_levels(int min_boxes);

/* Preconditioner apply (Algorithm 2, M = A^-1 approximately): a Woodbury
 * level whose box vectors (boxes times right-hand sides) number at least
 * min_vectors, and whose per-box vectors fit one workgroup's LDS, runs each
 * pass in one launch with a workgroup per box vector and its intermediates in
 * LDS; the other levels run the step's six to seven batched products.  The
 * two forms agree to rounding (different summation orders).  Affects later
 * applies of M (lsh_apply_precond with transpose = 0, and the
 * preconditioner inside lsh_solve); M^T (lsh_apply_precond with transpose = 1,
 * lsh_solve_adjoint) keeps the batched products.  Process-wide setting, not
 * thread-safe against concurrent applies: 0 never fuses, 1 fuses every such
 * level, -1 restores the default (128).  Returns LSH_ERR_INVALID_ARG below -1. */
int lsh_apply_fused_levels(int min_vectors);

#ifdef __cplusplus
}
#endif
#endif
