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

/* In place: A_b <- A_b^{-1} (c x c, leading dimension lda, stride sA) by
 * Gauss-Jordan elimination with partial pivoting.  info: device int[batch],
 * 0 or j+1 for a zero pivot at step j.  Allocates its own scratch. */
int lsh_dev_inverse(int prec, void* A, int c, long lda, long sA, int batch, int* info, void* stream);

#ifdef __cplusplus
}
#endif
#endif
