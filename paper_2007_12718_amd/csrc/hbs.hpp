// HBS compression / factor / apply kernels (host launchers).
#pragma once
#include "blas.hpp"

namespace lsh {

struct I2 {
  int x, y;
};

// out[i][j] = T[|dy|][|dx|], (dx, dy) = rows[i] - cols[j] (FP64 table lookup)
void gather_table(hipStream_t s, const z64* T, int D, const I2* rows, int m, const I2* cols, int np, z64* out,
                  long ld);

// Row interpolative decomposition A ~= U A[J, :] (U[J, :] = I) of the m x np
// FP64 matrix A (destroyed).  CPQR path: Householder QR with column pivoting
// of A^T in one workgroup; stops at the first |R_kk| <= thr.
// Outputs: J (m ints, first k used), U (m x m capacity, row-major with ld = m,
// first k columns used), rank in *k_dev.
void rowid_cpqr(hipStream_t s, z64* A, int m, int np, double thr, int* J, z64* U, int* k_dev, void* ws);
size_t rowid_cpqr_ws(int m);

// Gram path: M = A A^H, pivoted Cholesky with the stopping rule
// d_max <= thr^2, then U = L_k L11^{-1}.  Same pivots and U as CPQR in exact
// arithmetic; usable while thr / ||A|| stays above ~1e-7 (FP64 Gram).
// Returns the rank (synchronises on the stream).
int rowid_gram(hipStream_t s, const z64* A, int m, int np, double tol, int* J, z64* U, void* ws);
size_t rowid_gram_ws(int m);

// Gram path with block pivoting (left-looking, up to 32 pivots per step,
// chosen among the 48 largest Schur diagonals only while they remain the
// greedy choice over all rows): the greedy pivots and stopping rule.
// Returns the rank (synchronises on the stream once per step).
int rowid_bp(hipStream_t s, const z64* A, int m, int np, double tol, double alpha, int* J, z64* U, void* ws);
size_t rowid_bp_ws(int m);

// Leaf factor helpers (R = working precision)
template <typename R>
void leaf_build(hipStream_t s, cplx<R>* X, const cplx<R>* Gleaf, int mL, const double* b, double kappa2,
                const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n);
template <typename R>
void leaf_scale_U(hipStream_t s, cplx<R>* Y, const cplx<R>* U, int mL, int k, const double* b, double kappa2,
                  const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n);

// Apply, leaf level.  f, q: FP64 grid vectors [nrhs][n][n].  leaf_up takes
// U_L transposed (ULt, k x mL); the others U_L (mL x k).
template <typename R>
void leaf_up(hipStream_t s, const cplx<R>* X, const cplx<R>* ULt, int mL, int k, const z64* f, cplx<R>* r,
             cplx<R>* rt, const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n, int nrhs,
             const double* b = nullptr, double sb = 0);
// transpose pass, leaves: q = X^T (g + U_L w), XT = X transposed per leaf
template <typename R>
void leaf_tdown(hipStream_t s, const cplx<R>* XT, const cplx<R>* UL, int mL, int k, const cplx<R>* w, const z64* g,
                z64* q, const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n, int nrhs);
template <typename R>
void leaf_down(hipStream_t s, const cplx<R>* X, const cplx<R>* UL, int mL, int k, const cplx<R>* wt,
               const cplx<R>* r, z64* q, const double* b, double kappa2, const I2* leaf_origin,
               const I2* leaf_pts, int nleaf, int n, int nrhs);

}  // namespace lsh
