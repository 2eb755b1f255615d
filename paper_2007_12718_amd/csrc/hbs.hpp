// HBS compression / factor / apply kernels (host launchers).
#pragma once
#include <functional>
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

// The parent level's Gram matrix, built while this level's row ID finds its
// pivots.  The parent's candidate rows are this level's skeleton points in
// its two children (child c, pivot q); its proxy matrix rows hold the table
// entries between such a point and the parent's proxy points (order 4:
// T; order p > 4: T | T2).  Rows are stored interleaved (2q + c) as the
// pivots appear, and after each batch of pivot steps the new rows' products
// with every row so far fill the Gram rows 2q + c (columns up to the pivots
// so far), on the side stream gs: the same products as the whole Gram, done
// while the pivot steps run instead of after them.
struct NextGram {
  int cap = 0;                      // capacity in pivots (this level's candidate count)
  int np = 0, ncols = 0, D = 0;     // proxy points; columns (np, or 2 np with T2)
  const z64* T = nullptr;
  const z64* T2 = nullptr;
  const I2* cand = nullptr;         // this level's candidates (device, box-local)
  const I2* prox = nullptr;         // the parent's proxy points (device)
  I2 off[2] = {{0, 0}, {0, 0}};     // the children's origins in the parent box
  z64* A = nullptr;                 // [2 cap][ncols]
  z64* G = nullptr;                 // [2 cap][2 cap]
  hipStream_t gs = nullptr;
  int done = 0;                     // pivots whose rows are in
};
// rows and Gram rows of pivots [g.done, j) (J: this level's pivots, device;
// final on the device when called); launches on g.gs
void next_gram_rows(NextGram& g, const int* J, int j);
// M (2k x 2k, order c k + q) from the interleaved Gram rows of k pivots on s:
// entry (r, r') of the interleaved order read from row max(r, r'), so M is
// exactly Hermitian
void next_gram_pack(hipStream_t s, const NextGram& g, int k, z64* M);

// Gram path with block pivoting (left-looking, up to 32 pivots per step,
// chosen among the 48 largest Schur diagonals only while they remain the
// greedy choice over all rows): the greedy pivots and stopping rule.
// gram_ready: the Gram matrix is already in the workspace (its first m x m
// entries, from next_gram_pack; A unused).  next (or null): the parent
// level's Gram rows, fed after each batch of steps and at the end.
// Returns the rank (synchronises on the stream once per batch of steps).
// on_skel(k), when given, runs once the skeleton J[0..k) is final on the
// device (s synchronised), before the interpolation matrix U is formed.
int rowid_bp(hipStream_t s, const z64* A, int m, int np, double tol, double alpha, int* J, z64* U, void* ws,
             bool gram_ready = false, NextGram* next = nullptr, const std::function<void(int)>& on_skel = {});
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

// Apply, one Woodbury level in one launch per pass (a workgroup per box
// vector, the intermediates in LDS).  Shared: U (2c x k), Ut (k x 2c),
// Q = [L^T; R^T] (2r x c), Gab, Gba (c x c); per box b < nb: Ci = W' (2r x 2r)
// and Pa = [S_a L; S_b R] (two c x r blocks); per child: S (c x c).  All
// row-major and packed.  Box vector v belongs to box v mod nb.
template <typename R>
struct LevelApply {
  int c, k, r, nb;
  const cplx<R> *U, *Ut, *Q, *Gab, *Gba, *S, *Ci, *Pa;
};
// the LDS the box vectors of one workgroup may take (k + 6c + 4r entries)
constexpr size_t LEVEL_FUSED_LDS = 64 * 1024;
// out[v] (k) = U^T X_tau in[v] (in: [nvec][2c])
template <typename R>
void level_up_fused(hipStream_t s, const LevelApply<R>& A, const cplx<R>* in, cplx<R>* out, int nvec);
// wc[v] (2c) = Ghat X_tau (rtc[v] - diag(S) U wt[v]) + U wt[v]
template <typename R>
void level_down_fused(hipStream_t s, const LevelApply<R>& A, const cplx<R>* wt, const cplx<R>* rtc, cplx<R>* wc,
                      int nvec);

}  // namespace lsh
