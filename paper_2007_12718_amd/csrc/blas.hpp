// Batched complex dense linear algebra on gfx950 (host-side launchers).
//
// All matrices are row-major, interleaved complex (cplx<R>), R = float or
// double.  A "batch" is a set of equally sized problems at a fixed stride
// (stride 0 = one operand shared by every problem).
#pragma once
#include <array>
#include <vector>

#include "common.hpp"

namespace lsh {

// OP_R: conjugate without transposing (stored like OP_N)
enum Op : int { OP_N = 0, OP_T = 1, OP_C = 2, OP_R = 3 };

// C_b = alpha * op(A_b) * op(B_b) + beta * D_b (+ I if add_identity)
//   op(A) is M x K (A stored M x K for OP_N, K x M for OP_T / OP_C)
//   op(B) is K x N (B stored K x N for OP_N, N x K for OP_T / OP_C)
// D may alias C (in-place accumulate).  Runs on MFMA (16x16x4 f32 / f64).
// skip (optional, device): when *skip != 0 at launch time the call does nothing.
// lower (M == N): compute only the output tiles that reach the diagonal or
// lie below it (for Hermitian products, with mirror_lower afterwards).
template <typename R>
void cgemm(hipStream_t s, int M, int N, int K, cplx<R> alpha,
           const cplx<R>* A, long lda, long sA, Op opA,
           const cplx<R>* B, long ldb, long sB, Op opB,
           cplx<R> beta, const cplx<R>* D, long ldd, long sD,
           cplx<R>* C, long ldc, long sC, int batch, bool add_identity = false, const int* skip = nullptr,
           bool lower = false);

// As cgemm (no identity, skip flag or lower mode), but in FP32 a product
// with few output tiles splits K over workgroups, with ws (ws_bytes of
// device memory, stream-ordered scratch) holding the partial products;
// without room in ws, or in FP64, it is cgemm.
template <typename R>
void cgemm_ws(hipStream_t s, int M, int N, int K, cplx<R> alpha, const cplx<R>* A, long lda, long sA, Op opA,
              const cplx<R>* B, long ldb, long sB, Op opB, cplx<R> beta, const cplx<R>* D, long ldd, long sD,
              cplx<R>* C, long ldc, long sC, int batch, void* ws, size_t ws_bytes);

// C[i][j] = conj(C[j][i]) for j > i: completes a Hermitian matrix from its lower triangle
template <typename R>
void mirror_lower(hipStream_t s, cplx<R>* C, int n, long ldc);

// Many batched FP32 GEMMs of different shapes in one launch (64 x 64 tiles,
// the same arithmetic as cgemm<float>, so each result is bitwise that of
// the separate call).  dev: device buffer for the problem table (grown as
// needed; keep it alive until the stream has run the launch).
struct GemmItem {
  int M, N, K;
  c32 alpha, beta;
  const c32* A; long lda, sA; Op opA;
  const c32* B; long ldb, sB; Op opB;
  const c32* D; long ldd, sD;
  c32* C; long ldc, sC;
  int batch;
  bool addI;
};
void cgemm_grouped(hipStream_t s, const std::vector<GemmItem>& items, DevBuf& dev);
// bytes of the problem table of a grouped launch of this many items
size_t cgemm_grouped_table_bytes(size_t items);

// y_b = alpha * A_{b mod amod} x_b + beta * z_b   (A_b is M x N, op N).
// z may alias y; z may be null when beta == 0.
template <typename R>
void cgemv(hipStream_t s, int M, int N, cplx<R> alpha,
           const cplx<R>* A, long lda, long sA, int amod,
           const cplx<R>* x, long sx, cplx<R> beta, const cplx<R>* z, long sz,
           cplx<R>* y, long sy, int batch);

// Shared-matrix multi-vector product (rows of Mat streamed once):
//   Y[b][i] = alpha * sum_j Mat[i][j] X[b][j] + beta * Z[b][i],  b < nvec,
// Mat R x C row-major (ld ldm); X, Y, Z rows at strides ldx, ldy, ldz.
// Z may be null when beta == 0; Y must not overlap X.
template <typename R>
void cmgemv(hipStream_t s, int Rr, int C, cplx<R> alpha, const cplx<R>* Mat, long ldm, const cplx<R>* X, long ldx,
            cplx<R> beta, const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec);
// The same with the rows split in two blocks: rows i >= R1 read X + xoff2
// (each vector's second part), rows i < R1 read X; the second block's rows
// are Mat2's (row i - R1 of Mat2, ld ldm) when Mat2 is given, else Mat's.
template <typename R>
void cmgemv2(hipStream_t s, int Rr, int R1, long xoff2, int C, cplx<R> alpha, const cplx<R>* Mat, long ldm,
             const cplx<R>* X, long ldx, cplx<R> beta, const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec,
             const cplx<R>* Mat2 = nullptr);

// GEMM variants (tile shape and LDS depth; prec 1 = FP32, 0 = FP64) and
// their choice per shape: a tuned table keyed by half-octave buckets of
// (M, N, K, batch), else a model.  Every variant of a precision gives the
// same bits.
int gemm_variant_count(int prec);
const char* gemm_variant_name(int prec, int v);
void gemm_force_variant(int v);  // this thread's launches (-1: choose)
void gemm_tune_set(int prec, int M, int N, int K, int batch, int v);
void gemm_table_clear();
void gemm_table_save(const char* path);
int gemm_table_load(const char* path);
void gemm_record(bool on);  // record the (prec, M, N, K, batch) of every product
std::vector<std::array<int, 6>> gemm_recorded();

// In-place inverse of each c x c matrix by Gauss-Jordan elimination with
// partial (row) pivoting.  ws must hold inverse_ws_bytes(c, batch) bytes.
// info[b] = 0, or j+1 if a zero pivot was met at step j (matrix singular).
template <typename R>
size_t inverse_ws_bytes(int c, int batch);
template <typename R>
void inverse(hipStream_t s, cplx<R>* A, int c, long lda, long sA, int batch,
             void* ws, int* info);

// Many FP32 inverse batches of different orders at once (the LDS path for
// small orders and the blocked path for orders <= 1024 each in one set of
// launches; larger orders fall back to inverse()).  Same results as
// inverse<float>() per item.  Synchronises the stream.
struct InvItem {
  c32* A;
  int c;
  long lda, sA;
  int batch;
  int* info;  // batch ints (may be null)
};
size_t inverse_grouped_ws_bytes(const std::vector<InvItem>& items);
void inverse_grouped(hipStream_t s, const std::vector<InvItem>& items, void* ws, DevBuf& table);
// device memory inverse_grouped takes from the bound arena besides ws (its
// tables, and the workspace of orders beyond the grouped kernels), at most
size_t inverse_grouped_arena_bytes(const std::vector<InvItem>& items);

// One persistent launch per level step (FP32): for every box of every
// entry, the Woodbury merge of Algorithm 1 (S_a L, S_b R; Aw, Bw;
// C = (I - Bw Aw)^{-1}; W') and, with U set, the box's scattering matrix, in
// the layouts of the separate launches (Pst [nb][2][c][r], W [nb][2r][2r],
// S [nb][k][k]); the same bits.  T [nb][3][r][r], A12 [nb][2][c][k],
// Qb [nb][4][r][k], perm [nb][r] are temporaries; info [nb] the inverses'
// flags.  Only for r with merge_level_fits(r) (the inverse in LDS).
// counter: one device int (zeroed by the call); table: at least
// merge_level_table_bytes(levels.size()) bytes, else taken from the bound arena.
struct MergeLevelDev {
  const c32 *Sch, *Pm, *Qm, *U;
  c32 *Pst, *W, *S, *T, *A12, *Qb;
  int *info, *perm;
  int c, r, k, nb;
  long item0;
  // the scattering matrix's products with U skip its identity rows: U's
  // other rows Ur = U[rest, :] (n0 of them in half 0, n1 in half 1), the
  // candidate indices rest and skel (= J), and per box the gathered columns
  // G (c x (n0 + n1)) and rows Rg ((n0 + n1) x k)
  const c32* Ur;
  const int *rest, *skel;
  int n0, n1;
  c32 *G, *Rg;
};
bool merge_level_fits(int r);
size_t merge_level_table_bytes(size_t levels);
void merge_levels(hipStream_t s, const std::vector<MergeLevelDev>& levels, DevBuf& table, int* counter);

// out_b (cols x rows) = in_b^T (rows x cols), row-major, batch of contiguous matrices
template <typename R>
void ctranspose(hipStream_t s, const cplx<R>* in, int rows, int cols, cplx<R>* out, long batch = 1);

// dst_b = src_b for rows x cols blocks (leading dimensions lds, ldd; batch strides ss, sd)
// Y[v] = alpha X[v] + beta Z[v] (n entries each, nv vectors; Z may be null)
template <typename R>
void caxpby(hipStream_t s, int n, int nv, cplx<R> alpha, const cplx<R>* X, long ldx, cplx<R> beta, const cplx<R>* Z,
            long ldz, cplx<R>* Y, long ldy);
template <typename R>
void ccopy2d(hipStream_t s, int rows, int cols, const cplx<R>* src, long lds, long ss, cplx<R>* dst, long ldd,
             long sd, long batch = 1);

// dst_b[i][j] = src_b[i][idx[j] - off] where 0 <= idx[j] - off < lim, else 0
// (rows x cols outputs; leading dimensions lds, ldd; batch strides ss, sd)
template <typename R>
void gather_cols(hipStream_t s, int rows, int cols, const cplx<R>* src, long lds, long ss, const int* idx, int off,
                 int lim, cplx<R>* dst, long ldd, long sd, long batch);
// dst_b[i][:] = row t = idx[i] - off of [src0_b; src1_b] (rows t < c from
// src0, the others row t - c of src1; both with leading dimension lds and
// batch stride ss), cols entries each
template <typename R>
void gather_rows2(hipStream_t s, int rows, int cols, const cplx<R>* src0, const cplx<R>* src1, int c, long lds,
                  long ss, const int* idx, int off, cplx<R>* dst, long ldd, long sd, long batch);

// One launch of many FP32 gathers (batched factors): kind 0 as gather_cols
// (c: lim), kind 1 as gather_rows2.
struct GatherJob {
  int kind, rows, cols;
  const c32 *src0, *src1;
  int c;
  long lds, ss;
  const int* idx;
  int off;
  c32* dst;
  long ldd, sd, batch;
};
void gather_grouped(hipStream_t s, const std::vector<GatherJob>& jobs, DevBuf& dev);

// dst (R2) = src (R1), elementwise, n complex entries
template <typename R1, typename R2>
void ccast(hipStream_t s, const cplx<R1>* src, cplx<R2>* dst, long n);

}  // namespace lsh
