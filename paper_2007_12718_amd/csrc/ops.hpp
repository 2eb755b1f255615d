// FFT convolution operator, offset table and FGMRES vector kernels (FP64).
#pragma once
#include "common.hpp"
#include "weights.hpp"

namespace lsh {

// Power-of-two FP64 FFT of rows held in LDS (length <= 4096).
struct FFTPlan {
  int M = 0, logM = 0;
  DevBuf tw;  // exp(-2 pi i k / M), k < M
  void init(int M_, hipStream_t s);
};

// Batched row transforms: out[r][k] (k < nout) = DFT_M(in[r][0 .. nin)) (zero padded).
// inverse: conjugate twiddles, no scaling.
void fft_rows(hipStream_t s, const FFTPlan& P, const z64* in, long ldin, int nin, z64* out, long ldout,
              int nout, int nrows, bool inverse);
// out[c][r] = in[r][c]
void transpose_z(hipStream_t s, const z64* in, long ldin, z64* out, long ldout, int rows, int cols);

// y = x + kappa^2 b (K * x) (and the plain convolution u = K * x) with the
// zero-padded circulant embedding of size M x M, M = 2^k >= 2n.
struct ConvOperator {
  int n = 0, M = 0;
  double kappa = 0;
  FFTPlan fft;
  DevBuf khat;      // spectrum of the kernel scaled by 1/M^2, rows and columns 0 .. M/2 (even in both)
  DevBuf w1, w2;    // n x M and M x n work arrays
  // (device memory from the bound arena; scr: staging of the stencil)
  void init(hipStream_t s, int n_, double h, double kappa_, const z64* table, int D,
            const std::vector<StencilEntry>& stencil, mem::Arena& scr);
  // bytes that init takes from the bound arena, and from scr
  static size_t bytes(int n);
  static size_t scratch_bytes(int n);
  // b == nullptr: y = K * x ; otherwise y = x + kappa^2 b (K * x), or with
  // transpose the transposed operator y = x + K * (kappa^2 b x)
  void apply(hipStream_t s, const double* b, const z64* x, z64* y, int nrhs, bool transpose = false);
};

// Offset table T[dy][dx] = h^2 (i/4) H0(kappa h |d|) for 0 <= dx, dy <= D,
// with T[0][0] = h^2 tau0 (the 4th-order centre correction).
void build_offset_table(hipStream_t s, z64* T, int D, double h, double kappa, double tau0_re,
                        double tau0_im);
// T[|dy|][|dx|] += h^2 tau for the stencil entries off the origin (the
// order-p table; the origin value is set by build_offset_table)
void add_table_stencil(hipStream_t s, z64* T, int D, double h, const std::vector<StencilEntry>& stencil,
                       mem::Arena& scr);

// ---- FGMRES vector kernels (deterministic fixed-order reductions)
// out[v] = sum_i conj(V[v][i]) w[i], v < nv (V rows at stride ldv)
void multidot(hipStream_t s, const z64* V, long ldv, int nv, const z64* w, long N, z64* out, z64* partial);
size_t multidot_partial_bytes(int nv);
// w -= sum_v V[v] * h[v]
void multiaxpy(hipStream_t s, z64* w, const z64* V, long ldv, int nv, const z64* h, long N);
// y = x * (1 / sqrt(Re nrm2[0]))
void scale_by_invnorm(hipStream_t s, z64* y, const z64* x, const z64* nrm2, long N);
// y = sum_v V[v] * c[v]   (c on device)
void lincomb(hipStream_t s, z64* y, const z64* V, long ldv, int nv, const z64* c, long N);
// y = a * b .* x   (b real)
void scale_real(hipStream_t s, z64* y, const z64* x, const double* b, double a, long N);
// y = x - y
void sub_from(hipStream_t s, z64* y, const z64* x, long N);
void fill_zero(hipStream_t s, void* p, size_t bytes);
// y = conj(x)
void conj_copy(hipStream_t s, z64* y, const z64* x, long N);

}  // namespace lsh
