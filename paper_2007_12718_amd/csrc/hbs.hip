// HBS compression (paper Sec. 3.2), leaf factor (Alg. 1, leaf loop) and the
// leaf steps of the apply (Alg. 2) on gfx950.

#include <cmath>
#include <cstdlib>

#include <functional>
#include <vector>

#include "hbs.hpp"
#include "wave.hpp"
#include "ops.hpp"
#include "prof.hpp"

namespace lsh {

// ------------------------------------------------------------- gathers
__global__ void k_gather_table(const z64* __restrict__ T, int D, const I2* __restrict__ rows, int m,
                               const I2* __restrict__ cols, int np, z64* out, long ld) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= np) return;
  int dx = rows[i].x - cols[j].x, dy = rows[i].y - cols[j].y;
  dx = dx < 0 ? -dx : dx;
  dy = dy < 0 ? -dy : dy;
  out[(long)i * ld + j] = T[(long)dy * (D + 1) + dx];
}

void gather_table(hipStream_t s, const z64* T, int D, const I2* rows, int m, const I2* cols, int np, z64* out,
                  long ld) {
  if (m <= 0 || np <= 0) return;
  LSH_REQUIRE(m <= 65535 * 16, -6, "gather: too many rows");
  for (int i0 = 0; i0 < m; i0 += 65535) {
    int mm = m - i0 < 65535 ? m - i0 : 65535;
    hipLaunchKernelGGL(k_gather_table, dim3(ceil_div(np, 256), mm), dim3(256), 0, s, T, D, rows + i0, mm, cols,
                       np, out + (long)i0 * ld, ld);
    LSH_LAUNCH_CHECK();
  }
}

// rows r in [r0, r1) of the parent's proxy matrix, interleaved (r = 2q + c:
// pivot q of this level in child c): out[r][j] = T(point - prox[j]) (and
// T2 at column np + j), point = cand[J[q]] + off[c]
__global__ void k_next_gram_rows(const z64* __restrict__ T, const z64* __restrict__ T2, int D,
                                 const I2* __restrict__ cand, const int* __restrict__ J, I2 off0, I2 off1,
                                 const I2* __restrict__ prox, int np, int r0, z64* out, long ld) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = r0 + blockIdx.y;
  if (j >= np) return;
  const I2 c = cand[J[r >> 1]], o = (r & 1) ? off1 : off0;
  int dx = c.x + o.x - prox[j].x, dy = c.y + o.y - prox[j].y;
  dx = dx < 0 ? -dx : dx;
  dy = dy < 0 ? -dy : dy;
  const long t = (long)dy * (D + 1) + dx;
  out[(long)r * ld + j] = T[t];
  if (T2) out[(long)r * ld + np + j] = T2[t];
}

// M[c k + q][c' k + q'] from the interleaved rows r = 2q + c, r' = 2q' + c'
// (entry (r, r') stored when r >= r'; else the conjugate of (r', r))
__global__ void k_next_gram_pack(const z64* __restrict__ G, long ldg, int k, z64* M) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long m = 2L * k;
  if (e >= m * m) return;
  const int i = (int)(e / m), jj = (int)(e - (long)i * m);
  const int ci = i >= k, qi = i - ci * k, cj = jj >= k, qj = jj - cj * k;
  const long r = 2L * qi + ci, rr = 2L * qj + cj;
  M[e] = r >= rr ? G[r * ldg + rr] : conjg(G[rr * ldg + r]);
}

void next_gram_rows(NextGram& g, const int* J, int j) {
  if (j > g.cap) j = g.cap;
  if (j <= g.done) return;
  const int r0 = 2 * g.done, nr = 2 * (j - g.done);
  for (int a = 0; a < nr; a += 65535) {
    const int rows = nr - a < 65535 ? nr - a : 65535;
    hipLaunchKernelGGL(k_next_gram_rows, dim3(ceil_div(g.np, 256), rows), dim3(256), 0, g.gs, g.T, g.T2, g.D,
                       g.cand, J, g.off[0], g.off[1], g.prox, g.np, r0 + a, g.A, (long)g.ncols);
    LSH_LAUNCH_CHECK();
  }
  // G rows [r0, 2 j), columns [0, 2 j): the new rows against every row so far
  cgemm<double>(g.gs, nr, 2 * j, g.ncols, mk(1.0, 0.0), g.A + (long)r0 * g.ncols, g.ncols, 0, OP_N, g.A, g.ncols, 0,
                OP_C, mk(0.0, 0.0), nullptr, 0, 0, g.G + (long)r0 * 2 * g.cap, 2L * g.cap, 0, 1);
  g.done = j;
}

void next_gram_pack(hipStream_t s, const NextGram& g, int k, z64* M) {
  const long mm = 4L * k * k;
  hipLaunchKernelGGL(k_next_gram_pack, dim3(ceil_div(mm, 256L)), dim3(256), 0, s, g.G, 2L * g.cap, k, M);
  LSH_LAUNCH_CHECK();
}

__device__ __forceinline__ void wave_argmax_d(double& v, int& idx) {
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ----------------------------------------------- CPQR row ID (one workgroup)
// Columns of A^T are the rows of W (contiguous); Householder reflectors act
// on the proxy index.  After step j, W[i][j] (i > j) holds R[j][i].
constexpr int QR_NT = 1024, QR_NW = QR_NT / 64;

__global__ __launch_bounds__(QR_NT) void k_cpqr(z64* W, int m, int np, double thr, int* J, z64* U, int* k_out,
                                                 double* nrm, z64* Rd) {
  __shared__ double sb[QR_NW];
  __shared__ int si[QR_NW];
  __shared__ int s_p;
  __shared__ double s_val;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < m; i += QR_NT) J[i] = i;
  for (int i = wave; i < m; i += QR_NW) {
    double a = 0;
    for (int q = lane; q < np; q += 64) a += abs2(W[(long)i * np + q]);
    a = wave_sum_d(a);
    if (lane == 0) nrm[i] = a;
  }
  __syncthreads();
  const int kmax = m < np ? m : np;
  int k = kmax;
  for (int j = 0; j < kmax; ++j) {
    double best = -1;
    int bi = m;
    for (int i = j + tid; i < m; i += QR_NT) {
      const double a = nrm[i];
      if (a > best || (a == best && J[i] < (bi < m ? J[bi] : 1 << 30))) { best = a; bi = i; }
    }
    wave_argmax_d(best, bi);
    if (lane == 0) { sb[wave] = best; si[wave] = bi; }
    __syncthreads();
    if (tid == 0) {
      double bb = sb[0];
      int ii = si[0];
      for (int w = 1; w < QR_NW; ++w)
        if (sb[w] > bb) { bb = sb[w]; ii = si[w]; }
      s_p = ii;
      s_val = bb;
    }
    __syncthreads();
    const int p = s_p;
    if (!(sqrt(s_val) > thr)) { k = j; break; }
    if (p != j) {
      for (int q = tid; q < np; q += QR_NT) {
        const z64 t = W[(long)j * np + q];
        W[(long)j * np + q] = W[(long)p * np + q];
        W[(long)p * np + q] = t;
      }
      if (tid == 0) {
        const double tn = nrm[j]; nrm[j] = nrm[p]; nrm[p] = tn;
        const int tj = J[j]; J[j] = J[p]; J[p] = tj;
      }
    }
    __syncthreads();
    // Householder vector of row j, entries q >= j
    double a = 0;
    for (int q = j + tid; q < np; q += QR_NT) a += abs2(W[(long)j * np + q]);
    a = wave_sum_d(a);
    if (lane == 0) sb[wave] = a;
    __syncthreads();
    if (tid == 0) {
      double nx = 0;
      for (int w = 0; w < QR_NW; ++w) nx += sb[w];
      nx = sqrt(nx);
      const z64 x0 = W[(long)j * np + j];
      const double ax0 = sqrt(abs2(x0));
      const z64 ph = ax0 > 0 ? mk(x0.x / ax0, x0.y / ax0) : mk(1.0, 0.0);
      const z64 alpha = mk(-ph.x * nx, -ph.y * nx);
      const z64 v0 = x0 - alpha;
      const double vn2 = nx * nx - ax0 * ax0 + abs2(v0);
      Rd[j] = alpha;
      W[(long)j * np + j] = v0;
      s_val = vn2 > 0 ? 2.0 / vn2 : 0.0;
    }
    __syncthreads();
    const double beta = s_val;
    const z64* v = W + (long)j * np;
    for (int i = j + 1 + wave; i < m; i += QR_NW) {
      z64* w = W + (long)i * np;
      z64 sacc = mk(0.0, 0.0);
      for (int q = j + lane; q < np; q += 64) fma_acc(sacc, conjg(v[q]), w[q]);
      sacc.x = wave_sum_d(sacc.x);
      sacc.y = wave_sum_d(sacc.y);
      const z64 f = beta * sacc;
      double nn = 0;
      for (int q = j + lane; q < np; q += 64) {
        const z64 t = w[q] - f * v[q];
        w[q] = t;
        if (q > j) nn += abs2(t);
      }
      nn = wave_sum_d(nn);
      if (lane == 0) nrm[i] = nn;
    }
    __syncthreads();
  }
  // U: rows J[a] (a < k) are unit rows; rows J[k + c] hold (R11^{-1} R12)^T
  for (int c = tid; c < m - k; c += QR_NT) {
    z64* urow = U + (long)J[k + c] * k;
    for (int a = k - 1; a >= 0; --a) {
      z64 t = W[(long)(k + c) * np + a];  // R12[a][c]
      for (int b2 = a + 1; b2 < k; ++b2) t = t - W[(long)b2 * np + a] * urow[b2];  // R11[a][b2]
      urow[a] = cdiv(t, Rd[a]);
    }
  }
  for (int e = tid; e < k * k; e += QR_NT) {
    const int a = e / k, b2 = e % k;
    U[(long)J[a] * k + b2] = mk(a == b2 ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) *k_out = k;
}

size_t rowid_cpqr_ws(int m) { return (size_t)m * (sizeof(double) + sizeof(z64)) + 256; }

void rowid_cpqr(hipStream_t s, z64* A, int m, int np, double thr, int* J, z64* U, int* k_dev, void* ws) {
  ProfScope ps("cpqr", s, 16.0 * (double)m * np);
  double* nrm = static_cast<double*>(ws);
  z64* Rd = reinterpret_cast<z64*>(static_cast<char*>(ws) + ((m * sizeof(double) + 15) / 16) * 16);
  hipLaunchKernelGGL(k_cpqr, dim3(1), dim3(QR_NT), 0, s, A, m, np, thr, J, U, k_dev, nrm, Rd);
  LSH_LAUNCH_CHECK();
}

// ------------------------------------------- Gram / pivoted Cholesky row ID
__global__ void k_gram_init(const z64* M, int m, double* d, int* chosen, int* state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) { d[i] = M[(long)i * m + i].x; chosen[i] = 0; }
  if (i == 0) { state[0] = 0; state[1] = 0; }
}

// One-workgroup panel of nb <= PCH_NB pivots.  Per pivot: block argmax of the
// Schur diagonal over unchosen rows, then the new column
//   l_i = (conj(M[p][i]) - sum_{t in panel} L[i][t] conj(L[p][t])) / sqrt(d_p)
// where each thread first issues all its panel loads (independent, in
// registers) and the pivot row's panel entries come from LDS.
constexpr int PCH_NB = 32, PCH_MAXM = 4096;

__global__ __launch_bounds__(QR_NT) void k_pchol_panel(const z64* __restrict__ M, int m, double* d, int* chosen,
                                                        z64* Lt, int* piv, int j0, int nb, double thr2,
                                                        int* state) {
  constexpr int RPT = PCH_MAXM / QR_NT;  // rows per thread
  extern __shared__ unsigned char smem_raw[];
  double* ds = reinterpret_cast<double*>(smem_raw);        // Schur diagonal (m)
  unsigned char* cs = smem_raw + sizeof(double) * m;        // chosen flags (m)
  __shared__ double sb[QR_NW];
  __shared__ int si[QR_NW];
  __shared__ int s_p;
  __shared__ double s_d;
  __shared__ z64 lpc[PCH_NB];  // conj(L[p][t]) for the panel columns so far
  if (state[1]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < m; i += QR_NT) {
    ds[i] = d[i];
    cs[i] = (unsigned char)chosen[i];
  }
  __syncthreads();
  int jj = 0;
  bool stop = false;
  for (; jj < nb; ++jj) {
    const int j = j0 + jj;
    if (j >= m) {
      if (tid == 0) { state[0] = m; state[1] = 1; }
      stop = true;
      break;
    }
    double best = -1;
    int bi = m;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * QR_NT;
      if (i < m && !cs[i]) {
        const double a = ds[i];
        if (a > best || (a == best && i < bi)) { best = a; bi = i; }
      }
    }
    wave_argmax_d(best, bi);
    if (lane == 0) { sb[wave] = best; si[wave] = bi; }
    __syncthreads();
    if (tid < 64) {  // final reduction by one wave, then stage the pivot's panel row
      double bb = tid < QR_NW ? sb[tid] : -1.0;
      int ii = tid < QR_NW ? si[tid] : m;
      wave_argmax_d(bb, ii);
      if (tid == 0) { s_p = ii; s_d = bb; }
      if (tid < jj && ii < m) lpc[tid] = conjg(Lt[(long)(j0 + tid) * m + ii]);
    }
    __syncthreads();
    const int p = s_p;
    const double dp = s_d;
    if (!(dp > thr2)) {
      if (tid == 0) { state[0] = j; state[1] = 1; }
      stop = true;
      break;
    }
    const double sq = sqrt(dp), rs = 1.0 / sq;
    // issue every row's loads before any arithmetic
    z64 l[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * QR_NT;
      l[r] = (i < m) ? conjg(M[(long)p * m + i]) : mk(0.0, 0.0);
    }
    for (int t0 = 0; t0 < jj; t0 += 4) {
      z64 v[RPT][4];
#pragma unroll
      for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = tid + r * QR_NT;
          v[r][t] = (i < m && t0 + t < jj) ? Lt[(long)(j0 + t0 + t) * m + i] : mk(0.0, 0.0);
        }
#pragma unroll
      for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t0 + t < jj) l[r] = l[r] - v[r][t] * lpc[t0 + t];
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * QR_NT;
      if (i >= m) continue;
      z64 li;
      if (i == p) li = mk(sq, 0.0);
      else if (cs[i]) li = mk(0.0, 0.0);
      else {
        li = rs * l[r];
        ds[i] -= abs2(li);
      }
      Lt[(long)j * m + i] = li;
    }
    __syncthreads();
    if (tid == 0) { cs[p] = 1; piv[j] = p; ds[p] = 0; }
    __syncthreads();
  }
  for (int i = tid; i < m; i += QR_NT) {
    d[i] = ds[i];
    chosen[i] = cs[i];
  }
  if (!stop && tid == 0) state[0] = j0 + nb;
}


__global__ void k_gather_L11(const z64* Lt, int m, const int* piv, int k, z64* L11) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)k * k) return;
  const int a = (int)(e / k), b = (int)(e % k);
  L11[e] = Lt[(long)b * m + piv[a]];
}

// Lr[r][t] = L(rest[r], t)
__global__ void k_gather_rows(const z64* Lt, int m, const int* rest, int nr, int k, z64* Lr) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)nr * k) return;
  const int r = (int)(e / k), t = (int)(e % k);
  Lr[e] = Lt[(long)t * m + rest[r]];
}

// D[q] = diagonal block q of L11 (nb x nb), identity-padded past k
// Inverses of the 64 x 64 lower-triangular diagonal blocks of L11 (the last
// block padded with the identity) by forward substitution, one workgroup per
// block.  The four lanes of a quad share column c of the inverse, lane part
// holding rows 16 part .. 16 part + 15; step q finishes X[q][c] and passes it
// along the quad, whose later rows subtract L[r][q] X[q][c].
constexpr int TRI_B = 64;
__global__ __launch_bounds__(256) void k_trinv_blocks(const z64* L11, int k, z64* Dinv) {
  __shared__ z64 Ls[TRI_B][TRI_B];
  __shared__ z64 rd[TRI_B];  // 1 / L[q][q]
  const int tid = threadIdx.x, base = blockIdx.x * TRI_B;
  for (int e = tid; e < TRI_B * TRI_B; e += 256) {
    const int r = e / TRI_B, c = e % TRI_B, gi = base + r, gj = base + c;
    z64 v = mk(0.0, 0.0);
    if (gi < k && gj < k) v = L11[(long)gi * k + gj];
    else if (r == c) v = mk(1.0, 0.0);
    Ls[r][c] = v;
  }
  __syncthreads();
  if (tid < TRI_B) rd[tid] = crecip(Ls[tid][tid]);
  __syncthreads();
  const int c = tid >> 2, part = tid & 3, lane = tid & 63;
  z64 x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = mk(16 * part + i == c ? 1.0 : 0.0, 0.0);
  for (int q = 0; q < TRI_B; ++q) {
    z64 xq = mk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (16 * part + i == q) xq = x[i] * rd[q];
    const int src = (lane & ~3) | (q >> 4);
    xq.x = __shfl(xq.x, src);
    xq.y = __shfl(xq.y, src);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = 16 * part + i;
      if (r == q) x[i] = xq;
      else if (r > q) x[i] = x[i] - Ls[r][q] * xq;
    }
  }
  z64* D = Dinv + (long)blockIdx.x * TRI_B * TRI_B;
#pragma unroll
  for (int i = 0; i < 16; ++i) D[(16 * part + i) * TRI_B + c] = x[i];
}

// U[piv[a]] = e_a ; U[rest[r]] = X[r]
__global__ void k_scatter_U(z64* U, int k, const int* piv, const int* rest, int nr, const z64* X) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long tot = (long)(k + nr) * k;
  if (e >= tot) return;
  const int row = (int)(e / k), b = (int)(e % k);
  if (row < k) U[(long)piv[row] * k + b] = mk(row == b ? 1.0 : 0.0, 0.0);
  else U[(long)rest[row - k] * k + b] = X[(long)(row - k) * k + b];
}

// ------------------------------------ block-pivoted left-looking Cholesky
// The panels above take one pivot per workgroup-wide step and keep the whole
// Schur complement M - L L^H up to date (a rank-nb update of all m x m
// entries per panel).  The block variant below takes up to BP_NP pivots per
// step and never forms the trailing Schur complement:
//  1. candidates C = the BP_B unchosen rows with the largest Schur diagonal
//     d_i (radix selection), and dout = the largest d_i outside C;
//  2. S_C = M[C,C] - L[C,:] L[C,:]^H;
//  3. greedy pivoted Cholesky of S_C in one workgroup: pivots P, factor L_PP
//     and its inverse;
//  4. the new columns L[:, P] = (M[:, P] - L L[P,:]^H) L_PP^{-H} and
//     d_i -= |L[i, P]|^2.
// Step 3 stops before a pivot whose Schur diagonal falls below alpha * dout.
// Diagonals only decrease, so every pivot taken has a Schur diagonal of at
// least alpha times the largest over all rows.  With alpha = 1 each pivot is
// the greedy pivot, and the pivot sequence, the stopping point and the rank
// are those of one-at-a-time greedy pivoting (up to ties); alpha < 1 takes
// more pivots per step (alpha-greedy pivoting: the same stopping rule, so the
// same error bound, with a rank that can differ by a few).  All step state (rank so far,
// pivot count, done flag) lives on the device: the host queues steps in
// batches and reads the done flag once per batch; a step queued after the
// end returns at entry.
constexpr int BP_B = 48, BP_NP = 32, BP_KC = 128, BP_KCS = 64, BP_SUB = 32, BP_SEL = 16384;
// state words (int): 0 rank j, 1 done, 2 pivots of this step, 3 candidates,
// 4..5 dout (double), 6 error flag, 8..8+BP_B candidate rows, 120..121 the
// stopping threshold thr2 (double)
constexpr int BPS_J = 0, BPS_DONE = 1, BPS_NP = 2, BPS_NC = 3, BPS_DOUT = 4, BPS_ERR = 6, BPS_CAND = 8,
              BPS_THR = 120, BPS_WORDS = 128;
static_assert(BPS_CAND + BP_B <= BPS_THR && BPS_THR + 2 <= BPS_WORDS - 4, "step state layout");

// thr2 = tol^2 sum_i d_i (the squared Frobenius norm of the candidate
// matrix), in one workgroup with a fixed summation order
__global__ __launch_bounds__(1024) void k_bp_thr2(const double* d, int m, double tol2, int* st) {
  __shared__ double part[1024];
  double v = 0.0;
  for (int i = threadIdx.x; i < m; i += 1024) v += d[i];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) reinterpret_cast<double*>(st + BPS_THR)[0] = tol2 * part[0];
}

// selection key of candidate row i: the Schur diagonal's bits above the
// index field, then the complemented index (ties go to the lower row)
constexpr unsigned BP_IDX = 0x3FFF;  // index field: rows < BP_SEL
static_assert(BP_SEL <= BP_IDX + 1, "key index field");
__device__ __forceinline__ unsigned long long bp_key(double d, int i) {
  return d > 0.0 ? (((unsigned long long)__double_as_longlong(d) & ~(unsigned long long)BP_IDX) | (BP_IDX - i))
                 : 0ull;
}

// Candidates: the BP_B largest keys (unchosen rows, d > 0) by an 8-pass
// most-significant-digit radix selection of the BP_B-th largest key, then
// the <= BP_B keys at or above it, sorted descending.
// KPT keys per thread: m <= 1024 KPT
template <int KPT>
__global__ __launch_bounds__(1024) void k_bp_select(const double* d, const int* chosen, int m, int* st) {
  __shared__ unsigned int hist[256];
  __shared__ unsigned long long s_prefix, s_mask;
  __shared__ int s_rank, s_cnt, s_stop;
  __shared__ unsigned long long ck[64];
  __shared__ unsigned long long s_below;
  if (st[BPS_DONE]) return;
  const double thr2 = reinterpret_cast<const double*>(st + BPS_THR)[0];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the previous step's pivots join the rank here (every later kernel of
  // this step reads the rank after this kernel has ended)
  {
    const int jn = st[BPS_J] + st[BPS_NP];
    __syncthreads();
    if (tid == 0) {
      st[BPS_J] = jn;
      st[BPS_NP] = 0;
      if (jn >= m) st[BPS_DONE] = 1;
    }
    if (jn >= m) return;
  }
  unsigned long long key[KPT];
  int nz = 0;
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const int i = tid + r * 1024;
    key[r] = (i < m && !chosen[i]) ? bp_key(d[i], i) : 0ull;
    nz += key[r] != 0;
  }
  if (tid == 0) { s_prefix = 0; s_mask = 0; s_rank = BP_B; s_cnt = 0; s_below = 0; s_stop = 0; }
  // total nonzero keys: when at most BP_B, every one is a candidate
  for (int off = 32; off > 0; off >>= 1) nz += __shfl_xor(nz, off);
  __shared__ int wz[16];
  if (lane == 0) wz[wave] = nz;
  __syncthreads();
  int total = 0;
  for (int w = 0; w < 16; ++w) total += wz[w];
  unsigned long long thr = 1;  // keys >= thr are candidates
  if (total > BP_B) {
    for (int pass = 7; pass >= 0; --pass) {
      const int sh = 8 * pass;
      for (int b = tid; b < 256; b += 1024) hist[b] = 0;
      __syncthreads();
      const unsigned long long pre = s_prefix, msk = s_mask;
#pragma unroll
      for (int r = 0; r < KPT; ++r)
        if (key[r] && (key[r] & msk) == pre) atomicAdd(&hist[(key[r] >> sh) & 255], 1u);
      __syncthreads();
      if (wave == 0) {
        // bins from the top: lane l holds bins 255-4l .. 252-4l
        unsigned int c[4], sum = 0;
        for (int q = 0; q < 4; ++q) { c[q] = hist[255 - 4 * lane - q]; sum += c[q]; }
        unsigned int inc = sum;  // inclusive prefix over lanes
        for (int off = 1; off < 64; off <<= 1) {
          const unsigned int o = __shfl_up(inc, off);
          if (lane >= off) inc += o;
        }
        const unsigned int exc = inc - sum;
        const int rank = s_rank;
        if ((int)exc < rank && rank <= (int)inc) {
          unsigned int run = exc;
          for (int q = 0; q < 4; ++q) {
            if (rank <= (int)(run + c[q])) {
              const unsigned long long digit = 255 - 4 * lane - q;
              s_prefix = pre | (digit << sh);
              s_mask = msk | (255ull << sh);
              s_rank = rank - (int)run;
              // the whole bin is among the BP_B largest: keys >= the prefix
              // (lower digits zero) are exactly the candidates
              if (rank - (int)run == (int)c[q]) s_stop = 1;
              break;
            }
            run += c[q];
          }
        }
      }
      __syncthreads();
      if (s_stop) break;  // (uniform)
    }
    thr = s_prefix;
  }
  // gather the candidates and the largest key below them
  unsigned long long below = 0;
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    if (key[r] >= thr && key[r]) {
      const int slot = atomicAdd(&s_cnt, 1);
      if (slot < 64) ck[slot] = key[r];
    } else if (key[r] > below) {
      below = key[r];
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(below, off);
    below = o > below ? o : below;
  }
  if (lane == 0) atomicMax(&s_below, below);
  __syncthreads();
  if (wave == 0) {
    const int cnt = s_cnt < BP_B ? s_cnt : BP_B;
    unsigned long long k = lane < cnt ? ck[lane] : 0ull;
    // bitonic sort of 64 keys across the wave, descending
    for (int size = 2; size <= 64; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const unsigned long long o = __shfl_xor(k, stride);
        const bool up = (lane & size) == 0;  // descending blocks
        const bool lower = (lane & stride) == 0;
        const bool takeMax = (up == lower);
        k = takeMax ? (o > k ? o : k) : (o < k ? o : k);
      }
    const int row = k ? (int)(BP_IDX - (unsigned)(k & BP_IDX)) : -1;
    if (lane < BP_B) st[BPS_CAND + lane] = row;
    int valid = (lane < BP_B && row >= 0 && d[row] > thr2) ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) valid += __shfl_xor(valid, off);
    if (lane == 0) {
      st[BPS_NC] = valid;
      const unsigned long long kb = s_below;
      reinterpret_cast<double*>(st + BPS_DOUT)[0] = kb ? d[BP_IDX - (unsigned)(kb & BP_IDX)] : 0.0;
      if (valid == 0) st[BPS_DONE] = 1;
    }
  }
}

// S_C partial sums: blockIdx.x = depth chunk c (BP_KCS deep, staged BP_SUB
// at a time), blockIdx.y = output quadrant (rows a0.., columns b0.., each
// BP_B / 2 wide): part[c][a][b] = sum_{t in chunk, t < j} L(C_a, t) conj(L(C_b, t)).
__global__ __launch_bounds__(256) void k_bp_sc(const z64* Lt, int m, const int* st, z64* part) {
  constexpr int H = BP_B / 2, PER = (H * H + 255) / 256;
  __shared__ z64 La[BP_SUB][H + 1], Lb2[BP_SUB][H + 1];
  if (st[BPS_DONE]) return;
  const int j = st[BPS_J], nc = st[BPS_NC];
  const int c = blockIdx.x, t0 = c * BP_KCS;
  if (t0 >= j) return;
  const int a0 = (blockIdx.y >> 1) * H, b0 = (blockIdx.y & 1) * H;
  const int tid = threadIdx.x;
  const int* cand = st + BPS_CAND;
  z64 acc[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) acc[r] = mk(0.0, 0.0);
  const int tend = (j - t0) < BP_KCS ? j : t0 + BP_KCS;
  for (int s0 = t0; s0 < tend; s0 += BP_SUB) {
    __syncthreads();
    for (int e = tid; e < 2 * BP_SUB * H; e += 256) {
      const int half = e / (BP_SUB * H), f = e % (BP_SUB * H), t = f / H, a = f % H;
      const int row = (half ? b0 : a0) + a;
      const z64 v = (row < nc && s0 + t < tend) ? Lt[(long)(s0 + t) * m + cand[row]] : mk(0.0, 0.0);
      if (half) Lb2[t][a] = v;
      else La[t][a] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + r * 256;
      if (e < H * H) {
        const int a = e / H, b = e % H;
        z64 v = acc[r];
        for (int t = 0; t < BP_SUB; ++t) v = v + La[t][a] * conjg(Lb2[t][b]);
        acc[r] = v;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = tid + r * 256;
    if (e < H * H) {
      const int a = a0 + e / H, b = b0 + e % H;
      part[(long)c * BP_B * BP_B + a * BP_B + b] = acc[r];
    }
  }
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  return __longlong_as_double(
      (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), lane) << 32) |
                  (unsigned)__builtin_amdgcn_readlane((int)bits, lane)));
}

// Greedy pivoted Cholesky of the candidate block S_C = M[C,C] - sum_c
// part[c] (formed first, in LDS; zero past the nc candidates) while the
// pivot exceeds thr2 and, after the first, is not below alpha * dout; at
// most BP_NP pivots.  Writes J[j + q], the pivot count, Lpp (np x np, lower,
// pivot order) and Linv = Lpp^{-1}, both with ld BP_NP; sets done when no
// pivot qualifies.
//
// Four waves: lane b of wave w holds rows 12w..12w+11 of column b of S in
// registers, and every wave keeps all the Schur diagonals d_b (lane b).  Per
// pivot p: the pivot's lanes write column t of the factor (rl * S[:, p],
// zero in picked rows) to LDS, one barrier, then every lane updates its rows,
// S[:, b] -= L[:, t] conj(L[b, t]), and d_b -= |L[b, t]|^2.  The next
// pivot's search (a DPP maximum of d) is independent of the row updates, so
// the two run interleaved.  Pivot keys hold the top 26 bits of d (sign,
// exponent, 14 mantissa bits): diagonals within a relative 2^-14 of the
// largest count as ties, won by the lower candidate.  L_PP^{-1} follows by
// forward substitution inside each wave.
constexpr int BP_CW = 4, BP_CR = BP_B / BP_CW;  // waves, rows per wave
__global__ __launch_bounds__(64 * BP_CW) void k_bp_chol(const z64* M, const z64* part, int m, double alpha, int* J,
                                                        int* st, z64* Lpp, z64* Linv) {
  static_assert(BP_B <= 64 && BP_NP == 32 && BP_B % BP_CW == 0 && BP_CW * 8 == BP_NP,
                "one lane per candidate; 8 columns of L_PP^{-1} per wave");
  __shared__ z64 Ss[BP_B][BP_B + 1];   // S_C
  __shared__ z64 Lb[BP_B][BP_NP + 1];  // factor columns for every candidate row
  __shared__ z64 xs[BP_NP][BP_NP + 1]; // L_PP^{-1}
  __shared__ double rlv[BP_NP];        // 1 / L[t][t]
  __shared__ int piv[BP_NP];
  if (st[BPS_DONE]) return;
  const int tid = threadIdx.x, b = tid & 63, w = tid >> 6, r0 = w * BP_CR;
  const int nc = st[BPS_NC], j = st[BPS_J];
  const double dout = alpha * reinterpret_cast<const double*>(st + BPS_DOUT)[0];
  const double thr2 = reinterpret_cast<const double*>(st + BPS_THR)[0];
  const int* cand = st + BPS_CAND;
  {  // S_C: the Gram entries less the depth chunks' partial products, in chunk order.  Each thread
     // holds PE entries and loads CB chunks of all of them at a time (PE * CB loads in flight).
    const int nch = (j + BP_KCS - 1) / BP_KCS;
    constexpr long CS = (long)BP_B * BP_B;
    constexpr int PE = BP_B * BP_B / (64 * BP_CW), CB = 4;
    static_assert(PE * 64 * BP_CW == BP_B * BP_B, "entries per thread");
    z64 v[PE];
    bool live[PE];
#pragma unroll
    for (int i = 0; i < PE; ++i) {
      const int e = tid + i * 64 * BP_CW, a = e / BP_B, c2 = e % BP_B;
      live[i] = a < nc && c2 < nc;
      v[i] = live[i] ? M[(long)cand[a] * m + cand[c2]] : mk(0.0, 0.0);
    }
    int c = 0;
    for (; c + CB <= nch; c += CB) {
      z64 pv[CB][PE];
#pragma unroll
      for (int q = 0; q < CB; ++q)
#pragma unroll
        for (int i = 0; i < PE; ++i)
          pv[q][i] = live[i] ? part[(c + q) * CS + tid + i * 64 * BP_CW] : mk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < CB; ++q)
#pragma unroll
        for (int i = 0; i < PE; ++i) v[i] = v[i] - pv[q][i];
    }
    for (; c < nch; ++c)
#pragma unroll
      for (int i = 0; i < PE; ++i)
        if (live[i]) v[i] = v[i] - part[c * CS + tid + i * 64 * BP_CW];
#pragma unroll
    for (int i = 0; i < PE; ++i) {
      const int e = tid + i * 64 * BP_CW;
      Ss[e / BP_B][e % BP_B] = v[i];
    }
    __syncthreads();
  }
  z64 col[BP_CR];
#pragma unroll
  for (int i = 0; i < BP_CR; ++i) col[i] = (r0 + i < nc && b < nc) ? Ss[r0 + i][b] : mk(0.0, 0.0);
  double d = b < nc ? Ss[b][b].x : 0.0;
  unsigned long long picked = 0;  // (the same in every lane)
  auto pick = [&]() -> int {      // largest unpicked diagonal, or -1
    unsigned key = 0;
    if (b < nc && !((picked >> b) & 1ull) && d > 0.0)
      key = ((unsigned)((unsigned long long)__double_as_longlong(d) >> 32) & ~63u) | (unsigned)(63 - b);
    key = wave_max_u32_uniform(key);
    return key ? 63 - (int)(key & 63u) : -1;
  };
  int p = pick();
  double dp = (p >= 0 && p < nc) ? readlane_f64(d, p) : 0.0;
  bool go = p >= 0 && p < nc && dp > thr2;
  int np = 0;
  for (int t = 0; t < BP_NP && go; ++t) {
    // rl = 1 / sqrt(dp): hardware estimate and two Newton steps
    double rl = __builtin_amdgcn_rsq(dp);
    rl = rl * (1.5 - 0.5 * dp * rl * rl);
    rl = rl * (1.5 - 0.5 * dp * rl * rl);
    const double lpp = dp * rl;
    if (b == p) {
#pragma unroll
      for (int i = 0; i < BP_CR; ++i) {
        const int a = r0 + i;
        const bool zero = (picked >> a) & 1ull;
        z64 v = rl * col[i];
        v.x = a == p ? lpp : (zero ? 0.0 : v.x);
        v.y = (a == p || zero) ? 0.0 : v.y;
        Lb[a][t] = v;
      }
      if (w == 0) {
        rlv[t] = rl;
        piv[t] = p;
      }
    }
    __syncthreads();
    const z64 clb = conjg(Lb[b < BP_B ? b : 0][t]);
    d -= abs2(clb);
    if (b == p) d = 0.0;
    picked |= 1ull << p;
    np = t + 1;
    // the next pivot (rows outside the block have Schur diagonal <= dout /
    // alpha, since diagonals only decrease: an accepted pivot is
    // alpha-greedy over all rows) and this pivot's row updates
    const int pn = pick();
#pragma unroll
    for (int i = 0; i < BP_CR; ++i) col[i] = col[i] - Lb[r0 + i][t] * clb;
    dp = (pn >= 0 && pn < nc) ? readlane_f64(d, pn) : 0.0;
    go = pn >= 0 && pn < nc && dp > thr2 && dp >= dout;
    p = pn;
  }
  __syncthreads();
  // X = L_PP^{-1}: wave w takes columns c = 8w + lane / 8; lane k = lane % 8
  // of a column holds rows r = k + 8i.  Step q: the owner of row q finishes
  // X[q][c] and passes it to the column's lanes, which subtract
  // L[r][q] X[q][c] from their later rows.
  {
    const int c = 8 * w + (b >> 3), k = b & 7;
    z64 acc[BP_NP / 8];
    int pr[BP_NP / 8];
#pragma unroll
    for (int i = 0; i < BP_NP / 8; ++i) {
      const int r = k + 8 * i;
      acc[i] = mk(r == c ? 1.0 : 0.0, 0.0);
      pr[i] = r < np ? piv[r] : 0;
    }
    for (int q = 0; q < np; ++q) {
      z64 xq = mk(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < BP_NP / 8; ++i)
        if (i == (q >> 3)) xq = rlv[q] * acc[i];
      const int src = (b & ~7) | (q & 7);
      xq.x = __shfl(xq.x, src);
      xq.y = __shfl(xq.y, src);
      if (k == (q & 7)) xs[q][c] = xq;
#pragma unroll
      for (int i = 0; i < BP_NP / 8; ++i) {
        const int r = k + 8 * i;
        if (r > q && r < np) acc[i] = acc[i] - Lb[pr[i]][q] * xq;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < BP_NP * BP_NP; e += 64 * BP_CW) {
    const int q = e / BP_NP, r = e % BP_NP;
    const bool in = q < np && r <= q;
    Lpp[e] = in ? Lb[piv[q]][r] : mk(0.0, 0.0);
    Linv[e] = in ? xs[q][r] : mk(0.0, 0.0);
  }
  if (w == 0) {
    int bad = 0;
    if (b < np) {
      const int row = cand[piv[b]];
      bad = row < 0 || row >= m;  // (cannot happen: candidates are rows)
      J[j + b] = row;
    }
    bad = __any(bad);
    if (b == 0) {
      st[BPS_NP] = bad ? 0 : np;
      if (np == 0 || bad) st[BPS_DONE] = 1;
      if (bad) st[BPS_ERR] = 1;
    }
  }
}

// Wt partial sums over depth chunk c (BP_KC deep): part[c][q][i] =
// sum_{t in chunk, t < j} conj(L(P_q, t)) L(i, t) for q < np, as a product
// on the 16x16x4 FP64 matrix instruction: (pivots x depth) times (depth x
// rows).  The pivot rows' conjugated values for the chunk sit in LDS (real
// and imaginary planes); each wave owns 64 rows i and streams their factor
// entries from HBM (16 consecutive rows per instruction operand, the next
// four depths in flight).  Three real products per complex step (Gauss's
// form: t1 = ar br, t2 = ai bi, t3 = (ar + ai)(br + bi); Re = t1 - t2,
// Im = t3 - t1 - t2); the second pivot tile is skipped when np <= 16.  Rows
// already chosen are computed too (the new-columns kernel ignores them).
// rows per workgroup: four waves of 16 JT rows.  The MFMA work of a
// workgroup, not the memory, bounds a launch here (FP64 16x16x4 at 64 cycles
// a wave), and early steps have few depth chunks: small row blocks (JT = 1)
// keep every unit busy then.
constexpr int BP_WT_JT = 1, BP_WT_ROWS = 64 * BP_WT_JT;
__global__ __launch_bounds__(256) void k_bp_wt(const z64* Lt, const int* J, int m, const int* st, z64* part) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  __shared__ double Apr[BP_NP][BP_KC + 1], Api[BP_NP][BP_KC + 1];
  if (st[BPS_DONE]) return;
  const int j = st[BPS_J], np = st[BPS_NP];
  const int c = blockIdx.y, t0 = c * BP_KC;
  if (t0 >= j) return;
  const int tn = (j - t0) < BP_KC ? (j - t0) : BP_KC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int* Pq = J + j;
  for (int e = tid; e < BP_NP * BP_KC; e += 256) {
    const int q = e / BP_KC, t = e % BP_KC;
    const z64 v = (q < np && t < tn) ? Lt[(long)(t0 + t) * m + Pq[q]] : mk(0.0, 0.0);
    Apr[q][t] = v.x;
    Api[q][t] = -v.y;
  }
  __syncthreads();
  constexpr int JT = BP_WT_JT;
  const int i0 = blockIdx.x * BP_WT_ROWS + wave * 16 * JT, lr = lane & 15, lk = lane >> 4;
  const bool two = np > 16;
  d4 w1[2][JT], w2[2][JT], w3[2][JT];
#pragma unroll
  for (int qt = 0; qt < 2; ++qt)
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      w1[qt][jt] = d4{0.0, 0.0, 0.0, 0.0};
      w2[qt][jt] = d4{0.0, 0.0, 0.0, 0.0};
      w3[qt][jt] = d4{0.0, 0.0, 0.0, 0.0};
    }
  // B (the rows' factor entries) streams in stages of WT_DS depths: the next
  // stage's loads are issued before the current stage's MFMAs, so that a
  // stage of matrix work (WT_DS / 4 depth steps) covers the memory latency
  constexpr int WT_DS = 16, WT_SUB = WT_DS / 4;
  static_assert(BP_KC % WT_DS == 0, "stages tile the depth chunk");
  auto loadB = [&](int s0, double (&br)[WT_SUB][JT], double (&bi)[WT_SUB][JT]) {
#pragma unroll
    for (int u = 0; u < WT_SUB; ++u) {
      const int t = s0 + 4 * u + lk;
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        const int i = i0 + 16 * jt + lr;
        const z64 v = (t < tn && i < m) ? Lt[(long)(t0 + t) * m + i] : mk(0.0, 0.0);
        br[u][jt] = v.x;
        bi[u][jt] = v.y;
      }
    }
  };
  double br[WT_SUB][JT], bi[WT_SUB][JT];
  loadB(0, br, bi);
  for (int s0 = 0; s0 < tn; s0 += WT_DS) {
    double nbr[WT_SUB][JT], nbi[WT_SUB][JT];
    loadB(s0 + WT_DS, nbr, nbi);  // the next stage in flight meanwhile
#pragma unroll
    for (int u = 0; u < WT_SUB; ++u) {
      const int t = s0 + 4 * u + lk;  // (< BP_KC: s0 <= BP_KC - WT_DS, BP_KC % WT_DS == 0)
      double bs[JT];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) bs[jt] = br[u][jt] + bi[u][jt];
#pragma unroll
      for (int qt = 0; qt < 2; ++qt) {
        if (qt == 1 && !two) break;
        const double ar = Apr[16 * qt + lr][t], ai = Api[16 * qt + lr][t], as = ar + ai;
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          w1[qt][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br[u][jt], w1[qt][jt], 0, 0, 0);
          w2[qt][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi[u][jt], w2[qt][jt], 0, 0, 0);
          w3[qt][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, bs[jt], w3[qt][jt], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < WT_SUB; ++u)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        br[u][jt] = nbr[u][jt];
        bi[u][jt] = nbi[u][jt];
      }
  }
  // accumulator register r of lane l holds the pivot row lk + 4 r of its tile
  z64* pc = part + (long)c * BP_NP * m;
#pragma unroll
  for (int qt = 0; qt < 2; ++qt) {
    if (qt == 1 && !two) break;
#pragma unroll
    for (int jt = 0; jt < JT; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * qt + lk + 4 * r, i = i0 + 16 * jt + lr;
        if (q < np && i < m) {
          const double t1 = w1[qt][jt][r], t2 = w2[qt][jt][r];
          pc[(long)q * m + i] = mk(t1 - t2, w3[qt][jt][r] - t1 - t2);
        }
      }
  }
}

// New factor rows Lt[j+q][i] = sum_q' conj(Linv[q][q']) W[q'][i] with
// W[q'][i] = conj(M[P_q'][i]) - sum_c part[c][q'][i]; then rows already
// chosen get exact zeros, the pivot rows get Lpp exactly, other rows have
// their Schur diagonal reduced, and the pivots are marked chosen.  A
// workgroup takes 32 rows i; thread (q, i) forms W[q][i] (its chunk sum
// spread over all threads), the products go through LDS.
constexpr int BP_NCR = 32;
static_assert(BP_NCR == BP_NP && BP_NCR * BP_NP == 1024, "one thread per (pivot, row) pair");
__global__ __launch_bounds__(1024) void k_bp_newcols(z64* Lt, const z64* M, int m, const int* J, const z64* part,
                                                     const z64* Lpp, const z64* Linv, int* chosen, double* d,
                                                     const int* st) {
  __shared__ z64 W[BP_NP][BP_NCR + 1];
  __shared__ z64 Li[BP_NP][BP_NP + 1];
  __shared__ double sd[BP_NP][BP_NCR + 1];
  if (st[BPS_DONE]) return;
  const int j = st[BPS_J], np = st[BPS_NP];
  const int nch = (j + BP_KC - 1) / BP_KC;
  const int tid = threadIdx.x, q = tid / BP_NCR, ii = tid % BP_NCR;
  const int i = blockIdx.x * BP_NCR + ii;
  const int* Pq = J + j;
  Li[q][ii] = conjg(Linv[q * BP_NP + ii]);  // (BP_NCR == BP_NP: one entry per thread)
  z64 w = mk(0.0, 0.0);
  if (i < m && q < np && !chosen[i]) {
    w = conjg(M[(long)Pq[q] * m + i]);
    int c = 0;
    for (; c + 4 <= nch; c += 4) {
      const z64 p0 = part[((long)(c + 0) * BP_NP + q) * m + i], p1 = part[((long)(c + 1) * BP_NP + q) * m + i];
      const z64 p2 = part[((long)(c + 2) * BP_NP + q) * m + i], p3 = part[((long)(c + 3) * BP_NP + q) * m + i];
      w = w - p0;
      w = w - p1;
      w = w - p2;
      w = w - p3;
    }
    for (; c < nch; ++c) w = w - part[((long)c * BP_NP + q) * m + i];
  }
  W[q][ii] = w;
  __syncthreads();
  const bool live = i < m;
  int q0 = -1;
  for (int r = 0; r < np; ++r)
    if (live && Pq[r] == i) q0 = r;
  const bool was_chosen = live && chosen[i] != 0;
  z64 v = mk(0.0, 0.0);
  if (live && q < np) {
    if (q0 >= 0) v = Lpp[q0 * BP_NP + q];
    else if (!was_chosen)
      for (int r = 0; r <= q; ++r) v = v + Li[q][r] * W[r][ii];
    Lt[(long)(j + q) * m + i] = v;
  }
  sd[q][ii] = abs2(v);
  __syncthreads();
  if (live && q == 0) {
    if (q0 >= 0) {
      chosen[i] = 1;
      d[i] = 0.0;
    } else if (!was_chosen) {
      double t = 0.0;
      for (int r = 0; r < np; ++r) t += sd[r][ii];
      d[i] -= t;
    }
  }
}

size_t rowid_bp_ws(int m) {
  const size_t mm = (size_t)m * m, mp = (size_t)m + BP_KC;
  const size_t nch = mp / BP_KC + 1;
  return sizeof(z64) * (mm + mp * m + 2 * mm) + sizeof(double) * m + sizeof(int) * (3 * m + BPS_WORDS) +
         sizeof(z64) * (BP_B * BP_B + 2 * BP_NP * BP_NP + (mp / BP_KCS + 1) * BP_B * BP_B +
                        nch * (size_t)BP_NP * m) +
         inverse_ws_bytes<double>(64, m / 64 + 1) + sizeof(z64) * (size_t)(m / 64 + 1) * 64 * 64 + 32 * 256;
}

static int grid_of(long n) {
  const long g = (n + 255) / 256;
  return (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

// Linv[q] (diagonal block q of the k x k array, row-major, leading dimension
// k) = D[q] for the nb inverted 64 x 64 blocks (the last one cut at k)
__global__ void k_place_diag(const z64* D, int k, z64* Linv) {
  const int q = blockIdx.y, base = q * TRI_B;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < TRI_B * TRI_B; e += gridDim.x * blockDim.x) {
    const int r = e / TRI_B, c = e % TRI_B;
    if (base + r < k && base + c < k) Linv[(long)(base + r) * k + base + c] = D[(long)q * TRI_B * TRI_B + e];
  }
}

// U = L(rest, 0:k) L11^{-1} with U(J) = I, from the column-major factor Lt
// (shared by both Gram paths).  L11^{-1} is formed explicitly from the
// inverted 64 x 64 diagonal blocks by doubling (inv [[A, 0], [B, C]] =
// [[A^-1, 0], [-C^-1 B A^-1, C^-1]], all pairs of one size in two batched
// products), then U(rest) = L(rest) L11^{-1} is one product: a dozen wide
// launches instead of a block-by-block substitution chain.  Linv (k x k) and
// the pairs' temporaries T (at most k^2 / 4 entries) are scratch.
static void gram_interp(hipStream_t s, const z64* Lt, int m, int k, int* J, z64* U, int* rest, z64* L11, z64* Lr,
                        z64* Dinv, z64* Linv, z64* T) {
  const int DB = 64;
  std::vector<int> ph(k), rh;
  LSH_HIP(hipMemcpyAsync(ph.data(), J, sizeof(int) * k, hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  {
    std::vector<char> used(m, 0);
    for (int v : ph) used[v] = 1;
    for (int i = 0; i < m; ++i)
      if (!used[i]) rh.push_back(i);
  }
  const int nr = (int)rh.size();
  if (nr) LSH_HIP(hipMemcpyAsync(rest, rh.data(), sizeof(int) * nr, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_gather_L11, dim3(ceil_div((long)k * k, 256)), dim3(256), 0, s, Lt, m, J, k, L11);
  LSH_LAUNCH_CHECK();
  if (nr) {
    hipLaunchKernelGGL(k_gather_rows, dim3(ceil_div((long)nr * k, 256)), dim3(256), 0, s, Lt, m, rest, nr, k, Lr);
    LSH_LAUNCH_CHECK();
    const int nblk = ceil_div(k, DB);
    static_assert(DB == TRI_B, "diagonal block size");
    hipLaunchKernelGGL(k_trinv_blocks, dim3(nblk), dim3(256), 0, s, L11, k, Dinv);
    LSH_LAUNCH_CHECK();
    fill_zero(s, Linv, sizeof(z64) * (size_t)k * k);
    hipLaunchKernelGGL(k_place_diag, dim3(16, nblk), dim3(256), 0, s, Dinv, k, Linv);
    LSH_LAUNCH_CHECK();
    const z64 one = mk(1.0, 0.0), mone = mk(-1.0, 0.0), zero = mk(0.0, 0.0);
    for (int b = DB; b < k; b *= 2) {
      // pairs (A at rows i0 .. i0+b, C at i0+b .. min(i0+2b, k)), i0 = p 2b
      const int full = k / (2 * b);                  // pairs with a whole C block
      const long st = 2L * b * (k + 1);              // stride between pairs' diagonal positions
      if (full > 0) {
        // T_p = B_p A_p^{-1}, then Linv(C rows, A cols) = -C_p^{-1} T_p
        cgemm<double>(s, b, b, b, one, L11 + (long)b * k, k, st, OP_N, Linv, k, st, OP_N, zero, nullptr, 0, 0, T,
                      b, (long)b * b, full);
        cgemm<double>(s, b, b, b, mone, Linv + (long)b * (k + 1), k, st, OP_N, T, b, (long)b * b, OP_N, zero,
                      nullptr, 0, 0, Linv + (long)b * k, k, st, full);
      }
      const int i0 = full * 2 * b, c2 = k - i0 - b;  // a last pair with a partial C block
      if (c2 > 0) {
        cgemm<double>(s, c2, b, b, one, L11 + (long)(i0 + b) * k + i0, k, 0, OP_N, Linv + (long)i0 * (k + 1), k, 0,
                      OP_N, zero, nullptr, 0, 0, T, b, 0, 1);
        cgemm<double>(s, c2, b, c2, mone, Linv + (long)(i0 + b) * (k + 1), k, 0, OP_N, T, b, 0, OP_N, zero,
                      nullptr, 0, 0, Linv + (long)(i0 + b) * k + i0, k, 0, 1);
      }
    }
    z64* X = L11 + (size_t)k * k;  // (nr x k) after L11 in the same buffer
    cgemm<double>(s, nr, k, k, one, Lr, k, 0, OP_N, Linv, k, 0, OP_N, zero, nullptr, 0, 0, X, k, 0, 1);
    hipLaunchKernelGGL(k_scatter_U, dim3(ceil_div((long)(k + nr) * k, 256)), dim3(256), 0, s, U, k, J, rest, nr, X);
  } else {
    hipLaunchKernelGGL(k_scatter_U, dim3(ceil_div((long)k * k, 256)), dim3(256), 0, s, U, k, J, rest, 0, L11);
  }
  LSH_LAUNCH_CHECK();
}

int rowid_bp(hipStream_t s, const z64* A, int m, int np, double tol, double alpha, int* J, z64* U, void* ws,
             bool gram_ready, NextGram* next, const std::function<void(int)>& on_skel) {
  LSH_REQUIRE(alpha > 0.0 && alpha <= 1.0, -1, "row ID: alpha must lie in (0, 1]");
  LSH_REQUIRE(m <= BP_SEL, -6, "row ID: more than 16384 candidate rows in one level");
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) { char* r = p; p += ((bytes + 255) / 256) * 256; return (void*)r; };
  const size_t mp = (size_t)m + BP_KC;
  const int nch = (int)(mp / BP_KC) + 1, nchS = (int)(mp / BP_KCS) + 1;
  z64* M = static_cast<z64*>(take(sizeof(z64) * (size_t)m * m));
  z64* Lt = static_cast<z64*>(take(sizeof(z64) * mp * m));
  z64* L11 = static_cast<z64*>(take(sizeof(z64) * (size_t)m * m));
  z64* Lr = static_cast<z64*>(take(sizeof(z64) * (size_t)m * m));
  double* d = static_cast<double*>(take(sizeof(double) * m));
  int* chosen = static_cast<int*>(take(sizeof(int) * m));
  int* rest = static_cast<int*>(take(sizeof(int) * m));
  int* st = static_cast<int*>(take(sizeof(int) * BPS_WORDS));
  z64* Lpp = static_cast<z64*>(take(sizeof(z64) * BP_NP * BP_NP));
  z64* Linv = static_cast<z64*>(take(sizeof(z64) * BP_NP * BP_NP));
  z64* partS = static_cast<z64*>(take(sizeof(z64) * (size_t)nchS * BP_B * BP_B));
  z64* partW = static_cast<z64*>(take(sizeof(z64) * (size_t)nch * BP_NP * m));
  const int DB = 64;
  z64* Dinv = static_cast<z64*>(take(sizeof(z64) * (size_t)(m / DB + 1) * DB * DB));
  void* invws = take(inverse_ws_bytes<double>(DB, m / DB + 1));
  // Gram matrix and its diagonal; the factor starts at zero
  if (!gram_ready) {
    cgemm<double>(s, m, m, np, mk(1.0, 0.0), A, np, 0, OP_N, A, np, 0, OP_C, mk(0.0, 0.0), nullptr, 0, 0, M, m, 0,
                  1, false, nullptr, true);  // Hermitian: lower tiles, then the mirror
    mirror_lower<double>(s, M, m, m);
  }
  fill_zero(s, Lt, sizeof(z64) * mp * m);
  fill_zero(s, st, sizeof(int) * BPS_WORDS);
  hipLaunchKernelGGL(k_gram_init, dim3(ceil_div(m, 256)), dim3(256), 0, s, M, m, d, chosen, st + BPS_WORDS - 4);
  LSH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bp_thr2, dim3(1), dim3(1024), 0, s, d, m, tol * tol, st);
  LSH_LAUNCH_CHECK();
  const int gm = ceil_div(m, 256);
  // steps in batches; the first batches are short (the first step alone
  // can take every pivot of a small block).  With a parent Gram to feed, at
  // most 16 steps a batch, so that its last rows (after the final step) are
  // few.
  int batch = 4, host_st[4] = {0, 0, 0, 0};
  const int max_batch = next ? 16 : 32;
  while (true) {
    for (int b = 0; b < batch; ++b) {
      {
        ProfScope ps("bp_select", s, 16.0 * m);
        if (m <= 4096) hipLaunchKernelGGL(k_bp_select<4>, dim3(1), dim3(1024), 0, s, d, chosen, m, st);
        else if (m <= 8192) hipLaunchKernelGGL(k_bp_select<8>, dim3(1), dim3(1024), 0, s, d, chosen, m, st);
        else hipLaunchKernelGGL(k_bp_select<BP_SEL / 1024>, dim3(1), dim3(1024), 0, s, d, chosen, m, st);
      }
      LSH_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_bp_sc, dim3(nchS, 4), dim3(256), 0, s, Lt, m, st, partS);
      LSH_LAUNCH_CHECK();
      {
        ProfScope ps("bp_chol", s, 16.0 * BP_B * BP_B);
        hipLaunchKernelGGL(k_bp_chol, dim3(1), dim3(64 * BP_CW), 0, s, M, partS, m, alpha, J, st, Lpp, Linv);
      }
      LSH_LAUNCH_CHECK();
      {
        ProfScope ps("bp_wt", s, 16.0 * m * m);
        hipLaunchKernelGGL(k_bp_wt, dim3(ceil_div(m, BP_WT_ROWS), nch), dim3(256), 0, s, Lt, J, m, st, partW);
      }
      LSH_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_bp_newcols, dim3(ceil_div(m, BP_NCR)), dim3(1024), 0, s, Lt, M, m, J, partW, Lpp, Linv,
                         chosen, d, st);
      LSH_LAUNCH_CHECK();
    }
    LSH_HIP(hipMemcpyAsync(host_st, st, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    if (host_st[BPS_DONE]) break;
    if (next) next_gram_rows(*next, J, host_st[BPS_J] + host_st[BPS_NP]);
    batch = batch < max_batch ? batch * 2 : max_batch;
  }
  int j = 0;
  {
    int hs[8];
    LSH_HIP(hipMemcpyAsync(hs, st, sizeof(int) * 8, hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    LSH_REQUIRE(hs[BPS_ERR] == 0, -4, "row ID: pivot row out of range");
    j = hs[BPS_J] + hs[BPS_NP];  // (pivots of a step not yet advanced)
  }
  if (j < 1) {  // a zero block still gets one skeleton: row 0, U = e_0
    const int zero = 0;
    const z64 one = mk(1.0, 0.0);
    LSH_HIP(hipMemcpyAsync(J, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    fill_zero(s, U, sizeof(z64) * (size_t)m);
    LSH_HIP(hipMemcpyAsync(U, &one, sizeof(z64), hipMemcpyHostToDevice, s));
    LSH_HIP(hipStreamSynchronize(s));
    if (next) next_gram_rows(*next, J, 1);
    if (on_skel) on_skel(1);
    return 1;
  }
  if (next) next_gram_rows(*next, J, j);  // (J is final: the stream was synchronised)
  if (on_skel) on_skel(j);                // (before the interpolation matrix)
  // (the Gram is no longer needed: it holds L11^{-1}; the pairs' temporaries
  // follow the rest rows in Lr)
  gram_interp(s, Lt, m, j, J, U, rest, L11, Lr, Dinv, M, Lr + (size_t)(m - j) * j);
  (void)invws;
  return j;
}

size_t rowid_gram_ws(int m) {
  const size_t mm = (size_t)m * m;
  return sizeof(z64) * mm * 4 + sizeof(double) * m + sizeof(int) * (3 * m + 16) +
         inverse_ws_bytes<double>(64, m / 64 + 1) + sizeof(z64) * (size_t)(m / 64 + 1) * 64 * 64 +
         (sizeof(double) + sizeof(int)) * 512 + 16384;
}

int rowid_gram(hipStream_t s, const z64* A, int m, int np, double tol, int* J, z64* U, void* ws) {
  LSH_REQUIRE(m <= PCH_MAXM, -6, "row ID: more than 4096 candidate rows in one level");
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) { char* r = p; p += ((bytes + 255) / 256) * 256; return (void*)r; };
  z64* M = static_cast<z64*>(take(sizeof(z64) * (size_t)m * m));
  z64* Lt = static_cast<z64*>(take(sizeof(z64) * (size_t)m * m));
  z64* L11 = static_cast<z64*>(take(sizeof(z64) * (size_t)m * m));
  z64* Lr = static_cast<z64*>(take(sizeof(z64) * (size_t)m * m));
  double* d = static_cast<double*>(take(sizeof(double) * m));
  int* chosen = static_cast<int*>(take(sizeof(int) * m));
  int* rest = static_cast<int*>(take(sizeof(int) * m));
  int* state = static_cast<int*>(take(sizeof(int) * 16));
  const int DB = 64;
  z64* Dinv = static_cast<z64*>(take(sizeof(z64) * (size_t)(m / DB + 1) * DB * DB));
  void* invws = take(inverse_ws_bytes<double>(DB, m / DB + 1));
  cgemm<double>(s, m, m, np, mk(1.0, 0.0), A, np, 0, OP_N, A, np, 0, OP_C, mk(0.0, 0.0), nullptr, 0, 0, M, m, 0, 1,
                false, nullptr, true);  // Hermitian: lower tiles, then the mirror
  mirror_lower<double>(s, M, m, m);
  hipLaunchKernelGGL(k_gram_init, dim3(ceil_div(m, 256)), dim3(256), 0, s, M, m, d, chosen, state);
  LSH_LAUNCH_CHECK();
  // ||A||_F^2 = trace(M)
  std::vector<double> dh(m);
  LSH_HIP(hipMemcpyAsync(dh.data(), d, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  double fro2 = 0;
  for (double v : dh) fro2 += v;
  const double thr2 = tol * tol * fro2;
  static const int nb = [] {
    const char* e = std::getenv("LSH_PCHOL_NB");
    int v = e ? std::atoi(e) : 16;
    return (v >= 4 && v <= PCH_NB) ? v : 16;
  }();
  int rank = 0;
  // One workgroup per panel: the per-pivot cost is one workgroup's L2
  // stream of the panel, ~m * nb / 2 entries.  All panels and trailing updates are queued at once: each panel kernel
  // returns at entry once state[1] (done) is set, and each update is skipped
  // through the same flag, so the host reads the rank once per level.
  for (int j0 = 0; j0 < m; j0 += nb) {
    {
      ProfScope ps("pchol_panel", s, 16.0 * (double)m * nb);
      hipLaunchKernelGGL(k_pchol_panel, dim3(1), dim3(QR_NT), (size_t)m * (sizeof(double) + 1), s, M, m, d, chosen,
                         Lt, J, j0, nb, thr2, state);
    }
    LSH_LAUNCH_CHECK();
    if (j0 + nb < m)  // trailing update of the Schur complement: M -= Lp Lp^H
      cgemm<double>(s, m, m, nb, mk(-1.0, 0.0), Lt + (long)j0 * m, m, 0, OP_T, Lt + (long)j0 * m, m, 0, OP_R,
                    mk(1.0, 0.0), M, m, 0, M, m, 0, 1, false, state + 1);
  }
  {
    int st[2];
    LSH_HIP(hipMemcpyAsync(st, state, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    rank = st[0];
  }
  const int k = rank < 1 ? 1 : rank;
  gram_interp(s, Lt, m, k, J, U, rest, L11, Lr, Dinv, M, Lr + (size_t)(m - k) * k);
  (void)invws;
  return k;
}

// ------------------------------------------------------------- leaf factor
template <typename R>
__global__ void k_leaf_build(cplx<R>* X, const cplx<R>* __restrict__ G, int mL, const double* __restrict__ b,
                             double kappa2, const I2* __restrict__ org, const I2* __restrict__ pts, int n) {
  const long t = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mL * mL) return;
  const int i = e / mL, j = e % mL;
  const I2 o = org[t], pi = pts[i];
  const double bi = kappa2 * b[(long)(o.y + pi.y) * n + (o.x + pi.x)];
  cplx<R> v = (R)bi * G[e];
  if (i == j) v.x += R(1);
  X[t * (long)mL * mL + e] = v;
}

template <typename R>
void leaf_build(hipStream_t s, cplx<R>* X, const cplx<R>* Gleaf, int mL, const double* b, double kappa2,
                const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n) {
  LSH_REQUIRE(nleaf <= 65535 * 64, -6, "too many leaves");
  for (int t0 = 0; t0 < nleaf; t0 += 65535) {
    int nt = nleaf - t0 < 65535 ? nleaf - t0 : 65535;
    hipLaunchKernelGGL(k_leaf_build<R>, dim3(ceil_div(mL * mL, 256), nt), dim3(256), 0, s,
                       X + (long)t0 * mL * mL, Gleaf, mL, b, kappa2, leaf_origin + t0, leaf_pts, n);
    LSH_LAUNCH_CHECK();
  }
}

template <typename R>
__global__ void k_leaf_scale_U(cplx<R>* Y, const cplx<R>* __restrict__ U, int mL, int k,
                               const double* __restrict__ b, double kappa2, const I2* __restrict__ org,
                               const I2* __restrict__ pts, int n) {
  const long t = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mL * k) return;
  const int i = e / k;
  const I2 o = org[t], pi = pts[i];
  const double bi = kappa2 * b[(long)(o.y + pi.y) * n + (o.x + pi.x)];
  Y[t * (long)mL * k + e] = (R)bi * U[e];
}

template <typename R>
void leaf_scale_U(hipStream_t s, cplx<R>* Y, const cplx<R>* U, int mL, int k, const double* b, double kappa2,
                  const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n) {
  for (int t0 = 0; t0 < nleaf; t0 += 65535) {
    int nt = nleaf - t0 < 65535 ? nleaf - t0 : 65535;
    hipLaunchKernelGGL(k_leaf_scale_U<R>, dim3(ceil_div(mL * k, 256), nt), dim3(256), 0, s,
                       Y + (long)t0 * mL * k, U, mL, k, b, kappa2, leaf_origin + t0, leaf_pts, n);
    LSH_LAUNCH_CHECK();
  }
}

// -------------------------------------------------------------- leaf apply
// One workgroup per leaf and group of up to NV right-hand sides: the leaf's
// X_tau and U_L are read once for the group. Each right-hand side gets the
// same arithmetic, in the same order, as in a one-vector launch.
constexpr int LEAF_MAX = 144;
constexpr int LEAF_NV = 4;

// Rows i < nrows of the row-major matrix A (nrows x ncols) times NV vectors
// in LDS (ins[v][0 .. ncols)); fn(i, v, sum) once per row and vector v < nv.
// Rows of at most 64 (the leaf matrices and U_L of leaves up to 8 x 8): 16
// lanes per row in four 16-wide chunks, four rows per wave at a time and
// four such row groups per wave with every load issued before the products
// (16 loads in flight per lane); a lane adds its chunks as (s0 + s1) +
// (s2 + s3), then a DPP butterfly over the row's 16 lanes.  Longer rows: one
// wave per row, LEAF_RU rows at a time, butterfly over the wave.  Each vector
// gets the same arithmetic in the same order for any NV.
constexpr int LEAF_RU = 4;
template <typename R, int NV, typename Fn>
__device__ __forceinline__ void leaf_rows(const cplx<R>* __restrict__ A, int nrows, int ncols,
                                          const cplx<R> (*ins)[LEAF_MAX], int nv, Fn fn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (ncols <= 64) {
    constexpr int L = 16, NCH = 4, RW = 64 / L, P = 4;
    const int sub = lane & (L - 1), rs = lane / L;
    for (int base = wave * RW; base < nrows; base += 4 * RW * P) {
      cplx<R> a[P][NCH];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int i = base + p * 4 * RW + rs;
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          const int c = sub + u * L;
          a[p][u] = (i < nrows && c < ncols) ? A[(long)i * ncols + c] : mk<R>(0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (v >= nv) break;  // (uniform)
        cplx<R> xin[NCH];
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          const int c = sub + u * L;
          xin[u] = c < ncols ? ins[v][c] : mk<R>(0, 0);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
          cplx<R> a4[NCH];
#pragma unroll
          for (int u = 0; u < NCH; ++u) {
            a4[u] = mk<R>(0, 0);
            fma_acc(a4[u], a[p][u], xin[u]);
          }
          cplx<R> t = (a4[0] + a4[1]) + (a4[2] + a4[3]);
          t.x = group_sum<L>(t.x);
          t.y = group_sum<L>(t.y);
          const int i = base + p * 4 * RW + rs;
          if (sub == 0 && i < nrows) fn(i, v, t);
        }
      }
    }
    return;
  }
  for (int i0 = wave; i0 < nrows; i0 += 4 * LEAF_RU) {
    cplx<R> acc[LEAF_RU][NV];
#pragma unroll
    for (int u = 0; u < LEAF_RU; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[u][v] = mk<R>(0, 0);
    for (int j = lane; j < ncols; j += 64) {
      cplx<R> xv[LEAF_RU];
#pragma unroll
      for (int u = 0; u < LEAF_RU; ++u) {
        const int i = i0 + 4 * u;
        xv[u] = i < nrows ? A[(long)i * ncols + j] : mk<R>(0, 0);
      }
#pragma unroll
      for (int u = 0; u < LEAF_RU; ++u)
#pragma unroll
        for (int v = 0; v < NV; ++v) fma_acc(acc[u][v], xv[u], ins[v][j]);
    }
#pragma unroll
    for (int u = 0; u < LEAF_RU; ++u) {
      const int i = i0 + 4 * u;
      if (i >= nrows) break;  // (uniform across the wave)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (v >= nv) break;
        cplx<R> a = acc[u][v];
        a.x = group_sum<64>(a.x);
        a.y = group_sum<64>(a.y);
        if (lane == 0) fn(i, v, a);
      }
    }
  }
}

// Up: r = X_tau f_tau ; rt = U_L^T r  (ULt: U_L transposed, k x mL)
template <typename R, int NV>
__global__ __launch_bounds__(256) void k_leaf_up(const cplx<R>* __restrict__ X, const cplx<R>* __restrict__ ULt,
                                                 int mL, int k, const z64* __restrict__ f, cplx<R>* r, cplx<R>* rt,
                                                 const I2* __restrict__ org, const I2* __restrict__ pts, int n,
                                                 int nleaf, int nrhs, const double* __restrict__ b, double sb) {
  __shared__ cplx<R> fs[NV][LEAF_MAX];
  __shared__ cplx<R> rs[NV][LEAF_MAX];
  const long t = blockIdx.x, r0 = (long)blockIdx.y * NV;
  const int nv = nrhs - r0 < NV ? (int)(nrhs - r0) : NV;
  const I2 o = org[t];
  for (int i = threadIdx.x; i < mL; i += blockDim.x) {
    const I2 pi = pts[i];
    const long at = (long)(o.y + pi.y) * n + (o.x + pi.x);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      z64 val = mk(0.0, 0.0);
      if (v < nv) val = f[(r0 + v) * (long)n * n + at];
      fs[v][i] = mk<R>((R)val.x, (R)val.y);
    }
  }
  __syncthreads();
  leaf_rows<R, NV>(X + t * (long)mL * mL, mL, mL, fs, nv, [&](int i, int v, cplx<R> acc) { rs[v][i] = acc; });
  __syncthreads();
  for (int v = 0; v < nv; ++v) {
    if (r) {
      cplx<R>* rr = r + ((r0 + v) * nleaf + t) * (long)mL;
      for (int i = threadIdx.x; i < mL; i += blockDim.x) rr[i] = rs[v][i];
    }
    if (b) {  // transpose pass: rs <- sb * b .* rs before U_L^T
      for (int i = threadIdx.x; i < mL; i += blockDim.x) {
        const I2 pi = pts[i];
        rs[v][i] = (R)(sb * b[(long)(o.y + pi.y) * n + (o.x + pi.x)]) * rs[v][i];
      }
    }
  }
  if (b) __syncthreads();
  leaf_rows<R, NV>(ULt, k, mL, rs, nv,
                   [&](int a, int v, cplx<R> acc) { rt[((r0 + v) * nleaf + t) * (long)k + a] = acc; });
}

template <typename R>
void leaf_up(hipStream_t s, const cplx<R>* X, const cplx<R>* ULt, int mL, int k, const z64* f, cplx<R>* r,
             cplx<R>* rt, const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n, int nrhs, const double* b,
             double sb) {
  LSH_REQUIRE(mL <= LEAF_MAX, -6, "leaf too large");
  const int ng = nrhs == 1 ? 1 : ceil_div(nrhs, LEAF_NV);
  ProfScope ps("leaf_up", s, (double)sizeof(cplx<R>) * nleaf * ((double)ng * mL * mL + (double)nrhs * (2.0 * mL + k)) +
                                 16.0 * nrhs * (double)nleaf * mL);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_leaf_up<R, 1>), dim3(nleaf, 1), dim3(256), 0, s, X, ULt, mL, k, f, r, rt, leaf_origin,
                       leaf_pts, n, nleaf, nrhs, b, sb);
  else
    hipLaunchKernelGGL((k_leaf_up<R, LEAF_NV>), dim3(nleaf, ng), dim3(256), 0, s, X, ULt, mL, k, f, r, rt,
                       leaf_origin, leaf_pts, n, nleaf, nrhs, b, sb);
  LSH_LAUNCH_CHECK();
}

// Down: q_tau = r_tau - X_tau B_tau U_L wt_tau, written to the grid (FP64)
template <typename R, int NV>
__global__ __launch_bounds__(256) void k_leaf_down(const cplx<R>* __restrict__ X, const cplx<R>* __restrict__ UL,
                                                   int mL, int k, const cplx<R>* __restrict__ wt,
                                                   const cplx<R>* __restrict__ r, z64* q,
                                                   const double* __restrict__ b, double kappa2,
                                                   const I2* __restrict__ org, const I2* __restrict__ pts, int n,
                                                   int nleaf, int nrhs) {
  __shared__ cplx<R> us[NV][LEAF_MAX];
  __shared__ cplx<R> ws[NV][LEAF_MAX];
  __shared__ cplx<R> rl[NV][LEAF_MAX];  // r, then the result (stored to the grid together at the end)
  const long t = blockIdx.x, r0 = (long)blockIdx.y * NV;
  const int nv = nrhs - r0 < NV ? (int)(nrhs - r0) : NV;
  const I2 o = org[t];
  for (int a = threadIdx.x; a < k; a += blockDim.x)
#pragma unroll
    for (int v = 0; v < NV; ++v) ws[v][a] = v < nv ? wt[((r0 + v) * nleaf + t) * (long)k + a] : mk<R>(0, 0);
  for (int v = 0; v < nv; ++v)
    for (int i = threadIdx.x; i < mL; i += blockDim.x) rl[v][i] = r[((r0 + v) * nleaf + t) * (long)mL + i];
  __syncthreads();
  leaf_rows<R, NV>(UL, mL, k, ws, nv, [&](int i, int v, cplx<R> acc) {
    const I2 pi = pts[i];
    us[v][i] = (R)(kappa2 * b[(long)(o.y + pi.y) * n + (o.x + pi.x)]) * acc;
  });
  __syncthreads();
  leaf_rows<R, NV>(X + t * (long)mL * mL, mL, mL, us, nv,
                   [&](int i, int v, cplx<R> acc) { rl[v][i] = rl[v][i] - acc; });
  __syncthreads();
  for (int v = 0; v < nv; ++v)
    for (int i = threadIdx.x; i < mL; i += blockDim.x) {
      const I2 pi = pts[i];
      const cplx<R> val = rl[v][i];
      q[(r0 + v) * (long)n * n + (long)(o.y + pi.y) * n + (o.x + pi.x)] = mk((double)val.x, (double)val.y);
    }
}

template <typename R>
void leaf_down(hipStream_t s, const cplx<R>* X, const cplx<R>* UL, int mL, int k, const cplx<R>* wt,
               const cplx<R>* r, z64* q, const double* b, double kappa2, const I2* leaf_origin, const I2* leaf_pts,
               int nleaf, int n, int nrhs) {
  LSH_REQUIRE(mL <= LEAF_MAX, -6, "leaf too large");
  const int ng = nrhs == 1 ? 1 : ceil_div(nrhs, LEAF_NV);
  ProfScope ps("leaf_down", s, (double)sizeof(cplx<R>) * nleaf * ((double)ng * mL * mL + (double)nrhs * (mL + k)) +
                                   (16.0 + 8.0) * nrhs * (double)nleaf * mL);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_leaf_down<R, 1>), dim3(nleaf, 1), dim3(256), 0, s, X, UL, mL, k, wt, r, q, b, kappa2,
                       leaf_origin, leaf_pts, n, nleaf, nrhs);
  else
    hipLaunchKernelGGL((k_leaf_down<R, LEAF_NV>), dim3(nleaf, ng), dim3(256), 0, s, X, UL, mL, k, wt, r, q, b,
                       kappa2, leaf_origin, leaf_pts, n, nleaf, nrhs);
  LSH_LAUNCH_CHECK();
}

// Transpose pass, leaves: q_tau = X_tau^T (g_tau + U_L rb_tau) (X given transposed)
template <typename R, int NV>
__global__ __launch_bounds__(256) void k_leaf_tdown(const cplx<R>* __restrict__ XT, const cplx<R>* __restrict__ UL,
                                                    int mL, int k, const cplx<R>* __restrict__ w,
                                                    const z64* __restrict__ g, z64* q, const I2* __restrict__ org,
                                                    const I2* __restrict__ pts, int n, int nleaf, int nrhs) {
  __shared__ cplx<R> us[NV][LEAF_MAX];
  __shared__ cplx<R> ws[NV][LEAF_MAX];
  const long t = blockIdx.x, r0 = (long)blockIdx.y * NV;
  const int nv = nrhs - r0 < NV ? (int)(nrhs - r0) : NV;
  const I2 o = org[t];
  for (int a = threadIdx.x; a < k; a += blockDim.x)
#pragma unroll
    for (int v = 0; v < NV; ++v) ws[v][a] = v < nv ? w[((r0 + v) * nleaf + t) * (long)k + a] : mk<R>(0, 0);
  __syncthreads();
  leaf_rows<R, NV>(UL, mL, k, ws, nv, [&](int i, int v, cplx<R> acc) {
    const I2 pi = pts[i];
    const z64 gv = g[(r0 + v) * (long)n * n + (long)(o.y + pi.y) * n + (o.x + pi.x)];
    us[v][i] = acc + mk<R>((R)gv.x, (R)gv.y);
  });
  __syncthreads();
  // (ws is free once us is built: it stages the results for one store pass)
  leaf_rows<R, NV>(XT + t * (long)mL * mL, mL, mL, us, nv, [&](int i, int v, cplx<R> acc) { ws[v][i] = acc; });
  __syncthreads();
  for (int v = 0; v < nv; ++v)
    for (int i = threadIdx.x; i < mL; i += blockDim.x) {
      const I2 pi = pts[i];
      const cplx<R> val = ws[v][i];
      q[(r0 + v) * (long)n * n + (long)(o.y + pi.y) * n + (o.x + pi.x)] = mk((double)val.x, (double)val.y);
    }
}

template <typename R>
void leaf_tdown(hipStream_t s, const cplx<R>* XT, const cplx<R>* UL, int mL, int k, const cplx<R>* w, const z64* g,
                z64* q, const I2* leaf_origin, const I2* leaf_pts, int nleaf, int n, int nrhs) {
  LSH_REQUIRE(mL <= LEAF_MAX, -6, "leaf too large");
  const int ng = nrhs == 1 ? 1 : ceil_div(nrhs, LEAF_NV);
  ProfScope ps("leaf_tdown", s, (double)sizeof(cplx<R>) * nleaf * ((double)ng * mL * mL + (double)nrhs * (mL + k)) +
                                    32.0 * nrhs * (double)nleaf * mL);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_leaf_tdown<R, 1>), dim3(nleaf, 1), dim3(256), 0, s, XT, UL, mL, k, w, g, q, leaf_origin,
                       leaf_pts, n, nleaf, nrhs);
  else
    hipLaunchKernelGGL((k_leaf_tdown<R, LEAF_NV>), dim3(nleaf, ng), dim3(256), 0, s, XT, UL, mL, k, w, g, q,
                       leaf_origin, leaf_pts, n, nleaf, nrhs);
  LSH_LAUNCH_CHECK();
}

// ------------------------------------------- apply, one Woodbury level fused
// Rows of one box product inside a workgroup of NT threads: out(i, sum_j
// A_i[j] x_i[j]) for i < M, j < N, with x_i in LDS.  16 lanes per row (lane s
// takes columns s + 16u of each 64-column chunk), P rows per 16-lane group at
// a time with every load issued before the products; column u of a chunk goes
// to partial sum u, then (s0 + s1) + (s2 + s3) and a DPP butterfly over the
// 16 lanes.  (The same arithmetic for any NT.)
template <typename R, int P, int NT, typename RowA, typename RowX, typename Out>
__device__ __forceinline__ void box_rows(int M, int N, RowA rowA, RowX rowX, Out out) {
  constexpr int NG = NT / 16;
  const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
  for (int i0 = grp * P; i0 < M; i0 += NG * P) {
    cplx<R> acc[P][4];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[p][u] = mk<R>(0, 0);
    for (int j0 = 0; j0 < N; j0 += 64) {
      cplx<R> a[P][4], x[P][4];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int i = i0 + p < M ? i0 + p : M - 1;
        const cplx<R>* ar = rowA(i);
        const cplx<R>* xr = rowX(i);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jj = j0 + sub + 16 * u;
          const bool ok = i0 + p < M && jj < N;
          a[p][u] = ok ? ar[jj] : mk<R>(0, 0);
          x[p][u] = ok ? xr[jj] : mk<R>(0, 0);
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int u = 0; u < 4; ++u) fma_acc(acc[p][u], a[p][u], x[p][u]);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      cplx<R> t = (acc[p][0] + acc[p][1]) + (acc[p][2] + acc[p][3]);
      t.x = group_sum<16>(t.x);
      t.y = group_sum<16>(t.y);
      if (sub == 0 && i0 + p < M) out(i0 + p, t);
    }
  }
}

// Up, one level (Algorithm 2's upward step on a Woodbury level): per box
// vector v (box v mod nb) with input [rt_a; rt_b] (2c),
//   q = [L^T rt_a; R^T rt_b], y = W'_b q, t = in - [S_a L y1; S_b R y2],
//   out_v = U_l^T t (k),
// every intermediate in LDS: one workgroup of NT threads per box vector.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_level_up(LevelApply<R> A, const cplx<R>* __restrict__ in,
                                                 cplx<R>* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char lvl_lds[];
  const int c = A.c, k = A.k, r = A.r;
  const long v = blockIdx.x;
  const long b = v % A.nb;
  cplx<R>* xs = reinterpret_cast<cplx<R>*>(lvl_lds);  // [2c]
  cplx<R>* q = xs + 2 * c;                             // [2r]
  cplx<R>* y = q + 2 * r;                              // [2r]
  cplx<R>* t = y + 2 * r;                              // [2c]
  const cplx<R>* iv = in + v * 2 * c;
  for (int i = threadIdx.x; i < 2 * c; i += NT) xs[i] = iv[i];
  __syncthreads();
  box_rows<R, 2, NT>(2 * r, c, [&](int i) { return A.Q + (long)i * c; },
                     [&](int i) { return i < r ? xs : xs + c; }, [&](int i, cplx<R> s) { q[i] = s; });
  __syncthreads();
  const cplx<R>* Wb = A.Ci + b * 4 * r * r;
  box_rows<R, 2, NT>(2 * r, 2 * r, [&](int i) { return Wb + (long)i * 2 * r; },
                     [&](int) { return (const cplx<R>*)q; }, [&](int i, cplx<R> s) { y[i] = s; });
  __syncthreads();
  const cplx<R>* Pb = A.Pa + b * 2 * c * r;  // [S_a L; S_b R] of the two children, rows contiguous
  box_rows<R, 2, NT>(2 * c, r, [&](int i) { return Pb + (long)i * r; }, [&](int i) { return i < c ? y : y + r; },
                     [&](int i, cplx<R> s) { t[i] = xs[i] - s; });
  __syncthreads();
  cplx<R>* ov = out + v * k;
  box_rows<R, 2, NT>(k, 2 * c, [&](int i) { return A.Ut + (long)i * 2 * c; },
                     [&](int) { return (const cplx<R>*)t; }, [&](int i, cplx<R> s) { ov[i] = s; });
}

// Down, one level: per box vector v with wt_v (k) and the children's rt (2c),
//   u = U_l wt_v, d = rt - diag(S_a, S_b) u, o = X_tau d (the Woodbury form
//   as above), wt_children = [G_ab o_b; G_ba o_a] + u,
// every intermediate in LDS.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_level_down(LevelApply<R> A, const cplx<R>* __restrict__ wt,
                                                   const cplx<R>* __restrict__ rtc, cplx<R>* __restrict__ wc) {
  extern __shared__ __align__(16) unsigned char lvl_lds[];
  const int c = A.c, k = A.k, r = A.r;
  const long v = blockIdx.x;
  const long b = v % A.nb;
  cplx<R>* w = reinterpret_cast<cplx<R>*>(lvl_lds);  // [k]
  cplx<R>* u = w + k;                                 // [2c]
  cplx<R>* d = u + 2 * c;                             // [2c]
  cplx<R>* q = d + 2 * c;                             // [2r]
  cplx<R>* y = q + 2 * r;                             // [2r]
  cplx<R>* o = y + 2 * r;                             // [2c]
  const cplx<R>* wv = wt + v * k;
  for (int i = threadIdx.x; i < k; i += NT) w[i] = wv[i];
  __syncthreads();
  box_rows<R, 2, NT>(2 * c, k, [&](int i) { return A.U + (long)i * k; }, [&](int) { return (const cplx<R>*)w; },
                     [&](int i, cplx<R> s) { u[i] = s; });
  __syncthreads();
  const cplx<R>* Sb = A.S + b * 2 * c * c;  // S_a, S_b of the two children, rows contiguous
  const cplx<R>* rv = rtc + v * 2 * c;
  box_rows<R, 2, NT>(2 * c, c, [&](int i) { return Sb + (long)i * c; }, [&](int i) { return i < c ? u : u + c; },
                     [&](int i, cplx<R> s) { d[i] = rv[i] - s; });
  __syncthreads();
  box_rows<R, 2, NT>(2 * r, c, [&](int i) { return A.Q + (long)i * c; }, [&](int i) { return i < r ? d : d + c; },
                     [&](int i, cplx<R> s) { q[i] = s; });
  __syncthreads();
  const cplx<R>* Wb = A.Ci + b * 4 * r * r;
  box_rows<R, 2, NT>(2 * r, 2 * r, [&](int i) { return Wb + (long)i * 2 * r; },
                     [&](int) { return (const cplx<R>*)q; }, [&](int i, cplx<R> s) { y[i] = s; });
  __syncthreads();
  const cplx<R>* Pb = A.Pa + b * 2 * c * r;
  box_rows<R, 2, NT>(2 * c, r, [&](int i) { return Pb + (long)i * r; }, [&](int i) { return i < c ? y : y + r; },
                     [&](int i, cplx<R> s) { o[i] = d[i] - s; });
  __syncthreads();
  cplx<R>* ov = wc + v * 2 * c;
  box_rows<R, 2, NT>(2 * c, c, [&](int i) { return i < c ? A.Gab + (long)i * c : A.Gba + (long)(i - c) * c; },
                     [&](int i) { return i < c ? o + c : o; }, [&](int i, cplx<R> s) { ov[i] = s + u[i]; });
}

// threads per box vector: about 8192 waves in all (few vectors: more lanes on
// each vector's rows)
static int level_threads(int nvec) { return nvec <= 512 ? 1024 : nvec <= 1024 ? 512 : 256; }

template <typename R>
static void level_check(const LevelApply<R>& A, int nvec) {
  LSH_REQUIRE(A.c > 0 && A.k > 0 && A.r > 0 && A.nb > 0 && nvec > 0 && nvec % A.nb == 0, -6,
              "fused level apply: bad sizes");
  LSH_REQUIRE((size_t)(A.k + 6 * A.c + 4 * A.r) * sizeof(cplx<R>) <= LEVEL_FUSED_LDS, -6,
              "fused level apply: the box vectors exceed the workgroup's LDS");
}

template <typename R>
void level_up_fused(hipStream_t s, const LevelApply<R>& A, const cplx<R>* in, cplx<R>* out, int nvec) {
  level_check(A, nvec);
  const double e = (double)sizeof(cplx<R>);
  ProfScope ps(sizeof(R) == 4 ? "level_up_f32" : "level_up_f64", s,
               e * ((double)A.nb * (4.0 * A.r * A.r + 2.0 * A.c * A.r) + 2.0 * A.r * A.c + 2.0 * A.c * A.k +
                    (double)nvec * (2.0 * A.c + A.k)));
  const size_t lds = (size_t)(4 * A.c + 4 * A.r) * sizeof(cplx<R>);
  const int nt = level_threads(nvec);
  if (nt == 1024) hipLaunchKernelGGL((k_level_up<R, 1024>), dim3(nvec), dim3(1024), lds, s, A, in, out);
  else if (nt == 512) hipLaunchKernelGGL((k_level_up<R, 512>), dim3(nvec), dim3(512), lds, s, A, in, out);
  else hipLaunchKernelGGL((k_level_up<R, 256>), dim3(nvec), dim3(256), lds, s, A, in, out);
  LSH_LAUNCH_CHECK();
}

template <typename R>
void level_down_fused(hipStream_t s, const LevelApply<R>& A, const cplx<R>* wt, const cplx<R>* rtc, cplx<R>* wc,
                      int nvec) {
  level_check(A, nvec);
  const double e = (double)sizeof(cplx<R>);
  ProfScope ps(sizeof(R) == 4 ? "level_down_f32" : "level_down_f64", s,
               e * ((double)A.nb * (2.0 * A.c * A.c + 4.0 * A.r * A.r + 2.0 * A.c * A.r) + 2.0 * A.c * A.k +
                    2.0 * A.r * A.c + 2.0 * A.c * A.c + (double)nvec * (A.k + 4.0 * A.c)));
  const size_t lds = (size_t)(A.k + 6 * A.c + 4 * A.r) * sizeof(cplx<R>);
  const int nt = level_threads(nvec);
  if (nt == 1024) hipLaunchKernelGGL((k_level_down<R, 1024>), dim3(nvec), dim3(1024), lds, s, A, wt, rtc, wc);
  else if (nt == 512) hipLaunchKernelGGL((k_level_down<R, 512>), dim3(nvec), dim3(512), lds, s, A, wt, rtc, wc);
  else hipLaunchKernelGGL((k_level_down<R, 256>), dim3(nvec), dim3(256), lds, s, A, wt, rtc, wc);
  LSH_LAUNCH_CHECK();
}

#define LSH_HBS_INST(R)                                                                                       \
  template void leaf_build<R>(hipStream_t, cplx<R>*, const cplx<R>*, int, const double*, double, const I2*,   \
                              const I2*, int, int);                                                          \
  template void leaf_scale_U<R>(hipStream_t, cplx<R>*, const cplx<R>*, int, int, const double*, double,       \
                                const I2*, const I2*, int, int);                                             \
  template void leaf_up<R>(hipStream_t, const cplx<R>*, const cplx<R>*, int, int, const z64*, cplx<R>*,        \
                           cplx<R>*, const I2*, const I2*, int, int, int, const double*, double);           \
  template void leaf_tdown<R>(hipStream_t, const cplx<R>*, const cplx<R>*, int, int, const cplx<R>*, const z64*,  \
                              z64*, const I2*, const I2*, int, int, int);                                    \
  template void leaf_down<R>(hipStream_t, const cplx<R>*, const cplx<R>*, int, int, const cplx<R>*,           \
                             const cplx<R>*, z64*, const double*, double, const I2*, const I2*, int, int, int);    \
  template void level_up_fused<R>(hipStream_t, const LevelApply<R>&, const cplx<R>*, cplx<R>*, int);            \
  template void level_down_fused<R>(hipStream_t, const LevelApply<R>&, const cplx<R>*, const cplx<R>*, cplx<R>*, \
                                    int);
LSH_HBS_INST(float)
LSH_HBS_INST(double)

}  // namespace lsh
