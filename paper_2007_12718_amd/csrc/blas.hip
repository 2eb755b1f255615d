// Batched complex GEMM / GEMV / Gauss-Jordan inverse for gfx950.
//
// Complex products run on the real matrix cores: each complex k-step is four
// real 16x16x4 MFMAs (Re += ArBr - AiBi, Im += ArBi + AiBr) on LDS-staged
// 64x64 tiles; four 64-wide wavefronts each own a 32x32 quarter of the tile.
#include "blas.hpp"
#include "prof.hpp"

namespace lsh {

template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  // accumulator register r of lane l holds D[4 * (l / 16) + r][l % 16]
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  // accumulator register r of lane l holds D[l / 16 + 4 * r][l % 16]
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename R>
struct GemmP {
  int M, N, K;
  cplx<R> alpha, beta;
  const cplx<R>* A;
  long lda, sA;
  int opA;
  const cplx<R>* B;
  long ldb, sB;
  int opB;
  const cplx<R>* D;
  long ldd, sD;
  cplx<R>* C;
  long ldc, sC;
  int addI;
};

// Tile: 2 x 2 wavefronts, each owning WM x WN blocks of 16 x 16 outputs, so the
// workgroup tile is (32 WM) x (32 WN); K advances 16 at a time.  LDS holds
// separate real / imaginary planes laid out [row][k] with stride 17, which
// keeps both the coalesced global->LDS stores and the MFMA operand reads
// (16 rows x 4 k per instruction) within one extra bank conflict.  The next
// K tile is prefetched into registers while the current one is multiplied.
constexpr int GBK = 16, GLD = GBK + 1;

template <typename R, int WM, int WN>
__global__ __launch_bounds__(256) void k_cgemm(GemmP<R> P) {
  using M4 = Mfma<R>;
  using acc_t = typename M4::acc_t;
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int EA = BM * GBK / 256, EB = BN * GBK / 256;
  __shared__ R sAr[BM][GLD], sAi[BM][GLD];
  __shared__ R sBr[BN][GLD], sBi[BN][GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long b = blockIdx.z;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const cplx<R>* A = P.A + b * P.sA;
  const cplx<R>* B = P.B + b * P.sB;
  const bool aN = (P.opA == OP_N || P.opA == OP_R), bN = (P.opB == OP_N || P.opB == OP_R);
  const bool aC = (P.opA == OP_C || P.opA == OP_R), bC = (P.opB == OP_C || P.opB == OP_R);
  acc_t cr[WM][WN], ci[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) { cr[i][j][r] = 0; ci[i][j][r] = 0; }
  cplx<R> ra[EA], rb[EB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (aN) { m = idx / GBK; k = idx % GBK; }
      else { k = idx / BM; m = idx % BM; }
      const int gm = m0 + m, gk = k0 + k;
      cplx<R> v = mk<R>(0, 0);
      if (gm < P.M && gk < P.K) v = aN ? A[(long)gm * P.lda + gk] : A[(long)gk * P.lda + gm];
      if (aC) v.y = -v.y;
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      int n, k;
      if (bN) { k = idx / BN; n = idx % BN; }
      else { n = idx / GBK; k = idx % GBK; }
      const int gn = n0 + n, gk = k0 + k;
      cplx<R> v = mk<R>(0, 0);
      if (gn < P.N && gk < P.K) v = bN ? B[(long)gk * P.ldb + gn] : B[(long)gn * P.ldb + gk];
      if (bC) v.y = -v.y;
      rb[e] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (aN) { m = idx / GBK; k = idx % GBK; }
      else { k = idx / BM; m = idx % BM; }
      sAr[m][k] = ra[e].x;
      sAi[m][k] = ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      int n, k;
      if (bN) { k = idx / BN; n = idx % BN; }
      else { n = idx / GBK; k = idx % GBK; }
      sBr[n][k] = rb[e].x;
      sBi[n][k] = rb[e].y;
    }
  };
  load(0);
  store();
  __syncthreads();
  for (int k0 = 0; k0 < P.K; k0 += GBK) {
    const bool more = k0 + GBK < P.K;
    if (more) load(k0 + GBK);
#pragma unroll
    for (int kk = 0; kk < GBK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      R ar[WM], ai[WM], br[WN], bi[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        ar[i] = sAr[wm * 16 * WM + i * 16 + (lane & 15)][k];
        ai[i] = sAi[wm * 16 * WM + i * 16 + (lane & 15)][k];
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        br[j] = sBr[wn * 16 * WN + j * 16 + (lane & 15)][k];
        bi[j] = sBi[wn * 16 * WN + j * 16 + (lane & 15)][k];
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          cr[i][j] = M4::op(ar[i], br[j], cr[i][j]);
          cr[i][j] = M4::op(-ai[i], bi[j], cr[i][j]);
          ci[i][j] = M4::op(ar[i], bi[j], ci[i][j]);
          ci[i][j] = M4::op(ai[i], br[j], ci[i][j]);
        }
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
  cplx<R>* C = P.C + b * P.sC;
  const cplx<R>* D = P.D ? P.D + b * P.sD : nullptr;
  const bool useD = D && (P.beta.x != R(0) || P.beta.y != R(0));
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 16 * WM + i * 16 + M4::row(lane, r);
        const int n = n0 + wn * 16 * WN + j * 16 + (lane & 15);
        if (m < P.M && n < P.N) {
          cplx<R> v = P.alpha * mk<R>(cr[i][j][r], ci[i][j][r]);
          if (useD) v = v + P.beta * D[(long)m * P.ldd + n];
          if (P.addI && m == n) v.x += R(1);
          C[(long)m * P.ldc + n] = v;
        }
      }
}

template <typename R, int WM, int WN>
static void launch_gemm(hipStream_t s, const GemmP<R>& P, const cplx<R>* A, const cplx<R>* B, const cplx<R>* D,
                        cplx<R>* C, long sA, long sB, long sD, long sC, int batch) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  for (int b0 = 0; b0 < batch; b0 += 65535) {
    int nb = batch - b0 < 65535 ? batch - b0 : 65535;
    GemmP<R> Q = P;
    Q.A = A + b0 * sA; Q.B = B + b0 * sB; Q.C = C + b0 * sC;
    if (D) Q.D = D + b0 * sD;
    dim3 grid(ceil_div(P.N, BN), ceil_div(P.M, BM), nb);
    hipLaunchKernelGGL((k_cgemm<R, WM, WN>), grid, dim3(256), 0, s, Q);
    LSH_LAUNCH_CHECK();
  }
}

template <typename R>
void cgemm(hipStream_t s, int M, int N, int K, cplx<R> alpha,
           const cplx<R>* A, long lda, long sA, Op opA,
           const cplx<R>* B, long ldb, long sB, Op opB,
           cplx<R> beta, const cplx<R>* D, long ldd, long sD,
           cplx<R>* C, long ldc, long sC, int batch, bool add_identity) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  ProfScope ps(sizeof(R) == 4 ? "cgemm_f32" : "cgemm_f64", s, 8.0 * M * N * K * (double)batch);
  GemmP<R> P;
  P.M = M; P.N = N; P.K = K; P.alpha = alpha; P.beta = beta;
  P.A = A; P.lda = lda; P.sA = sA; P.opA = opA;
  P.B = B; P.ldb = ldb; P.sB = sB; P.opB = opB;
  P.D = D; P.ldd = ldd; P.sD = sD;
  P.C = C; P.ldc = ldc; P.sC = sC; P.addI = add_identity ? 1 : 0;
  // large tiles when they still leave a few waves of workgroups in flight
  const double big_tiles = (double)ceil_div(M, 128) * ceil_div(N, sizeof(R) == 4 ? 128 : 64) * batch;
  if (M >= 128 && N >= 64 && K >= 32 && big_tiles >= 128) {
    if (sizeof(R) == 4) launch_gemm<R, 4, 4>(s, P, A, B, D, C, sA, sB, sD, sC, batch);
    else launch_gemm<R, 4, 2>(s, P, A, B, D, C, sA, sB, sD, sC, batch);
  } else {
    launch_gemm<R, 2, 2>(s, P, A, B, D, C, sA, sB, sD, sC, batch);
  }
}

// ---------------------------------------------------------------- GEMV
// One wavefront per row, lanes stride the row (coalesced); x_b staged in LDS.
constexpr int GV_ROWS = 16;

template <typename R>
__global__ __launch_bounds__(256) void k_cgemv(int M, int N, cplx<R> alpha,
                                               const cplx<R>* __restrict__ A, long lda, long sA, int amod,
                                               const cplx<R>* __restrict__ x, long sx, cplx<R> beta,
                                               const cplx<R>* z, long sz, cplx<R>* y, long sy) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* xs = reinterpret_cast<cplx<R>*>(smem_raw);
  const long b = blockIdx.x;  // problem index (unbounded grid dimension)
  const cplx<R>* Ab = A + (b % amod) * sA;
  const cplx<R>* xb = x + b * sx;
  for (int j = threadIdx.x; j < N; j += blockDim.x) xs[j] = xb[j];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int rr = 0; rr < GV_ROWS / 4; ++rr) {
    const int i = blockIdx.y * GV_ROWS + wave * (GV_ROWS / 4) + rr;
    if (i >= M) break;
    const cplx<R>* row = Ab + (long)i * lda;
    cplx<R> acc = mk<R>(0, 0);
    for (int j = lane; j < N; j += 64) fma_acc(acc, row[j], xs[j]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if (lane == 0) {
      cplx<R> v = alpha * acc;
      if (z && (beta.x != R(0) || beta.y != R(0))) v = v + beta * z[b * sz + i];
      y[b * sy + i] = v;
    }
  }
}

template <typename R>
void cgemv(hipStream_t s, int M, int N, cplx<R> alpha,
           const cplx<R>* A, long lda, long sA, int amod,
           const cplx<R>* x, long sx, cplx<R> beta, const cplx<R>* z, long sz,
           cplx<R>* y, long sy, int batch) {
  if (M <= 0 || batch <= 0) return;
  LSH_REQUIRE((size_t)N * sizeof(cplx<R>) <= 65536, -6, "cgemv: row length too large for LDS staging");
  // algorithmic bytes: every distinct matrix once, x, z and y once per problem
  const int nmat = amod < batch ? amod : batch;
  ProfScope ps(sizeof(R) == 4 ? "cgemv_f32" : "cgemv_f64", s,
               (double)sizeof(cplx<R>) * ((double)nmat * M * N + (double)batch * (N + (z ? 2.0 : 1.0) * M)));
  LSH_REQUIRE(ceil_div(M, GV_ROWS) <= 65535, -6, "cgemv: too many rows");
  dim3 grid(batch, ceil_div(M, GV_ROWS));
  hipLaunchKernelGGL(k_cgemv<R>, grid, dim3(256), N * sizeof(cplx<R>), s, M, N, alpha, A, lda, sA,
                     amod > 0 ? amod : 1, x, sx, beta, z, sz, y, sy);
  LSH_LAUNCH_CHECK();
}

// ------------------------------------------------ shared-matrix multi-GEMV
// One wavefront per row of Mat (lanes stride the row), up to MG_VEC vectors
// accumulated in registers; X is read through the caches by every wave.
constexpr int MG_VEC = 8;

template <typename R>
__global__ __launch_bounds__(256) void k_cmgemv(int Rr, int C, cplx<R> alpha, const cplx<R>* __restrict__ Mat,
                                                long ldm, const cplx<R>* __restrict__ X, long ldx, cplx<R> beta,
                                                const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + wave;
  if (i >= Rr) return;
  const cplx<R>* row = Mat + (long)i * ldm;
  for (int b0 = 0; b0 < nvec; b0 += MG_VEC) {
    const int nb = nvec - b0 < MG_VEC ? nvec - b0 : MG_VEC;
    cplx<R> acc[MG_VEC];
#pragma unroll
    for (int v = 0; v < MG_VEC; ++v) acc[v] = mk<R>(0, 0);
    for (int j = lane; j < C; j += 64) {
      const cplx<R> a = row[j];
#pragma unroll
      for (int v = 0; v < MG_VEC; ++v)
        if (v < nb) fma_acc(acc[v], a, X[(long)(b0 + v) * ldx + j]);
    }
#pragma unroll
    for (int v = 0; v < MG_VEC; ++v) {
      if (v >= nb) break;
      cplx<R> a = acc[v];
      for (int off = 32; off > 0; off >>= 1) {
        a.x += __shfl_xor(a.x, off);
        a.y += __shfl_xor(a.y, off);
      }
      if (lane == 0) {
        cplx<R> r = alpha * a;
        if (Z && (beta.x != R(0) || beta.y != R(0))) r = r + beta * Z[(long)(b0 + v) * ldz + i];
        Y[(long)(b0 + v) * ldy + i] = r;
      }
    }
  }
}

template <typename R>
void cmgemv(hipStream_t s, int Rr, int C, cplx<R> alpha, const cplx<R>* Mat, long ldm, const cplx<R>* X, long ldx,
            cplx<R> beta, const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec) {
  if (Rr <= 0 || nvec <= 0) return;
  ProfScope ps(sizeof(R) == 4 ? "cmgemv_f32" : "cmgemv_f64", s,
               (double)sizeof(cplx<R>) * ((double)Rr * C + (double)nvec * (C + (Z ? 2.0 : 1.0) * Rr)));
  hipLaunchKernelGGL(k_cmgemv<R>, dim3(ceil_div(Rr, 4)), dim3(256), 0, s, Rr, C, alpha, Mat, ldm, X, ldx, beta, Z,
                     ldz, Y, ldy, nvec);
  LSH_LAUNCH_CHECK();
}

// ------------------------------------------------- Gauss-Jordan inverse
// Small matrices: the whole matrix lives in LDS, one workgroup per matrix.
template <typename R>
__device__ void wave_argmax(R& v, int& idx) {
  for (int off = 32; off > 0; off >>= 1) {
    R ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_inv_small(cplx<R>* A, int c, long lda, long sA, int* info, int* permg) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* S = reinterpret_cast<cplx<R>*>(smem_raw);  // c*c
  __shared__ int s_piv;
  __shared__ int s_bad;
  const long b = blockIdx.x;
  cplx<R>* Ab = A + b * sA;
  int* perm = permg + b * c;  // row interchanges (global scratch, one row per matrix)
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < c * c; e += nt) S[e] = Ab[(long)(e / c) * lda + (e % c)];
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    if (tid < 64) {
      R best = -1;
      int bi = j;
      for (int i = j + tid; i < c; i += 64) {
        R a = abs2(S[i * c + j]);
        if (a > best || (a == best && i < bi)) { best = a; bi = i; }
      }
      wave_argmax(best, bi);
      if (tid == 0) {
        s_piv = bi;
        perm[j] = bi;
        if (!(best > R(0)) && !s_bad) s_bad = j + 1;
      }
    }
    __syncthreads();
    const int p = s_piv;
    if (p != j)
      for (int k = tid; k < c; k += nt) {
        cplx<R> t = S[j * c + k];
        S[j * c + k] = S[p * c + k];
        S[p * c + k] = t;
      }
    __syncthreads();
    const cplx<R> rp = crecip(S[j * c + j]);
    for (int k = tid; k < c; k += nt)
      if (k != j) S[j * c + k] = S[j * c + k] * rp;
    __syncthreads();
    // phase A: every entry outside row j and column j (column j is only read)
    for (int e = tid; e < c * c; e += nt) {
      const int i = e / c, k = e % c;
      if (i != j && k != j) S[e] = S[e] - S[i * c + j] * S[j * c + k];
    }
    __syncthreads();
    // phase B: column j becomes the elimination operator's column
    for (int i = tid; i < c; i += nt) S[i * c + j] = (i == j) ? rp : mk<R>(0, 0) - S[i * c + j] * rp;
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int j = c - 1; j >= 0; --j) {
    const int p = perm[j];
    if (p != j)
      for (int i = tid; i < c; i += nt) {
        cplx<R> t = S[i * c + j];
        S[i * c + j] = S[i * c + p];
        S[i * c + p] = t;
      }
    __syncthreads();
  }
  for (int e = tid; e < c * c; e += nt) Ab[(long)(e / c) * lda + (e % c)] = S[e];
  if (tid == 0 && info) info[b] = s_bad;
}

// Large matrices: blocked in-place Gauss-Jordan.  Per block K of NB columns:
//  1. k_gj_panel: one workgroup per matrix keeps the c x NB panel in
//     registers, chooses NB pivots by partial pivoting among the unused rows,
//     and applies the NB elementary Gauss-Jordan steps to the panel (which
//     ends up holding the K columns of the block's elimination operator E);
//  2. k_gj_swap: applies the row interchanges to the other columns, copies
//     rows K of the other columns to T (nb x c, zero in K) and writes
//     F = E(:,K) - I(:,K);
//  3. GEMM: A += F T  (updates every column outside K).
// At the end the row interchanges are undone as column interchanges.
constexpr int GJ_NB = 8, GJ_NT = 1024;

template <typename R, int RPT>
__global__ __launch_bounds__(GJ_NT) void k_gj_panel(cplx<R>* A, int c, long lda, long sA, int j0, int* perm,
                                                    int* info) {
  __shared__ cplx<R> prow[GJ_NB];
  __shared__ cplx<R> rowbuf[2][GJ_NB];
  __shared__ R wbest[GJ_NT / 64];
  __shared__ int widx[GJ_NT / 64];
  __shared__ int s_p;
  const long b = blockIdx.x;
  cplx<R>* Ab = A + b * sA;
  int* pb = perm + b * c;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = (c - j0) < GJ_NB ? (c - j0) : GJ_NB;
  cplx<R> P[RPT][GJ_NB];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * GJ_NT;
#pragma unroll
    for (int q = 0; q < GJ_NB; ++q)
      P[r][q] = (i < c && q < nb) ? Ab[(long)i * lda + j0 + q] : mk<R>(0, 0);
  }
  for (int jj = 0; jj < nb; ++jj) {
    const int j = j0 + jj;
    R best = -1;
    int bi = c;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * GJ_NT;
      if (i >= j && i < c) {
        cplx<R> v = P[r][0];
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q)
          if (q == jj) v = P[r][q];
        const R a = abs2(v);
        if (a > best || (a == best && i < bi)) { best = a; bi = i; }
      }
    }
    wave_argmax(best, bi);
    if (lane == 0) { wbest[wave] = best; widx[wave] = bi; }
    __syncthreads();
    if (tid < 64) {
      R bb = tid < GJ_NT / 64 ? wbest[tid] : R(-1);
      int ii = tid < GJ_NT / 64 ? widx[tid] : c;
      wave_argmax(bb, ii);
      if (tid == 0) {
        s_p = ii;
        pb[j] = ii;
        if (!(bb > R(0)) && info && info[b] == 0) info[b] = j + 1;
      }
    }
    __syncthreads();
    const int p = s_p;
    // publish rows j and p, then swap them
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * GJ_NT;
      if (i == j)
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q) rowbuf[0][q] = P[r][q];
      if (i == p)
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q) rowbuf[1][q] = P[r][q];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * GJ_NT;
      if (i == j && p != j)
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q) P[r][q] = rowbuf[1][q];
      if (i == p && p != j)
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q) P[r][q] = rowbuf[0][q];
    }
    if (tid < GJ_NB) prow[tid] = rowbuf[1][tid];  // the new row j
    __syncthreads();
    cplx<R> piv = prow[0];
#pragma unroll
    for (int q = 0; q < GJ_NB; ++q)
      if (q == jj) piv = prow[q];
    const cplx<R> rp = crecip(piv);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * GJ_NT;
      if (i >= c) continue;
      if (i == j) {
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q) P[r][q] = (q == jj) ? rp : prow[q] * rp;
      } else {
        cplx<R> f = P[r][0];
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q)
          if (q == jj) f = P[r][q];
        const cplx<R> fr = f * rp;
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q) P[r][q] = (q == jj) ? mk<R>(0, 0) - fr : P[r][q] - fr * prow[q];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * GJ_NT;
    if (i < c)
#pragma unroll
      for (int q = 0; q < GJ_NB; ++q)
        if (q < nb) Ab[(long)i * lda + j0 + q] = P[r][q];
  }
}

template <typename R>
__global__ void k_gj_swap(cplx<R>* A, int c, long lda, long sA, int j0, int nb, const int* perm,
                          cplx<R>* T, cplx<R>* F) {
  const long b = blockIdx.y;
  cplx<R>* Ab = A + b * sA;
  const int* pb = perm + b * c;
  cplx<R>* Tb = T + b * (long)GJ_NB * c;
  cplx<R>* Fb = F + b * (long)c * GJ_NB;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < c) {
    const bool inK = (k >= j0 && k < j0 + nb);
    if (!inK)
      for (int q = 0; q < nb; ++q) {
        const int j = j0 + q, p = pb[j];
        if (p != j) {
          cplx<R> t = Ab[(long)j * lda + k];
          Ab[(long)j * lda + k] = Ab[(long)p * lda + k];
          Ab[(long)p * lda + k] = t;
        }
      }
    for (int q = 0; q < GJ_NB; ++q)
      Tb[(long)q * c + k] = (!inK && q < nb) ? Ab[(long)(j0 + q) * lda + k] : mk<R>(0, 0);
    // F = panel - I(:,K), row k of F
    for (int q = 0; q < GJ_NB; ++q) {
      cplx<R> v = q < nb ? Ab[(long)k * lda + j0 + q] : mk<R>(0, 0);
      if (q < nb && k == j0 + q) v.x -= R(1);
      Fb[(long)k * GJ_NB + q] = v;
    }
  }
}

template <typename R>
__global__ void k_gj_colperm(cplx<R>* A, int c, long lda, long sA, const int* perm) {
  const long b = blockIdx.y;
  cplx<R>* Ab = A + b * sA;
  const int* pb = perm + b * c;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c) return;
  cplx<R>* row = Ab + (long)i * lda;
  for (int j = c - 1; j >= 0; --j) {
    const int p = pb[j];
    if (p != j) {
      cplx<R> t = row[j];
      row[j] = row[p];
      row[p] = t;
    }
  }
}

__global__ void k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename R>
static size_t small_inv_lds(int c) {
  return (size_t)c * c * sizeof(cplx<R>);
}

template <typename R>
size_t inverse_ws_bytes(int c, int batch) {
  if (small_inv_lds<R>(c) <= 65536) return (size_t)batch * c * sizeof(int) + 256;
  // perm (int c) + T (NB x c) + F (c x NB) per matrix
  return (size_t)batch * ((size_t)c * sizeof(int) + 2 * (size_t)GJ_NB * c * sizeof(cplx<R>)) + 256;
}

template <typename R>
void inverse(hipStream_t s, cplx<R>* A, int c, long lda, long sA, int batch, void* ws, int* info) {
  if (c <= 0 || batch <= 0) return;
  ProfScope ps(sizeof(R) == 4 ? "inverse_f32" : "inverse_f64", s, 8.0 * (double)c * c * c * batch);
  if (info) hipLaunchKernelGGL(k_zero_int, dim3(ceil_div(batch, 256)), dim3(256), 0, s, info, batch);
  const size_t lds = small_inv_lds<R>(c);
  if (lds <= 65536) {
    int* permg = static_cast<int*>(ws);
    hipLaunchKernelGGL(k_inv_small<R>, dim3(batch), dim3(256), lds, s, A, c, lda, sA, info, permg);
    LSH_LAUNCH_CHECK();
    return;
  }
  LSH_REQUIRE(c <= 4 * GJ_NT, -6, "inverse: matrix order above 4096 is not supported");
  LSH_REQUIRE(batch <= 65535, -6, "inverse: batch too large for the blocked path");
  int* perm = static_cast<int*>(ws);
  cplx<R>* T = reinterpret_cast<cplx<R>*>(static_cast<char*>(ws) +
                                          (((size_t)batch * c * sizeof(int) + 255) / 256) * 256);
  cplx<R>* F = T + (size_t)batch * GJ_NB * c;
  const int rpt = ceil_div(c, GJ_NT);
  for (int j0 = 0; j0 < c; j0 += GJ_NB) {
    const int nb = (c - j0) < GJ_NB ? (c - j0) : GJ_NB;
    switch (rpt) {
      case 1: hipLaunchKernelGGL((k_gj_panel<R, 1>), dim3(batch), dim3(GJ_NT), 0, s, A, c, lda, sA, j0, perm, info); break;
      case 2: hipLaunchKernelGGL((k_gj_panel<R, 2>), dim3(batch), dim3(GJ_NT), 0, s, A, c, lda, sA, j0, perm, info); break;
      case 3: hipLaunchKernelGGL((k_gj_panel<R, 3>), dim3(batch), dim3(GJ_NT), 0, s, A, c, lda, sA, j0, perm, info); break;
      default: hipLaunchKernelGGL((k_gj_panel<R, 4>), dim3(batch), dim3(GJ_NT), 0, s, A, c, lda, sA, j0, perm, info); break;
    }
    LSH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gj_swap<R>, dim3(ceil_div(c, 256), batch), dim3(256), 0, s, A, c, lda, sA, j0, nb, perm, T, F);
    LSH_LAUNCH_CHECK();
    cgemm<R>(s, c, c, GJ_NB, mk<R>(1, 0), F, GJ_NB, (long)c * GJ_NB, OP_N, T, c, (long)GJ_NB * c, OP_N,
             mk<R>(1, 0), A, lda, sA, A, lda, sA, batch);
  }
  hipLaunchKernelGGL(k_gj_colperm<R>, dim3(ceil_div(c, 256), batch), dim3(256), 0, s, A, c, lda, sA, perm);
  LSH_LAUNCH_CHECK();
}

template <typename R>
__global__ void k_ctranspose(const cplx<R>* in, int rows, int cols, cplx<R>* out, long batch) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long per = (long)rows * cols;
  if (e >= per * batch) return;
  const long bb = e / per, q = e % per;
  const int r = (int)(q / cols), c = (int)(q % cols);
  out[bb * per + (long)c * rows + r] = in[e];
}

template <typename R>
void ctranspose(hipStream_t s, const cplx<R>* in, int rows, int cols, cplx<R>* out, long batch) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(k_ctranspose<R>, dim3(ceil_div((long)rows * cols * batch, 256)), dim3(256), 0, s, in, rows,
                     cols, out, batch);
  LSH_LAUNCH_CHECK();
}

template <typename R1, typename R2>
__global__ void k_ccast(const cplx<R1>* src, cplx<R2>* dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = mk<R2>((R2)src[i].x, (R2)src[i].y);
}

template <typename R1, typename R2>
void ccast(hipStream_t s, const cplx<R1>* src, cplx<R2>* dst, long n) {
  if (n <= 0) return;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_ccast<R1, R2>), dim3(blocks), dim3(256), 0, s, src, dst, n);
  LSH_LAUNCH_CHECK();
}

#define LSH_INST(R)                                                                                        \
  template void cgemm<R>(hipStream_t, int, int, int, cplx<R>, const cplx<R>*, long, long, Op, const cplx<R>*, \
                         long, long, Op, cplx<R>, const cplx<R>*, long, long, cplx<R>*, long, long, int, bool); \
  template void cgemv<R>(hipStream_t, int, int, cplx<R>, const cplx<R>*, long, long, int, const cplx<R>*, long, \
                         cplx<R>, const cplx<R>*, long, cplx<R>*, long, int);                               \
  template void cmgemv<R>(hipStream_t, int, int, cplx<R>, const cplx<R>*, long, const cplx<R>*, long, cplx<R>, \
                          const cplx<R>*, long, cplx<R>*, long, int);                                        \
  template void ctranspose<R>(hipStream_t, const cplx<R>*, int, int, cplx<R>*, long);                       \
  template size_t inverse_ws_bytes<R>(int, int);                                                           \
  template void inverse<R>(hipStream_t, cplx<R>*, int, long, long, int, void*, int*);
LSH_INST(float)
LSH_INST(double)
template void ccast<double, float>(hipStream_t, const cplx<double>*, cplx<float>*, long);
template void ccast<float, double>(hipStream_t, const cplx<float>*, cplx<double>*, long);
template void ccast<double, double>(hipStream_t, const cplx<double>*, cplx<double>*, long);

}  // namespace lsh
