// Batched complex GEMM / GEMV / Gauss-Jordan inverse for gfx950.
//
// Complex products run on the real matrix cores: each complex k-step is four
// real 16x16x4 MFMAs (Re += ArBr - AiBi, Im += ArBi + AiBr) on LDS-staged
// 64x64 tiles; four 64-wide wavefronts each own a 32x32 quarter of the tile.
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <tuple>

#include "blas.hpp"
#include "wave.hpp"
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
  const int* skip;  // optional device flag: the whole launch is a no-op when *skip != 0
  int lower;        // 1: only tiles that reach the diagonal or below it (M == N)
  // split K (k_cgemm_x32_splitk): partial products [batch][nsplit][M][N],
  // chunks of kchunk along K
  cplx<R>* part = nullptr;
  int nsplit = 1, kchunk = 0;
};

// Tile: 2 x 2 wavefronts, each owning WM x WN blocks of 16 x 16 outputs, so the
// workgroup tile is (32 WM) x (32 WN); K advances GBK (16 or 32) at a time.  LDS holds
// separate real / imaginary planes laid out [row][k] with stride 17, which
// keeps both the coalesced global->LDS stores and the MFMA operand reads
// (16 rows x 4 k per instruction) within one extra bank conflict.  The next
// K tile is prefetched into registers while the current one is multiplied.

template <typename R, int WM, int WN, int GBK = 16>
__global__ __launch_bounds__(256) void k_cgemm(GemmP<R> P) {
  constexpr int GLD = GBK + 1;
  using M4 = Mfma<R>;
  using acc_t = typename M4::acc_t;
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int EA = BM * GBK / 256, EB = BN * GBK / 256;
  if (P.skip && *P.skip) return;  // uniform across the launch
  __shared__ R sAr[BM][GLD], sAi[BM][GLD];
  __shared__ R sBr[BN][GLD], sBi[BN][GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
  // renumber them to give each XCD a contiguous run of tiles (neighbouring
  // tiles share A rows / B columns in that XCD's L2).
  const long T = (long)gridDim.x * gridDim.y * gridDim.z;
  long L = blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z);
  const long T8 = (T / 8) * 8;
  // (lower-triangle mode keeps round-robin order: contiguous row bands per
  // XCD would leave the bottom band with nearly all the work)
  if (L < T8 && !P.lower) L = (L % 8) * (T / 8) + L / 8;
  const int tn = (int)(L % gridDim.x);
  const int tm = (int)((L / gridDim.x) % gridDim.y);
  const long b = L / ((long)gridDim.x * gridDim.y);
  const int m0 = tm * BM, n0 = tn * BN;
  if (P.lower && n0 >= m0 + BM) return;  // strictly above the diagonal
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
      sAi[m][k] = aC ? -ra[e].y : ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      int n, k;
      if (bN) { k = idx / BN; n = idx % BN; }
      else { n = idx / GBK; k = idx % GBK; }
      sBr[n][k] = rb[e].x;
      sBi[n][k] = bC ? -rb[e].y : rb[e].y;
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

// FP32 variant on the 32x32x2 matrix instruction (the higher-throughput FP32
// shape), three real products per complex step (Gauss's form, 25 % fewer
// matrix instructions; the imaginary part is a difference of products, which
// stays within FP32 rounding of |A||B| sums): 2 x 2 wavefronts, each owning
// WM x WN blocks of 32 x 32 outputs, so
// the workgroup tile is (64 WM) x (64 WN), K advancing BK (a multiple of 32)
// per LDS tile.  The sum over k inside one instruction does not care which k
// each lane group supplies, so in each 32-deep chunk lane group g (lanes
// 32g .. 32g+31) takes k = 16g + s at step s: each lane then reads its
// operands for four steps with one 16-byte LDS load per plane.  Row stride
// BK + 4 floats keeps those loads free of bank conflicts.  Every tile shape
// and depth issues the same instructions per output in the same order.
// Accumulator register r of lane l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
constexpr int X32_BK = 32;  // K depth of the split-K chunks' tiles

// One (64 WM) x (64 WN) output tile of problem b of P, at (m0, n0), K
// advancing BK per LDS tile.
template <int WM, int WN, int BK = 32>
__device__ __forceinline__ void cgemm_x32_tile(const GemmP<float>& P, long b, int m0, int n0) {
  typedef float f16v __attribute__((ext_vector_type(16)));
  typedef float f4v __attribute__((ext_vector_type(4)));
  constexpr int BM = 64 * WM, BN = 64 * WN, LDK = BK + 4;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  __shared__ __align__(16) float sAr[BM][LDK], sAi[BM][LDK];
  __shared__ __align__(16) float sBr[BN][LDK], sBi[BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int g = lane >> 5, l32 = lane & 31;
  const cplx<float>* A = P.A + b * P.sA;
  const cplx<float>* B = P.B + b * P.sB;
  const bool aN = (P.opA == OP_N || P.opA == OP_R), bN = (P.opB == OP_N || P.opB == OP_R);
  const bool aC = (P.opA == OP_C || P.opA == OP_R), bC = (P.opB == OP_C || P.opB == OP_R);
  // three real products per complex step (Gauss): t1 = Ar Br, t2 = Ai Bi,
  // t3 = (Ar + Ai)(Br + Bi); Re = t1 - t2, Im = t3 - t1 - t2
  f16v t1[WM][WN], t2[WM][WN], t3[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) { t1[i][j][r] = 0; t2[i][j][r] = 0; t3[i][j][r] = 0; }
  cplx<float> ra[EA], rb[EB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (aN) { m = idx / BK; k = idx % BK; }
      else { k = idx / BM; m = idx % BM; }
      const int gm = m0 + m, gk = k0 + k;
      cplx<float> v = mk<float>(0, 0);
      if (gm < P.M && gk < P.K) v = aN ? A[(long)gm * P.lda + gk] : A[(long)gk * P.lda + gm];
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      int n, k;
      if (bN) { k = idx / BN; n = idx % BN; }
      else { n = idx / BK; k = idx % BK; }
      const int gn = n0 + n, gk = k0 + k;
      cplx<float> v = mk<float>(0, 0);
      if (gn < P.N && gk < P.K) v = bN ? B[(long)gk * P.ldb + gn] : B[(long)gn * P.ldb + gk];
      rb[e] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (aN) { m = idx / BK; k = idx % BK; }
      else { k = idx / BM; m = idx % BM; }
      sAr[m][k] = ra[e].x;
      sAi[m][k] = aC ? -ra[e].y : ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * 256;
      int n, k;
      if (bN) { k = idx / BN; n = idx % BN; }
      else { n = idx / BK; k = idx % BK; }
      sBr[n][k] = rb[e].x;
      sBi[n][k] = bC ? -rb[e].y : rb[e].y;
    }
  };
  load(0);
  store();
  __syncthreads();
  for (int k0 = 0; k0 < P.K; k0 += BK) {
    const bool more = k0 + BK < P.K;
    if (more) load(k0 + BK);
#pragma unroll
    for (int h = 0; h < BK / 8; ++h) {  // groups of four k steps
      f4v ar[WM], ai[WM], as[WM], br[WN], bi[WN], bs[WN];
      // within each 32-deep chunk lane group g takes k = 16 g + 4 (h % 4) + step:
      // every BK adds the same products in the same order (the same bits)
      const int kq = 32 * (h >> 2) + 16 * g + 4 * (h & 3);
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int row = wm * 32 * WM + i * 32 + l32;
        ar[i] = *reinterpret_cast<const f4v*>(&sAr[row][kq]);
        ai[i] = *reinterpret_cast<const f4v*>(&sAi[row][kq]);
        as[i] = ar[i] + ai[i];
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int col = wn * 32 * WN + j * 32 + l32;
        br[j] = *reinterpret_cast<const f4v*>(&sBr[col][kq]);
        bi[j] = *reinterpret_cast<const f4v*>(&sBi[col][kq]);
        bs[j] = br[j] + bi[j];
      }
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i][st], br[j][st], t1[i][j], 0, 0, 0);
            t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i][st], bi[j][st], t2[i][j], 0, 0, 0);
            t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[i][st], bs[j][st], t3[i][j], 0, 0, 0);
          }
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
  cplx<float>* C = P.C + b * P.sC;
  const cplx<float>* D = P.D ? P.D + b * P.sD : nullptr;
  const bool useD = D && (P.beta.x != 0.f || P.beta.y != 0.f);
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 * WM + i * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
        const int n = n0 + wn * 32 * WN + j * 32 + l32;
        if (m < P.M && n < P.N) {
          const float re = t1[i][j][r] - t2[i][j][r], im = t3[i][j][r] - t1[i][j][r] - t2[i][j][r];
          cplx<float> v = P.alpha * mk<float>(re, im);
          if (useD) v = v + P.beta * D[(long)m * P.ldd + n];
          if (P.addI && m == n) v.x += 1.f;
          C[(long)m * P.ldc + n] = v;
        }
      }
}

template <int WM, int WN, int BK>
__global__ __launch_bounds__(256, (WM * WN >= 4 ? 1 : 2)) void k_cgemm_x32(GemmP<float> P) {
  constexpr int BM = 64 * WM, BN = 64 * WN;
  if (P.skip && *P.skip) return;  // uniform across the launch
  // XCD-aware tile order (see k_cgemm)
  const long T = (long)gridDim.x * gridDim.y * gridDim.z;
  long L = blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z);
  const long T8 = (T / 8) * 8;
  if (L < T8 && !P.lower) L = (L % 8) * (T / 8) + L / 8;
  const int tn = (int)(L % gridDim.x);
  const int tm = (int)((L / gridDim.x) % gridDim.y);
  const long b = L / ((long)gridDim.x * gridDim.y);
  if (P.lower && tn * BN >= (tm + 1) * BM) return;  // strictly above the diagonal
  cgemm_x32_tile<WM, WN, BK>(P, b, tm * BM, tn * BN);
}

// Split K (64 x 64 tiles, XCD-aware order as above): grid z runs over
// (problem, K chunk); chunk ks of problem b writes its partial product to
// part + (b nsplit + ks) M N.
__global__ __launch_bounds__(256, 2) void k_cgemm_x32_splitk(GemmP<float> P) {
  const long T = (long)gridDim.x * gridDim.y * gridDim.z;
  long L = blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z);
  const long T8 = (T / 8) * 8;
  if (L < T8) L = (L % 8) * (T / 8) + L / 8;
  const int tn = (int)(L % gridDim.x);
  const int tm = (int)((L / gridDim.x) % gridDim.y);
  const long b = L / ((long)gridDim.x * gridDim.y);
  const int ks = (int)(b % P.nsplit);
  const long bb = b / P.nsplit;
  const long k0 = (long)ks * P.kchunk;
  const bool aN = (P.opA == OP_N || P.opA == OP_R), bN = (P.opB == OP_N || P.opB == OP_R);
  GemmP<float> Q = P;
  Q.A = P.A + (aN ? k0 : k0 * P.lda);
  Q.B = P.B + (bN ? k0 * P.ldb : k0);
  Q.K = (int)(P.K - k0 < P.kchunk ? P.K - k0 : P.kchunk);
  Q.C = P.part + b * (long)P.M * P.N;
  Q.ldc = P.N;
  Q.sC = 0;
  Q.D = nullptr;
  Q.beta = mk<float>(0, 0);
  Q.addI = 0;
  cgemm_x32_tile<1, 1>(Q, bb, tm * 64, tn * 64);
}

// C = sum of the nsplit partial products + beta D (+ I)
template <typename R>
__global__ __launch_bounds__(256) void k_splitk_reduce(const cplx<R>* __restrict__ part, int nsplit, int M, int N,
                                                       long total, cplx<R> beta, const cplx<R>* D, long ldd, long sD,
                                                       cplx<R>* C, long ldc, long sC, int addI) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const long mn = (long)M * N;
  const long b = e / mn, r = e - b * mn;
  const int m = (int)(r / N), n = (int)(r - (long)m * N);
  const cplx<R>* p = part + b * nsplit * mn + r;
  cplx<R> v = p[0];
  for (int ks = 1; ks < nsplit; ++ks) v = v + p[ks * mn];
  if (D && (beta.x != R(0) || beta.y != R(0))) v = v + beta * D[b * sD + (long)m * ldd + n];
  if (addI && m == n) v.x += R(1);
  C[b * sC + (long)m * ldc + n] = v;
}

// Grouped form: problem g of the table has tiles_m x tiles_n x batch tiles
// starting at flat tile index tile0; one workgroup per tile of every problem.
struct GemmGroupDev {
  GemmP<float> p;
  int batch, tiles_m, tiles_n;
  long tile0;
};

__global__ __launch_bounds__(256, 4) void k_cgemm_x32_grouped(const GemmGroupDev* G, int ng) {
  const long L = blockIdx.x + (long)gridDim.x * blockIdx.y;
  int lo = 0, hi = ng - 1;  // last group with tile0 <= L
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (G[mid].tile0 <= L) lo = mid;
    else hi = mid - 1;
  }
  const GemmGroupDev& gd = G[lo];
  const long t = L - gd.tile0;
  if (t >= (long)gd.tiles_m * gd.tiles_n * gd.batch) return;
  const int tn = (int)(t % gd.tiles_n);
  const int tm = (int)((t / gd.tiles_n) % gd.tiles_m);
  const long b = t / ((long)gd.tiles_n * gd.tiles_m);
  cgemm_x32_tile<1, 1>(gd.p, b, tm * 64, tn * 64);
}

template <int WM, int WN, int BK>
static void launch_gemm_x32(hipStream_t s, const GemmP<float>& P, const cplx<float>* A, const cplx<float>* B,
                            const cplx<float>* D, cplx<float>* C, long sA, long sB, long sD, long sC, int batch,
                            const char* name) {
  constexpr int BM = 64 * WM, BN = 64 * WN;
  for (int b0 = 0; b0 < batch; b0 += 65535) {
    int nb = batch - b0 < 65535 ? batch - b0 : 65535;
    // algorithmic bytes: each distinct operand once, the result (and D) once per problem
    const double bytes = 8.0 * ((double)P.M * P.K * (sA ? nb : 1) + (double)P.K * P.N * (sB ? nb : 1) +
                                (double)P.M * P.N * nb * (D ? 2 : 1));
    ProfScope ps(name, s, 8.0 * P.M * P.N * P.K * (double)nb, bytes);
    GemmP<float> Q = P;
    Q.A = A + b0 * sA; Q.B = B + b0 * sB; Q.C = C + b0 * sC;
    if (D) Q.D = D + b0 * sD;
    dim3 grid(ceil_div(P.N, BN), ceil_div(P.M, BM), nb);
    hipLaunchKernelGGL((k_cgemm_x32<WM, WN, BK>), grid, dim3(256), 0, s, Q);
    LSH_LAUNCH_CHECK();
  }
}

template <typename R, int WM, int WN, int BK = 16>
static void launch_gemm(hipStream_t s, const GemmP<R>& P, const cplx<R>* A, const cplx<R>* B, const cplx<R>* D,
                        cplx<R>* C, long sA, long sB, long sD, long sC, int batch) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  const char* name = sizeof(R) == 4 ? (BM == 128 ? "cgemm_f32_128x128" : "cgemm_f32_64x64")
                                    : (BM == 128 ? "cgemm_f64_128x64" : BK == 32 ? "cgemm_f64_64x64k32"
                                                                                 : "cgemm_f64_64x64");
  for (int b0 = 0; b0 < batch; b0 += 65535) {
    int nb = batch - b0 < 65535 ? batch - b0 : 65535;
    // algorithmic bytes: each distinct operand once, the result (and D) once per problem
    const double e = sizeof(cplx<R>);
    const double bytes = e * ((double)P.M * P.K * (sA ? nb : 1) + (double)P.K * P.N * (sB ? nb : 1) +
                              (double)P.M * P.N * nb * (D ? 2 : 1));
    ProfScope ps(name, s, 8.0 * P.M * P.N * P.K * (double)nb, bytes);
    GemmP<R> Q = P;
    Q.A = A + b0 * sA; Q.B = B + b0 * sB; Q.C = C + b0 * sC;
    if (D) Q.D = D + b0 * sD;
    dim3 grid(ceil_div(P.N, BN), ceil_div(P.M, BM), nb);
    hipLaunchKernelGGL((k_cgemm<R, WM, WN, BK>), grid, dim3(256), 0, s, Q);
    LSH_LAUNCH_CHECK();
  }
}

// ---- GEMM variants and their choice
//
// FP32: tile (64 WM) x (64 WN) with K depth BK.  FP64: 64 x 64 (16 or 32 deep) or 128 x 64.
// All variants of one precision add the same products in the same order, so
// the choice changes the time, never the bits.
struct GemmVariant { int wm, wn, bk; const char* name; };
static const GemmVariant kF32Variants[] = {
    {1, 1, 32, "cgemm_f32_64x64"},   {2, 1, 32, "cgemm_f32_128x64"},    {2, 2, 32, "cgemm_f32_128x128"},
    {1, 1, 64, "cgemm_f32_64x64k64"}, {2, 1, 64, "cgemm_f32_128x64k64"}, {1, 2, 32, "cgemm_f32_64x128"}};
static const GemmVariant kF64Variants[] = {
    {2, 2, 16, "cgemm_f64_64x64"}, {4, 2, 16, "cgemm_f64_128x64"}, {2, 2, 32, "cgemm_f64_64x64k32"}};
constexpr int kNumF32Variants = sizeof(kF32Variants) / sizeof(kF32Variants[0]);
constexpr int kNumF64Variants = sizeof(kF64Variants) / sizeof(kF64Variants[0]);

int gemm_variant_count(int prec) { return prec == 1 ? kNumF32Variants : kNumF64Variants; }
const char* gemm_variant_name(int prec, int v) {
  return prec == 1 ? kF32Variants[v].name : kF64Variants[v].name;
}

// Without a tuned entry: a wave-quantisation model for FP32 (a launch takes
// ceil(tiles / (256 CUs x resident workgroups per CU)) rounds, and a full
// round costs (resident workgroups x tile area) / (per-CU efficiency of that
// tile)), and the 32-deep 64 x 64 tile for FP64 (47-50 TF/s alone on the
// plan's Gram and interpolation shapes, against 45-48 with 16-deep and 23-42
// with 128 x 64 tiles).
struct TileModel { int variant, bm, bn, resident; double eff; };
static const TileModel kF32Model[2] = {{1, 128, 64, 2, 0.60}, {0, 64, 64, 4, 0.69}};

static int model_variant(int prec, int M, int N, int batch) {
  if (prec != 1) return 2;
  int best = 0;
  double bt = 1e300;
  for (const TileModel& tm : kF32Model) {
    const double tiles = (double)ceil_div(M, tm.bm) * ceil_div(N, tm.bn) * batch;
    const double rounds = std::ceil(tiles / (256.0 * tm.resident));
    const double cost = rounds * tm.resident * tm.bm * tm.bn / tm.eff;
    if (cost < bt * 0.999) { bt = cost; best = tm.variant; }
  }
  return best;
}

// Tuned choices, keyed by precision and the half-octave buckets of M, N, K
// and the batch (lsh_gemm_tune fills it; lsh_gemm_table_load reads a file).
namespace {
struct TuneKey {
  int prec, m, n, k, b;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, m, n, k, b) < std::tie(o.prec, o.m, o.n, o.k, o.b);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
thread_local int g_forced_variant = -1;  // (the tuner's timing runs)
bool g_record = false;
std::map<std::array<int, 5>, int> g_recorded;  // shape -> number of products

int half_octave(long x) { return x <= 1 ? 0 : (int)std::lround(2.0 * std::log2((double)x)); }
TuneKey tune_key(int prec, int M, int N, int K, int batch) {
  return {prec, half_octave(M), half_octave(N), half_octave(K), half_octave(batch)};
}
}  // namespace

static int choose_variant(int prec, int M, int N, int K, int batch) {
  if (g_forced_variant >= 0) return g_forced_variant;
  static const int env = [] {
    const char* e = getenv("LSH_GEMM_VARIANT");
    return e ? atoi(e) : -1;
  }();
  const int nv = gemm_variant_count(prec);
  if (env >= 0 && env < nv) return env;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (g_record) ++g_recorded[{prec, M, N, K, batch}];
    auto it = g_tune.find(tune_key(prec, M, N, K, batch));
    if (it != g_tune.end() && it->second < nv) return it->second;
  }
  return model_variant(prec, M, N, batch);
}

void gemm_force_variant(int v) { g_forced_variant = v; }

void gemm_tune_set(int prec, int M, int N, int K, int batch, int v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[tune_key(prec, M, N, K, batch)] = v;
}

void gemm_table_clear() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
}

// Text file, one entry per line: prec m n k batch (bucket indices) variant.
void gemm_table_save(const char* path) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  LSH_REQUIRE(f, -1, std::string("gemm table: cannot open ") + path);
  std::fprintf(f, "# prec(0 FP64, 1 FP32) M N K batch (half-octave buckets, round(2 log2 x)) variant name\n");
  for (auto& kv : g_tune)
    std::fprintf(f, "%d %d %d %d %d %d %s\n", kv.first.prec, kv.first.m, kv.first.n, kv.first.k, kv.first.b,
                 kv.second, gemm_variant_name(kv.first.prec, kv.second));
  std::fclose(f);
}

int gemm_table_load(const char* path) {
  FILE* f = std::fopen(path, "r");
  LSH_REQUIRE(f, -1, std::string("gemm table: cannot open ") + path);
  char line[256];
  int n = 0;
  std::lock_guard<std::mutex> g(g_tune_mu);
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    TuneKey k;
    int v;
    if (std::sscanf(line, "%d %d %d %d %d %d", &k.prec, &k.m, &k.n, &k.k, &k.b, &v) == 6 && (k.prec == 0 || k.prec == 1) &&
        v >= 0 && v < gemm_variant_count(k.prec)) {
      g_tune[k] = v;
      ++n;
    }
  }
  std::fclose(f);
  return n;
}

void gemm_record(bool on) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_record = on;
  if (on) g_recorded.clear();
}

std::vector<std::array<int, 6>> gemm_recorded() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::vector<std::array<int, 6>> v;
  for (auto& kv : g_recorded) v.push_back({kv.first[0], kv.first[1], kv.first[2], kv.first[3], kv.first[4], kv.second});
  return v;
}

template <typename R>
void cgemm(hipStream_t s, int M, int N, int K, cplx<R> alpha,
           const cplx<R>* A, long lda, long sA, Op opA,
           const cplx<R>* B, long ldb, long sB, Op opB,
           cplx<R> beta, const cplx<R>* D, long ldd, long sD,
           cplx<R>* C, long ldc, long sC, int batch, bool add_identity, const int* skip, bool lower) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  LSH_REQUIRE(!lower || M == N, -1, "cgemm: lower-triangle mode needs a square result");
  GemmP<R> P;
  P.skip = skip;
  P.lower = lower ? 1 : 0;
  P.M = M; P.N = N; P.K = K; P.alpha = alpha; P.beta = beta;
  P.A = A; P.lda = lda; P.sA = sA; P.opA = opA;
  P.B = B; P.ldb = ldb; P.sB = sB; P.opB = opB;
  P.D = D; P.ldd = ldd; P.sD = sD;
  P.C = C; P.ldc = ldc; P.sC = sC; P.addI = add_identity ? 1 : 0;
  if constexpr (sizeof(R) == 4) {
    const int v = lower ? 0 : choose_variant(1, M, N, K, batch);
    const char* nm = kF32Variants[v].name;
    switch (v) {
      case 1: launch_gemm_x32<2, 1, 32>(s, P, A, B, D, C, sA, sB, sD, sC, batch, nm); break;
      case 2: launch_gemm_x32<2, 2, 32>(s, P, A, B, D, C, sA, sB, sD, sC, batch, nm); break;
      case 3: launch_gemm_x32<1, 1, 64>(s, P, A, B, D, C, sA, sB, sD, sC, batch, nm); break;
      case 4: launch_gemm_x32<2, 1, 64>(s, P, A, B, D, C, sA, sB, sD, sC, batch, nm); break;
      case 5: launch_gemm_x32<1, 2, 32>(s, P, A, B, D, C, sA, sB, sD, sC, batch, nm); break;
      default: launch_gemm_x32<1, 1, 32>(s, P, A, B, D, C, sA, sB, sD, sC, batch, nm); break;
    }
  } else {
    // (Hermitian Grams in lower mode: the 32-deep 64 x 64 tile, fastest on every measured shape)
    const int v = lower ? 2 : choose_variant(0, M, N, K, batch);
    if (v == 1) launch_gemm<R, 4, 2>(s, P, A, B, D, C, sA, sB, sD, sC, batch);
    else if (v == 2) launch_gemm<R, 2, 2, 32>(s, P, A, B, D, C, sA, sB, sD, sC, batch);
    else launch_gemm<R, 2, 2>(s, P, A, B, D, C, sA, sB, sD, sC, batch);
  }
}

// Products with too few output tiles to fill the device (shared box
// matrices: a few hundred boxes times a few hundred rows at the upper
// levels, thousands of boxes times a few dozen rows at the lower ones)
// split K over workgroups into ws, then sum the partial tiles.
// (fourier-1024, one FP32 apply: 3.38 ms without the 32 < K < 128 and 128..255-tile splits, 3.19 ms with them)
constexpr long SPLIT_TILES = 256;  // split below this many 64 x 64 output tiles
constexpr long SPLIT_WG = 512;     // aim for about this many workgroups
constexpr int SPLIT_KMIN = 32;     // at least one K tile per chunk

template <typename R>
void cgemm_ws(hipStream_t s, int M, int N, int K, cplx<R> alpha, const cplx<R>* A, long lda, long sA, Op opA,
              const cplx<R>* B, long ldb, long sB, Op opB, cplx<R> beta, const cplx<R>* D, long ldd, long sD,
              cplx<R>* C, long ldc, long sC, int batch, void* ws, size_t ws_bytes) {
  if constexpr (sizeof(R) == 4) {
    const long tiles = (long)ceil_div(M, 64) * ceil_div(N, 64) * batch;
    if (ws && M > 0 && N > 0 && batch > 0 && tiles < SPLIT_TILES && K >= 2 * SPLIT_KMIN) {
      long ns = (SPLIT_WG + tiles - 1) / tiles;
      if (ns > K / SPLIT_KMIN) ns = K / SPLIT_KMIN;
      const size_t per = sizeof(cplx<R>) * (size_t)M * N * batch;
      if ((size_t)ns > ws_bytes / per) ns = (long)(ws_bytes / per);
      if (ns >= 2) {
        const int kchunk = ceil_div(ceil_div(K, (int)ns), X32_BK) * X32_BK;
        const int nsplit = ceil_div(K, kchunk);
        GemmP<R> P;
        P.skip = nullptr;
        P.lower = 0;
        P.M = M; P.N = N; P.K = K; P.alpha = alpha; P.beta = mk<R>(0, 0);
        P.A = A; P.lda = lda; P.sA = sA; P.opA = opA;
        P.B = B; P.ldb = ldb; P.sB = sB; P.opB = opB;
        P.D = nullptr; P.ldd = 0; P.sD = 0;
        P.C = nullptr; P.ldc = N; P.sC = 0; P.addI = 0;
        P.part = static_cast<cplx<R>*>(ws);
        P.nsplit = nsplit;
        P.kchunk = kchunk;
        ProfScope ps("cgemm_f32_splitk", s, 8.0 * M * N * (double)K * batch);
        hipLaunchKernelGGL(k_cgemm_x32_splitk, dim3(ceil_div(N, 64), ceil_div(M, 64), batch * nsplit), dim3(256), 0,
                           s, P);
        LSH_LAUNCH_CHECK();
        const long total = (long)batch * M * N;
        hipLaunchKernelGGL(k_splitk_reduce<R>, dim3((unsigned)ceil_div(total, 256L)), dim3(256), 0, s,
                           P.part, nsplit, M, N, total, beta, D, ldd, sD, C, ldc, sC, 0);
        LSH_LAUNCH_CHECK();
        return;
      }
    }
  }
  cgemm<R>(s, M, N, K, alpha, A, lda, sA, opA, B, ldb, sB, opB, beta, D, ldd, sD, C, ldc, sC, batch);
}

void cgemm_grouped(hipStream_t s, const std::vector<GemmItem>& items, DevBuf& dev) {
  std::vector<GemmGroupDev> h;
  long tiles = 0;
  double flops = 0;
  for (const GemmItem& it : items) {
    if (it.M <= 0 || it.N <= 0 || it.batch <= 0) continue;
    GemmGroupDev g;
    GemmP<float>& P = g.p;
    P.M = it.M; P.N = it.N; P.K = it.K; P.alpha = it.alpha; P.beta = it.beta;
    P.A = it.A; P.lda = it.lda; P.sA = it.sA; P.opA = it.opA;
    P.B = it.B; P.ldb = it.ldb; P.sB = it.sB; P.opB = it.opB;
    P.D = it.D; P.ldd = it.ldd; P.sD = it.sD;
    P.C = it.C; P.ldc = it.ldc; P.sC = it.sC; P.addI = it.addI ? 1 : 0; P.skip = nullptr; P.lower = 0;
    g.batch = it.batch;
    g.tiles_m = ceil_div(it.M, 64);
    g.tiles_n = ceil_div(it.N, 64);
    g.tile0 = tiles;
    tiles += (long)g.tiles_m * g.tiles_n * g.batch;
    flops += 8.0 * it.M * it.N * it.K * it.batch;
    h.push_back(g);
  }
  if (h.empty()) return;
  const size_t bytes = sizeof(GemmGroupDev) * h.size();
  if (dev.bytes < bytes) dev.alloc(bytes);
  LSH_HIP(hipMemcpyAsync(dev.p, h.data(), bytes, hipMemcpyHostToDevice, s));
  ProfScope ps("cgemm_f32_grouped", s, flops);
  const long gx = tiles < 65535 ? tiles : 65535;
  const dim3 grid((unsigned)gx, (unsigned)((tiles + gx - 1) / gx));
  hipLaunchKernelGGL(k_cgemm_x32_grouped, grid, dim3(256), 0, s, dev.as<GemmGroupDev>(), (int)h.size());
  LSH_LAUNCH_CHECK();
  // the table must outlive the copy: pageable copies are staged before
  // hipMemcpyAsync returns, so the host vector may go out of scope here
}

// C[i][j] = conj(C[j][i]) for j > i (32 x 32 tiles through LDS)
template <typename R>
__global__ __launch_bounds__(256) void k_mirror_lower(cplx<R>* C, int n, long ldc) {
  __shared__ cplx<R> t[32][33];
  const int tr = blockIdx.y, tc = blockIdx.x;  // destination tile (row tr, column tc), tc >= tr
  if (tc < tr) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {  // source: rows of tile (tc, tr)
    const int i = tc * 32 + r, j = tr * 32 + tx;
    t[r][tx] = (i < n && j < n) ? C[(long)i * ldc + j] : mk<R>(0, 0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = tr * 32 + r, j = tc * 32 + tx;
    if (i < n && j < n && j > i) C[(long)i * ldc + j] = conjg(t[tx][r]);
  }
}

template <typename R>
void mirror_lower(hipStream_t s, cplx<R>* C, int n, long ldc) {
  if (n <= 1) return;
  const int nt = ceil_div(n, 32);
  hipLaunchKernelGGL(k_mirror_lower<R>, dim3(nt, nt), dim3(256), 0, s, C, n, ldc);
  LSH_LAUNCH_CHECK();
}
template void mirror_lower<double>(hipStream_t, cplx<double>*, int, long);
template void mirror_lower<float>(hipStream_t, cplx<float>*, int, long);

// ---------------------------------------------------------------- GEMV
// One wavefront per row, lanes stride the row (coalesced); x_b staged in LDS.

// Per-problem GEMV over the rows of all problems: y[v amod + b] = alpha A_b
// x[v amod + b] + beta z[...] for rows i of problem b < nb (matrix b mod
// amod) and v < nv vectors per matrix (nv = 1: one vector per problem, any
// batch; nv > 1: the vectors of one matrix share its row loads).  Global row
// g = b M + i.  L lanes share a row (a power of two chosen from the row
// length, at most 64); a wave takes 64 / L rows per pass and P passes.  Short
// and medium rows (NCH = the row's chunks of L, at most 8): every load of the
// P rows is issued before the products, so small boxes still keep
// 2 P NCH loads in flight per lane; long rows (NCH = 0) loop over chunks of
// 8 L.  A lane adds its products in chunk order into four partial sums
// (chunk u into sum u mod 4), then (s0 + s1) + (s2 + s3), then a butterfly
// over the row's L lanes: every vector of a matrix gets the arithmetic of a
// one-vector call (same lanes, same order), so columns come out bitwise the
// same either way.  x is read through the caches (the rows of one problem
// share it).
template <typename R, int L, int NCH, int P, int NV>
__global__ __launch_bounds__(256) void k_cgemv(int M, int N, cplx<R> alpha, const cplx<R>* __restrict__ A, long lda,
                                               long sA, int amod, int nv, const cplx<R>* __restrict__ x, long sx,
                                               cplx<R> beta, const cplx<R>* z, long sz, cplx<R>* y, long sy,
                                               long rows) {
  constexpr int RW = 64 / L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, sub = lane & (L - 1);
  // rows < 2^31 (checked by the launcher): 32-bit problem / row split, once
  const unsigned g0 = ((blockIdx.x * 4u + wave) * P) * RW + lane / L;
  unsigned bp[P], ip[P];
  {
    unsigned b = g0 / (unsigned)M, i = g0 - b * (unsigned)M;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      bp[p] = b;
      ip[p] = i;
      i += RW;
      while (i >= (unsigned)M) { i -= M; ++b; }
    }
  }
  cplx<R> out[P][NV];
  if constexpr (NCH > 0) {
    cplx<R> a[P][NCH];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const bool live = (long)g0 + (long)p * RW < rows;
      const cplx<R>* row = A + (long)(bp[p] % (unsigned)amod) * sA + (long)ip[p] * lda;
#pragma unroll
      for (int u = 0; u < NCH; ++u) {
        const int col = sub + u * L;
        a[p][u] = (live && col < N) ? row[col] : mk<R>(0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      cplx<R> xv[P][NCH];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const bool live = v < nv && (long)g0 + (long)p * RW < rows;
        const cplx<R>* xb = x + ((long)v * amod + bp[p]) * sx;
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          const int col = sub + u * L;
          xv[p][u] = (live && col < N) ? xb[col] : mk<R>(0, 0);
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) {
        cplx<R> a4[4] = {mk<R>(0, 0), mk<R>(0, 0), mk<R>(0, 0), mk<R>(0, 0)};
#pragma unroll
        for (int u = 0; u < NCH; ++u) fma_acc(a4[u & 3], a[p][u], xv[p][u]);
        out[p][v] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      }
    }
  } else {  // long rows (L == 64): eight independent loads per lane per chunk
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
      for (int v = 0; v < NV; ++v) out[p][v] = mk<R>(0, 0);
      const long g = (long)g0 + (long)p * RW;
      if (g >= rows) break;
      const cplx<R>* row = A + (long)(bp[p] % (unsigned)amod) * sA + (long)ip[p] * lda;
      cplx<R> a4[NV][4];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int u = 0; u < 4; ++u) a4[v][u] = mk<R>(0, 0);
      for (int j = sub; j < N; j += 8 * L) {
        cplx<R> w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int jj = j + u * L;
          w[u] = jj < N ? row[jj] : mk<R>(0, 0);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (v >= nv) break;
          const cplx<R>* xb = x + ((long)v * amod + bp[p]) * sx;
          cplx<R> xw[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int jj = j + u * L;
            xw[u] = jj < N ? xb[jj] : mk<R>(0, 0);
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) fma_acc(a4[v][u & 3], w[u], xw[u]);
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) out[p][v] = (a4[v][0] + a4[v][1]) + (a4[v][2] + a4[v][3]);
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      cplx<R> t = out[p][v];
      t.x = group_sum<L>(t.x);  // (stays inside the row's L lanes)
      t.y = group_sum<L>(t.y);
      const long g = (long)g0 + (long)p * RW;
      if (v < nv && sub == 0 && g < rows) {
        const long pb = (long)v * amod + bp[p], i = ip[p];
        cplx<R> o = alpha * t;
        if (z && (beta.x != R(0) || beta.y != R(0))) o = o + beta * z[pb * sz + i];
        y[pb * sy + i] = o;
      }
    }
}

template <typename R, int L, int NCH, int P, int NV>
static void cgemv_launch(hipStream_t s, int M, int N, cplx<R> alpha, const cplx<R>* A, long lda, long sA, int amod,
                         int nv, const cplx<R>* x, long sx, cplx<R> beta, const cplx<R>* z, long sz, cplx<R>* y,
                         long sy, long rows) {
  const long per_wg = 4L * P * (64 / L);
  const long g = (rows + per_wg - 1) / per_wg;
  LSH_REQUIRE(rows + per_wg < 2147483647L, -6, "cgemv: too many rows");
  hipLaunchKernelGGL((k_cgemv<R, L, NCH, P, NV>), dim3((unsigned)g), dim3(256), 0, s, M, N, alpha, A, lda, sA, amod,
                     nv, x, sx, beta, z, sz, y, sy, rows);
}

// Lanes per row and chunk count from the row length N: L = the power of two
// >= N / 4 (8..64), NCH = the power of two >= N / L; rows past 8 x 64 loop.
// P keeps P NCH near 16 for one FP32 vector; halved for several vectors and
// again for FP64, so the loads and sums stay near 80 registers.
template <typename R, int NV>
static void cgemv_dispatch(hipStream_t s, int M, int N, cplx<R> alpha, const cplx<R>* A, long lda, long sA, int amod,
                           int nv, const cplx<R>* x, long sx, cplx<R> beta, const cplx<R>* z, long sz, cplx<R>* y,
                           long sy, long rows) {
  constexpr int DIV = (NV > 1 ? 2 : 1) * (sizeof(R) == 8 ? 2 : 1);
#define LSH_GV(LL, NC, PP) \
  cgemv_launch<R, LL, NC, ((PP) / DIV > 0 ? (PP) / DIV : 1), NV>(s, M, N, alpha, A, lda, sA, amod, nv, x, sx, beta, \
                                                                 z, sz, y, sy, rows)
  if (N > 512) { LSH_GV(64, 0, 1); return; }
  int L = 8;
  while (L < 64 && 4 * L < N) L *= 2;
  const int nch = (N + L - 1) / L;  // 1 .. 8
  switch (L) {
    case 8:
      if (nch <= 1) LSH_GV(8, 1, 8); else if (nch <= 2) LSH_GV(8, 2, 8); else LSH_GV(8, 4, 4);
      break;
    case 16:
      if (nch <= 2) LSH_GV(16, 2, 8); else LSH_GV(16, 4, 4);
      break;
    case 32:
      if (nch <= 2) LSH_GV(32, 2, 8); else LSH_GV(32, 4, 4);
      break;
    default:
      if (nch <= 2) LSH_GV(64, 2, 8); else if (nch <= 4) LSH_GV(64, 4, 4); else LSH_GV(64, 8, 2);
      break;
  }
#undef LSH_GV
}

template <typename R>
void cgemv(hipStream_t s, int M, int N, cplx<R> alpha,
           const cplx<R>* A, long lda, long sA, int amod,
           const cplx<R>* x, long sx, cplx<R> beta, const cplx<R>* z, long sz,
           cplx<R>* y, long sy, int batch) {
  if (M <= 0 || batch <= 0) return;
  // algorithmic bytes: every distinct matrix once, x, z and y once per problem
  const int nmat = amod < batch ? amod : batch;
  ProfScope ps(sizeof(R) == 4 ? "cgemv_f32" : "cgemv_f64", s,
               (double)sizeof(cplx<R>) * ((double)nmat * M * N + (double)batch * (N + (z ? 2.0 : 1.0) * M)));
  const int am = amod > 0 ? amod : 1;
  if (batch > am && batch % am == 0 && batch / am <= 64) {
    // several vectors per matrix: groups of four read each matrix once
    const int nvec = batch / am;
    for (int v0 = 0; v0 < nvec; v0 += 4) {
      const int nv = nvec - v0 < 4 ? nvec - v0 : 4;
      const long o = (long)v0 * am;
      const cplx<R>* zv = z ? z + o * sz : nullptr;
      cgemv_dispatch<R, 4>(s, M, N, alpha, A, lda, sA, am, nv, x + o * sx, sx, beta, zv, sz, y + o * sy, sy,
                           (long)am * M);
      LSH_LAUNCH_CHECK();
    }
    return;
  }
  cgemv_dispatch<R, 1>(s, M, N, alpha, A, lda, sA, am, 1, x, sx, beta, z, sz, y, sy, (long)batch * M);
  LSH_LAUNCH_CHECK();
}

// ------------------------------------------------ shared-matrix multi-GEMV
// Y[v] = alpha Mat X[v] + beta Z[v] for v < nvec and one shared matrix
// (rows x C, row-major): the preconditioner's shared box products (U_l,
// G_ab, [L^T; R^T], [L; R]) for up to a thousand box vectors.  A workgroup
// takes a block of rows of one block of Mat (the rows from R1 on read
// X + xoff2: the two halves of Q v in one launch) and NV vectors (grid y
// runs over the groups of NV).  WS = 4 (long rows): the four waves split the
// columns of RR rows (wave w takes columns 64(w + 4q) + lane, two chunks per
// step) and meet in LDS; WS = 1 (rows under 1024): each wave takes RR rows of
// its own over all columns.  Each loaded piece of x serves RR rows, and a
// lane keeps 2 (RR + NV) loads in flight.  Sums in a fixed order: per lane
// over its chunks, a butterfly over the wave's lanes, then (WS = 4) the
// waves in order.
template <typename R, int RR, int NV, int WS>
__global__ __launch_bounds__(256) void k_cmgemv(int Rr, int R1, int wg1, int C, cplx<R> alpha,
                                                const cplx<R>* __restrict__ Mat,
                                                const cplx<R>* __restrict__ Mat2, long ldm,
                                                const cplx<R>* __restrict__ X, long ldx, long xoff2, cplx<R> beta,
                                                const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec) {
  constexpr int ROWS = WS == 4 ? RR : 4 * RR;  // rows per workgroup
  __shared__ cplx<R> red[WS == 4 ? 4 : 1][RR * NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int i0, iend;
  const cplx<R>* Xb = X;
  const cplx<R>* Mb = Mat;
  int mrow0 = 0;  // the block's first row in Mb
  if ((int)blockIdx.x < wg1) {
    i0 = blockIdx.x * ROWS;
    iend = R1;
  } else {
    i0 = R1 + (blockIdx.x - wg1) * ROWS;
    iend = Rr;
    Xb = X + xoff2;
    Mb = Mat2;  // (row i of the second block is row i - R1 of Mat2)
    mrow0 = R1;
  }
  if (WS == 1) i0 += wave * RR;
  const int nr = iend - i0 < RR ? iend - i0 : RR;  // (<= 0: this wave has no rows)
  const int v0 = blockIdx.y * NV;
  const int nv = nvec - v0 < NV ? nvec - v0 : NV;
  const cplx<R>* row0 = Mb + (long)(i0 - mrow0) * ldm;
  const cplx<R>* xv = Xb + (long)v0 * ldx;
  cplx<R> acc[RR][NV];
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[r][v] = mk<R>(0, 0);
  constexpr int STEP = 64 * WS;  // columns per chunk
  for (int j = (WS == 4 ? wave * 64 : 0) + lane; j < C && nr > 0; j += 2 * STEP) {
    const int j2 = j + STEP;
    cplx<R> a[2][RR], x[2][NV];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      a[0][r] = r < nr ? row0[(long)r * ldm + j] : mk<R>(0, 0);
      a[1][r] = (r < nr && j2 < C) ? row0[(long)r * ldm + j2] : mk<R>(0, 0);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      x[0][v] = v < nv ? xv[(long)v * ldx + j] : mk<R>(0, 0);
      x[1][v] = (v < nv && j2 < C) ? xv[(long)v * ldx + j2] : mk<R>(0, 0);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v) fma_acc(acc[r][v], a[h][r], x[h][v]);
  }
  auto store = [&](int r, int v, cplx<R> t) {
    const long yi = (long)(v0 + v);
    cplx<R> o = alpha * t;
    if (Z && (beta.x != R(0) || beta.y != R(0))) o = o + beta * Z[yi * ldz + i0 + r];
    Y[yi * ldy + i0 + r] = o;
  };
  if (WS == 1) {
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        cplx<R> t = acc[r][v];
        t.x = group_sum<64>(t.x);
        t.y = group_sum<64>(t.y);
        if (lane == 0 && r < nr && v < nv) store(r, v, t);
      }
    return;
  }
#pragma unroll
  for (int r = 0; r < RR; ++r)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      cplx<R> t = acc[r][v];
      t.x = group_sum<64>(t.x);
      t.y = group_sum<64>(t.y);
      if (lane == 0) red[WS == 4 ? wave : 0][r * NV + v] = t;
    }
  __syncthreads();
  if (threadIdx.x < RR * NV) {
    const int r = threadIdx.x / NV, v = threadIdx.x % NV;
    if (r < nr && v < nv) {
      const int e = threadIdx.x, w3 = WS == 4 ? 3 : 0, w2 = WS == 4 ? 2 : 0, w1 = WS == 4 ? 1 : 0;
      store(r, v, (red[0][e] + red[w1][e]) + (red[w2][e] + red[w3][e]));
    }
  }
}

template <typename R, int RR, int NV, int WS>
static void cmgemv_launch(hipStream_t s, int Rr, int R1, long xoff2, int C, cplx<R> alpha, const cplx<R>* Mat,
                          const cplx<R>* Mat2, long ldm, const cplx<R>* X, long ldx, cplx<R> beta,
                          const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec) {
  constexpr int ROWS = WS == 4 ? RR : 4 * RR;
  const int wg1 = ceil_div(R1, ROWS), wg2 = ceil_div(Rr - R1, ROWS);
  LSH_REQUIRE(ceil_div(nvec, NV) <= 65535, -6, "cmgemv: too many vectors");
  hipLaunchKernelGGL((k_cmgemv<R, RR, NV, WS>), dim3(wg1 + wg2, ceil_div(nvec, NV)), dim3(256), 0, s, Rr, R1, wg1,
                     C, alpha, Mat, Mat2, ldm, X, ldx, xoff2, beta, Z, ldz, Y, ldy, nvec);
}

template <typename R>
void cmgemv2(hipStream_t s, int Rr, int R1, long xoff2, int C, cplx<R> alpha, const cplx<R>* Mat, long ldm,
             const cplx<R>* X, long ldx, cplx<R> beta, const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec,
             const cplx<R>* Mat2) {
  if (Rr <= 0 || nvec <= 0) return;
  if (R1 > Rr) R1 = Rr;
  if (!Mat2) Mat2 = Mat + (long)R1 * ldm;
  ProfScope ps(sizeof(R) == 4 ? "cmgemv_f32" : "cmgemv_f64", s,
               (double)sizeof(cplx<R>) * ((double)Rr * C + (double)nvec * ((R1 < Rr ? 2.0 : 1.0) * C +
                                                                          (Z ? 2.0 : 1.0) * Rr)));
  constexpr int RR = sizeof(R) == 4 ? 4 : 2;  // (FP64: the accumulators in half the rows)
  // Launches that would give fewer than two workgroups per compute unit take
  // one row per wave instead (each row's sum is the same either way).
  const int nvs = nvec == 1 ? 1 : nvec == 2 ? 2 : nvec <= 4 ? 4 : 8;
  const int rows = C >= 1024 ? RR : 4 * RR;
  const long wgs = (long)(ceil_div(R1, rows) + ceil_div(Rr - R1, rows)) * ceil_div(nvec, nvs);
  const bool thin = wgs < 512;
#define LSH_MG(RRV, NVV, WSS) \
  cmgemv_launch<R, RRV, NVV, WSS>(s, Rr, R1, xoff2, C, alpha, Mat, Mat2, ldm, X, ldx, beta, Z, ldz, Y, ldy, nvec)
#define LSH_MG_NV(RRV, WSS)           \
  if (nvs == 1) LSH_MG(RRV, 1, WSS);  \
  else if (nvs == 2) LSH_MG(RRV, 2, WSS); \
  else if (nvs == 4) LSH_MG(RRV, 4, WSS); \
  else LSH_MG(RRV, 8, WSS);
  if (C >= 1024) {
    if (thin) { LSH_MG_NV(1, 4) }
    else { LSH_MG_NV(RR, 4) }
  } else {
    if (thin) { LSH_MG_NV(1, 1) }
    else { LSH_MG_NV(RR, 1) }
  }
#undef LSH_MG_NV
#undef LSH_MG
  LSH_LAUNCH_CHECK();
}

template <typename R>
void cmgemv(hipStream_t s, int Rr, int C, cplx<R> alpha, const cplx<R>* Mat, long ldm, const cplx<R>* X, long ldx,
            cplx<R> beta, const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy, int nvec) {
  cmgemv2<R>(s, Rr, Rr, 0, C, alpha, Mat, ldm, X, ldx, beta, Z, ldz, Y, ldy, nvec, nullptr);
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

// One c x c matrix in LDS (one workgroup); perm: c ints of global scratch.
template <typename R>
__device__ void inv_small_body(cplx<R>* Ab, int c, long lda, int* infob, int* perm) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* S = reinterpret_cast<cplx<R>*>(smem_raw);  // c*c
  __shared__ int s_piv;
  __shared__ int s_bad;
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
  if (tid == 0 && infob) *infob = s_bad;
}

template <typename R>
__global__ __launch_bounds__(256) void k_inv_small(cplx<R>* A, int c, long lda, long sA, int* info, int* permg) {
  const long b = blockIdx.x;
  inv_small_body<R>(A + b * sA, c, lda, info ? info + b : nullptr, permg + b * c);
}

// Large matrices: two-level blocked in-place Gauss-Jordan without row
// interchanges.  The pivot of column j is the largest |a_ij|^2 among the rows
// not yet used as pivots (partial pivoting); that row p_j stays where it is.
// One elementary step E_j = I + w_j e_{p_j}^T makes column j the unit vector
// e_{p_j}; in place, column j receives E_j's column p_j instead (1/pivot in
// row p_j, -a_ij/pivot elsewhere) and every other column is updated.  With
// Q = [e_{p_0} .. e_{p_{c-1}}] the array ends as S = E Q where E A = Q, so
//     A^{-1} = Q^T S Q^T,   A^{-1}[a][b] = S[p_a][pinv_b].
// Blocking: slabs of NB2 columns, panels of NB columns within a slab.
//  1. k_gj_panel: one workgroup per matrix holds the c x NB panel in
//     registers (loaded and stored through LDS so that the global accesses
//     are coalesced) and applies its NB steps.  One barrier per column: each
//     wave posts its best candidate row and key, every thread reduces the
//     posts itself.
//  2. k_gj_gather + GEMM on the rest of the slab: the block's steps combine to
//     E_K = I + F R_K^T (R_K selects rows p_K, F = S(:,K) - I(:,p_K)), so
//     slab += F T with T = slab rows p_K (zero in the panel's columns).
//  3. After the slab: the same with the slab's NB2 steps on every column
//     outside it, one GEMM of depth NB2.
//  4. k_gj_unperm: the permutation above, through a copy.
constexpr int GJ_NT = 1024;
constexpr int GJ_NB2_DEFAULT = 64, GJ_NB2_MAX = 256;
constexpr int GJ_STAGE_BYTES = 32768;

static int gj_nb2() {
  static int v = [] {
    const char* e = getenv("LSH_GJ_NB2");
    int x = e ? atoi(e) : GJ_NB2_DEFAULT;
    if (x < 8) x = 8;
    if (x > GJ_NB2_MAX) x = GJ_NB2_MAX;
    return x & ~7;
  }();
  return v;
}

// Pivot search keys: a 32-bit integer whose maximum is, up to the low bits
// of the value, the largest |a|^2, and among values equal in the kept bits the
// smallest row.  Non-negative IEEE values order like their bit patterns: the
// key keeps the value's top 19 bits (FP32: exponent and 10 mantissa bits;
// FP64, from its top word: exponent and 7 mantissa bits) above 8191 - row
// (rows < 4096).  So a pivot is chosen among the values within 2^-10 (FP32)
// or 2^-7 (FP64) of the largest, a threshold partial pivoting.  A NaN value
// counts as 0.  Every key of a candidate row is nonzero; 0 = no candidate.
template <typename R>
struct PivKey;
template <>
struct PivKey<float> {
  static __device__ __forceinline__ unsigned make(float a, int i) {
    return ((a >= 0.f ? __float_as_uint(a) : 0u) & ~0x1FFFu) | (unsigned)(0x1FFF - i);
  }
  static __device__ __forceinline__ int row(unsigned k) { return 0x1FFF - (int)(k & 0x1FFF); }
};
template <>
struct PivKey<double> {
  static __device__ __forceinline__ unsigned make(double a, int i) {
    const unsigned v = a >= 0.0 ? (unsigned)((unsigned long long)__double_as_longlong(a) >> 32) : 0u;
    return (v & ~0x1FFFu) | (unsigned)(0x1FFF - i);
  }
  static __device__ __forceinline__ int row(unsigned k) { return 0x1FFF - (int)(k & 0x1FFF); }
};

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a - f p with four fused multiply-adds
template <typename R>
__device__ __forceinline__ cplx<R> cfms(cplx<R> a, cplx<R> f, cplx<R> p) {
  return mk<R>(fmaR(f.y, p.y, fmaR(-f.x, p.x, a.x)), fmaR(-f.y, p.x, fmaR(-f.x, p.y, a.y)));
}

// Workgroup barrier that orders LDS only: the panel kernel's global stores
// (pivot records, the panel itself) are read by later launches only, so the
// barrier need not wait for them.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Staging rounds move GJ_KR(R) x blockDim elements of the row-major panel
// between global memory (coalesced) and the row owners (through LDS).
template <typename R>
constexpr int gj_kr() { return GJ_STAGE_BYTES / (GJ_NT * (int)sizeof(cplx<R>)); }

// After its columns, the panel writes Tb[q][t] = A[p_{j0+q}][s0 + t] for the
// other columns of its slab (zero in its own), the pivot rows the slab
// update needs before any of them changes (Tb null or w2 <= nb: no update).
template <typename R, int RPT, int NB>
__device__ __forceinline__ void gj_panel_body(cplx<R>* Ab, int c, long lda, int j0, int* pb, int* ub, int* infob,
                                              int s0, int w2, cplx<R>* Tb) {
  constexpr int KR = gj_kr<R>();
  __shared__ cplx<R> stg[KR * GJ_NT];
  __shared__ int pvs[NB];
  __shared__ cplx<R> cand[2][GJ_NT / 64][NB];  // each wave's best candidate row (double-buffered)
  __shared__ unsigned ckey[2][GJ_NT / 64];
  const int nt = blockDim.x, nw = nt >> 6;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = (c - j0) < NB ? (c - j0) : NB;
  const int ne = c * NB;     // panel elements, row-major
  const int S = KR * nt;     // elements per staging round (a multiple of NB)
  const int nrounds = (ne + S - 1) / S;
  cplx<R> P[RPT][NB];
  bool avail[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * nt;
    avail[r] = i < c && !ub[i];
#pragma unroll
    for (int q = 0; q < NB; ++q) P[r][q] = mk<R>(0, 0);
  }
  {
    cplx<R> V[KR], Vn[KR];
    auto fetch = [&](cplx<R>(&v)[KR], int lo) {
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int e = lo + tid + k * nt, q = e & (NB - 1);
        v[k] = (e < ne && q < nb) ? Ab[(long)(e / NB) * lda + j0 + q] : mk<R>(0, 0);
      }
    };
    fetch(V, 0);
    for (int rd = 0; rd < nrounds; ++rd) {
      const int lo = rd * S;
      if (rd + 1 < nrounds) fetch(Vn, lo + S);  // next round in flight meanwhile
#pragma unroll
      for (int k = 0; k < KR; ++k) stg[tid + k * nt] = V[k];
      lds_sync();
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int o = (tid + r * nt) * NB - lo;
        if (o >= 0 && o < S && o < ne - lo)
#pragma unroll
          for (int q = 0; q < NB; ++q) P[r][q] = stg[o + q];
      }
      lds_sync();
#pragma unroll
      for (int k = 0; k < KR; ++k) V[k] = Vn[k];
    }
  }
  // the column loop is unrolled so that every register index is static
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    if (jj >= nb) break;
    const int j = j0 + jj, buf = jj & 1;
    unsigned key = 0;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      if (avail[r]) {
        const unsigned k = PivKey<R>::make(abs2(P[r][jj]), tid + r * nt);
        key = k > key ? k : key;
      }
    key = wave_max_u32_uniform(key);
    const int bi = key ? PivKey<R>::row(key) : -1;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      if (tid + r * nt == bi)
#pragma unroll
        for (int q = 0; q < NB; ++q) cand[buf][wave][q] = P[r][q];
    if (lane == 0) ckey[buf][wave] = key;
    lds_sync();
    // block maximum: every lane reads the waves' posts (the same words)
    unsigned kb = 0;
#pragma unroll
    for (int w = 0; w < GJ_NT / 64; ++w)
      if (w < nw) kb = ckey[buf][w] > kb ? ckey[buf][w] : kb;
    // fewer than c pivots are in use, so some row is a candidate (kb != 0);
    // row p is held by thread p mod nt, so its post is that thread's wave's
    const int p = PivKey<R>::row(kb);
    const int pw = (p % nt) >> 6;
    cplx<R> pr[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) pr[q] = cand[buf][pw][q];
    if (tid == 0) {
      pb[j] = p;
      ub[p] = 1;
      pvs[jj] = p;
      if (!(abs2(pr[jj]) > R(0)) && infob && *infob == 0) *infob = j + 1;
    }
    const cplx<R> rp = crecip(pr[jj]);
    // every row as a non-pivot row; the pivot row is overwritten below
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const cplx<R> fr = P[r][jj] * rp;
#pragma unroll
      for (int q = 0; q < NB; ++q) P[r][q] = (q == jj) ? mk<R>(0, 0) - fr : cfms(P[r][q], fr, pr[q]);
    }
    if (wave == pw) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (tid + r * nt == p) {
#pragma unroll
          for (int q = 0; q < NB; ++q) P[r][q] = (q == jj) ? rp : pr[q] * rp;
          avail[r] = false;
        }
    }
  }
  // rows to LDS, then coalesced stores (never waited for inside the kernel)
  for (int rd = 0; rd < nrounds; ++rd) {
    const int lo = rd * S;
    lds_sync();
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int o = (tid + r * nt) * NB - lo;
      if (o >= 0 && o < S && o < ne - lo)
#pragma unroll
        for (int q = 0; q < NB; ++q) stg[o + q] = P[r][q];
    }
    lds_sync();
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int e = lo + tid + k * nt, q = e & (NB - 1);
      if (e < ne && q < nb) Ab[(long)(e / NB) * lda + j0 + q] = stg[tid + k * nt];
    }
  }
  if (Tb && w2 > nb) {
    lds_sync();  // (pvs)
    for (int e = tid; e < nb * w2; e += nt) {
      const int q = e / w2, col = s0 + e % w2;
      Tb[e] = (col >= j0 && col < j0 + nb) ? mk<R>(0, 0) : Ab[(long)pvs[q] * lda + col];
    }
  }
}

// The rest of slab [s0, s0 + w2) after the panel [j0, j0 + nb): row i gets
// A[i][col] += sum_q F[i][q] T[q][col] with F[i][q] = A[i][j0 + q] -
// [i == p_{j0+q}] (the panel's finished columns) and T from the panel.  The
// 64 lanes of a wave take one row, a column each.
template <typename R>
__device__ __forceinline__ void gj_slab_update_body(cplx<R>* Ab, int c, long lda, int j0, int nb, int s0, int w2,
                                                    const int* pb, const cplx<R>* Tb, int i, int lane) {
  if (i >= c) return;
  cplx<R> f[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    f[q] = q < nb ? Ab[(long)i * lda + j0 + q] : mk<R>(0, 0);
    if (q < nb && i == pb[q]) f[q].x -= R(1);
  }
  for (int t = lane; t < w2; t += 64) {
    const int col = s0 + t;
    if (col >= j0 && col < j0 + nb) continue;
    cplx<R> acc = Ab[(long)i * lda + col];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < nb) {
        const cplx<R> tv = Tb[q * w2 + t];
        acc.x = fmaR(f[q].x, tv.x, acc.x);
        acc.x = fmaR(-f[q].y, tv.y, acc.x);
        acc.y = fmaR(f[q].x, tv.y, acc.y);
        acc.y = fmaR(f[q].y, tv.x, acc.y);
      }
    Ab[(long)i * lda + col] = acc;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_gj_slab_update(cplx<R>* A, int c, long lda, long sA, int j0, int nb, int s0,
                                                        int w2, const int* perm, const cplx<R>* T, int nb2) {
  const long b = blockIdx.y;
  gj_slab_update_body<R>(A + b * sA, c, lda, j0, nb, s0, w2, perm + b * c + j0, T + b * (long)nb2 * c,
                         blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

template <typename R, int RPT, int NB>
__global__ __launch_bounds__(GJ_NT) void k_gj_panel(cplx<R>* A, int c, long lda, long sA, int j0, int* perm,
                                                    int* used, int* info, int s0, int w2, cplx<R>* T, int nb2) {
  const long b = blockIdx.x;
  gj_panel_body<R, RPT, NB>(A + b * sA, c, lda, j0, perm + b * c, used + b * c, info ? info + b : nullptr, s0, w2,
                            T + b * (long)nb2 * c);
}

// Block K = columns [kb, kb+nbk) with pivot rows perm[kb ..]:
//   T[q][t] = A[perm[kb+q]][cs+t] for the columns cs+t (t < ncol) outside K,
//             0 inside K (ld ncol);
//   F[i][q] = A[i][kb+q] - [i == perm[kb+q]]   (ld nbk).
// Both index spaces run along contiguous memory.
// (Tb, Fb: this matrix's T and F; pb: its pivot rows of the block, perm + kb)
template <typename R>
__device__ __forceinline__ void gj_gather_body(const cplx<R>* Ab, int c, long lda, int kb, int nbk, int cs,
                                               int ncol, const int* pb, cplx<R>* Tb, cplx<R>* Fb) {
  const long nT = (long)nbk * ncol, nF = (long)c * nbk;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nT + nF; e += (long)gridDim.x * blockDim.x) {
    if (e < nT) {
      const int q = (int)(e / ncol), t = (int)(e % ncol), k = cs + t;
      Tb[e] = (k >= kb && k < kb + nbk) ? mk<R>(0, 0) : Ab[(long)pb[q] * lda + k];
    } else {
      const long f = e - nT;
      const int i = (int)(f / nbk), q = (int)(f % nbk);
      cplx<R> v = Ab[(long)i * lda + kb + q];
      if (i == pb[q]) v.x -= R(1);
      Fb[f] = v;
    }
  }
}

template <typename R>
__global__ void k_gj_gather(const cplx<R>* A, int c, long lda, long sA, int kb, int nbk, int cs, int ncol,
                            const int* perm, cplx<R>* T, cplx<R>* F) {
  const long b = blockIdx.y;
  gj_gather_body<R>(A + b * sA, c, lda, kb, nbk, cs, ncol, perm + b * c + kb, T + b * (long)nbk * ncol,
                    F + b * (long)c * nbk);
}

// tmp[a][b] = S[perm[a]][pinv[b]] (pinv[perm[j]] = j), then copied back
template <typename R>
__global__ void k_gj_pinv(const int* perm, int* pinv, int c, int batch) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)c * batch) return;
  const long b = e / c;
  pinv[b * c + perm[e]] = (int)(e % c);
}

template <typename R>
__global__ void k_gj_unperm(const cplx<R>* A, int c, long lda, long sA, const int* perm, const int* pinv,
                            cplx<R>* tmp) {
  const long b = blockIdx.y;
  const long n = (long)c * c;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int a = (int)(e / c), bb = (int)(e % c);
    tmp[b * n + e] = A[b * sA + (long)perm[b * c + a] * lda + pinv[b * c + bb]];
  }
}

template <typename R>
__global__ void k_gj_copyback(cplx<R>* A, int c, long lda, long sA, const cplx<R>* tmp) {
  const long b = blockIdx.y;
  const long n = (long)c * c;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    A[b * sA + (e / c) * lda + (e % c)] = tmp[b * n + e];
}

__global__ void k_zero_int(int* p, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename R>
static size_t small_inv_lds(int c) {
  return (size_t)c * c * sizeof(cplx<R>);
}

// blocked-path workspace per matrix: perm, pinv, used (int c each), T (NB2 x c),
// F (c x NB2), the copy for the final permutation (c x c)
template <typename R>
static size_t gj_ws_per_matrix(int c) {
  return 3 * (size_t)c * sizeof(int) + (2 * (size_t)gj_nb2() * c + (size_t)c * c) * sizeof(cplx<R>);
}

template <typename R>
size_t inverse_ws_bytes(int c, int batch) {
  if (small_inv_lds<R>(c) <= 65536) return (size_t)batch * c * sizeof(int) + 256;
  return (size_t)batch * gj_ws_per_matrix<R>(c) + 8 * 256;
}

template <typename R, int NB>
static void gj_panel_launch(hipStream_t s, int rpt, int nt, cplx<R>* A, int c, long lda, long sA, int j0,
                            int* perm, int* used, int batch, int* info, int s0, int w2, cplx<R>* T, int nb2) {
  const size_t lds = 0;
  switch (rpt) {
    case 1: hipLaunchKernelGGL((k_gj_panel<R, 1, NB>), dim3(batch), dim3(nt), lds, s, A, c, lda, sA, j0, perm, used, info, s0, w2, T, nb2); break;
    case 2: hipLaunchKernelGGL((k_gj_panel<R, 2, NB>), dim3(batch), dim3(nt), lds, s, A, c, lda, sA, j0, perm, used, info, s0, w2, T, nb2); break;
    case 3: hipLaunchKernelGGL((k_gj_panel<R, 3, NB>), dim3(batch), dim3(nt), lds, s, A, c, lda, sA, j0, perm, used, info, s0, w2, T, nb2); break;
    default: hipLaunchKernelGGL((k_gj_panel<R, 4, NB>), dim3(batch), dim3(nt), lds, s, A, c, lda, sA, j0, perm, used, info, s0, w2, T, nb2); break;
  }
  LSH_LAUNCH_CHECK();
}

static int grid_for(long n) {
  const long g = (n + 255) / 256;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

template <typename R>
void inverse(hipStream_t s, cplx<R>* A, int c, long lda, long sA, int batch, void* ws, int* info) {
  if (c <= 0 || batch <= 0) return;
  ProfScope ps(sizeof(R) == 4 ? "op_inverse_f32" : "op_inverse_f64", s, 8.0 * (double)c * c * c * batch);
  if (info) hipLaunchKernelGGL(k_zero_int, dim3(ceil_div(batch, 256)), dim3(256), 0, s, info, (long)batch);
  const size_t lds = small_inv_lds<R>(c);
  if (lds <= 65536) {
    int* permg = static_cast<int*>(ws);
    hipLaunchKernelGGL(k_inv_small<R>, dim3(batch), dim3(256), lds, s, A, c, lda, sA, info, permg);
    LSH_LAUNCH_CHECK();
    return;
  }
  LSH_REQUIRE(c <= 4 * GJ_NT, -6, "inverse: matrix order above 4096 is not supported");
  LSH_REQUIRE(batch <= 65535, -6, "inverse: batch too large for the blocked path");
  const int NB2 = gj_nb2();
  char* w = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    char* p = w;
    w += (bytes + 255) / 256 * 256;
    return p;
  };
  int* perm = reinterpret_cast<int*>(take((size_t)batch * c * sizeof(int)));
  int* pinv = reinterpret_cast<int*>(take((size_t)batch * c * sizeof(int)));
  int* used = reinterpret_cast<int*>(take((size_t)batch * c * sizeof(int)));
  cplx<R>* T = reinterpret_cast<cplx<R>*>(take((size_t)batch * NB2 * c * sizeof(cplx<R>)));
  cplx<R>* F = reinterpret_cast<cplx<R>*>(take((size_t)batch * NB2 * c * sizeof(cplx<R>)));
  cplx<R>* tmp = reinterpret_cast<cplx<R>*>(take((size_t)batch * c * c * sizeof(cplx<R>)));
  hipLaunchKernelGGL(k_zero_int, dim3(ceil_div((long)batch * c, 256)), dim3(256), 0, s, used, (long)batch * c);
  LSH_LAUNCH_CHECK();
  const int rpt = ceil_div(c, GJ_NT);
  const int nt = ceil_div(ceil_div(c, rpt), 64) * 64;
  // panel width: 8 columns, 4 for FP64 with more than one row per thread (register budget)
  const int NB = (sizeof(R) == 8 && rpt > 1) ? 4 : 8;
  const cplx<R> one = mk<R>(1, 0);
  for (int s0 = 0; s0 < c; s0 += NB2) {
    const int w2 = (c - s0) < NB2 ? (c - s0) : NB2;
    for (int j0 = s0; j0 < s0 + w2; j0 += NB) {
      const int nb = (s0 + w2 - j0) < NB ? (s0 + w2 - j0) : NB;
      if (NB == 8) gj_panel_launch<R, 8>(s, rpt, nt, A, c, lda, sA, j0, perm, used, batch, info, s0, w2, T, NB2);
      else gj_panel_launch<R, 4>(s, rpt, nt, A, c, lda, sA, j0, perm, used, batch, info, s0, w2, T, NB2);
      if (w2 > nb) {  // the rest of the slab
        hipLaunchKernelGGL(k_gj_slab_update<R>, dim3(ceil_div(c, 4), batch), dim3(256), 0, s, A, c, lda, sA, j0, nb,
                           s0, w2, perm, T, NB2);
        LSH_LAUNCH_CHECK();
      }
    }
    if (c > w2) {  // every column outside the slab, depth w2
      hipLaunchKernelGGL(k_gj_gather<R>, dim3(grid_for((long)2 * w2 * c), batch), dim3(256), 0, s, A, c, lda, sA,
                         s0, w2, 0, c, perm, T, F);
      LSH_LAUNCH_CHECK();
      if (s0 > 0)
        cgemm<R>(s, c, s0, w2, one, F, w2, (long)c * w2, OP_N, T, c, (long)w2 * c, OP_N, one, A, lda, sA, A, lda,
                 sA, batch);
      const int e = s0 + w2;
      if (e < c)
        cgemm<R>(s, c, c - e, w2, one, F, w2, (long)c * w2, OP_N, T + e, c, (long)w2 * c, OP_N, one, A + e, lda,
                 sA, A + e, lda, sA, batch);
    }
  }
  hipLaunchKernelGGL(k_gj_pinv<R>, dim3(ceil_div((long)batch * c, 256)), dim3(256), 0, s, perm, pinv, c, batch);
  LSH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gj_unperm<R>, dim3(grid_for((long)c * c), batch), dim3(256), 0, s, A, c, lda, sA, perm,
                     pinv, tmp);
  LSH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gj_copyback<R>, dim3(grid_for((long)c * c), batch), dim3(256), 0, s, A, c, lda, sA, tmp);
  LSH_LAUNCH_CHECK();
}

// ------------------------------------------------ grouped FP32 inverses
// Many batches of different orders in one set of launches: every kernel
// walks a device table of the items and one workgroup (or a block row of
// workgroups) per matrix of every item; an item whose order is past the
// current column step returns at once.  Per matrix the arithmetic is the
// one of inverse<float>(), so each result is bitwise the separate call's.
struct InvDev {
  c32* A;
  int c, batch;
  long lda, sA;
  int* info;
  int *perm, *pinv, *used;
  c32 *T, *F, *tmp;
  long mat0;  // first global matrix index of this item
};

__device__ __forceinline__ int inv_item_of(const InvDev* G, int ng, long gm) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (G[mid].mat0 <= gm) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_inv_small_grouped(const InvDev* G, int ng) {
  const long gm = blockIdx.x;
  const InvDev& it = G[inv_item_of(G, ng, gm)];
  const long b = gm - it.mat0;
  inv_small_body<float>(it.A + b * it.sA, it.c, it.lda, it.info ? it.info + b : nullptr, it.perm + b * it.c);
}

__global__ void k_inv_grouped_init(const InvDev* G, int ng) {
  const long gm = blockIdx.y;
  const InvDev& it = G[inv_item_of(G, ng, gm)];
  const long b = gm - it.mat0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < it.c; i += gridDim.x * blockDim.x) it.used[b * it.c + i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && it.info) it.info[b] = 0;
}

// panel j0 of slab s0 (items with j0 inside their slab)
__global__ __launch_bounds__(GJ_NT) void k_gj_panel_grouped(const InvDev* G, int ng, int s0, int nb2, int j0) {
  const long gm = blockIdx.x;
  const InvDev& it = G[inv_item_of(G, ng, gm)];
  const int c = it.c, se = (s0 + nb2) < c ? s0 + nb2 : c;
  if (j0 >= se) return;
  const long b = gm - it.mat0;
  gj_panel_body<float, 1, 8>(it.A + b * it.sA, c, it.lda, j0, it.perm + b * c, it.used + b * c,
                             it.info ? it.info + b : nullptr, s0, se - s0, it.T + b * (long)nb2 * c);
}

// the rest of slab s0 after panel j0 (items with such a rest)
__global__ __launch_bounds__(256) void k_gj_slab_update_grouped(const InvDev* G, int ng, int s0, int nb2, int j0) {
  const long gm = blockIdx.y;
  const InvDev& it = G[inv_item_of(G, ng, gm)];
  const int c = it.c;
  if (s0 >= c) return;
  const int w2 = (c - s0) < nb2 ? c - s0 : nb2;
  if (j0 >= s0 + w2) return;
  const int nb = (s0 + w2 - j0) < 8 ? s0 + w2 - j0 : 8;
  if (w2 <= nb) return;
  const long b = gm - it.mat0;
  gj_slab_update_body<float>(it.A + b * it.sA, c, it.lda, j0, nb, s0, w2, it.perm + b * c + j0,
                             it.T + b * (long)nb2 * c, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// mode 0: the rest of slab s0 after panel j0 (block [j0, j0+nb), columns of
// the slab); mode 1: every column outside slab s0 (block = the slab)
__global__ void k_gj_gather_grouped(const InvDev* G, int ng, int mode, int s0, int nb2, int j0) {
  const long gm = blockIdx.y;
  const InvDev& it = G[inv_item_of(G, ng, gm)];
  const int c = it.c;
  if (s0 >= c) return;
  const int w2 = (c - s0) < nb2 ? c - s0 : nb2;
  int kb, nbk, cs, ncol;
  if (mode == 0) {
    if (j0 >= s0 + w2) return;
    nbk = (s0 + w2 - j0) < 8 ? s0 + w2 - j0 : 8;
    if (w2 <= nbk) return;
    kb = j0; cs = s0; ncol = w2;
  } else {
    if (c <= w2) return;
    kb = s0; nbk = w2; cs = 0; ncol = c;
  }
  const long b = gm - it.mat0;
  gj_gather_body<float>(it.A + b * it.sA, c, it.lda, kb, nbk, cs, ncol, it.perm + b * c + kb,
                        it.T + b * (long)nbk * ncol, it.F + b * (long)c * nbk);
}

__global__ void k_gj_unperm_grouped(const InvDev* G, int ng, int phase) {
  const long gm = blockIdx.y;
  const InvDev& it = G[inv_item_of(G, ng, gm)];
  const int c = it.c;
  const long b = gm - it.mat0;
  const int* pb = it.perm + b * c;
  int* qb = it.pinv + b * c;
  const long n = (long)c * c;
  c32* Ab = it.A + b * it.sA;
  c32* tb = it.tmp + b * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (phase == 0 ? c : n);
       e += (long)gridDim.x * blockDim.x) {
    if (phase == 0) qb[pb[e]] = (int)e;
    else if (phase == 1) tb[e] = Ab[(long)pb[e / c] * it.lda + qb[e % c]];
    else Ab[(e / c) * it.lda + (e % c)] = tb[e];
  }
}

size_t inverse_grouped_ws_bytes(const std::vector<InvItem>& items) {
  size_t t = 0;
  for (const InvItem& it : items) {
    const size_t c = it.c, b = it.batch;
    if (small_inv_lds<float>(it.c) <= 65536) t += ((b * c * sizeof(int) + 255) / 256) * 256;
    else t += ((3 * b * c * sizeof(int) + 255) / 256) * 256 +
              ((b * (2 * (size_t)gj_nb2() * c + c * c) * sizeof(c32) + 255) / 256) * 256 + 4 * 256;
  }
  return t + 256;
}

size_t cgemm_grouped_table_bytes(size_t items) { return mem::round_up(sizeof(GemmGroupDev) * (items ? items : 1)); }

size_t inverse_grouped_arena_bytes(const std::vector<InvItem>& items) {
  size_t t = mem::round_up(sizeof(InvDev) * (items.size() ? items.size() : 1));  // problem table
  int cmax = 0;
  size_t nblocked = 0;
  for (const InvItem& it : items) {
    if (it.c <= 0 || it.batch <= 0) continue;
    if (small_inv_lds<float>(it.c) <= 65536) continue;
    if (it.c <= GJ_NT) {
      cmax = it.c > cmax ? it.c : cmax;
      ++nblocked;
    } else {
      t += mem::round_up(inverse_ws_bytes<float>(it.c, it.batch));  // one-by-one fallback
    }
  }
  // the blocked path's slab GEMM tables (two problems per matrix batch per slab)
  const int NB2 = gj_nb2();
  t += (size_t)((cmax + NB2 - 1) / NB2) * cgemm_grouped_table_bytes(2 * nblocked);
  return t;
}

void inverse_grouped(hipStream_t s, const std::vector<InvItem>& items, void* ws, DevBuf& table) {
  const int NB2 = gj_nb2();
  std::vector<InvDev> small, blocked;
  std::vector<const InvItem*> big;
  char* w = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    char* p = w;
    w += (bytes + 255) / 256 * 256;
    return p;
  };
  long msmall = 0, mblocked = 0;
  int cmax_small = 0, cmax_blocked = 0;
  double flops = 0;
  for (const InvItem& it : items) {
    if (it.c <= 0 || it.batch <= 0) continue;
    flops += 8.0 * it.c * it.c * it.c * it.batch;
    InvDev d{};
    d.A = it.A; d.c = it.c; d.batch = it.batch; d.lda = it.lda; d.sA = it.sA; d.info = it.info;
    if (small_inv_lds<float>(it.c) <= 65536) {
      d.perm = reinterpret_cast<int*>(take((size_t)it.batch * it.c * sizeof(int)));
      d.mat0 = msmall;
      msmall += it.batch;
      cmax_small = it.c > cmax_small ? it.c : cmax_small;
      small.push_back(d);
    } else if (it.c <= GJ_NT) {
      const size_t bc = (size_t)it.batch * it.c;
      d.perm = reinterpret_cast<int*>(take(3 * bc * sizeof(int)));
      d.pinv = d.perm + bc;
      d.used = d.pinv + bc;
      d.T = reinterpret_cast<c32*>(take(sizeof(c32) * bc * NB2));
      d.F = reinterpret_cast<c32*>(take(sizeof(c32) * bc * NB2));
      d.tmp = reinterpret_cast<c32*>(take(sizeof(c32) * bc * it.c));
      d.mat0 = mblocked;
      mblocked += it.batch;
      cmax_blocked = it.c > cmax_blocked ? it.c : cmax_blocked;
      blocked.push_back(d);
    } else {
      big.push_back(&it);
    }
  }
  ProfScope ps("op_inverse_f32_grouped", s, flops);
  LSH_REQUIRE(msmall <= 2147483647L && mblocked <= 65535, -6, "grouped inverse: too many matrices");
  const size_t bytes = sizeof(InvDev) * (small.size() + blocked.size());
  if (bytes && table.bytes < bytes) table.alloc(bytes);
  InvDev* Ts = table.as<InvDev>();
  InvDev* Tb = Ts + small.size();
  if (!small.empty()) {
    LSH_HIP(hipMemcpyAsync(Ts, small.data(), sizeof(InvDev) * small.size(), hipMemcpyHostToDevice, s));
    for (const InvDev& d : small)
      if (d.info) hipLaunchKernelGGL(k_zero_int, dim3(ceil_div((long)d.batch, 256)), dim3(256), 0, s, d.info, (long)d.batch);
    hipLaunchKernelGGL(k_inv_small_grouped, dim3((unsigned)msmall), dim3(256),
                       small_inv_lds<float>(cmax_small), s, Ts, (int)small.size());
    LSH_LAUNCH_CHECK();
  }
  if (!blocked.empty()) {
    const int ng = (int)blocked.size();
    LSH_HIP(hipMemcpyAsync(Tb, blocked.data(), sizeof(InvDev) * ng, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_inv_grouped_init, dim3(ceil_div(cmax_blocked, 256), (unsigned)mblocked), dim3(256), 0, s,
                       Tb, ng);
    LSH_LAUNCH_CHECK();
    const int nt = ceil_div(cmax_blocked, 64) * 64;
    const c32 one = mk<float>(1, 0);
    std::vector<GemmItem> gi;
    DevBuf gtab;
    std::vector<DevBuf> keep;  // GEMM tables of earlier steps stay alive until the end
    auto gemms = [&](std::vector<GemmItem>& v) {
      if (v.empty()) return;
      keep.emplace_back();
      cgemm_grouped(s, v, keep.back());
      v.clear();
    };
    for (int s0 = 0; s0 < cmax_blocked; s0 += NB2) {
      for (int j0 = s0; j0 < s0 + NB2 && j0 < cmax_blocked; j0 += 8) {
        hipLaunchKernelGGL(k_gj_panel_grouped, dim3((unsigned)mblocked), dim3(nt), 0, s, Tb, ng, s0, NB2, j0);
        LSH_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gj_slab_update_grouped, dim3(ceil_div(cmax_blocked, 4), (unsigned)mblocked), dim3(256),
                           0, s, Tb, ng, s0, NB2, j0);
        LSH_LAUNCH_CHECK();
      }
      hipLaunchKernelGGL(k_gj_gather_grouped, dim3(64, (unsigned)mblocked), dim3(256), 0, s, Tb, ng, 1, s0, NB2, 0);
      LSH_LAUNCH_CHECK();
      for (const InvDev& d : blocked) {
        if (s0 >= d.c) continue;
        const int w2 = (d.c - s0) < NB2 ? d.c - s0 : NB2;
        if (d.c <= w2) continue;
        if (s0 > 0)
          gi.push_back({d.c, s0, w2, one, one, d.F, w2, (long)d.c * w2, OP_N, d.T, d.c, (long)w2 * d.c, OP_N, d.A,
                        d.lda, d.sA, d.A, d.lda, d.sA, d.batch, false});
        const int e = s0 + w2;
        if (e < d.c)
          gi.push_back({d.c, d.c - e, w2, one, one, d.F, w2, (long)d.c * w2, OP_N, d.T + e, d.c, (long)w2 * d.c,
                        OP_N, d.A + e, d.lda, d.sA, d.A + e, d.lda, d.sA, d.batch, false});
      }
      gemms(gi);
    }
    for (int phase = 0; phase < 3; ++phase) {
      hipLaunchKernelGGL(k_gj_unperm_grouped, dim3(64, (unsigned)mblocked), dim3(256), 0, s, Tb, ng, phase);
      LSH_LAUNCH_CHECK();
    }
    LSH_HIP(hipStreamSynchronize(s));  // the GEMM tables in keep die here
  }
  for (const InvItem* it : big) {
    DevBuf wsb(inverse_ws_bytes<float>(it->c, it->batch));
    inverse<float>(s, it->A, it->c, it->lda, it->sA, it->batch, wsb.p, it->info);
    LSH_HIP(hipStreamSynchronize(s));
  }
}

// ---- One persistent launch per level: the Woodbury merge (Algorithm 1 with
// eq. (blockinv) restored) and the scattering matrices of every box of every
// instance in the launch.  A fixed grid of workgroups takes boxes from a work
// counter; a workgroup runs the whole chain of its box (each product as a
// loop over 64 x 64 output tiles of the FP32 tile routine, the order-r
// inverse in LDS), so the box's intermediates are made and used on one
// compute unit, and a level is one launch instead of about a dozen.  Every
// product and the inverse are the same instructions as in the separate
// launches, so the factor has the same bits.
namespace {
__device__ __forceinline__ void gemm_all_tiles(const GemmP<float>& P, long b) {
  for (int m0 = 0; m0 < P.M; m0 += 64)
    for (int n0 = 0; n0 < P.N; n0 += 64) cgemm_x32_tile<1, 1, 32>(P, b, m0, n0);
  __syncthreads();  // (the outputs are read by other threads of the workgroup next)
}

__device__ __forceinline__ GemmP<float> gp(int M, int N, int K, float alpha, const c32* A, long lda, long sA, int opA,
                                           const c32* B, long ldb, long sB, int opB, float beta, const c32* D,
                                           long ldd, long sD, c32* C, long ldc, long sC, int addI) {
  GemmP<float> P;
  P.M = M; P.N = N; P.K = K;
  P.alpha = mk<float>(alpha, 0); P.beta = mk<float>(beta, 0);
  P.A = A; P.lda = lda; P.sA = sA; P.opA = opA;
  P.B = B; P.ldb = ldb; P.sB = sB; P.opB = opB;
  P.D = D; P.ldd = ldd; P.sD = sD;
  P.C = C; P.ldc = ldc; P.sC = sC;
  P.addI = addI; P.skip = nullptr; P.lower = 0;
  return P;
}
}  // namespace

__global__ __launch_bounds__(256) void k_merge_level(const MergeLevelDev* G, int ng, long total, int* counter) {
  __shared__ long s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const long item = s_item;
    __syncthreads();
    if (item >= total) break;  // (uniform: every wave of the workgroup leaves)
    int lo = 0, hi = ng - 1;   // last level entry with item0 <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (G[mid].item0 <= item) lo = mid;
      else hi = mid - 1;
    }
    const MergeLevelDev& g = G[lo];
    const long t = item - g.item0;
    const int c = g.c, r = g.r, k = g.k;
    const long cc = (long)c * c, cr = (long)c * r, rr = (long)r * r, r2 = 2L * r, w4 = 4L * rr;
    const long ck = (long)c * k, rk = (long)r * k;
    const c32* Lm = g.Pm;           // L (c x r)
    const c32* Rm = g.Pm + cr;      // R (c x r)
    const c32* Lt = g.Qm;           // L^T (r x c)
    const c32* Rt = g.Qm + cr;      // R^T (r x c)
    c32* Pst = g.Pst + t * 2 * cr;  // [S_a L; S_b R]
    c32* W = g.W + t * w4;
    c32* Aw = g.T + t * 3 * rr;
    c32* Bw = Aw + rr;
    c32* Cm = Bw + rr;
    const c32* Sa = g.Sch + 2 * t * cc;
    // S_a L, S_b R
    gemm_all_tiles(gp(c, r, c, 1, Sa, c, 0, OP_N, Lm, r, 0, OP_N, 0, nullptr, 0, 0, Pst, r, 0, 0), 0);
    gemm_all_tiles(gp(c, r, c, 1, Sa + cc, c, 0, OP_N, Rm, r, 0, OP_N, 0, nullptr, 0, 0, Pst + cr, r, 0, 0), 0);
    // Aw = R^T (S_b R), Bw = L^T (S_a L), C = I - Bw Aw
    gemm_all_tiles(gp(r, r, c, 1, Rt, c, 0, OP_N, Pst + cr, r, 0, OP_N, 0, nullptr, 0, 0, Aw, r, 0, 0), 0);
    gemm_all_tiles(gp(r, r, c, 1, Lt, c, 0, OP_N, Pst, r, 0, OP_N, 0, nullptr, 0, 0, Bw, r, 0, 0), 0);
    gemm_all_tiles(gp(r, r, r, -1, Bw, r, 0, OP_N, Aw, r, 0, OP_N, 0, nullptr, 0, 0, Cm, r, 0, 1), 0);
    // C^{-1} in LDS
    inv_small_body<float>(Cm, r, r, g.info + t, g.perm + t * r);
    __syncthreads();
    // W' = [[-Aw C, I + Aw C Bw], [C, -C Bw]]
    for (long e = threadIdx.x; e < rr; e += blockDim.x) W[r * r2 + (e / r) * r2 + (e % r)] = Cm[e];
    __syncthreads();
    gemm_all_tiles(gp(r, r, r, -1, Aw, r, 0, OP_N, Cm, r, 0, OP_N, 0, nullptr, 0, 0, W, r2, 0, 0), 0);
    gemm_all_tiles(gp(r, r, r, -1, W, r2, 0, OP_N, Bw, r, 0, OP_N, 0, nullptr, 0, 0, W + r, r2, 0, 1), 0);
    gemm_all_tiles(gp(r, r, r, -1, Cm, r, 0, OP_N, Bw, r, 0, OP_N, 0, nullptr, 0, 0, W + r * r2 + r, r2, 0, 0), 0);
    if (!g.U) continue;  // (the root has no scattering matrix)
    // X [a1; a2] = [a1; a2] - P W' [L^T a1; R^T a2] with a = [S_a U1; S_b U2], then S = U^T X D U,
    // the products with U through its rows off the skeleton (as the separate launches)
    c32* a = g.A12 + t * 2 * ck;
    c32* q = g.Qb + t * 4 * rk;
    c32* y = q + 2 * rk;
    const int nh[2] = {g.n0, g.n1}, nr = g.n0 + g.n1;
    c32* Gb = g.G + t * (long)c * nr;
    c32* Rb = g.Rg + t * (long)nr * k;
    for (int h = 0; h < 2; ++h) {  // a_h: the skeleton columns of S_h placed; S_h[:, rest_h] gathered
      const c32* Sh = Sa + h * cc;
      c32* ah = a + h * ck;
      for (long e = threadIdx.x; e < ck; e += blockDim.x) {
        const int col = g.skel[e % k] - h * c;
        ah[e] = (col >= 0 && col < c) ? Sh[(e / k) * c + col] : mk<float>(0, 0);
      }
      c32* Gh = Gb + (h ? (long)c * nh[0] : 0L);
      const int* rh = g.rest + (h ? nh[0] : 0);
      for (long e = threadIdx.x; e < (long)c * nh[h]; e += blockDim.x)
        Gh[e] = Sh[(e / nh[h]) * c + rh[e % nh[h]] - h * c];
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h)
      if (nh[h] > 0)
        gemm_all_tiles(gp(c, k, nh[h], 1, Gb + (h ? (long)c * nh[0] : 0L), nh[h], 0, OP_N,
                          g.Ur + (h ? (long)nh[0] * k : 0L), k, 0, OP_N, 1, a + h * ck, k, 0, a + h * ck, k, 0, 0),
                       0);
    gemm_all_tiles(gp(r, k, c, 1, Lt, c, 0, OP_N, a, k, 0, OP_N, 0, nullptr, 0, 0, q, k, 0, 0), 0);
    gemm_all_tiles(gp(r, k, c, 1, Rt, c, 0, OP_N, a + ck, k, 0, OP_N, 0, nullptr, 0, 0, q + rk, k, 0, 0), 0);
    gemm_all_tiles(gp(2 * r, k, 2 * r, 1, W, r2, 0, OP_N, q, k, 0, OP_N, 0, nullptr, 0, 0, y, k, 0, 0), 0);
    gemm_all_tiles(gp(c, k, r, -1, Pst, r, 0, OP_N, y, k, 0, OP_N, 1, a, k, 0, a, k, 0, 0), 0);
    gemm_all_tiles(gp(c, k, r, -1, Pst + cr, r, 0, OP_N, y + rk, k, 0, OP_N, 1, a + ck, k, 0, a + ck, k, 0, 0), 0);
    c32* S = g.S + t * (long)k * k;
    // S: the skeleton rows of a placed; a_h[rest_h, :] gathered; then T_h^T of them added
    for (long e = threadIdx.x; e < (long)k * k; e += blockDim.x) S[e] = a[(long)g.skel[e / k] * k + e % k];
    for (long e = threadIdx.x; e < (long)nr * k; e += blockDim.x) Rb[e] = a[(long)g.rest[e / k] * k + e % k];
    __syncthreads();
    for (int h = 0; h < 2; ++h)
      if (nh[h] > 0)
        gemm_all_tiles(gp(k, k, nh[h], 1, g.Ur + (h ? (long)nh[0] * k : 0L), k, 0, OP_T,
                          Rb + (h ? (long)nh[0] * k : 0L), k, 0, OP_N, 1, S, k, 0, S, k, 0, 0),
                       0);
  }
}

bool merge_level_fits(int r) { return r >= 1 && small_inv_lds<float>(r) <= 65536; }

size_t merge_level_table_bytes(size_t levels) { return mem::round_up(sizeof(MergeLevelDev) * (levels ? levels : 1)); }

void merge_levels(hipStream_t s, const std::vector<MergeLevelDev>& levels, DevBuf& table, int* counter) {
  std::vector<MergeLevelDev> h;
  long total = 0;
  int rmax = 1;
  double flops = 0;
  for (MergeLevelDev g : levels) {
    LSH_REQUIRE(merge_level_fits(g.r), -6, "merge_levels: inverse order beyond the in-LDS form");
    g.item0 = total;
    total += g.nb;
    rmax = g.r > rmax ? g.r : rmax;
    const double c = g.c, r = g.r, k = g.k;
    const double nr = g.n0 + g.n1;
    flops += 8.0 * g.nb * (2 * c * r * c + 2 * r * r * c + 4 * r * r * r +
                           (g.U ? c * k * nr + 2 * r * k * c + 4 * r * r * k + 2 * c * k * r + k * k * nr : 0));
    h.push_back(g);
  }
  if (h.empty()) return;
  if (table.bytes < sizeof(MergeLevelDev) * h.size()) table.alloc(sizeof(MergeLevelDev) * h.size());
  LSH_HIP(hipMemcpyAsync(table.p, h.data(), sizeof(MergeLevelDev) * h.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, counter, 1L);
  LSH_LAUNCH_CHECK();
  int dev = 0, ncu = 0;
  LSH_HIP(hipGetDevice(&dev));
  LSH_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const size_t lds = small_inv_lds<float>(rmax);
  const long grid = std::min<long>(total, (long)ncu * (lds <= 16384 ? 3 : lds <= 40960 ? 2 : 1));
  ProfScope ps("merge_level_f32", s, flops);
  hipLaunchKernelGGL(k_merge_level, dim3((unsigned)grid), dim3(256), lds, s, table.as<MergeLevelDev>(),
                     (int)h.size(), total, counter);
  LSH_LAUNCH_CHECK();
}

// dst[b][i][j] = src[b][i][j] for rows x cols blocks with their own leading
// dimensions and batch strides
template <typename R>
__global__ void k_ccopy2d(int rows, int cols, const cplx<R>* __restrict__ src, long lds, long ss, cplx<R>* dst,
                          long ldd, long sd, long total) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long b = e / ((long)rows * cols), q = e - b * rows * cols;
    const long i = q / cols, j = q - i * cols;
    dst[b * sd + i * ldd + j] = src[b * ss + i * lds + j];
  }
}

template <typename R>
void ccopy2d(hipStream_t s, int rows, int cols, const cplx<R>* src, long lds, long ss, cplx<R>* dst, long ldd,
             long sd, long batch) {
  const long total = (long)rows * cols * batch;
  if (total <= 0) return;
  const long g = std::min<long>(ceil_div(total, 256L), 65536L);
  hipLaunchKernelGGL(k_ccopy2d<R>, dim3((unsigned)g), dim3(256), 0, s, rows, cols, src, lds, ss, dst, ldd, sd, total);
  LSH_LAUNCH_CHECK();
}

// dst[b][i][j] = src[b][i][idx[j] - off] where 0 <= idx[j] - off < lim, else 0
template <typename R>
__global__ void k_gather_cols(int rows, int cols, const cplx<R>* __restrict__ src, long lds, long ss,
                              const int* __restrict__ idx, int off, int lim, cplx<R>* dst, long ldd, long sd,
                              long total) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long b = e / ((long)rows * cols), q = e - b * rows * cols;
    const long i = q / cols, j = q - i * cols;
    const int col = idx[j] - off;
    dst[b * sd + i * ldd + j] = (col >= 0 && col < lim) ? src[b * ss + i * lds + col] : mk<R>(0, 0);
  }
}

template <typename R>
void gather_cols(hipStream_t s, int rows, int cols, const cplx<R>* src, long lds, long ss, const int* idx, int off,
                 int lim, cplx<R>* dst, long ldd, long sd, long batch) {
  const long total = (long)rows * cols * batch;
  if (total <= 0) return;
  const long g = std::min<long>(ceil_div(total, 256L), 65536L);
  hipLaunchKernelGGL(k_gather_cols<R>, dim3((unsigned)g), dim3(256), 0, s, rows, cols, src, lds, ss, idx, off, lim,
                     dst, ldd, sd, total);
  LSH_LAUNCH_CHECK();
}

// dst[b][i][j] = row t = idx[i] - off of [src0[b]; src1[b]] (rows t < c of
// src0, the others row t - c of src1), column j
template <typename R>
__global__ void k_gather_rows2(int rows, int cols, const cplx<R>* __restrict__ src0, const cplx<R>* __restrict__ src1,
                               int c, long lds, long ss, const int* __restrict__ idx, int off, cplx<R>* dst,
                               long ldd, long sd, long total) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long b = e / ((long)rows * cols), q = e - b * rows * cols;
    const long i = q / cols, j = q - i * cols;
    const int t = idx[i] - off;
    const cplx<R>* src = t < c ? src0 + b * ss + (long)t * lds : src1 + b * ss + (long)(t - c) * lds;
    dst[b * sd + i * ldd + j] = src[j];
  }
}

template <typename R>
void gather_rows2(hipStream_t s, int rows, int cols, const cplx<R>* src0, const cplx<R>* src1, int c, long lds,
                  long ss, const int* idx, int off, cplx<R>* dst, long ldd, long sd, long batch) {
  const long total = (long)rows * cols * batch;
  if (total <= 0) return;
  const long g = std::min<long>(ceil_div(total, 256L), 65536L);
  hipLaunchKernelGGL(k_gather_rows2<R>, dim3((unsigned)g), dim3(256), 0, s, rows, cols, src0, src1, c, lds, ss, idx,
                     off, dst, ldd, sd, total);
  LSH_LAUNCH_CHECK();
}

// Many gathers of FP32 blocks in one launch: grid row y takes job y (the
// elements of gather_cols when its kind is 0, of gather_rows2 when 1, with
// the same arguments), grid columns stride over the job's elements.
__global__ __launch_bounds__(256) void k_gather_grouped(const GatherJob* __restrict__ J) {
  const GatherJob& g = J[blockIdx.y];
  const long per = (long)g.rows * g.cols, total = per * g.batch;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long b = e / per, q = e - b * per;
    const long i = q / g.cols, j = q - i * g.cols;
    c32 v;
    if (g.kind == 0) {
      const int col = g.idx[j] - g.off;
      v = (col >= 0 && col < g.c) ? g.src0[b * g.ss + i * g.lds + col] : mk<float>(0, 0);
    } else {
      const int t = g.idx[i] - g.off;
      v = t < g.c ? g.src0[b * g.ss + (long)t * g.lds + j] : g.src1[b * g.ss + (long)(t - g.c) * g.lds + j];
    }
    g.dst[b * g.sd + i * g.ldd + j] = v;
  }
}

void gather_grouped(hipStream_t s, const std::vector<GatherJob>& jobs, DevBuf& dev) {
  std::vector<GatherJob> h;
  long most = 0;
  for (GatherJob g : jobs) {
    const long n = (long)g.rows * g.cols * g.batch;
    if (n <= 0) continue;
    most = std::max(most, n);
    h.push_back(g);
  }
  if (h.empty()) return;
  LSH_REQUIRE(h.size() <= 65535, -6, "gather_grouped: too many jobs");
  const size_t bytes = sizeof(GatherJob) * h.size();
  if (dev.bytes < bytes) dev.alloc(bytes);
  LSH_HIP(hipMemcpyAsync(dev.p, h.data(), bytes, hipMemcpyHostToDevice, s));
  const long gx = std::min<long>(ceil_div(most, 256L), 1024L);
  hipLaunchKernelGGL(k_gather_grouped, dim3((unsigned)gx, (unsigned)h.size()), dim3(256), 0, s,
                     dev.as<GatherJob>());
  LSH_LAUNCH_CHECK();
  // (pageable copies are staged before hipMemcpyAsync returns: h may go now)
}

// Y[v][i] = alpha X[v][i] + beta Z[v][i] for i < n, v < nv (Z may be null)
template <typename R>
__global__ void k_caxpby(int n, int nv, cplx<R> alpha, const cplx<R>* __restrict__ X, long ldx, cplx<R> beta,
                         const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * nv) return;
  const long v = e / n, i = e - v * n;
  cplx<R> o = alpha * X[v * ldx + i];
  if (Z) o = o + beta * Z[v * ldz + i];
  Y[v * ldy + i] = o;
}

template <typename R>
void caxpby(hipStream_t s, int n, int nv, cplx<R> alpha, const cplx<R>* X, long ldx, cplx<R> beta, const cplx<R>* Z,
            long ldz, cplx<R>* Y, long ldy) {
  const long total = (long)n * nv;
  if (total <= 0) return;
  if (beta.x == R(0) && beta.y == R(0)) Z = nullptr;
  hipLaunchKernelGGL(k_caxpby<R>, dim3((unsigned)ceil_div(total, 256L)), dim3(256), 0, s, n, nv, alpha, X, ldx, beta,
                     Z, ldz, Y, ldy);
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
                         long, long, Op, cplx<R>, const cplx<R>*, long, long, cplx<R>*, long, long, int, bool, \
                         const int*, bool);                                                                \
  template void cgemv<R>(hipStream_t, int, int, cplx<R>, const cplx<R>*, long, long, int, const cplx<R>*, long, \
                         cplx<R>, const cplx<R>*, long, cplx<R>*, long, int);                               \
  template void cmgemv<R>(hipStream_t, int, int, cplx<R>, const cplx<R>*, long, const cplx<R>*, long, cplx<R>, \
                          const cplx<R>*, long, cplx<R>*, long, int);                                        \
  template void ctranspose<R>(hipStream_t, const cplx<R>*, int, int, cplx<R>*, long);                       \
  template void cgemm_ws<R>(hipStream_t, int, int, int, cplx<R>, const cplx<R>*, long, long, Op,              \
                            const cplx<R>*, long, long, Op, cplx<R>, const cplx<R>*, long, long, cplx<R>*,   \
                            long, long, int, void*, size_t);                                                 \
  template void cmgemv2<R>(hipStream_t, int, int, long, int, cplx<R>, const cplx<R>*, long, const cplx<R>*,   \
                           long, cplx<R>, const cplx<R>*, long, cplx<R>*, long, int, const cplx<R>*);                        \
  template void ccopy2d<R>(hipStream_t, int, int, const cplx<R>*, long, long, cplx<R>*, long, long, long);   \
  template void gather_cols<R>(hipStream_t, int, int, const cplx<R>*, long, long, const int*, int, int,      \
                               cplx<R>*, long, long, long);                                                  \
  template void gather_rows2<R>(hipStream_t, int, int, const cplx<R>*, const cplx<R>*, int, long, long,      \
                                const int*, int, cplx<R>*, long, long, long);                                \
  template void caxpby<R>(hipStream_t, int, int, cplx<R>, const cplx<R>*, long, cplx<R>, const cplx<R>*, long,  \
                          cplx<R>*, long);                                                                  \
  template size_t inverse_ws_bytes<R>(int, int);                                                           \
  template void inverse<R>(hipStream_t, cplx<R>*, int, long, long, int, void*, int*);
LSH_INST(float)
LSH_INST(double)
template void ccast<double, float>(hipStream_t, const cplx<double>*, cplx<float>*, long);
template void ccast<float, double>(hipStream_t, const cplx<float>*, cplx<double>*, long);
template void ccast<double, double>(hipStream_t, const cplx<double>*, cplx<double>*, long);

}  // namespace lsh
