// FFT convolution operator (paper Sec. 2.2 end and Sec. 5: G + T is a
// convolution on the regular grid, applied by FFT), kernel-entry generator
// and FGMRES vector kernels.  All FP64.
#include <cmath>

#include "ops.hpp"
#include "prof.hpp"

namespace lsh {

// ------------------------------------------------------------ offset table
__global__ void k_offset_table(z64* T, int D, double h, double kappa, double t0r, double t0i) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long W = D + 1;
  if (e >= W * W) return;
  const int dy = (int)(e / W), dx = (int)(e % W);
  z64 v;
  if (dx == 0 && dy == 0) {
    v = mk(t0r, t0i);
  } else {
    const double r = kappa * h * sqrt((double)dx * dx + (double)dy * dy);
    // (i/4) H0(r) = (i/4)(J0 + i Y0) = -Y0/4 + i J0/4
    v = mk(-0.25 * y0(r), 0.25 * j0(r));
  }
  T[e] = (h * h) * v;
}

void build_offset_table(hipStream_t s, z64* T, int D, double h, double kappa, double tau0_re, double tau0_im) {
  const long W = D + 1;
  hipLaunchKernelGGL(k_offset_table, dim3(ceil_div(W * W, 256)), dim3(256), 0, s, T, D, h, kappa, tau0_re,
                     tau0_im);
  LSH_LAUNCH_CHECK();
}

__global__ void k_table_add(z64* T, int D, const int* dxy, const z64* w, int cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  const int dx = dxy[2 * k], dy = dxy[2 * k + 1];
  T[(long)dy * (D + 1) + dx] = T[(long)dy * (D + 1) + dx] + w[k];
}

void add_table_stencil(hipStream_t s, z64* T, int D, double h, const std::vector<StencilEntry>& stencil,
                       mem::Arena& scr) {
  std::vector<int> dxy;
  std::vector<z64> wv;
  for (auto& e : stencil) {  // one representative per offset (|dx|, |dy|): the stencil is symmetric
    if (e.dx < 0 || e.dy < 0 || (e.dx == 0 && e.dy == 0) || e.dx > D || e.dy > D) continue;
    dxy.push_back(e.dx);
    dxy.push_back(e.dy);
    wv.push_back(mk(h * h * e.re, h * h * e.im));
  }
  if (wv.empty()) return;
  int* ddxy = static_cast<int*>(scr.take(sizeof(int) * dxy.size()));
  z64* dw = static_cast<z64*>(scr.take(sizeof(z64) * wv.size()));
  LSH_HIP(hipMemcpyAsync(ddxy, dxy.data(), sizeof(int) * dxy.size(), hipMemcpyHostToDevice, s));
  LSH_HIP(hipMemcpyAsync(dw, wv.data(), sizeof(z64) * wv.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_table_add, dim3(ceil_div((int)wv.size(), 64)), dim3(64), 0, s, T, D, ddxy, dw,
                     (int)wv.size());
  LSH_LAUNCH_CHECK();
  LSH_HIP(hipStreamSynchronize(s));  // the host staging vectors die here
}

// ------------------------------------------------------------------- FFT
void FFTPlan::init(int M_, hipStream_t s) {
  M = M_;
  logM = 0;
  while ((1 << logM) < M) ++logM;
  LSH_REQUIRE((1 << logM) == M && M >= 2 && M <= 4096, -6, "FFT length must be a power of two <= 4096");
  std::vector<z64> h(M);
  for (int k = 0; k < M; ++k) {
    long double a = -2.0L * 3.141592653589793238462643383279502884L * k / M;
    h[k] = mk((double)std::cos(a), (double)std::sin(a));
  }
  tw.alloc(sizeof(z64) * h.size());
  // on the caller's stream: a plain hipMemcpy would also wait for every
  // blocking stream of the device (a factorisation running beside the plan)
  LSH_HIP(hipMemcpyAsync(tw.p, h.data(), sizeof(z64) * h.size(), hipMemcpyHostToDevice, s));
  LSH_HIP(hipStreamSynchronize(s));  // h dies here
}

// In-place radix-2 decimation-in-time transform of x (bit-reversed input).
__device__ __forceinline__ void fft_lds(z64* x, int M, int logM, const z64* __restrict__ W, bool inv) {
  for (int st = 0; st < logM; ++st) {
    const int half = 1 << st;
    const int ts = M >> (st + 1);
    for (int bf = threadIdx.x; bf < (M >> 1); bf += blockDim.x) {
      const int pos = bf & (half - 1);
      const int i = ((bf >> st) << (st + 1)) + pos, j = i + half;
      z64 w = W[pos * ts];
      if (inv) w.y = -w.y;
      const z64 t = w * x[j];
      const z64 u = x[i];
      x[i] = u + t;
      x[j] = u - t;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int i, int logM) { return (int)(__brev((unsigned)i) >> (32 - logM)); }

// mode 0: plain rows; mode 1: multiply by spectrum row then inverse transform;
// mode 2: epilogue y = x + kb2 * b * v; mode 4: epilogue y = x + v.
// preb (optional): the input row is scaled by prek * preb on load.
__global__ __launch_bounds__(256) void k_fft_rows(const z64* __restrict__ in, long ldin, int nin, z64* out,
                                                  long ldout, int nout, int M, int logM,
                                                  const z64* __restrict__ W, int inv, int mode,
                                                  const z64* __restrict__ spec, long ldspec,
                                                  const z64* __restrict__ xadd, const double* __restrict__ b,
                                                  double kb2, const double* __restrict__ preb, double prek) {
  extern __shared__ unsigned char smem_raw[];
  z64* x = reinterpret_cast<z64*>(smem_raw);
  const long r = blockIdx.x;
  const z64* src = in + r * ldin;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    z64 v = i < nin ? src[i] : mk(0.0, 0.0);
    if (preb && i < nin) v = (prek * preb[r * ldin + i]) * v;
    x[bitrev(i, logM)] = v;
  }
  __syncthreads();
  fft_lds(x, M, logM, W, inv != 0);
  if (mode == 1) {  // spectrum row min(r, M - r), entry min(i, M - i)
    const z64* sp = spec + (r <= M - r ? r : M - r) * ldspec;
    for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = x[i] * sp[i <= M - i ? i : M - i];
    __syncthreads();
    // back to bit-reversed order for the inverse transform
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
      const int j = bitrev(i, logM);
      if (i < j) { z64 t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    __syncthreads();
    fft_lds(x, M, logM, W, true);
  }
  z64* dst = out + r * ldout;
  if (mode == 2) {
    for (int i = threadIdx.x; i < nout; i += blockDim.x) {
      const long g = r * ldout + i;
      dst[i] = xadd[g] + (kb2 * b[g]) * x[i];
    }
  } else if (mode == 4) {
    for (int i = threadIdx.x; i < nout; i += blockDim.x) dst[i] = xadd[r * ldout + i] + x[i];
  } else {
    for (int i = threadIdx.x; i < nout; i += blockDim.x) dst[i] = x[i];
  }
}

// ---------------------------------------------- Stockham FFT in registers
// Length M = 2^LOGM >= 64: T = M / 16 threads per row, each holding 16
// values.  Passes of radix 16 (a last one of radix 2, 4 or 8 when LOGM is not
// a multiple of 4) in Stockham's self-sorting form: with NS the product of the
// earlier radices, butterfly j (< M / R) takes x[j + r M / R] (r < R),
// multiplies entry r by w_M^(r (j mod NS) M / (NS R)), transforms the R values
// in registers and puts entry r at (j / NS) NS R + (j mod NS) + r NS.  Input
// and output are in natural order, so the first pass reads global memory and
// the last writes it, coalesced, and only the exchanges between passes go
// through LDS (one padded slot per 16 values keeps the radix-16 writes free
// of bank conflicts).  Thread t runs butterflies t + T q, q < 16 / R.
namespace fft16 {

constexpr double kC[8] = {1.0,
                          0.92387953251128675613,
                          0.70710678118654752440,
                          0.38268343236508977173,
                          0.0,
                          -0.38268343236508977173,
                          -0.70710678118654752440,
                          -0.92387953251128675613};  // cos(2 pi p / 16)
constexpr double kS[8] = {0.0,
                          0.38268343236508977173,
                          0.70710678118654752440,
                          0.92387953251128675613,
                          1.0,
                          0.92387953251128675613,
                          0.70710678118654752440,
                          0.38268343236508977173};  // sin(2 pi p / 16)

constexpr int brev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}
constexpr int lg(int R) { return R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4; }

// a * w_16^p (forward: w = exp(-2 pi i / 16); inverse: its conjugate)
template <int P, bool INV>
__device__ __forceinline__ z64 rot16(z64 a) {
  if (P == 0) return a;
  if (P == 4) return INV ? mk(-a.y, a.x) : mk(a.y, -a.x);
  const double c = kC[P], sn = INV ? kS[P] : -kS[P];
  return mk(a.x * c - a.y * sn, a.x * sn + a.y * c);
}

// In-register DFT of v[OFF .. OFF + R): out[k] = sum_r v[r] w_R^(r k), by
// radix-2 decimation in time (bit-reversed loads, natural-order result).
template <int R, bool INV, int OFF>
__device__ __forceinline__ void dft(z64 (&v)[16]) {
  constexpr int B = lg(R);
  z64 a[R];
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = v[OFF + brev(i, B)];
#pragma unroll
  for (int half = 1; half < R; half <<= 1)
#pragma unroll
    for (int i = 0; i < R; i += 2 * half)
#pragma unroll
      for (int p = 0; p < half; ++p) {
        const int e = p * (16 / (2 * half));
        z64 t;
        switch (e) {  // compile-time after unrolling
          case 0: t = rot16<0, INV>(a[i + p + half]); break;
          case 1: t = rot16<1, INV>(a[i + p + half]); break;
          case 2: t = rot16<2, INV>(a[i + p + half]); break;
          case 3: t = rot16<3, INV>(a[i + p + half]); break;
          case 4: t = rot16<4, INV>(a[i + p + half]); break;
          case 5: t = rot16<5, INV>(a[i + p + half]); break;
          case 6: t = rot16<6, INV>(a[i + p + half]); break;
          default: t = rot16<7, INV>(a[i + p + half]); break;
        }
        const z64 u = a[i + p];
        a[i + p] = u + t;
        a[i + p + half] = u - t;
      }
#pragma unroll
  for (int i = 0; i < R; ++i) v[OFF + i] = a[i];
}

template <int R, bool INV, int Q = 0>
__device__ __forceinline__ void dft_all(z64 (&v)[16]) {
  if constexpr (Q < 16 / R) {
    dft<R, INV, Q * R>(v);
    dft_all<R, INV, Q + 1>(v);
  }
}

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// twiddles of pass (R, NS) for thread t: w[q R + r] = w_M^(r (j mod NS) M / (NS R))
template <int M, int R, int NS, bool INV>
__device__ __forceinline__ void load_tw(z64 (&w)[16], int t, const z64* __restrict__ W) {
  constexpr int T = M / 16, S = M / (NS * R);
#pragma unroll
  for (int q = 0; q < 16 / R; ++q) {
    const int jm = (t + T * q) & (NS - 1);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      z64 x = W[r * jm * S];
      if (INV) x.y = -x.y;
      w[q * R + r] = x;
    }
  }
}

// passes from NS on; v holds the inputs of pass (R, NS) for thread t and w
// its twiddles (loaded before the exchange that filled v, so that their
// latency overlaps it)
template <int M, int NS, bool INV>
__device__ __forceinline__ void passes(z64 (&v)[16], z64 (&w)[16], z64* L, int t, const z64* __restrict__ W) {
  constexpr int T = M / 16, R = (M / NS >= 16) ? 16 : M / NS;
  if constexpr (NS > 1) {
#pragma unroll
    for (int q = 0; q < 16 / R; ++q)
#pragma unroll
      for (int r = 1; r < R; ++r) v[q * R + r] = v[q * R + r] * w[q * R + r];
  }
  dft_all<R, INV>(v);
  if constexpr (NS * R < M) {
    constexpr int R2 = (M / (NS * R) >= 16) ? 16 : M / (NS * R);
    load_tw<M, R2, NS * R, INV>(w, t, W);
    __syncthreads();  // every read of L by the previous exchange is done
#pragma unroll
    for (int q = 0; q < 16 / R; ++q) {
      const int j = t + T * q, base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) L[lpad(base + r * NS)] = v[q * R + r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16 / R2; ++q)
#pragma unroll
      for (int r = 0; r < R2; ++r) v[q * R2 + r] = L[lpad(t + T * q + r * (M / R2))];
    passes<M, NS * R, INV>(v, w, L, t, W);
  }
}

// radix and stride of the last pass: thread t ends holding, for q < 16 / RL
// and r < RL, v[q RL + r] = X[t + T q + r M / RL]
template <int M>
struct Last {
  static constexpr int RL = (M & 0x1111) ? 16 : (M & 0x2222) ? 2 : (M & 0x4444) ? 4 : 8;
  static constexpr int NSL = M / RL;
};

}  // namespace fft16

// Same arguments and modes as k_fft_rows; rows = ceil(grid / ...) handled by
// ROWS rows per workgroup for short lengths.
template <int LOGM>
__global__ __launch_bounds__(256) void k_fft16_rows(const z64* __restrict__ in, long ldin, int nin, z64* out,
                                                    long ldout, int nout, int nrows, const z64* __restrict__ W,
                                                    int inv, int mode, const z64* __restrict__ spec, long ldspec,
                                                    const z64* __restrict__ xadd, const double* __restrict__ b,
                                                    double kb2, const double* __restrict__ preb, double prek) {
  using namespace fft16;
  constexpr int M = 1 << LOGM, T = M / 16, ROWS = T >= 64 ? 1 : 64 / T, LR = M + M / 16;
  constexpr int RL = Last<M>::RL, NSL = Last<M>::NSL;
  extern __shared__ unsigned char smem_raw[];
  const int rw = threadIdx.x / T, t = threadIdx.x % T;
  const long r = (long)blockIdx.x * ROWS + rw;
  const bool ok = r < nrows;
  z64* L = reinterpret_cast<z64*>(smem_raw) + rw * LR;
  z64 v[16];
  {
    const z64* src = in + r * ldin;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int k = t + i * T;
      z64 x = mk(0.0, 0.0);
      if (ok && k < nin) {
        x = src[k];
        if (preb) x = (prek * preb[r * ldin + k]) * x;
      }
      v[i] = x;
    }
  }
  z64 w[16];
  if (inv) passes<M, 1, true>(v, w, L, t, W);
  else passes<M, 1, false>(v, w, L, t, W);
  if (mode == 1) {  // times the spectrum row (min(r, M - r), entry min(k, M - k)), then the inverse transform
    const z64* sp = spec + (r <= M - r ? r : M - r) * ldspec;
#pragma unroll
    for (int q = 0; q < 16 / RL; ++q)
#pragma unroll
      for (int e = 0; e < RL; ++e) {
        const int k = t + T * q + e * NSL;
        if (ok) v[q * RL + e] = v[q * RL + e] * sp[k <= M - k ? k : M - k];
      }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16 / RL; ++q)
#pragma unroll
      for (int e = 0; e < RL; ++e) L[lpad(t + T * q + e * NSL)] = v[q * RL + e];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = L[lpad(t + i * T)];
    passes<M, 1, true>(v, w, L, t, W);
  }
  if (!ok) return;
  z64* dst = out + r * ldout;
#pragma unroll
  for (int q = 0; q < 16 / RL; ++q)
#pragma unroll
    for (int e = 0; e < RL; ++e) {
      const int k = t + T * q + e * NSL;
      if (k >= nout) continue;
      const z64 x = v[q * RL + e];
      if (mode == 2) {
        const long g = r * ldout + k;
        dst[k] = xadd[g] + (kb2 * b[g]) * x;
      } else if (mode == 4) {
        dst[k] = xadd[r * ldout + k] + x;
      } else {
        dst[k] = x;
      }
    }
}

// One launch of the row transform (modes as k_fft_rows) on nrows rows.
static void launch_fft_rows(hipStream_t s, const FFTPlan& P, int nrows, const z64* in, long ldin, int nin, z64* out,
                            long ldout, int nout, int inv, int mode, const z64* spec, long ldspec, const z64* xadd,
                            const double* b, double kb2, const double* preb, double prek) {
  const z64* W = P.tw.as<z64>();
  if (P.logM < 6) {
    hipLaunchKernelGGL(k_fft_rows, dim3(nrows), dim3(256), P.M * sizeof(z64), s, in, ldin, nin, out, ldout, nout,
                       P.M, P.logM, W, inv, mode, spec, ldspec, xadd, b, kb2, preb, prek);
    LSH_LAUNCH_CHECK();
    return;
  }
  const int T = P.M / 16, rows = T >= 64 ? 1 : 64 / T;
  const size_t lds = sizeof(z64) * (size_t)rows * (P.M + P.M / 16);
  const dim3 grid(ceil_div(nrows, rows)), block(rows * T);
#define LSH_FFT16(LG)                                                                                         \
  case LG:                                                                                                    \
    hipLaunchKernelGGL(k_fft16_rows<LG>, grid, block, lds, s, in, ldin, nin, out, ldout, nout, nrows, W, inv, \
                       mode, spec, ldspec, xadd, b, kb2, preb, prek);                                         \
    break;
  if (P.logM == 12) {  // 68 KB of LDS (above the 64 KB default of a launch)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft16_rows<12>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    LSH_HIP(attr);
  }
  switch (P.logM) {
    LSH_FFT16(6)
    LSH_FFT16(7)
    LSH_FFT16(8)
    LSH_FFT16(9)
    LSH_FFT16(10)
    LSH_FFT16(11)
    LSH_FFT16(12)
    default: LSH_REQUIRE(false, -6, "FFT length must be a power of two <= 4096");
  }
#undef LSH_FFT16
  LSH_LAUNCH_CHECK();
}

void fft_rows(hipStream_t s, const FFTPlan& P, const z64* in, long ldin, int nin, z64* out, long ldout, int nout,
              int nrows, bool inverse) {
  launch_fft_rows(s, P, nrows, in, ldin, nin, out, ldout, nout, inverse ? 1 : 0, 0, nullptr, 0L, nullptr, nullptr,
                  0.0, nullptr, 0.0);
}

constexpr int TT = 32;
__global__ __launch_bounds__(256) void k_transpose(const z64* __restrict__ in, long ldin, z64* __restrict__ out,
                                                   long ldout, int rows, int cols) {
  __shared__ z64 tile[TT][TT + 1];
  const int c0 = blockIdx.x * TT, r0 = blockIdx.y * TT;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < TT; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = in[(long)r * ldin + c];
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) out[(long)c * ldout + r] = tile[tx][k];
  }
}

void transpose_z(hipStream_t s, const z64* in, long ldin, z64* out, long ldout, int rows, int cols) {
  dim3 grid(ceil_div(cols, TT), ceil_div(rows, TT));
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, in, ldin, out, ldout, rows, cols);
  LSH_LAUNCH_CHECK();
}

// C[dy mod M][dx mod M] = h^2 (G(h|d|)[d != 0] + tau_d) for |dx|, |dy| < n
__global__ void k_fill_circulant(z64* C, int M, int n, const z64* __restrict__ T, int D) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)M * M) return;
  const int iy = (int)(e / M), ix = (int)(e % M);
  const int dy = iy < n ? iy : iy - M, dx = ix < n ? ix : ix - M;
  z64 v = mk(0.0, 0.0);
  const int ady = dy < 0 ? -dy : dy, adx = dx < 0 ? -dx : dx;
  if (ady < n && adx < n && ady <= D && adx <= D && !(dx == 0 && dy == 0)) v = T[(long)ady * (D + 1) + adx];
  C[e] = v;
}

__global__ void k_add_stencil(z64* C, int M, const int* dxy, const z64* w, int cnt) {
  const int k = threadIdx.x;
  if (k >= cnt) return;
  const int dx = dxy[2 * k], dy = dxy[2 * k + 1];
  const int ix = (dx + M) % M, iy = (dy + M) % M;
  C[(long)iy * M + ix] = C[(long)iy * M + ix] + w[k];
}

// khat[a][c] = s Kt[a][c] for a, c <= M / 2 (ld M / 2 + 1)
__global__ void k_spectrum_quarter(const z64* __restrict__ Kt, int M, double s, z64* khat) {
  const int H = M / 2 + 1;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)H * H) return;
  const int a = (int)(e / H), c = (int)(e % H);
  khat[e] = s * Kt[(long)a * M + c];
}

static int pad_len(int n) {
  int M = 1;
  while (M < 2 * n) M <<= 1;
  return M;
}

size_t ConvOperator::bytes(int n) {
  const size_t M = pad_len(n), H = M / 2 + 1;
  mem::Sizer z;
  z.add_n<z64>(M);                 // twiddles
  z.add_n<z64>(H * H);             // khat (one quarter)
  z.add_n<z64>((size_t)n * M);     // w1
  z.add_n<z64>((size_t)n * M);     // w2
  return z.total;
}

size_t ConvOperator::scratch_bytes(int n) {
  const size_t M = pad_len(n);
  return 2 * mem::round_up(sizeof(z64) * 64) + 2 * mem::round_up(sizeof(z64) * M * M);
}

void ConvOperator::init(hipStream_t s, int n_, double h, double kappa_, const z64* table, int D,
                        const std::vector<StencilEntry>& stencil, mem::Arena& scr) {
  n = n_;
  kappa = kappa_;
  M = pad_len(n);
  const int H = M / 2 + 1;
  fft.init(M, s);
  khat.alloc(sizeof(z64) * (size_t)H * H);
  w1.alloc(sizeof(z64) * (size_t)n * M);
  w2.alloc(sizeof(z64) * (size_t)n * M);
  z64* C = static_cast<z64*>(scr.take(sizeof(z64) * (size_t)M * M));
  z64* Kt = static_cast<z64*>(scr.take(sizeof(z64) * (size_t)M * M));
  hipLaunchKernelGGL(k_fill_circulant, dim3(ceil_div((long)M * M, 256)), dim3(256), 0, s, C, M, n, table, D);
  LSH_LAUNCH_CHECK();
  std::vector<int> dxy;
  std::vector<z64> wv;
  for (auto& e : stencil) {
    if (std::abs(e.dx) >= n || std::abs(e.dy) >= n) continue;
    dxy.push_back(e.dx);
    dxy.push_back(e.dy);
    wv.push_back(mk(h * h * e.re, h * h * e.im));
  }
  int* ddxy = static_cast<int*>(scr.take(sizeof(int) * dxy.size()));
  z64* dw = static_cast<z64*>(scr.take(sizeof(z64) * wv.size()));
  LSH_HIP(hipMemcpyAsync(ddxy, dxy.data(), sizeof(int) * dxy.size(), hipMemcpyHostToDevice, s));
  LSH_HIP(hipMemcpyAsync(dw, wv.data(), sizeof(z64) * wv.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_add_stencil, dim3(1), dim3(64), 0, s, C, M, ddxy, dw, (int)wv.size());
  LSH_LAUNCH_CHECK();
  // full 2-D transform, transposed: Kt[k1][k2].  The kernel is even in each
  // offset (G depends on |d|; the correction stencil covers whole symmetry
  // orbits), so its transform is too: Kt[k1][k2] = Kt[M - k1][k2] =
  // Kt[k1][M - k2] up to rounding, and only the quarter k1, k2 <= M / 2 is kept.
  fft_rows(s, fft, C, M, M, C, M, M, M, false);
  transpose_z(s, C, M, Kt, M, M, M);
  fft_rows(s, fft, Kt, M, M, Kt, M, M, M, false);
  hipLaunchKernelGGL(k_spectrum_quarter, dim3(ceil_div((long)H * H, 256)), dim3(256), 0, s, Kt, M,
                     1.0 / ((double)M * M), khat.as<z64>());
  LSH_LAUNCH_CHECK();
  LSH_HIP(hipStreamSynchronize(s));  // the staging and scratch buffers die here
}

void ConvOperator::apply(hipStream_t s, const double* b, const z64* x, z64* y, int nrhs, bool transpose) {
  // algorithmic bytes: read x (and b), write y, read the spectrum quarter once
  const double H = M / 2 + 1;
  ProfScope ps("op_fft_operator", s, (double)nrhs * (16.0 * 2 * n * n + (b ? 8.0 * n * n : 0.0)) + 16.0 * H * H);
  z64* W1 = w1.as<z64>();
  z64* W2 = w2.as<z64>();
  const double k2 = kappa * kappa;
  const z64* nz = nullptr;
  const double* nd = nullptr;
  for (int r = 0; r < nrhs; ++r) {
    const z64* xr = x + (long)r * n * n;
    z64* yr = y + (long)r * n * n;
    // rows (x1 direction) of the n data rows, padded to M (A^T: scaled by kappa^2 b first)
    launch_fft_rows(s, fft, n, xr, (long)n, n, W1, (long)M, M, 0, 0, nz, 0L, nz, nd, 0.0,
                    (transpose && b) ? b : nd, k2);
    transpose_z(s, W1, M, W2, n, n, M);  // W2: M x n
    // columns: transform, multiply by the spectrum, transform back, keep n
    launch_fft_rows(s, fft, M, W2, (long)n, n, W2, (long)n, n, 0, 1, khat.as<z64>(), (long)(M / 2 + 1), nz, nd, 0.0,
                    nd, 0.0);
    transpose_z(s, W2, n, W1, M, M, n);  // W1: n x M
    const int mode = !b ? 3 : (transpose ? 4 : 2);
    launch_fft_rows(s, fft, n, W1, (long)M, M, yr, (long)n, n, 1, mode, nz, 0L, b ? xr : nz, b, k2, nd, 0.0);
  }
}

// --------------------------------------------------------- vector kernels
constexpr int MD_BLOCKS = 1024, MD_NT = 256, MD_MAXV = 128;

__global__ __launch_bounds__(MD_NT) void k_multidot(const z64* __restrict__ V, long ldv, int nv,
                                                    const z64* __restrict__ w, long N, z64* partial) {
  __shared__ z64 red[MD_MAXV][MD_NT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = 0; v < nv; ++v) {
    const z64* Vv = V + v * ldv;
    z64 acc = mk(0.0, 0.0);
    for (long i = blockIdx.x * (long)MD_NT + threadIdx.x; i < N; i += (long)MD_BLOCKS * MD_NT)
      fma_acc(acc, conjg(Vv[i]), w[i]);
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if (lane == 0) red[v][wave] = acc;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += MD_NT) {
    z64 a = red[v][0];
    for (int k = 1; k < MD_NT / 64; ++k) a = a + red[v][k];
    partial[(long)v * MD_BLOCKS + blockIdx.x] = a;
  }
}

__global__ __launch_bounds__(256) void k_reduce_partials(const z64* partial, int nparts, z64* out) {
  __shared__ z64 red[256];
  const int v = blockIdx.x;
  z64 a = mk(0.0, 0.0);
  for (int k = threadIdx.x; k < nparts; k += 256) a = a + partial[(long)v * nparts + k];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = red[0];
}

size_t multidot_partial_bytes(int nv) { return sizeof(z64) * (size_t)nv * MD_BLOCKS; }

void multidot(hipStream_t s, const z64* V, long ldv, int nv, const z64* w, long N, z64* out, z64* partial) {
  ProfScope ps("op_multidot", s, 16.0 * (double)N * (nv + 1));
  LSH_REQUIRE(nv <= MD_MAXV, -6, "multidot: too many vectors");
  hipLaunchKernelGGL(k_multidot, dim3(MD_BLOCKS), dim3(MD_NT), 0, s, V, ldv, nv, w, N, partial);
  LSH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_partials, dim3(nv), dim3(256), 0, s, partial, MD_BLOCKS, out);
  LSH_LAUNCH_CHECK();
}

__global__ void k_multiaxpy(z64* w, const z64* __restrict__ V, long ldv, int nv, const z64* __restrict__ h, long N) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    z64 a = w[i];
    for (int v = 0; v < nv; ++v) a = a - V[v * ldv + i] * h[v];
    w[i] = a;
  }
}

void multiaxpy(hipStream_t s, z64* w, const z64* V, long ldv, int nv, const z64* h, long N) {
  ProfScope ps("multiaxpy", s, 16.0 * (double)N * (nv + 2));
  hipLaunchKernelGGL(k_multiaxpy, dim3(2048), dim3(256), 0, s, w, V, ldv, nv, h, N);
  LSH_LAUNCH_CHECK();
}

__global__ void k_scale_invnorm(z64* y, const z64* x, const z64* nrm2, long N) {
  const double s = 1.0 / sqrt(nrm2[0].x);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    y[i] = s * x[i];
}

void scale_by_invnorm(hipStream_t s, z64* y, const z64* x, const z64* nrm2, long N) {
  hipLaunchKernelGGL(k_scale_invnorm, dim3(2048), dim3(256), 0, s, y, x, nrm2, N);
  LSH_LAUNCH_CHECK();
}

__global__ void k_lincomb(z64* y, const z64* __restrict__ V, long ldv, int nv, const z64* __restrict__ c, long N) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    z64 a = mk(0.0, 0.0);
    for (int v = 0; v < nv; ++v) fma_acc(a, V[v * ldv + i], c[v]);
    y[i] = a;
  }
}

void lincomb(hipStream_t s, z64* y, const z64* V, long ldv, int nv, const z64* c, long N) {
  hipLaunchKernelGGL(k_lincomb, dim3(2048), dim3(256), 0, s, y, V, ldv, nv, c, N);
  LSH_LAUNCH_CHECK();
}

__global__ void k_scale_real(z64* y, const z64* x, const double* b, double a, long N, long nb) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    y[i] = (a * b[i % nb]) * x[i];
}

void scale_real(hipStream_t s, z64* y, const z64* x, const double* b, double a, long N) {
  hipLaunchKernelGGL(k_scale_real, dim3(2048), dim3(256), 0, s, y, x, b, a, N, N);
  LSH_LAUNCH_CHECK();
}

__global__ void k_sub_from(z64* y, const z64* x, long N) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    y[i] = x[i] - y[i];
}

void sub_from(hipStream_t s, z64* y, const z64* x, long N) {
  hipLaunchKernelGGL(k_sub_from, dim3(2048), dim3(256), 0, s, y, x, N);
  LSH_LAUNCH_CHECK();
}

__global__ void k_conj(z64* y, const z64* x, long N) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    y[i] = conjg(x[i]);
}

void conj_copy(hipStream_t s, z64* y, const z64* x, long N) {
  hipLaunchKernelGGL(k_conj, dim3(2048), dim3(256), 0, s, y, x, N);
  LSH_LAUNCH_CHECK();
}

__global__ void k_fill_zero(uint32_t* p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0;
}

void fill_zero(hipStream_t s, void* p, size_t bytes) {
  if (!bytes) return;
  LSH_REQUIRE(bytes % 4 == 0, -1, "fill_zero: size must be a multiple of 4");
  long n = (long)(bytes / 4);
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), n);
  LSH_LAUNCH_CHECK();
}

}  // namespace lsh
