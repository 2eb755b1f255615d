// Woodbury levels with at least this many box vectors (lsh_apply_fused_levels;
// 0: never) whose box vectors fit one workgroup's LDS run each apply pass in
// one launch (level_up_fused / level_down_fused) instead of six to seven.
constexpr int kApplyFusedMin = 128;
static int g_apply_fused_min = kApplyFusedMin;

// Host orchestration and the C ABI (include/lsh.h).
//
// plan   : tree (Sec. 3.1-3.2), correction weights (Sec. 2.2), kernel table,
//          per-level row IDs and sibling blocks (Sec. 3.2), FFT spectrum.
// factor : Algorithm 1, with the parent inverse in Schur-complement form
//          X = [[I, Pa],[Pb, I]]^{-1}, Pa = S_a G_ab, Pb = S_b G_ba,
//          C = I - Pb Pa:  X [a; b] = [a - Pa y; y], y = C^{-1} (b - Pb a).
// apply  : Algorithm 2 (up l = L-1..1, root solve, down l = 1..L-1, leaves).
// solve  : right-preconditioned flexible GMRES on the order-p FFT operator.
#include <array>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "../../include/lsh.h"
#include "blas.hpp"
#include "hbs.hpp"
#include "ops.hpp"
#include "plancache.hpp"
#include "prof.hpp"
#include "weights.hpp"

namespace lsh {
namespace prof {
void set(bool enable);
void set_only(const char* prefix);
int query(const char* name, int* launches, double* ms, double* work, double* bytes);
std::string names();
}  // namespace prof
}  // namespace lsh

using namespace lsh;

namespace {

thread_local std::string g_last_error;

struct Level {
  int sx = 0, sy = 0;  // box size
  int m = 0, k = 0;    // candidate rows and rank (levels 1..L)
  std::vector<I2> cand;
  std::vector<int> J;
  std::vector<I2> ra, rb;  // skeleton points of the two children (sibling-block rows / columns)
  DevBuf U64, U32;       // m x k
  DevBuf Ut64, Ut32;     // k x m (transpose, for row-streamed products)
  bool ident = false;    // U = I (k = m): the level keeps all its candidates
  // cand, m, J and k are known (set once: the sibling blocks read them while
  // the interpolation matrix of this level is still being formed)
  bool skel_known = false;
  bool host_ready = false;  // an uncompressed level prepared ahead from its children
  // U is the identity on the skeleton rows J.  For the factor's products
  // with U (levels 1 .. L-1, candidates of half h: h m/2 .. h m/2 + m/2 - 1):
  // the other rows ("rest", ascending; nrest0 of them in half 0), and on the
  // device their indices, J, and T = U[rest, :] ((m - k) x k).
  std::vector<int> rest;
  int nrest0 = 0;
  DevBuf restIdx, skelIdx;
  DevBuf T64, T32;
  DevBuf Gab64, Gab32;   // sibling block of this parent level (c x c, c = k of level+1)
  DevBuf Gabt64, Gabt32; // its transpose
  int c = 0;
  // low-rank form G_ab ~= L R^T (merge by the Woodbury form); wr = 0: Schur form
  int wr = 0;
  std::vector<I2> wrows;  // skeleton points J of G_ab's row ID (upload source)
  DevBuf WU64;            // U of G_ab's row ID (c x r; kept: freeing it mid-build would sync the device)
  DevBuf Pm64, Pm32;      // [L; R] (2c x wr): L = U of the row ID, R = G_ab[J, :]^T
  DevBuf Qm64, Qm32;      // [L^T; R^T] (2 wr x c)
};

}  // namespace

struct lsh_plan_s {
  lsh_desc d{};
  int n = 0, L = 0, ls = 0, mL = 0, D = 0, nleaf = 0;
  double h = 0, kappa = 0;
  std::vector<Level> lev;
  std::vector<I2> leaf_origin_h, leaf_pts_h;
  DevBuf leaf_origin, leaf_pts;
  DevBuf table;   // 4th-order offset table (operator circulant, inspection)
  DevBuf htable;  // offset table of the compressed matrix when hbs_order > 4
  DevBuf Gleaf64, Gleaf32;
  int hbs_order = 4;
  const z64* hbs_table() const { return htable.p ? htable.as<z64>() : table.as<z64>(); }
  // Device memory, all from the caller's plan workspace: persist holds what
  // the plan keeps; sid and ssib hold the temporaries of the level row IDs
  // and of the sibling blocks (the two plan threads of lsh_build), each
  // rewound at the start of its next level, after a stream synchronisation;
  // sgram holds the parent level's Gram rows built during a level's row ID
  // (rewound once they are packed into the parent's row-ID workspace).
  mem::Arena persist, sid, ssib, sgram;
  // side stream for the parent Gram rows while a plan is built (null: the
  // Gram of each level is formed after its candidates are known)
  hipStream_t gs = nullptr;
  // called (on the row-ID thread) once the skeleton of a level is known,
  // before its interpolation matrix: lsh_build starts the sibling blocks
  // that need it
  std::function<void(int)> skel_cb;
  NextGram ng;          // the parent Gram in progress or done
  int ng_level = -1;    // the level whose Gram ng holds (-1: none)
  std::vector<I2> ng_prox;  // (host source of its proxy upload)
  ConvOperator op;
  std::vector<StencilEntry> st4;
  double tau0_re = 0, tau0_im = 0;
  template <typename R>
  const cplx<R>* U(int l) const;
  template <typename R>
  const cplx<R>* Gab(int l) const;
  template <typename R>
  const cplx<R>* Gleaf() const;
  template <typename R>
  const cplx<R>* Ut(int l) const;
  template <typename R>
  const cplx<R>* Gabt(int l) const;
  template <typename R>
  const cplx<R>* T(int l) const {
    return static_cast<const cplx<R>*>(sizeof(R) == 8 ? lev[l].T64.p : lev[l].T32.p);
  }
  // low-rank sibling factors of parent level l: 0 L, 1 L^T, 2 R, 3 R^T
  // (L and R stacked in [L; R], L^T and R^T in [L^T; R^T])
  template <typename R>
  const cplx<R>* W(int l, int which) const {
    const Level& v = lev[l];
    const DevBuf& b = (which & 1) ? (sizeof(R) == 8 ? v.Qm64 : v.Qm32) : (sizeof(R) == 8 ? v.Pm64 : v.Pm32);
    return static_cast<const cplx<R>*>(b.p) + (which >= 2 ? (long)v.c * v.wr : 0L);
  }
};

template <>
const cplx<double>* lsh_plan_s::Ut<double>(int l) const {
  return lev[l].ident ? lev[l].U64.as<z64>() : lev[l].Ut64.as<z64>();
}
template <>
const cplx<float>* lsh_plan_s::Ut<float>(int l) const {
  return lev[l].ident ? lev[l].U32.as<c32>() : lev[l].Ut32.as<c32>();
}
template <>
const cplx<double>* lsh_plan_s::Gabt<double>(int l) const { return lev[l].Gabt64.as<z64>(); }
template <>
const cplx<float>* lsh_plan_s::Gabt<float>(int l) const { return lev[l].Gabt32.as<c32>(); }

template <>
const cplx<double>* lsh_plan_s::U<double>(int l) const { return lev[l].U64.as<z64>(); }
template <>
const cplx<float>* lsh_plan_s::U<float>(int l) const { return lev[l].U32.as<c32>(); }
template <>
const cplx<double>* lsh_plan_s::Gab<double>(int l) const { return lev[l].Gab64.as<z64>(); }
template <>
const cplx<float>* lsh_plan_s::Gab<float>(int l) const { return lev[l].Gab32.as<c32>(); }
template <>
const cplx<double>* lsh_plan_s::Gleaf<double>() const { return Gleaf64.as<z64>(); }
template <>
const cplx<float>* lsh_plan_s::Gleaf<float>() const { return Gleaf32.as<c32>(); }

namespace {

// box (origin, size) of box t on a level: vertical cuts (split x1) from even
// levels, horizontal cuts (split x2) from odd levels; child 2t is the half
// with the smaller coordinates.
void box_of(int n, int level, long t, int& ox, int& oy, int& sx, int& sy) {
  ox = oy = 0;
  sx = sy = n;
  for (int m = 1; m <= level; ++m) {
    const int bit = (int)((t >> (level - m)) & 1);
    if ((m - 1) % 2 == 0) {
      sx /= 2;
      ox += bit * sx;
    } else {
      sy /= 2;
      oy += bit * sy;
    }
  }
}

std::vector<I2> proxy_ring(int sx, int sy, int w) {
  std::vector<I2> p;
  for (int b = -w; b < sy + w; ++b)
    for (int a = -w; a < sx + w; ++a)
      if (!(a >= 0 && a < sx && b >= 0 && b < sy)) p.push_back(I2{a, b});
  return p;
}

template <typename T>
DevBuf upload(const std::vector<T>& v, hipStream_t s) {
  DevBuf b(sizeof(T) * (v.size() ? v.size() : 1));
  if (!v.empty()) LSH_HIP(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
  return b;
}

// copy of a host vector in a temporary arena (the host vector must outlive
// the copy: the callers synchronise the stream before it goes)
template <typename T>
T* upload_to(mem::Arena& a, const std::vector<T>& v, hipStream_t s) {
  T* p = static_cast<T*>(a.take(sizeof(T) * (v.size() ? v.size() : 1)));
  if (!v.empty()) LSH_HIP(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
  return p;
}

void validate(const lsh_desc& d) {
  LSH_REQUIRE(d.n >= 4 && d.n <= 2048, LSH_ERR_INVALID_ARG, "n must be in [4, 2048]");
  LSH_REQUIRE(d.h > 0 && std::isfinite(d.h), LSH_ERR_INVALID_ARG, "h must be positive");
  LSH_REQUIRE(d.kappa > 0 && std::isfinite(d.kappa), LSH_ERR_INVALID_ARG, "kappa must be positive");
  LSH_REQUIRE(d.op_order == 4 || d.op_order == 6 || d.op_order == 8 || d.op_order == 10, LSH_ERR_INVALID_ARG,
              "op_order must be 4, 6, 8 or 10");
  LSH_REQUIRE(d.leaf >= 2 && d.leaf <= 12 && d.n % d.leaf == 0, LSH_ERR_INVALID_ARG, "leaf must divide n (2..12)");
  const int p = d.n / d.leaf;
  LSH_REQUIRE(p >= 2 && (p & (p - 1)) == 0, LSH_ERR_INVALID_ARG, "n / leaf must be a power of two >= 2");
  LSH_REQUIRE(d.tol >= 0 && d.tol < 1, LSH_ERR_INVALID_ARG, "tol must be in [0, 1)");
  LSH_REQUIRE(d.proxy_width >= 1 && d.proxy_width <= 3, LSH_ERR_INVALID_ARG, "proxy_width must be 1..3");
  LSH_REQUIRE(d.hbs_prec == LSH_FP64 || d.hbs_prec == LSH_FP32, LSH_ERR_INVALID_ARG, "hbs_prec");
  LSH_REQUIRE(d.merge >= LSH_MERGE_AUTO && d.merge <= LSH_MERGE_LOWRANK, LSH_ERR_INVALID_ARG, "merge");
  LSH_REQUIRE(d.hbs_order == 0 || d.hbs_order == 4 || d.hbs_order == 6 || d.hbs_order == 8 || d.hbs_order == 10,
              LSH_ERR_INVALID_ARG, "hbs_order must be 0, 4, 6, 8 or 10");
  const int reach = d.hbs_order > 4 ? d.hbs_order / 2 - 2 : 0;  // stencil reach of order 6/8/10: 1/2/3
  LSH_REQUIRE(d.proxy_width >= reach, LSH_ERR_INVALID_ARG,
              "proxy_width must reach the correction stencil of hbs_order (6: 1, 8: 2, 10: 3)");
  int lg = 0;
  while ((1 << lg) < p) ++lg;
  LSH_REQUIRE(d.full_levels >= 0 && d.full_levels < 2 * lg, LSH_ERR_INVALID_ARG,
              "full_levels must be in [0, L) (L = 2 log2(n / leaf) levels below the root)");
}

__global__ void k_identity(z64* U, int m) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)m * m) U[e] = mk(e / m == e % m ? 1.0 : 0.0, 0.0);
}

// The exact "row ID" of m rows: J = all rows, U = I (on the device).
int identity_id(int m, std::vector<int>& Jh, DevBuf& U64, hipStream_t s) {
  Jh.resize(m);
  for (int i = 0; i < m; ++i) Jh[i] = i;
  U64.alloc(sizeof(z64) * (size_t)m * m);
  hipLaunchKernelGGL(k_identity, dim3(ceil_div((long)m * m, 256L)), dim3(256), 0, s, U64.as<z64>(), m);
  LSH_LAUNCH_CHECK();
  return m;
}

// Row ID A ~= U A[J, :] of a device matrix A (m x np, FP64; overwritten) at
// the plan's tolerance: J to the host, U (m x k) to a new buffer of the
// bound arena, temporaries from scr; returns k.  Synchronises s.
//
// gram (block-pivoted path only): called with the row-ID workspace's Gram
// block before the pivot steps; it may fill that block (ready = true: A is
// then unused) and return the parent level's Gram rows to feed (or null).
int row_id_matrix(lsh_plan_s& P, z64* A, int m, int np, std::vector<int>& Jh, DevBuf& U64, mem::Arena& scr,
                  hipStream_t s, const std::function<NextGram*(z64*, bool&)>& gram = {},
                  const std::function<void(int)>& on_skel = {}) {
  if (P.d.tol == 0) {  // exact full-rank form
    const int k = identity_id(m, Jh, U64, s);
    if (on_skel) on_skel(k);
    return k;
  }
  int* J = static_cast<int*>(scr.take(sizeof(int) * m));
  z64* Ufull = static_cast<z64*>(scr.take(sizeof(z64) * (size_t)m * m));
  int k = 0;
  // the skeleton to the host once it is final (J is written once), then on_skel
  bool told = false;
  auto skel = [&](int kk) {
    Jh.resize(kk);
    LSH_HIP(hipMemcpyAsync(Jh.data(), J, sizeof(int) * kk, hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    told = true;
    if (on_skel) on_skel(kk);
  };
  // Gram + pivoted Cholesky squares the conditioning: FP64 resolves the
  // stopping rule only while tol stays above ~1e-7; below that, CPQR.
  if (P.d.tol < 1e-7) {
    // ||A||_F for the stopping rule |R_kk| <= tol ||A||_F (computed on device)
    void* ws = scr.take(rowid_cpqr_ws(m));
    int* kd = static_cast<int*>(scr.take(sizeof(int)));
    z64* fro = static_cast<z64*>(scr.take(sizeof(z64)));
    z64* part = static_cast<z64*>(scr.take(multidot_partial_bytes(1)));
    multidot(s, A, 0, 1, A, (long)m * np, fro, part);
    z64 f2;
    LSH_HIP(hipMemcpyAsync(&f2, fro, sizeof(z64), hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    const double thr = P.d.tol * std::sqrt(f2.x);
    rowid_cpqr(s, A, m, np, thr, J, Ufull, kd, ws);
    LSH_HIP(hipMemcpyAsync(&k, kd, sizeof(int), hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    if (k < 1) k = 1;  // (a zero block still gets one skeleton)
  } else {
    // block-pivoted left-looking Cholesky by default (alpha-greedy with
    // alpha = LSH_BP_ALPHA, default 0.65; 1 = greedy); LSH_ROWID=panel selects
    // the one-pivot-at-a-time panels (greedy)
    const char* e = std::getenv("LSH_ROWID");
    const bool block = !(e && std::string(e) == "panel");
    const char* ea = std::getenv("LSH_BP_ALPHA");
    const double alpha = (ea && *ea) ? std::atof(ea) : 0.65;
    if (!block)
      k = rowid_gram(s, A, m, np, P.d.tol, J, Ufull, scr.take(rowid_gram_ws(m)));
    else {
      // (the Gram matrix is the first m x m block of the workspace)
      void* ws = scr.take(rowid_bp_ws(m));
      bool ready = false;
      NextGram* next = gram ? gram(static_cast<z64*>(ws), ready) : nullptr;
      k = rowid_bp(s, A, m, np, P.d.tol, alpha, J, Ufull, ws, ready, next, skel);
    }
  }
  if (!told) skel(k);
  U64.alloc(sizeof(z64) * (size_t)m * k);
  LSH_HIP(hipMemcpyAsync(U64.p, Ufull, sizeof(z64) * (size_t)m * k, hipMemcpyDeviceToDevice, s));
  LSH_HIP(hipStreamSynchronize(s));
  return k;
}

// Cache key of a row ID (kind 0: a level's proxy matrix, 1: a sibling
// block) of the box sx x sy: everything the pivots and U depend on.
pcache::Key cache_key(const lsh_plan_s& P, int kind, int sx, int sy) {
  pcache::Key k;
  LSH_HIP(hipGetDevice(&k.dev));
  k.kind = kind;
  k.sx = sx;
  k.sy = sy;
  k.w = P.d.proxy_width;
  k.order = P.hbs_order;
  const double kh = P.d.kappa * P.d.h, tol = P.d.tol;
  std::memcpy(&k.kh, &kh, sizeof(double));
  std::memcpy(&k.tol, &tol, sizeof(double));
  const char* e = std::getenv("LSH_ROWID");
  const char* ea = std::getenv("LSH_BP_ALPHA");
  const double alpha = (ea && *ea) ? std::atof(ea) : 0.65;
  k.method = tol == 0 ? 0 : tol < 1e-7 ? 1 : (e && std::string(e) == "panel") ? 2 : 3;
  if (k.method == 3) std::memcpy(&k.alpha, &alpha, sizeof(double));
  return k;
}

// Row ID of the level's proxy matrix (FP64); fills lv.J (host) and lv.U64.
// Levels with at least this many candidates build their parent's Gram rows
// during their row ID (below it the parent's Gram is cheap).
constexpr int kNextGramMin = 256;

// The block-pivoted Gram row ID is in use (not CPQR, not the one-pivot panels).
bool block_pivots(const lsh_plan_s& P) {
  if (P.d.tol == 0 || P.d.tol < 1e-7) return false;
  const char* e = std::getenv("LSH_ROWID");
  return !(e && std::string(e) == "panel");
}

// Row ID of level l (candidates lv.cand, proxy ring prox).  With a side
// stream, the Gram of level l (built during the row ID of level l + 1) is
// packed instead of formed here, and the rows of level l - 1's Gram are
// built while this row ID runs.
// the candidates of level l < L: the skeleton points of its two children, in
// the coordinates of box 0 of level l
void level_candidates(const lsh_plan_s& P, int l, Level& lv) {
  lv.cand.clear();
  int ox, oy, sx, sy;
  box_of(P.d.n, l, 0, ox, oy, sx, sy);
  for (int c = 0; c < 2; ++c) {
    int cx, cy, csx, csy;
    box_of(P.d.n, l + 1, c, cx, cy, csx, csy);
    const Level& ch = P.lev[l + 1];
    for (int j : ch.J) lv.cand.push_back(I2{ch.cand[j].x + cx - ox, ch.cand[j].y + cy - oy});
  }
  lv.m = (int)lv.cand.size();
}

// level l's skeleton is known: note it, prepare the uncompressed levels above
// it (their candidates, skeleton and rank follow from it), and tell the plan's
// owner
void skeleton_known(lsh_plan_s& P, int l) {
  P.lev[l].skel_known = true;
  int top = l;
  while (top - 1 >= 1 && (P.d.tol == 0 || top - 1 <= P.d.full_levels)) {
    Level& up = P.lev[top - 1];
    level_candidates(P, top - 1, up);
    up.ident = true;
    up.J.resize(up.m);
    for (int i = 0; i < up.m; ++i) up.J[i] = i;
    up.k = up.m;
    up.host_ready = up.skel_known = true;
    --top;
  }
  if (P.skel_cb) P.skel_cb(top);
}

void level_id(lsh_plan_s& P, int l, Level& lv, const std::vector<I2>& prox, hipStream_t s) {
  const int m = lv.m, np = (int)prox.size();
  if (!lv.host_ready) lv.ident = P.d.tol == 0 || l <= P.d.full_levels;
  if (lv.ident) {  // every candidate kept (exact form, or an uncompressed top level)
    std::vector<int> Jtmp;  // (J and k already set when prepared ahead)
    const int k = identity_id(m, lv.host_ready ? Jtmp : lv.J, lv.U64, s);
    if (!lv.host_ready) lv.k = k;
    return;
  }
  pcache::Key key;
  if (P.d.plan_cache) {
    key = cache_key(P, 0, lv.sx, lv.sy);
    if (pcache::find(key, lv.cand, lv.J, lv.k, lv.U64, s)) return;
  }
  const bool block = block_pivots(P);
  const bool pre = block && P.gs && P.ng_level == l && P.ng.done * 2 == m;
  const I2* dc = upload_to(P.sid, lv.cand, s);
  const int ncols = P.hbs_order == 4 ? np : 2 * np;
  z64* A = nullptr;
  if (!pre) {
    const I2* dp = upload_to(P.sid, prox, s);
    A = static_cast<z64*>(P.sid.take(sizeof(z64) * (size_t)m * ncols));
    gather_table(s, P.table.as<z64>(), P.D, dc, m, dp, np, A, ncols);
    // order > 4: the rows must also span the corrected entries against the
    // ring's points (the actual near neighbours, within the stencil's
    // reach), beside plain G on the ring (the representation of everything
    // farther)
    if (P.hbs_order > 4) gather_table(s, P.hbs_table(), P.D, dc, m, dp, np, A + np, ncols);
  }
  auto gram = [&](z64* M, bool& ready) -> NextGram* {
    if (pre) {  // (the side stream was synchronised at the start of this level)
      next_gram_pack(s, P.ng, m / 2, M);
      ready = true;
    }
    P.ng_level = -1;
    if (!(block && P.gs && l - 1 > P.d.full_levels && l >= 2 && m >= kNextGramMin && !P.d.plan_cache)) return nullptr;
    // the parent level l - 1: its box, the children's origins in it, its ring
    P.sgram.reset(0);  // (after the pack above, on s; the new rows start after a sync of s)
    int ox, oy, psx, psy, cx, cy, csx, csy;
    box_of(P.d.n, l - 1, 0, ox, oy, psx, psy);
    NextGram& g = P.ng;
    g = NextGram();
    for (int c = 0; c < 2; ++c) {
      box_of(P.d.n, l, c, cx, cy, csx, csy);
      g.off[c] = I2{cx - ox, cy - oy};
    }
    P.ng_prox = proxy_ring(psx, psy, P.d.proxy_width);
    g.cap = m;
    g.np = (int)P.ng_prox.size();
    g.ncols = P.hbs_order == 4 ? g.np : 2 * g.np;
    g.D = P.D;
    g.T = P.table.as<z64>();
    g.T2 = P.hbs_order > 4 ? P.hbs_table() : nullptr;
    g.cand = dc;
    g.prox = upload_to(P.sgram, P.ng_prox, s);
    g.A = static_cast<z64*>(P.sgram.take(sizeof(z64) * 2 * (size_t)m * g.ncols));
    g.G = static_cast<z64*>(P.sgram.take(sizeof(z64) * 4 * (size_t)m * m));
    g.gs = P.gs;
    P.ng_level = l - 1;
    return &g;
  };
  row_id_matrix(P, A, m, ncols, lv.J, lv.U64, P.sid, s, block ? gram : std::function<NextGram*(z64*, bool&)>(),
                [&](int k) {
                  lv.k = k;
                  skeleton_known(P, l);
                });
  if (P.d.plan_cache) pcache::insert(key, lv.cand, lv.J, m, lv.k, lv.U64, s);
}

// Plan in three phases so that the factor can follow it level by level:
// plan_init (weights, table, leaf geometry), plan_level(l) for l = L..0 (the
// row ID of level l and the sibling block of parent level l, in the working
// precision and transposed), plan_finish (the FFT spectrum).
void plan_init(lsh_plan_s& P, hipStream_t s) {
  const lsh_desc& d = P.d;
  P.n = d.n;
  P.h = d.h;
  P.kappa = d.kappa;
  P.ls = d.leaf;
  int p = d.n / d.leaf, lg = 0;
  while ((1 << lg) < p) ++lg;
  P.L = 2 * lg;
  LSH_REQUIRE(P.L < LSH_MAX_LEVELS, LSH_ERR_UNSUPPORTED, "too many levels");
  P.nleaf = 1 << P.L;
  P.mL = d.leaf * d.leaf;
  P.D = d.n + d.proxy_width + 1;
  // weights (Sec. 2.2) and the offset table
  P.st4 = correction_stencil(4, d.kappa * d.h);
  P.tau0_re = P.st4[0].re;
  P.tau0_im = P.st4[0].im;
  P.table.alloc(sizeof(z64) * (size_t)(P.D + 1) * (P.D + 1));
  build_offset_table(s, P.table.as<z64>(), P.D, d.h, d.kappa, P.tau0_re, P.tau0_im);
  P.hbs_order = d.hbs_order > 4 ? d.hbs_order : 4;
  P.htable.release();
  if (P.hbs_order > 4) {  // direct-solver mode: the compressed matrix carries the order-p corrections
    const std::vector<StencilEntry> st = correction_stencil(P.hbs_order, d.kappa * d.h);
    P.htable.alloc(sizeof(z64) * (size_t)(P.D + 1) * (P.D + 1));
    build_offset_table(s, P.htable.as<z64>(), P.D, d.h, d.kappa, st[0].re, st[0].im);
    add_table_stencil(s, P.htable.as<z64>(), P.D, d.h, st, P.sid);
  }
  // leaves
  P.leaf_origin_h.resize(P.nleaf);
  for (int t = 0; t < P.nleaf; ++t) {
    int ox, oy, sx, sy;
    box_of(d.n, P.L, t, ox, oy, sx, sy);
    P.leaf_origin_h[t] = I2{ox, oy};
  }
  P.leaf_pts_h.clear();
  for (int iy = 0; iy < d.leaf; ++iy)
    for (int ix = 0; ix < d.leaf; ++ix) P.leaf_pts_h.push_back(I2{ix, iy});
  P.leaf_origin = upload(P.leaf_origin_h, s);
  P.leaf_pts = upload(P.leaf_pts_h, s);
  P.lev.clear();
  P.lev.resize(P.L + 1);
  for (int l = 0; l <= P.L; ++l) {
    int ox, oy;
    box_of(d.n, l, 0, ox, oy, P.lev[l].sx, P.lev[l].sy);
  }
  P.Gleaf64.alloc(sizeof(z64) * (size_t)P.mL * P.mL);
  gather_table(s, P.hbs_table(), P.D, P.leaf_pts.as<I2>(), P.mL, P.leaf_pts.as<I2>(), P.mL, P.Gleaf64.as<z64>(),
               P.mL);
  if (d.hbs_prec == LSH_FP32) {
    P.Gleaf32.alloc(sizeof(c32) * (size_t)P.mL * P.mL);
    ccast<double, float>(s, P.Gleaf64.as<z64>(), P.Gleaf32.as<c32>(), (long)P.mL * P.mL);
  }
  LSH_HIP(hipStreamSynchronize(s));
}

// row ID of level l (needs level l + 1)
// The interpolation rows of level l's U (the rows off the skeleton J), for
// products with U that skip its identity rows.
void plan_interp_rows(lsh_plan_s& P, int l, hipStream_t s) {
  Level& lv = P.lev[l];
  const int m = lv.m, k = lv.k, half = m / 2;
  std::vector<char> skel(m, 0);
  for (int q = 0; q < k; ++q) {
    LSH_REQUIRE(lv.J[q] >= 0 && lv.J[q] < m && !skel[lv.J[q]], -4, "row ID: skeleton rows not distinct");
    skel[lv.J[q]] = 1;
  }
  lv.rest.clear();
  lv.nrest0 = 0;
  for (int i = 0; i < m; ++i)
    if (!skel[i]) {
      lv.rest.push_back(i);
      if (i < half) ++lv.nrest0;
    }
  const int nr = (int)lv.rest.size();
  lv.restIdx.alloc(sizeof(int) * std::max(nr, 1));
  lv.skelIdx.alloc(sizeof(int) * k);
  if (nr) LSH_HIP(hipMemcpyAsync(lv.restIdx.p, lv.rest.data(), sizeof(int) * nr, hipMemcpyHostToDevice, s));
  LSH_HIP(hipMemcpyAsync(lv.skelIdx.p, lv.J.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
  lv.T64.alloc(sizeof(z64) * std::max((size_t)nr * k, (size_t)1));
  gather_rows2<double>(s, nr, k, lv.U64.as<z64>(), lv.U64.as<z64>(), m, k, 0, lv.restIdx.as<int>(), 0,
                       lv.T64.as<z64>(), k, 0, 1);
  if (P.d.hbs_prec == LSH_FP32) {
    lv.T32.alloc(sizeof(c32) * std::max((size_t)nr * k, (size_t)1));
    gather_rows2<float>(s, nr, k, lv.U32.as<c32>(), lv.U32.as<c32>(), m, k, 0, lv.restIdx.as<int>(), 0,
                        lv.T32.as<c32>(), k, 0, 1);
  }
}

void plan_id(lsh_plan_s& P, int l, hipStream_t s) {
  const lsh_desc& d = P.d;
  const bool f32 = d.hbs_prec == LSH_FP32;
  if (l >= 1) {  // row ID of level l (Sec. 3.2)
    LSH_HIP(hipStreamSynchronize(s));
    if (P.gs) LSH_HIP(hipStreamSynchronize(P.gs));  // (this level's Gram rows, read from the previous sid)
    P.sid.reset(0);  // (the previous level's temporaries are no longer in use)
    Level& lv = P.lev[l];
    if (!lv.host_ready) {
      if (l == P.L) {
        lv.cand = P.leaf_pts_h;
        lv.m = (int)lv.cand.size();
      } else {
        level_candidates(P, l, lv);
      }
    }
    level_id(P, l, lv, proxy_ring(lv.sx, lv.sy, d.proxy_width), s);
    if (!lv.skel_known) skeleton_known(P, l);
    if (f32) {
      lv.U32.alloc(sizeof(c32) * (size_t)lv.m * lv.k);
      ccast<double, float>(s, lv.U64.as<z64>(), lv.U32.as<c32>(), (long)lv.m * lv.k);
    }
    if (!lv.ident) {  // (U = I is its own transpose: Ut(l) then reads U)
      lv.Ut64.alloc(sizeof(z64) * (size_t)lv.m * lv.k);
      ctranspose<double>(s, lv.U64.as<z64>(), lv.m, lv.k, lv.Ut64.as<z64>());
      if (f32) {
        lv.Ut32.alloc(sizeof(c32) * (size_t)lv.m * lv.k);
        ctranspose<float>(s, lv.U32.as<c32>(), lv.m, lv.k, lv.Ut32.as<c32>());
      }
      if (l < P.L) plan_interp_rows(P, l, s);
    }
  }
}

// Low-rank form of parent level l's sibling block for the Woodbury merge:
// G_ab ~= L R^T with L = U and R^T = G_ab[J, :] from the row ID of G_ab at
// the compression tolerance (the remark after Algorithm 2; rank about a
// quarter to two fifths of c at tol 1e-4).  AUTO keeps the Schur form where
// r > 0.6 c, where the Woodbury products stop saving work.
void plan_lowrank(lsh_plan_s& P, int l, hipStream_t s, mem::Arena& tmp) {
  const lsh_desc& d = P.d;
  Level& lv = P.lev[l];
  lv.wr = 0;
  const int c = lv.c;
  if (d.merge == LSH_MERGE_SCHUR || (d.merge == LSH_MERGE_AUTO && d.tol == 0)) return;
  const long cc = (long)c * c;
  std::vector<int> J;
  DevBuf& U = lv.WU64;
  int r = 0;
  std::vector<I2> sk;  // the sibling skeletons: the cache entry's identity
  pcache::Key key;
  bool hit = false;
  if (P.d.plan_cache && d.tol > 0) {
    sk = lv.ra;
    sk.insert(sk.end(), lv.rb.begin(), lv.rb.end());
    int psx, psy, ox, oy;
    box_of(d.n, l, 0, ox, oy, psx, psy);
    key = cache_key(P, 1, psx, psy);
    hit = pcache::find(key, sk, J, r, U, s);
  }
  if (!hit) {
    z64* A = static_cast<z64*>(tmp.take(sizeof(z64) * cc));
    LSH_HIP(hipMemcpyAsync(A, lv.Gab64.p, sizeof(z64) * cc, hipMemcpyDeviceToDevice, s));
    r = row_id_matrix(P, A, c, c, J, U, tmp, s);
    if (P.d.plan_cache && d.tol > 0) pcache::insert(key, sk, J, c, r, U, s);  // U = L: c x r
  }
  if (d.merge == LSH_MERGE_AUTO && 10 * r > 6 * c) return;
  const bool f32 = d.hbs_prec == LSH_FP32;
  const long cr = (long)c * r;
  lv.wr = r;
  std::vector<I2>& rows = lv.wrows;
  rows.resize(r);
  for (int i = 0; i < r; ++i) rows[i] = lv.ra[J[i]];
  const I2* dr = upload_to(tmp, rows, s);
  const I2* db = upload_to(tmp, lv.rb, s);
  lv.Pm64.alloc(sizeof(z64) * 2 * cr);
  lv.Qm64.alloc(sizeof(z64) * 2 * cr);
  z64* Pm = lv.Pm64.as<z64>();
  z64* Qm = lv.Qm64.as<z64>();
  LSH_HIP(hipMemcpyAsync(Pm, U.p, sizeof(z64) * cr, hipMemcpyDeviceToDevice, s));       // L
  gather_table(s, P.hbs_table(), P.D, dr, r, db, c, Qm + cr, c);  // R^T = G_ab[J, :]
  ctranspose<double>(s, Pm, c, r, Qm);                                                 // L^T
  ctranspose<double>(s, Qm + cr, r, c, Pm + cr);                                       // R
  if (f32) {
    lv.Pm32.alloc(sizeof(c32) * 2 * cr);
    lv.Qm32.alloc(sizeof(c32) * 2 * cr);
    ccast<double, float>(s, Pm, lv.Pm32.as<c32>(), 2 * cr);
    ccast<double, float>(s, Qm, lv.Qm32.as<c32>(), 2 * cr);
  }
  LSH_HIP(hipStreamSynchronize(s));
}

// sibling block of parent level l (needs the skeletons of level l + 1);
// temporaries from tmp, rewound first (after a synchronisation of s)
void plan_sibling(lsh_plan_s& P, int l, hipStream_t s, mem::Arena& tmp) {
  const lsh_desc& d = P.d;
  const bool f32 = d.hbs_prec == LSH_FP32;
  if (l < P.L) {  // sibling block G_ab of parent level l (eq. (sibint)): children 0 and 1 of box 0
    LSH_HIP(hipStreamSynchronize(s));
    tmp.reset(0);  // (the previous sibling block's temporaries are no longer in use)
    const Level& ch = P.lev[l + 1];
    int ax, ay, bx, by, sx, sy;
    box_of(d.n, l + 1, 0, ax, ay, sx, sy);
    box_of(d.n, l + 1, 1, bx, by, sx, sy);
    Level& lv = P.lev[l];
    // (kept in the level: the host source of the uploads below outlives them)
    std::vector<I2>& ra = lv.ra;
    std::vector<I2>& rb = lv.rb;
    ra.clear();
    rb.clear();
    for (int j : ch.J) {
      ra.push_back(I2{ch.cand[j].x + ax, ch.cand[j].y + ay});
      rb.push_back(I2{ch.cand[j].x + bx, ch.cand[j].y + by});
    }
    lv.c = ch.k;
    const I2* da = upload_to(tmp, ra, s);
    const I2* db = upload_to(tmp, rb, s);
    const long cc = (long)lv.c * lv.c;
    lv.Gab64.alloc(sizeof(z64) * cc);
    gather_table(s, P.hbs_table(), P.D, da, lv.c, db, lv.c, lv.Gab64.as<z64>(), lv.c);
    lv.Gabt64.alloc(sizeof(z64) * cc);
    ctranspose<double>(s, lv.Gab64.as<z64>(), lv.c, lv.c, lv.Gabt64.as<z64>());
    if (f32) {
      lv.Gab32.alloc(sizeof(c32) * cc);
      ccast<double, float>(s, lv.Gab64.as<z64>(), lv.Gab32.as<c32>(), cc);
      lv.Gabt32.alloc(sizeof(c32) * cc);
      ctranspose<float>(s, lv.Gab32.as<c32>(), lv.c, lv.c, lv.Gabt32.as<c32>());
    }
    plan_lowrank(P, l, s, tmp);
  }
}

void plan_level(lsh_plan_s& P, int l, hipStream_t s) {
  plan_sibling(P, l, s, P.ssib);
  plan_id(P, l, s);
}

void plan_finish(lsh_plan_s& P, hipStream_t s) {
  const lsh_desc& d = P.d;
  // operator spectrum (order op_order)
  LSH_HIP(hipStreamSynchronize(s));
  P.sid.reset(0);
  P.op.init(s, d.n, d.h, d.kappa, P.table.as<z64>(), P.D, correction_stencil(d.op_order, d.kappa * d.h), P.sid);
  LSH_HIP(hipStreamSynchronize(s));
}

void plan_build(lsh_plan_s& P, hipStream_t s) {
  plan_init(P, s);
  for (int l = P.L; l >= 0; --l) plan_level(P, l, s);
  plan_finish(P, s);
}

// ------------------------------------------------------------ workspace sizes
// The ranks are known only once the row IDs have run, so the plan's
// workspace is sized by bounds: a level's rank is at most its number of
// candidate rows (twice the children's rank; the leaf's nodes) and at most
// its number of proxy columns (the ring, twice that for an order-p
// compression); a sibling block's rank is at most its order.  Given a plan,
// the factor's size is exact; so is the solve's.

struct PlanBytes {
  size_t persist = 0, sid = 0, ssib = 0, sgram = 0;
  size_t total() const { return persist + sid + ssib + sgram; }
};

// Per-level sizes that the factor's memory depends on: ranks k, merge
// orders c, Woodbury ranks r and which merge forms may occur (bit 0: Schur,
// bit 1: Woodbury).
struct Profile {
  long N = 0;
  int L = 0, nleaf = 0, mL = 0;
  bool f32 = false;
  std::vector<long> k, c, r;
  std::vector<long> nr;  // level l: rows of T (both halves), at most (0: U = I)
  std::vector<int> form;
};

size_t rowid_scratch_bytes(long m, double tol) {
  if (tol == 0) return 0;  // (U = I goes to the plan's own memory)
  mem::Sizer z, q;
  z.add_n<int>(m);
  z.add_n<z64>((size_t)m * m);
  q.add(rowid_cpqr_ws((int)m));
  q.add(sizeof(int));
  q.add(sizeof(z64));
  q.add(multidot_partial_bytes(1));
  return z.total + std::max({q.total, mem::round_up(rowid_gram_ws((int)m)), mem::round_up(rowid_bp_ws((int)m))});
}

// Plan sizes (bounds) and the factor's rank profile under the same bounds.
PlanBytes plan_bytes(const lsh_desc& d, Profile* prof) {
  int p = d.n / d.leaf, lg = 0;
  while ((1 << lg) < p) ++lg;
  const int L = 2 * lg, nleaf = 1 << L, mL = d.leaf * d.leaf, D = d.n + d.proxy_width + 1, w = d.proxy_width;
  const bool f32 = d.hbs_prec == LSH_FP32;
  const int horder = d.hbs_order > 4 ? d.hbs_order : 4;
  const bool lowrank = !(d.merge == LSH_MERGE_SCHUR || (d.merge == LSH_MERGE_AUTO && d.tol == 0));
  const size_t e = f32 ? sizeof(c32) : 0;  // extra FP32 copies
  std::vector<long> m(L + 2, 0), k(L + 2, 0), np(L + 1, 0);
  for (int l = L; l >= 1; --l) {
    int ox, oy, sx, sy;
    box_of(d.n, l, 0, ox, oy, sx, sy);
    np[l] = (long)(sx + 2 * w) * (sy + 2 * w) - (long)sx * sy;
    const long ncols = (horder > 4 ? 2 : 1) * np[l];
    m[l] = l == L ? mL : 2 * k[l + 1];
    k[l] = (d.tol == 0 || l <= d.full_levels) ? m[l] : std::max(1L, std::min(m[l], ncols));
  }
  PlanBytes b;
  mem::Sizer z;
  z.add_n<z64>((size_t)(D + 1) * (D + 1));                      // table
  if (horder > 4) z.add_n<z64>((size_t)(D + 1) * (D + 1));      // htable
  z.add_n<I2>(nleaf);                                           // leaf_origin
  z.add_n<I2>(mL);                                              // leaf_pts
  z.add_n<z64>((size_t)mL * mL);                                // Gleaf64
  if (f32) z.add(e * mL * mL);                                  // Gleaf32
  size_t sid = mem::round_up(4096) + ConvOperator::scratch_bytes(d.n), ssib = 0, sgram = 0;
  for (int l = 1; l <= L; ++l) {
    const size_t mk = (size_t)m[l] * k[l];
    z.add_n<z64>(mk);  // U64
    z.add_n<z64>(mk);  // Ut64
    if (f32) { z.add(e * mk); z.add(e * mk); }
    if (l < L && !(d.tol == 0 || l <= d.full_levels)) {  // T = U[rest, :] ((m - k) x k, rank k <= k[l]), indices
      const size_t mm = m[l], kb = k[l];
      const size_t tb = std::max<size_t>(2 * kb >= mm ? (mm / 2) * (mm - mm / 2) : (mm - kb) * kb, 1);
      z.add_n<z64>(tb);
      if (f32) z.add(e * tb);
      z.add_n<int>(mm);
      z.add_n<int>(kb);
    }
    const long ncols = (horder > 4 ? 2 : 1) * np[l];
    mem::Sizer t;
    t.add_n<I2>(m[l]);
    t.add_n<I2>(np[l]);
    if (d.tol > 0) t.add_n<z64>((size_t)m[l] * ncols);
    sid = std::max(sid, t.total + rowid_scratch_bytes(m[l], d.tol));
    // the parent's Gram rows, built during this row ID (level_id)
    if (d.tol >= 1e-7 && !d.plan_cache && l >= 2 && l - 1 > d.full_levels && m[l] >= kNextGramMin) {
      const long pcols = (horder > 4 ? 2 : 1) * np[l - 1];
      mem::Sizer g;
      g.add_n<I2>(np[l - 1]);
      g.add_n<z64>(2 * (size_t)m[l] * pcols);
      g.add_n<z64>(4 * (size_t)m[l] * m[l]);
      sgram = std::max(sgram, g.total);
    }
  }
  for (int l = 0; l < L; ++l) {
    // r <= c; AUTO keeps the low-rank factors only where 10 r <= 6 c
    const size_t c = k[l + 1], cc = c * c, cr = c * (d.merge == LSH_MERGE_AUTO ? c * 6 / 10 : c);
    z.add_n<z64>(cc);
    z.add_n<z64>(cc);
    if (f32) { z.add(e * cc); z.add(e * cc); }
    mem::Sizer t;
    t.add_n<I2>(c);
    t.add_n<I2>(c);
    if (lowrank) {
      z.add_n<z64>(cc);                     // U of the sibling block's row ID
      z.add_n<z64>(2 * cr);                 // [L; R]
      z.add_n<z64>(2 * cr);                 // [L^T; R^T]
      if (f32) { z.add(e * 2 * cr); z.add(e * 2 * cr); }
      t.add_n<z64>(cc);                     // copy of G_ab (overwritten by the row ID)
      t.add_n<I2>(c);
      t.add_n<I2>(c);
      ssib = std::max(ssib, t.total + rowid_scratch_bytes((long)c, d.tol));
    } else {
      ssib = std::max(ssib, t.total);
    }
  }
  z.add(ConvOperator::bytes(d.n));
  b.persist = z.total;
  b.sid = std::max(sid, ssib);  // (lsh_build's row-ID thread may take the last sibling blocks)
  b.ssib = ssib;
  b.sgram = sgram;
  if (prof) {
    Profile& P = *prof;
    P.N = (long)d.n * d.n;
    P.L = L;
    P.nleaf = nleaf;
    P.mL = mL;
    P.f32 = f32;
    P.k.assign(k.begin(), k.begin() + L + 1);
    P.c.resize(L);
    P.r.resize(L);
    P.nr.assign(L, 0);
    P.form.resize(L);
    for (int l = 0; l < L; ++l) {
      P.c[l] = k[l + 1];
      if (l >= 1 && !(d.tol == 0 || l <= d.full_levels)) P.nr[l] = m[l];
      if (!lowrank) { P.form[l] = 1; P.r[l] = 0; }
      else if (d.merge == LSH_MERGE_LOWRANK) { P.form[l] = 2; P.r[l] = P.c[l]; }
      else { P.form[l] = 3; P.r[l] = P.c[l] * 6 / 10; }  // AUTO: Woodbury only where 10 r <= 6 c
    }
  }
  return b;
}

Profile plan_profile(const lsh_plan_s& P) {
  Profile f;
  f.N = (long)P.n * P.n;
  f.L = P.L;
  f.nleaf = P.nleaf;
  f.mL = P.mL;
  f.f32 = P.d.hbs_prec == LSH_FP32;
  f.k.resize(P.L + 1);
  f.c.resize(P.L);
  f.r.resize(P.L);
  f.form.resize(P.L);
  for (int l = 0; l <= P.L; ++l) f.k[l] = P.lev[l].k;
  f.nr.assign(P.L, 0);
  for (int l = 0; l < P.L; ++l) {
    const Level& v = P.lev[l];
    if (l >= 1 && !v.ident) f.nr[l] = std::max<long>(1, (long)v.rest.size());
    f.c[l] = P.lev[l].c;
    f.r[l] = P.lev[l].wr;
    f.form[l] = P.lev[l].wr > 0 ? 2 : 1;
  }
  return f;
}

struct FactorBytes {
  size_t keep = 0, scr = 0;
  size_t total() const { return keep + scr; }
};

// Right-hand sides per apply of the preconditioner (larger calls are split).
constexpr int APPLY_GROUP = 8;
// FP32 partial products of the apply's split-K shared products.
constexpr size_t kSplitKBytes = size_t(24) << 20;

template <typename R>
FactorBytes factor_bytes_t(const Profile& f, bool want_T) {
  const size_t e = sizeof(cplx<R>);
  const long L = f.L, nleaf = f.nleaf, mL = f.mL, kL = f.k[L];
  mem::Sizer z;
  z.add_n<double>(f.N);                                 // b
  z.add(sizeof(int));                                   // input check flag
  z.add(e * nleaf * mL * mL);                           // X
  z.add_n<int>(nleaf);                                  // leaf flags
  z.add(e * nleaf * kL * kL);                           // S_L
  size_t scr = mem::round_up(inverse_ws_bytes<R>((int)mL, (int)nleaf)) + 2 * mem::round_up(e * nleaf * mL * kL);
  for (long l = L - 1; l >= 0; --l) {
    const long nb = 1L << l, c = f.c[l], r = f.r[l], k = f.k[l];
    size_t keep_l = 0, scr_l = 0;
    if (f.form[l] & 2) {  // Woodbury
      mem::Sizer a, t;
      a.add(e * nb * 2 * c * r);
      a.add(e * nb * 4 * r * r);
      if (want_T) { a.add(e * nb * 2 * c * r); a.add(e * nb * 4 * r * r); }
      t.add(e * nb * 3 * r * r);
      t.add(inverse_ws_bytes<R>((int)std::max(1L, r), (int)nb));
      t.add(merge_level_table_bytes(1));  // (a level in one persistent launch: its table and counter)
      t.add(sizeof(int));
      if (l >= 1) { t.add(e * nb * 2 * c * k); t.add(e * nb * 4 * r * k); }
      if (l >= 1 && f.nr[l] > 0) { t.add(e * nb * c * f.nr[l]); t.add(e * nb * f.nr[l] * k); }
      keep_l = std::max(keep_l, a.total);
      scr_l = std::max(scr_l, t.total);
    }
    if (f.form[l] & 1) {  // Schur
      mem::Sizer a, t;
      for (int q = 0; q < (want_T ? 6 : 3); ++q) a.add(e * nb * c * c);
      t.add(inverse_ws_bytes<R>((int)c, (int)nb));
      if (l >= 1) for (int q = 0; q < 3; ++q) t.add(e * nb * c * k);
      if (l >= 1 && f.nr[l] > 0) { t.add(e * nb * c * f.nr[l]); t.add(e * nb * f.nr[l] * k); }
      keep_l = std::max(keep_l, a.total);
      scr_l = std::max(scr_l, t.total);
    }
    z.add(keep_l);
    z.add_n<int>(nb);                                   // merge flags
    if (l >= 1) z.add(e * nb * k * k);                  // S_l
    scr = std::max(scr, scr_l);
  }
  // apply vectors for APPLY_GROUP right-hand sides
  const long G = APPLY_GROUP;
  z.add(e * G * nleaf * mL);
  size_t big = 0;
  for (long l = 1; l <= L; ++l) {
    const size_t v = (size_t)G * ((size_t)1 << l) * f.k[l];
    z.add(e * v);
    z.add(e * v);
    big = std::max(big, v);
  }
  for (int q = 0; q < 5; ++q) z.add(e * big);
  if (sizeof(R) == 4) z.add(kSplitKBytes);
  if (want_T) {  // transposed leaf and scattering matrices, transpose-pass vectors
    z.add(e * nleaf * mL * mL);
    for (long l = 1; l <= L; ++l) z.add(e * ((size_t)1 << l) * f.k[l] * f.k[l]);
    for (long l = 1; l < L; ++l) z.add(e * G * ((size_t)1 << l) * 2 * f.c[l]);
  }
  FactorBytes b;
  b.keep = z.total;
  b.scr = scr;
  return b;
}

FactorBytes factor_bytes(const Profile& f, bool want_T) {
  return f.f32 ? factor_bytes_t<float>(f, want_T) : factor_bytes_t<double>(f, want_T);
}

// ------------------------------------------------------------ factor
template <typename R>
struct FactorData {
  using real_t = R;
  DevBuf X;                       // leaf inverses [nleaf][mL][mL]
  std::vector<DevBuf> S;          // S[l], l = 1..L : [2^l][k_l][k_l]
  std::vector<DevBuf> Pa, Pb, Ci; // parent level l = 0..L-1 : [2^l][c][c]
  // Woodbury levels (wr[l] = r > 0): Pa = [S_a L; S_b R] per box
  // ([2^l][2][c][r]) and Ci = W', the inverse of I + Q P with its two column
  // blocks swapped ([2^l][2r][2r]); Pb unused
  std::vector<int> wr;
  // apply workspace
  int ws_nrhs = 0;
  DevBuf r;                       // [nrhs][nleaf][mL]
  std::vector<DevBuf> rt, wt;     // [nrhs][2^l][k_l]
  DevBuf t1, t2, t3, ty, tw;      // scratch
  DevBuf tk;                      // partial products of split-K shared products
  // transposed per-box matrices for M^T (built on first use)
  bool has_T = false;
  DevBuf XT;
  std::vector<DevBuf> ST, PaT, PbT, CiT;
  std::vector<DevBuf> vb;         // transpose pass: per parent level [nrhs][2^l][2c]
  // singularity flags of the local inverses, read back once when the factor ends
  std::vector<DevBuf> info;
  // The factor's arenas (its workspace): keep holds the factor, the apply
  // vectors and the transposed copies; scr the temporaries of the build,
  // rewound at the start of every level (all of the build runs on one
  // stream, so a level's temporaries are reused only after the previous
  // level's kernels).
  mem::Arena* keep = nullptr;
  mem::Arena* scr = nullptr;
  bool want_T = false;  // room for the transposed copies was reserved
  template <typename T = void>
  T* scratch_buf(size_t bytes) {
    return static_cast<T*>(scr->take(bytes));
  }
  void scratch_reset() { scr->reset(0); }
  std::vector<int> info_n;
  std::vector<std::string> info_what;
};

// Read back every pending singularity flag (one synchronisation) and raise
// on the first singular local matrix.
template <typename R>
void factor_check(FactorData<R>& F, hipStream_t s) {
  std::vector<std::vector<int>> h(F.info.size());
  for (size_t q = 0; q < F.info.size(); ++q) {
    h[q].resize(F.info_n[q]);
    LSH_HIP(hipMemcpyAsync(h[q].data(), F.info[q].p, sizeof(int) * F.info_n[q], hipMemcpyDeviceToHost, s));
  }
  LSH_HIP(hipStreamSynchronize(s));
  for (size_t q = 0; q < h.size(); ++q)
    for (int v : h[q]) LSH_REQUIRE(!v, LSH_ERR_SINGULAR, F.info_what[q]);
  F.info.clear();
  F.info_n.clear();
  F.info_what.clear();
}

int check_info(const DevBuf& info, int batch, hipStream_t s) {
  std::vector<int> h(batch);
  LSH_HIP(hipMemcpyAsync(h.data(), info.p, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  for (int v : h)
    if (v) return v;
  return 0;
}

// Algorithm 1 in stages: factor_leaves (needs plan level L), then
// factor_level(l) for l = L-1..0 (needs plan level l).
template <typename R>
void factor_init(const lsh_plan_s& P, FactorData<R>& F) {
  F.S.clear();
  F.S.resize(P.L + 1);
  F.Pa.clear(); F.Pb.clear(); F.Ci.clear();
  F.Pa.resize(P.L); F.Pb.resize(P.L); F.Ci.resize(P.L);
  F.wr.assign(P.L, 0);
}

template <typename R>
void factor_leaves(const lsh_plan_s& P, const double* b, FactorData<R>& F, hipStream_t s) {
  const int L = P.L, nleaf = P.nleaf, mL = P.mL, kL = P.lev[L].k;
  const double k2 = P.kappa * P.kappa;
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0);
  mem::Bind bind(F.keep);
  F.scratch_reset();
  // leaves: X = (I + B G_leaf)^{-1}, S = U^T X B U
  F.X.alloc(sizeof(cplx<R>) * (size_t)nleaf * mL * mL);
  cplx<R>* X = F.X.template as<cplx<R>>();
  leaf_build<R>(s, X, P.Gleaf<R>(), mL, b, k2, P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), nleaf, P.n);
  {
    void* ws = F.scratch_buf(inverse_ws_bytes<R>(mL, nleaf));
    F.info.emplace_back(sizeof(int) * nleaf);
    F.info_n.push_back(nleaf);
    F.info_what.push_back("singular leaf matrix I + B G");
    inverse<R>(s, X, mL, mL, (long)mL * mL, nleaf, ws, F.info.back().template as<int>());
  }
  cplx<R>* Y = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * (size_t)nleaf * mL * kL);
  cplx<R>* Z = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * (size_t)nleaf * mL * kL);
  leaf_scale_U<R>(s, Y, P.U<R>(L), mL, kL, b, k2, P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), nleaf, P.n);
  cgemm<R>(s, mL, kL, mL, one, X, mL, (long)mL * mL, OP_N, Y, kL, (long)mL * kL, OP_N, zero, nullptr, 0, 0, Z, kL,
           (long)mL * kL, nleaf);
  F.S[L].alloc(sizeof(cplx<R>) * (size_t)nleaf * kL * kL);
  cgemm<R>(s, kL, kL, mL, one, P.U<R>(L), kL, 0, OP_T, Z, kL, (long)mL * kL, OP_N, zero,
           nullptr, 0, 0, F.S[L].template as<cplx<R>>(), kL, (long)kL * kL, nleaf);
}

// Woodbury merge of parent level l (G_ab ~= L R^T, rank r): with
// P = diag(S_a L, S_b R) and Q = [[0, R^T], [L^T, 0]] the merge matrix is
// I + P Q, so X = I - P (I + Q P)^{-1} Q.  I + Q P = [[I, Aw], [Bw, I]]
// (Aw = R^T S_b R, Bw = L^T S_a L) is inverted by its own Schur step,
// C = (I - Bw Aw)^{-1}:  (I + Q P)^{-1} = [[I + Aw C Bw, -Aw C], [-C Bw, C]].
// Stored: W' = that inverse with its column blocks swapped,
// [[-Aw C, I + Aw C Bw], [C, -C Bw]], which takes Q v in the order
// [L^T v_a; R^T v_b] (so that both halves of Q v, and of Q^T z, are one
// strided product).
template <typename R>
void factor_merge_lowrank(const lsh_plan_s& P, FactorData<R>& F, int l, hipStream_t s) {
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
  const int c = P.lev[l].c, r = P.lev[l].wr, nb = 1 << l;
  const long cc = (long)c * c, cr = (long)c * r, rr = (long)r * r, r2 = 2L * r, w4 = 4L * rr;
  const cplx<R>* Sch = F.S[l + 1].template as<cplx<R>>();
  mem::Bind bind(F.keep);
  F.wr[l] = r;
  F.Pa[l].alloc(sizeof(cplx<R>) * nb * 2 * cr);
  F.Ci[l].alloc(sizeof(cplx<R>) * nb * w4);
  cplx<R>* Pst = F.Pa[l].template as<cplx<R>>();
  cplx<R>* W = F.Ci[l].template as<cplx<R>>();
  cplx<R>* Aw = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * 3 * rr);
  cplx<R>* Bw = Aw + nb * rr;
  cplx<R>* C = Bw + nb * rr;
  // S_a L, S_b R
  cgemm<R>(s, c, r, c, one, Sch, c, 2 * cc, OP_N, P.W<R>(l, 0), r, 0, OP_N, zero, nullptr, 0, 0, Pst, r, 2 * cr, nb);
  cgemm<R>(s, c, r, c, one, Sch + cc, c, 2 * cc, OP_N, P.W<R>(l, 2), r, 0, OP_N, zero, nullptr, 0, 0, Pst + cr, r,
           2 * cr, nb);
  // Aw = R^T (S_b R), Bw = L^T (S_a L), C = (I - Bw Aw)^{-1}
  cgemm<R>(s, r, r, c, one, P.W<R>(l, 3), c, 0, OP_N, Pst + cr, r, 2 * cr, OP_N, zero, nullptr, 0, 0, Aw, r, rr, nb);
  cgemm<R>(s, r, r, c, one, P.W<R>(l, 1), c, 0, OP_N, Pst, r, 2 * cr, OP_N, zero, nullptr, 0, 0, Bw, r, rr, nb);
  cgemm<R>(s, r, r, r, mone, Bw, r, rr, OP_N, Aw, r, rr, OP_N, zero, nullptr, 0, 0, C, r, rr, nb, true);
  {
    void* ws = F.scratch_buf(inverse_ws_bytes<R>(r, nb));
    F.info.emplace_back(sizeof(int) * nb);
    F.info_n.push_back(nb);
    F.info_what.push_back("singular merge matrix I - Bw Aw at level " + std::to_string(l));
    inverse<R>(s, C, r, r, rr, nb, ws, F.info.back().template as<int>());
  }
  // W' = [[-Aw C, I + Aw C Bw], [C, -C Bw]]  (row blocks of 2r entries)
  ccopy2d<R>(s, r, r, C, r, rr, W + r * r2, r2, w4, nb);
  cgemm<R>(s, r, r, r, mone, Aw, r, rr, OP_N, C, r, rr, OP_N, zero, nullptr, 0, 0, W, r2, w4, nb);
  cgemm<R>(s, r, r, r, mone, W, r2, w4, OP_N, Bw, r, rr, OP_N, zero, nullptr, 0, 0, W + r, r2, w4, nb, true);
  cgemm<R>(s, r, r, r, mone, C, r, rr, OP_N, Bw, r, rr, OP_N, zero, nullptr, 0, 0, W + r * r2 + r, r2, w4, nb);
}

// merge of parent level l: P_a, P_b, C^{-1} (needs G_ab of level l)
template <typename R>
void factor_merge(const lsh_plan_s& P, FactorData<R>& F, int l, hipStream_t s) {
  F.scratch_reset();  // (a new level: the previous level's temporaries are done in stream order)
  if (P.lev[l].wr > 0) return factor_merge_lowrank(P, F, l, s);
  mem::Bind bind(F.keep);
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
  const int c = P.lev[l].c, nb = 1 << l;
  const long cc = (long)c * c;
  const cplx<R>* Sch = F.S[l + 1].template as<cplx<R>>();
  F.wr[l] = 0;
  const cplx<R>* G = P.Gab<R>(l);
  F.Pa[l].alloc(sizeof(cplx<R>) * nb * cc);
  F.Pb[l].alloc(sizeof(cplx<R>) * nb * cc);
  F.Ci[l].alloc(sizeof(cplx<R>) * nb * cc);
  cplx<R>* Pa = F.Pa[l].template as<cplx<R>>();
  cplx<R>* Pb = F.Pb[l].template as<cplx<R>>();
  cplx<R>* Ci = F.Ci[l].template as<cplx<R>>();
  cgemm<R>(s, c, c, c, one, Sch, c, 2 * cc, OP_N, G, c, 0, OP_N, zero, nullptr, 0, 0, Pa, c, cc, nb);
  cgemm<R>(s, c, c, c, one, Sch + cc, c, 2 * cc, OP_N, G, c, 0, OP_T, zero, nullptr, 0, 0, Pb, c, cc, nb);
  cgemm<R>(s, c, c, c, mone, Pb, c, cc, OP_N, Pa, c, cc, OP_N, zero, nullptr, 0, 0, Ci, c, cc, nb, true);
  {
    void* ws = F.scratch_buf(inverse_ws_bytes<R>(c, nb));
    F.info.emplace_back(sizeof(int) * nb);
    F.info_n.push_back(nb);
    F.info_what.push_back("singular merge matrix I - Pb Pa at level " + std::to_string(l));
    inverse<R>(s, Ci, c, c, cc, nb, ws, F.info.back().template as<int>());
  }
}

// Products with U_l that skip its identity rows (U = I on the skeleton rows
// J; T = U[rest, :] holds the others, nh[0] of them in half 0, nh[1] in half 1):
//   a_h = S_h U_h: the columns J of S_h placed (zero elsewhere), plus
//                  S_h[:, rest_h] T_h                        (both halves h)
//   S = U^T [b_0; b_1]: the rows J of [b_0; b_1] placed, plus
//                  T_h^T b_h[rest_h, :]                       (both halves h)
// over the nb boxes of parent level l.  Each box's S_h (c x c) sits at
// Sch + 2 c^2 box + c^2 h; a_h and b_h are c x k at stride sa / sb per box.
// The *_prep functions launch the placements and the gathers of S_h's
// columns rest_h (into G: nb c x nh[h] blocks per half) or of b_h's rows
// rest_h (into Rg: nb nh[h] x k blocks per half) on s, and return the
// products C += A B that complete the result (beta 1, in stream order after
// the gathers), for one launch each or a grouped launch.
template <typename R>
struct ScatterGemm {
  int M, N, K;
  const cplx<R>* A;
  long lda, sA;
  Op opA;
  const cplx<R>* B;
  long ldb, sB;
  cplx<R>* C;
  long ldc, sC;
  int batch;
};

inline void rest_counts(const Level& lv, int nh[2]) {
  nh[0] = lv.nrest0;
  nh[1] = (int)lv.rest.size() - lv.nrest0;
}

// entries of G (and of Rg per column) that one box needs
inline long rest_total(const Level& lv) { return std::max<long>(1, (long)lv.rest.size()); }

// one gather (kind 0: gather_cols with lim c; 1: gather_rows2), launched on s
// or, with a sink (FP32), kept for one grouped launch
template <typename R>
void gather_job(std::vector<GatherJob>* sink, hipStream_t s, int kind, int rows, int cols, const cplx<R>* src0,
                const cplx<R>* src1, int c, long lds, long ss, const int* idx, int off, cplx<R>* dst, long ldd,
                long sd, long batch) {
  if constexpr (sizeof(R) == 4) {
    if (sink) {
      sink->push_back({kind, rows, cols, src0, src1, c, lds, ss, idx, off, dst, ldd, sd, batch});
      return;
    }
  }
  if (kind == 0) gather_cols<R>(s, rows, cols, src0, lds, ss, idx, off, c, dst, ldd, sd, batch);
  else gather_rows2<R>(s, rows, cols, src0, src1, c, lds, ss, idx, off, dst, ldd, sd, batch);
}

template <typename R>
int scatter_su_prep(const lsh_plan_s& P, int l, const cplx<R>* Sch, cplx<R>* a0, cplx<R>* a1, long sa, cplx<R>* G,
                    hipStream_t s, ScatterGemm<R> out[2], std::vector<GatherJob>* sink = nullptr) {
  const Level& lv = P.lev[l];
  const int c = lv.c, k = lv.k, nb = 1 << l;
  const long cc = (long)c * c;
  int nh[2];
  rest_counts(lv, nh);
  cplx<R>* ah[2] = {a0, a1};
  int n = 0;
  for (int h = 0; h < 2; ++h) {
    const cplx<R>* Sh = Sch + h * cc;
    gather_job<R>(sink, s, 0, c, k, Sh, nullptr, c, c, 2 * cc, lv.skelIdx.as<int>(), h * c, ah[h], k, sa, nb);
    if (nh[h] == 0) continue;
    const int* rh = lv.restIdx.as<int>() + (h ? nh[0] : 0);
    cplx<R>* Gh = G + (h ? (long)nb * c * nh[0] : 0L);
    gather_job<R>(sink, s, 0, c, nh[h], Sh, nullptr, c, c, 2 * cc, rh, h * c, Gh, nh[h], (long)c * nh[h], nb);
    out[n++] = {c, k, nh[h], Gh, nh[h], (long)c * nh[h], OP_N, P.T<R>(l) + (h ? (long)nh[0] * k : 0L), k, 0,
                ah[h], k, sa, nb};
  }
  return n;
}

template <typename R>
int scatter_utb_prep(const lsh_plan_s& P, int l, const cplx<R>* b0, const cplx<R>* b1, long sb, cplx<R>* S,
                     cplx<R>* Rg, hipStream_t s, ScatterGemm<R> out[2], std::vector<GatherJob>* sink = nullptr) {
  const Level& lv = P.lev[l];
  const int c = lv.c, k = lv.k, nb = 1 << l;
  const long kk = (long)k * k;
  int nh[2];
  rest_counts(lv, nh);
  gather_job<R>(sink, s, 1, k, k, b0, b1, c, k, sb, lv.skelIdx.as<int>(), 0, S, k, kk, nb);
  const cplx<R>* bh[2] = {b0, b1};
  int n = 0;
  for (int h = 0; h < 2; ++h) {
    if (nh[h] == 0) continue;
    const int* rh = lv.restIdx.as<int>() + (h ? nh[0] : 0);
    cplx<R>* Rh = Rg + (h ? (long)nb * nh[0] * k : 0L);
    gather_job<R>(sink, s, 1, nh[h], k, bh[h], bh[h], c, k, sb, rh, h * c, Rh, k, (long)nh[h] * k, nb);
    out[n++] = {k, k, nh[h], P.T<R>(l) + (h ? (long)nh[0] * k : 0L), k, 0, OP_T, Rh, k, (long)nh[h] * k, S, k, kk,
                nb};
  }
  return n;
}

template <typename R>
void run_scatter_gemms(hipStream_t s, const ScatterGemm<R>* g, int n) {
  const cplx<R> one = mk<R>(1, 0);
  for (int i = 0; i < n; ++i)
    cgemm<R>(s, g[i].M, g[i].N, g[i].K, one, g[i].A, g[i].lda, g[i].sA, g[i].opA, g[i].B, g[i].ldb, g[i].sB, OP_N,
             one, g[i].C, g[i].ldc, g[i].sC, g[i].C, g[i].ldc, g[i].sC, g[i].batch);
}

template <typename R>
void scatter_su(const lsh_plan_s& P, int l, const cplx<R>* Sch, cplx<R>* a0, cplx<R>* a1, long sa, cplx<R>* G,
                hipStream_t s) {
  ScatterGemm<R> g[2];
  run_scatter_gemms<R>(s, g, scatter_su_prep<R>(P, l, Sch, a0, a1, sa, G, s, g));
}

template <typename R>
void scatter_utb(const lsh_plan_s& P, int l, const cplx<R>* b0, const cplx<R>* b1, long sb, cplx<R>* S,
                 cplx<R>* Rg, hipStream_t s) {
  ScatterGemm<R> g[2];
  run_scatter_gemms<R>(s, g, scatter_utb_prep<R>(P, l, b0, b1, sb, S, Rg, s, g));
}

// scattering matrices of level l (needs U_l)
template <typename R>
void factor_scatter(const lsh_plan_s& P, FactorData<R>& F, int l, hipStream_t s) {
  if (l == 0) return;
  mem::Bind bind(F.keep);
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
  const int c = P.lev[l].c, nb = 1 << l;
  const long cc = (long)c * c;
  const cplx<R>* Sch = F.S[l + 1].template as<cplx<R>>();
  const cplx<R>* Pa = F.Pa[l].template as<cplx<R>>();
  const cplx<R>* Pb = F.Pb[l].template as<cplx<R>>();
  const cplx<R>* Ci = F.Ci[l].template as<cplx<R>>();
  const int k = P.lev[l].k;
  const long ck = (long)c * k;
  if (P.lev[l].ident) {  // U_l = I (k = 2c): the products with U are placements
    F.S[l].alloc(sizeof(cplx<R>) * nb * (long)k * k);
    cplx<R>* S = F.S[l].template as<cplx<R>>();
    const long kk = (long)k * k;
    // S = [[S_a, 0], [0, S_b]] per box: the rows U_1^T a1 and U_2^T a2 start from
    fill_zero(s, S, sizeof(cplx<R>) * nb * kk);
    ccopy2d<R>(s, c, c, Sch, c, 2 * cc, S, k, kk, nb);
    ccopy2d<R>(s, c, c, Sch + cc, c, 2 * cc, S + ck + c, k, kk, nb);
    if (F.wr[l] > 0) {  // S <- S - P W' [L^T a1; R^T a2], in place (as below with U = I)
      // a1 = [S_a, 0] and a2 = [0, S_b], so [L^T a1; R^T a2] = [[L^T S_a, 0], [0, R^T S_b]] and
      // W' times it is [W'_1 L^T S_a, W'_2 R^T S_b] (W'_1, W'_2: W''s first and last r columns)
      const int r = F.wr[l];
      const long rk = (long)r * k, cr = (long)c * r, w4 = 4L * r * r;
      cplx<R>* q = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * 4 * rk);
      cplx<R>* yv = q + nb * 2 * rk;
      cgemm<R>(s, r, c, c, one, P.W<R>(l, 1), c, 0, OP_N, S, k, kk, OP_N, zero, nullptr, 0, 0, q, k, 2 * rk, nb);
      cgemm<R>(s, r, c, c, one, P.W<R>(l, 3), c, 0, OP_N, S + ck + c, k, kk, OP_N, zero, nullptr, 0, 0, q + rk + c, k,
               2 * rk, nb);
      cgemm<R>(s, 2 * r, c, r, one, Ci, 2 * r, w4, OP_N, q, k, 2 * rk, OP_N, zero, nullptr, 0, 0, yv, k, 2 * rk, nb);
      cgemm<R>(s, 2 * r, c, r, one, Ci + r, 2 * r, w4, OP_N, q + rk + c, k, 2 * rk, OP_N, zero, nullptr, 0, 0, yv + c,
               k, 2 * rk, nb);
      cgemm<R>(s, c, k, r, mone, Pa, r, cr, OP_N, yv, k, rk, OP_N, one, S, k, ck, S, k, ck, 2 * nb);
      return;
    }
    // Schur form: a2 = [0, S_b] - Pb a1, y = C^{-1} a2 (the lower rows of S), then a1 - Pa y (the upper rows)
    cplx<R>* a2 = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * ck);
    ccopy2d<R>(s, c, k, S + ck, k, kk, a2, k, ck, nb);
    cgemm<R>(s, c, k, c, mone, Pb, c, cc, OP_N, S, k, kk, OP_N, one, a2, k, ck, a2, k, ck, nb);
    cgemm<R>(s, c, k, c, one, Ci, c, cc, OP_N, a2, k, ck, OP_N, zero, nullptr, 0, 0, S + ck, k, kk, nb);
    cgemm<R>(s, c, k, c, mone, Pa, c, cc, OP_N, S + ck, k, kk, OP_N, one, S, k, kk, S, k, kk, nb);
    return;
  }
  const long nrt = rest_total(P.lev[l]);
  cplx<R>* G = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * c * nrt);
  cplx<R>* Rg = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * nrt * k);
  if (F.wr[l] > 0) {
    // X [a1; a2] = [a1; a2] - P W' [L^T a1; R^T a2] (a1, a2 interleaved per box in A12)
    const int r = F.wr[l];
    const long rk = (long)r * k, cr = (long)c * r, w4 = 4L * r * r;
    cplx<R>* a = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * 2 * ck);
    cplx<R>* q = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * 4 * rk);
    cplx<R>* yv = q + nb * 2 * rk;
    scatter_su<R>(P, l, Sch, a, a + ck, 2 * ck, G, s);
    cgemm<R>(s, r, k, c, one, P.W<R>(l, 1), c, 0, OP_N, a, k, 2 * ck, OP_N, zero, nullptr, 0, 0, q, k, 2 * rk, nb);
    cgemm<R>(s, r, k, c, one, P.W<R>(l, 3), c, 0, OP_N, a + ck, k, 2 * ck, OP_N, zero, nullptr, 0, 0, q + rk, k,
             2 * rk, nb);
    cgemm<R>(s, 2 * r, k, 2 * r, one, Ci, 2 * r, w4, OP_N, q, k, 2 * rk, OP_N, zero, nullptr, 0, 0, yv, k, 2 * rk,
             nb);
    cgemm<R>(s, c, k, r, mone, Pa, r, cr, OP_N, yv, k, rk, OP_N, one, a, k, ck, a, k, ck, 2 * nb);
    F.S[l].alloc(sizeof(cplx<R>) * nb * (long)k * k);
    scatter_utb<R>(P, l, a, a + ck, 2 * ck, F.S[l].template as<cplx<R>>(), Rg, s);
    return;
  }
  cplx<R>* a1 = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * ck);
  cplx<R>* a2 = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * ck);
  cplx<R>* y = F.template scratch_buf<cplx<R>>(sizeof(cplx<R>) * nb * ck);
  scatter_su<R>(P, l, Sch, a1, a2, ck, G, s);
  {
    // a2 <- A2 - Pb A1 ; y = C^{-1} a2 ; a1 <- A1 - Pa y
    cgemm<R>(s, c, k, c, mone, Pb, c, cc, OP_N, a1, k, ck, OP_N, one, a2, k, ck, a2, k, ck, nb);
    cgemm<R>(s, c, k, c, one, Ci, c, cc, OP_N, a2, k, ck, OP_N, zero, nullptr, 0, 0, y, k, ck, nb);
    cgemm<R>(s, c, k, c, mone, Pa, c, cc, OP_N, y, k, ck, OP_N, one, a1, k, ck, a1, k, ck, nb);
  }
  F.S[l].alloc(sizeof(cplx<R>) * nb * (long)k * k);
  scatter_utb<R>(P, l, a1, y, ck, F.S[l].template as<cplx<R>>(), Rg, s);
}  // (scratch freed in stream order)

// Woodbury levels whose inverse order fits the in-LDS Gauss-Jordan run as one
// persistent launch (merge and scattering matrices of every box;
// merge_levels) when they have at least lsh_fused_levels(min_boxes) boxes;
// 0 switches this off (the separate launches; the same bits).
constexpr int kFusedMinBoxes = 0;  // (measured slower than the separate launches on MI355X)
int g_fused_min_boxes = kFusedMinBoxes;  // fuse levels with at least this many boxes (0: never)

template <typename R>
bool level_fused(const lsh_plan_s& P, int l) {
  return sizeof(R) == 4 && g_fused_min_boxes > 0 && (1 << l) >= g_fused_min_boxes && P.lev[l].wr > 0 &&
         !P.lev[l].ident && merge_level_fits(P.lev[l].wr);
}

// The level-l entry of a persistent merge launch for one FP32 factor:
// the factor's own parts from keep, the temporaries from tmp.
MergeLevelDev merge_entry(const lsh_plan_s& P, FactorData<float>& F, int l, mem::Arena& keep, mem::Arena& tmp,
                          int* info) {
  const int c = P.lev[l].c, r = P.lev[l].wr, nb = 1 << l, k = l >= 1 ? P.lev[l].k : 0;
  const long cr = (long)c * r, rr = (long)r * r, ck = (long)c * k, rk = (long)r * k;
  F.wr[l] = r;
  F.Pa[l].alloc_in(keep, sizeof(c32) * nb * 2 * cr);
  F.Ci[l].alloc_in(keep, sizeof(c32) * nb * 4 * rr);
  if (l >= 1) F.S[l].alloc_in(keep, sizeof(c32) * nb * (long)k * k);
  MergeLevelDev g{};
  g.Sch = F.S[l + 1].as<c32>();
  g.Pm = P.W<float>(l, 0);
  g.Qm = P.W<float>(l, 1);
  g.U = l >= 1 ? P.U<float>(l) : nullptr;
  g.Pst = F.Pa[l].as<c32>();
  g.W = F.Ci[l].as<c32>();
  g.S = l >= 1 ? F.S[l].as<c32>() : nullptr;
  g.T = static_cast<c32*>(tmp.take(sizeof(c32) * nb * 3 * rr));
  g.A12 = l >= 1 ? static_cast<c32*>(tmp.take(sizeof(c32) * nb * 2 * ck)) : nullptr;
  g.Qb = l >= 1 ? static_cast<c32*>(tmp.take(sizeof(c32) * nb * 4 * rk)) : nullptr;
  g.perm = static_cast<int*>(tmp.take(sizeof(int) * nb * r));
  if (l >= 1) {
    const Level& v = P.lev[l];
    const long nrt = rest_total(v);
    g.Ur = P.T<float>(l);
    g.rest = v.restIdx.as<int>();
    g.skel = v.skelIdx.as<int>();
    g.n0 = v.nrest0;
    g.n1 = (int)v.rest.size() - v.nrest0;
    g.G = static_cast<c32*>(tmp.take(sizeof(c32) * nb * (long)c * nrt));
    g.Rg = static_cast<c32*>(tmp.take(sizeof(c32) * nb * nrt * k));
  }
  g.info = info;
  g.c = c;
  g.r = r;
  g.k = k;
  g.nb = nb;
  return g;
}

// merge and scattering matrices of level l in one launch (needs G_l and U_l)
template <typename R>
void factor_level_fused(const lsh_plan_s& P, FactorData<R>& F, int l, hipStream_t s) {
  if constexpr (sizeof(R) == 4) {
    F.scratch_reset();
    mem::Bind bind(F.keep);
    const int nb = 1 << l;
    F.info.emplace_back(sizeof(int) * nb);
    F.info_n.push_back(nb);
    F.info_what.push_back("singular merge matrix I - Bw Aw at level " + std::to_string(l));
    std::vector<MergeLevelDev> e{merge_entry(P, F, l, *F.keep, *F.scr, F.info.back().template as<int>())};
    DevBuf table;
    table.alloc_in(*F.scr, merge_level_table_bytes(1));
    int* counter = F.template scratch_buf<int>(sizeof(int));
    merge_levels(s, e, table, counter);
  }
}

template <typename R>
void factor_level(const lsh_plan_s& P, FactorData<R>& F, int l, hipStream_t s) {
  if (level_fused<R>(P, l)) return factor_level_fused(P, F, l, s);
  factor_merge(P, F, l, s);
  factor_scatter(P, F, l, s);
}

// The apply vectors (for APPLY_GROUP right-hand sides), from the factor's keep arena.
template <typename R>
void ensure_apply_ws(const lsh_plan_s& P, FactorData<R>& F) {
  if (F.ws_nrhs) return;
  mem::Bind bind(F.keep);
  const int L = P.L, nrhs = APPLY_GROUP;
  F.r.alloc(sizeof(cplx<R>) * (size_t)nrhs * P.nleaf * P.mL);
  F.rt.clear();
  F.wt.clear();
  F.rt.resize(L + 1);
  F.wt.resize(L + 1);
  size_t big = 0;
  for (int l = 1; l <= L; ++l) {
    const size_t e = (size_t)nrhs * ((size_t)1 << l) * P.lev[l].k;
    F.rt[l].alloc(sizeof(cplx<R>) * e);
    F.wt[l].alloc(sizeof(cplx<R>) * e);
    if (e > big) big = e;
  }
  F.t1.alloc(sizeof(cplx<R>) * big);
  F.t2.alloc(sizeof(cplx<R>) * big);
  F.t3.alloc(sizeof(cplx<R>) * big);
  F.ty.alloc(sizeof(cplx<R>) * big);
  F.tw.alloc(sizeof(cplx<R>) * big);
  if (sizeof(R) == 4) F.tk.alloc(kSplitKBytes);  // (FP64 products do not split)
  F.ws_nrhs = nrhs;
}

template <typename R>
void factor_build(const lsh_plan_s& P, const double* b, FactorData<R>& F, hipStream_t s) {
  factor_init(P, F);
  factor_leaves(P, b, F, s);
  for (int l = P.L - 1; l >= 0; --l) factor_level(P, F, l, s);
  factor_check(F, s);
  ensure_apply_ws(P, F);
}

// up to this many box vectors the shared products stream the matrix rows
// (multi-vector GEMV over vector groups); above it they are MFMA GEMMs,
// split along K when they have few output tiles (FP32).  fourier-1024, one
// apply, with 8 / 64 / 256 / 1024 / 8192: FP32 2.62 / 2.64 / 2.61 / 2.61 /
// 2.86 ms, FP64 7.14 / 4.40 / 3.69 / 3.45 / 3.76 ms.
template <typename R>
constexpr int skinny() { return 1024; }

// Y[v] = alpha M X[v] + beta Z[v] for B vectors (strides ldx, ldz, ldy) and
// one shared matrix M (rows x cols, row-major); (MtB, ldb, opB) give M^T as
// the B operand of the GEMM used for many vectors.
template <typename R>
void shared_mv(hipStream_t s, int rows, int cols, cplx<R> alpha, const cplx<R>* M, const cplx<R>* MtB, long ldb,
               Op opB, const cplx<R>* X, long ldx, cplx<R> beta, const cplx<R>* Z, long ldz, cplx<R>* Y, long ldy,
               int B, DevBuf& ws, bool ident = false) {
  if (ident) {  // M = I (a level that keeps all its candidates)
    caxpby<R>(s, rows, B, alpha, X, ldx, beta, Z, ldz, Y, ldy);
    return;
  }
  if (B <= skinny<R>())
    cmgemv<R>(s, rows, cols, alpha, M, cols, X, ldx, beta, Z, ldz, Y, ldy, B);
  else
    cgemm_ws<R>(s, B, rows, cols, alpha, X, ldx, 0, OP_N, MtB, ldb, 0, opB, beta, Z, ldz, 0, Y, ldy, 0, 1, ws.p,
                ws.bytes);
}

// out = X_tau in on a Woodbury level, three launches:
//   q = [L^T a; R^T b]  (shared [L^T; R^T], one two-block product),
//   y = W' q            (per box, 2r x 2r),
//   out = in - [S_a L y1; S_b R y2]  (per box, as 2B problems of c x r).
// Transposed: X^T = I - Q^T (I + Q P)^{-T} P^T with Q^T = [[0, L], [R, 0]]:
//   p = [(S_a L)^T a; (S_b R)^T b], z = W'^T p = [z2; z1],
//   out = in - [L z2; R z1]  (shared [L; R], one two-block product).
template <typename R>
void apply_X_lowrank(const lsh_plan_s& P, FactorData<R>& F, int l, int nrhs, const cplx<R>* in, cplx<R>* out,
                     hipStream_t s, bool transposed) {
  const int c = P.lev[l].c, r = F.wr[l], nb = 1 << l, B = nrhs * nb;
  const long cr = (long)c * r, w4 = 4L * r * r;
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
  cplx<R>* q = F.tw.template as<cplx<R>>();  // [B][2r]
  cplx<R>* y = F.ty.template as<cplx<R>>();  // [B][2r]
  const cplx<R>* Pm = P.W<R>(l, 0);  // [L; R]
  const cplx<R>* Qm = P.W<R>(l, 1);  // [L^T; R^T]
  if (!transposed) {
    if (B <= skinny<R>())
      cmgemv2<R>(s, 2 * r, r, c, c, one, Qm, c, in, 2 * c, zero, nullptr, 0, q, 2 * r, B);
    else  // two strided products: (a, L) and (b, R)
      cgemm_ws<R>(s, B, r, c, one, in, 2 * c, c, OP_N, Pm, r, cr, OP_N, zero, nullptr, 0, 0, q, 2 * r, r, 2, F.tk.p,
                  F.tk.bytes);
    cgemv<R>(s, 2 * r, 2 * r, one, F.Ci[l].template as<cplx<R>>(), 2 * r, w4, nb, q, 2 * r, zero, nullptr, 0, y,
             2 * r, B);
    cgemv<R>(s, c, r, mone, F.Pa[l].template as<cplx<R>>(), r, cr, 2 * nb, y, r, one, in, c, out, c, 2 * B);
  } else {
    cgemv<R>(s, r, c, one, F.PaT[l].template as<cplx<R>>(), c, cr, 2 * nb, in, c, zero, nullptr, 0, q, r, 2 * B);
    cgemv<R>(s, 2 * r, 2 * r, one, F.CiT[l].template as<cplx<R>>(), 2 * r, w4, nb, q, 2 * r, zero, nullptr, 0, y,
             2 * r, B);
    if (B <= skinny<R>())
      cmgemv2<R>(s, 2 * c, c, r, r, mone, Pm, r, y, 2 * r, one, in, 2 * c, out, 2 * c, B);
    else  // (z2, L^T) -> a, (z1, R^T) -> b
      cgemm_ws<R>(s, B, c, r, mone, y, 2 * r, r, OP_N, Qm, c, cr, OP_N, one, in, 2 * c, c, out, 2 * c, c, 2,
                  F.tk.p, F.tk.bytes);
  }
}

// out = X_tau in for every box of parent level l (B = nrhs * 2^l problems, [B][2c])
template <typename R>
void apply_X(const lsh_plan_s& P, FactorData<R>& F, int l, int nrhs, const cplx<R>* in, cplx<R>* out,
             hipStream_t s, bool transposed = false) {
  if (F.wr[l] > 0) return apply_X_lowrank(P, F, l, nrhs, in, out, s, transposed);
  const int c = P.lev[l].c, nb = 1 << l, B = nrhs * nb;
  const long cc = (long)c * c;
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
  cplx<R>* ty = F.ty.template as<cplx<R>>();
  // X = [[I, Pa], [Pb, I]]^{-1};  X^T has the same form with Pa -> Pb^T, Pb -> Pa^T, C^{-1} -> C^{-T}
  const cplx<R>* Pa = (transposed ? F.PbT[l] : F.Pa[l]).template as<cplx<R>>();
  const cplx<R>* Pb = (transposed ? F.PaT[l] : F.Pb[l]).template as<cplx<R>>();
  const cplx<R>* Ci = (transposed ? F.CiT[l] : F.Ci[l]).template as<cplx<R>>();
  // ty = b - Pb a
  cgemv<R>(s, c, c, mone, Pb, c, cc, nb, in, 2 * c, one, in + c, 2 * c, ty, c, B);
  // y = C^{-1} ty  -> second half of out
  cgemv<R>(s, c, c, one, Ci, c, cc, nb, ty, c, zero, nullptr, 0, out + c, 2 * c, B);
  // top = a - Pa y -> first half of out
  cgemv<R>(s, c, c, mone, Pa, c, cc, nb, out + c, 2 * c, one, in, 2 * c, out, 2 * c, B);
}

template <typename R>
void ensure_transposed(const lsh_plan_s& P, FactorData<R>& F, hipStream_t s) {
  if (F.has_T) return;
  LSH_REQUIRE(F.want_T, LSH_ERR_INVALID_ARG,
              "M^T needs a factor created with LSH_FACTOR_TRANSPOSE (room for the transposed copies)");
  mem::Bind bind(F.keep);
  const int L = P.L;
  F.XT.alloc(F.X.bytes);
  ctranspose<R>(s, F.X.template as<cplx<R>>(), P.mL, P.mL, F.XT.template as<cplx<R>>(), P.nleaf);
  F.ST.clear(); F.PaT.clear(); F.PbT.clear(); F.CiT.clear();
  F.ST.resize(L + 1); F.PaT.resize(L); F.PbT.resize(L); F.CiT.resize(L);
  for (int l = 1; l <= L; ++l) {
    const int k = P.lev[l].k;
    F.ST[l].alloc(F.S[l].bytes);
    ctranspose<R>(s, F.S[l].template as<cplx<R>>(), k, k, F.ST[l].template as<cplx<R>>(), 1L << l);
  }
  for (int l = 0; l < L; ++l) {
    const int c = P.lev[l].c;
    if (F.wr[l] > 0) {  // Woodbury level: [S_a L; S_b R] blocks (c x r) and W' (2r x 2r)
      const int r = F.wr[l];
      F.PaT[l].alloc(F.Pa[l].bytes);
      F.CiT[l].alloc(F.Ci[l].bytes);
      ctranspose<R>(s, F.Pa[l].template as<cplx<R>>(), c, r, F.PaT[l].template as<cplx<R>>(), 2L << l);
      ctranspose<R>(s, F.Ci[l].template as<cplx<R>>(), 2 * r, 2 * r, F.CiT[l].template as<cplx<R>>(), 1L << l);
      continue;
    }
    F.PaT[l].alloc(F.Pa[l].bytes);
    F.PbT[l].alloc(F.Pb[l].bytes);
    F.CiT[l].alloc(F.Ci[l].bytes);
    ctranspose<R>(s, F.Pa[l].template as<cplx<R>>(), c, c, F.PaT[l].template as<cplx<R>>(), 1L << l);
    ctranspose<R>(s, F.Pb[l].template as<cplx<R>>(), c, c, F.PbT[l].template as<cplx<R>>(), 1L << l);
    ctranspose<R>(s, F.Ci[l].template as<cplx<R>>(), c, c, F.CiT[l].template as<cplx<R>>(), 1L << l);
  }
  F.vb.clear();
  F.vb.resize(L);
  for (int l = 1; l < L; ++l)
    F.vb[l].alloc(sizeof(cplx<R>) * (size_t)APPLY_GROUP * ((size_t)1 << l) * 2 * P.lev[l].c);
  LSH_HIP(hipStreamSynchronize(s));
  F.has_T = true;
}

// Woodbury levels with at least this many box vectors (LSH_LEVEL_FUSED
// overrides it) whose box vectors fit one workgroup's LDS run each pass in one
// launch (level_up_fused / level_down_fused) instead of six to seven.
int level_fused_min() {
  static const int v = [] {
    const char* e = std::getenv("LSH_LEVEL_FUSED");
    return e && *e ? std::atoi(e) : 512;
  }();
  return v;
}

template <typename R>
bool level_fused(const lsh_plan_s& P, FactorData<R>& F, int l, int B, LevelApply<R>& A) {
  if (g_apply_fused_min <= 0 || B < g_apply_fused_min || l < 1 || l >= P.L || P.lev[l].ident || F.wr[l] <= 0)
    return false;
  const int c = P.lev[l].c, k = P.lev[l].k, r = F.wr[l];
  if ((size_t)(k + 6 * c + 4 * r) * sizeof(cplx<R>) > LEVEL_FUSED_LDS) return false;
  A = {c, k, r, 1 << l, P.U<R>(l), P.Ut<R>(l), P.W<R>(l, 1), P.Gab<R>(l), P.Gabt<R>(l),
       F.S[l + 1].template as<cplx<R>>(), F.Ci[l].template as<cplx<R>>(), F.Pa[l].template as<cplx<R>>()};
  return true;
}

template <typename R>
void apply_M(const lsh_plan_s& P, const double* b, FactorData<R>& F, const z64* f, z64* q, int nrhs,
             hipStream_t s) {
  LSH_REQUIRE(F.ws_nrhs >= nrhs, LSH_ERR_INVALID_ARG, "internal: apply workspace");
  const int L = P.L;
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
  const double k2 = P.kappa * P.kappa;
  cplx<R>* r = F.r.template as<cplx<R>>();
  cplx<R>* t1 = F.t1.template as<cplx<R>>();
  cplx<R>* t2 = F.t2.template as<cplx<R>>();
  cplx<R>* t3 = F.t3.template as<cplx<R>>();
  leaf_up<R>(s, F.X.template as<cplx<R>>(), P.Ut<R>(L), P.mL, P.lev[L].k, f, r, F.rt[L].template as<cplx<R>>(),
             P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), P.nleaf, P.n, nrhs);
  // upward pass
  for (int l = L - 1; l >= 1; --l) {
    const int c = P.lev[l].c, k = P.lev[l].k, B = nrhs << l;
    LevelApply<R> A;
    if (level_fused(P, F, l, B, A)) {
      level_up_fused<R>(s, A, F.rt[l + 1].template as<cplx<R>>(), F.rt[l].template as<cplx<R>>(), B);
      continue;
    }
    apply_X<R>(P, F, l, nrhs, F.rt[l + 1].template as<cplx<R>>(), t1, s);
    // rt_l = U_l^T xv
    shared_mv<R>(s, k, 2 * c, one, P.Ut<R>(l), P.U<R>(l), k, OP_N, t1, 2 * c, zero, nullptr, 0,
                 F.rt[l].template as<cplx<R>>(), k, B, F.tk, P.lev[l].ident);
  }
  // root: w_children = Ghat X_root [rt_a; rt_b]
  {
    const int c = P.lev[0].c;
    apply_X<R>(P, F, 0, nrhs, F.rt[1].template as<cplx<R>>(), t1, s);
    cplx<R>* w1 = F.wt[1].template as<cplx<R>>();
    cmgemv2<R>(s, 2 * c, c, -c, c, one, P.Gab<R>(0), c, t1 + c, 2 * c, zero, nullptr, 0, w1, 2 * c, nrhs,
               P.Gabt<R>(0));
  }
  // downward pass
  for (int l = 1; l <= L - 1; ++l) {
    const int c = P.lev[l].c, k = P.lev[l].k, nb = 1 << l, B = nrhs * nb;
    const long cc = (long)c * c;
    LevelApply<R> A;
    if (level_fused(P, F, l, B, A)) {
      level_down_fused<R>(s, A, F.wt[l].template as<cplx<R>>(), F.rt[l + 1].template as<cplx<R>>(),
                          F.wt[l + 1].template as<cplx<R>>(), B);
      continue;
    }
    // u = U_l wt_l  ([B][2c])
    shared_mv<R>(s, 2 * c, k, one, P.U<R>(l), P.U<R>(l), k, OP_T, F.wt[l].template as<cplx<R>>(), k, zero, nullptr,
                 0, t1, 2 * c, B, F.tk, P.lev[l].ident);
    // d = rt_children - diag(S_a, S_b) u  ([2B][c])
    cgemv<R>(s, c, c, mone, F.S[l + 1].template as<cplx<R>>(), c, cc, 2 * nb, t1, c, one,
             F.rt[l + 1].template as<cplx<R>>(), c, t2, c, 2 * B);
    // qt = X_tau d
    apply_X<R>(P, F, l, nrhs, t2, t3, s);
    // wt_children = Ghat qt + u
    cplx<R>* wc = F.wt[l + 1].template as<cplx<R>>();
    if (B <= skinny<R>()) {  // both blocks in one launch
      cmgemv2<R>(s, 2 * c, c, -c, c, one, P.Gab<R>(l), c, t3 + c, 2 * c, one, t1, 2 * c, wc, 2 * c, B,
                 P.Gabt<R>(l));
    } else {
      shared_mv<R>(s, c, c, one, P.Gab<R>(l), P.Gab<R>(l), c, OP_T, t3 + c, 2 * c, one, t1, 2 * c, wc, 2 * c, B,
                   F.tk);
      shared_mv<R>(s, c, c, one, P.Gabt<R>(l), P.Gab<R>(l), c, OP_N, t3, 2 * c, one, t1 + c, 2 * c, wc + c, 2 * c,
                   B, F.tk);
    }
  }
  leaf_down<R>(s, F.X.template as<cplx<R>>(), P.U<R>(L), P.mL, P.lev[L].k, F.wt[L].template as<cplx<R>>(), r, q,
               b, k2, P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), P.nleaf, P.n, nrhs);
}

// q = M^T g: the steps of Algorithm 2 transposed, in reverse order.
template <typename R>
void apply_MT(const lsh_plan_s& P, const double* b, FactorData<R>& F, const z64* g, z64* q, int nrhs,
              hipStream_t s) {
  LSH_REQUIRE(F.ws_nrhs >= nrhs, LSH_ERR_INVALID_ARG, "internal: apply workspace");
  ensure_transposed(P, F, s);
  const int L = P.L;
  const cplx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
  const double k2 = P.kappa * P.kappa;
  cplx<R>* t1 = F.t1.template as<cplx<R>>();
  cplx<R>* t2 = F.t2.template as<cplx<R>>();
  cplx<R>* t3 = F.t3.template as<cplx<R>>();
  // leaves: wb_L = -U_L^T B X^T g
  leaf_up<R>(s, F.XT.template as<cplx<R>>(), P.Ut<R>(L), P.mL, P.lev[L].k, g, nullptr,
             F.wt[L].template as<cplx<R>>(), P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), P.nleaf, P.n, nrhs, b, -k2);
  // transposed downward pass, leaves upward
  for (int l = L - 1; l >= 1; --l) {
    const int c = P.lev[l].c, k = P.lev[l].k, nb = 1 << l, B = nrhs * nb;
    const long cc = (long)c * c;
    const cplx<R>* wc = F.wt[l + 1].template as<cplx<R>>();
    cplx<R>* vb = F.vb[l].template as<cplx<R>>();
    // vb = Ghat wc
    if (B <= skinny<R>()) {  // both blocks in one launch
      cmgemv2<R>(s, 2 * c, c, -c, c, one, P.Gab<R>(l), c, wc + c, 2 * c, zero, nullptr, 0, vb, 2 * c, B,
                 P.Gabt<R>(l));
    } else {
      shared_mv<R>(s, c, c, one, P.Gab<R>(l), P.Gab<R>(l), c, OP_T, wc + c, 2 * c, zero, nullptr, 0, vb, 2 * c, B,
                   F.tk);
      shared_mv<R>(s, c, c, one, P.Gabt<R>(l), P.Gab<R>(l), c, OP_N, wc, 2 * c, zero, nullptr, 0, vb + c, 2 * c, B,
                   F.tk);
    }
    // t3 = X^T vb ; t2 = wc - diag(S_a^T, S_b^T) t3
    apply_X<R>(P, F, l, nrhs, vb, t3, s, true);
    cgemv<R>(s, c, c, mone, F.ST[l + 1].template as<cplx<R>>(), c, cc, 2 * nb, t3, c, one, wc, c, t2, c, 2 * B);
    // wb_l = U_l^T t2
    shared_mv<R>(s, k, 2 * c, one, P.Ut<R>(l), P.U<R>(l), k, OP_N, t2, 2 * c, zero, nullptr, 0,
                 F.wt[l].template as<cplx<R>>(), k, B, F.tk, P.lev[l].ident);
  }
  // root: rb_1 = X_root^T Ghat wb_1
  {
    const int c = P.lev[0].c;
    const cplx<R>* wc = F.wt[1].template as<cplx<R>>();
    cmgemv2<R>(s, 2 * c, c, -c, c, one, P.Gab<R>(0), c, wc + c, 2 * c, zero, nullptr, 0, t1, 2 * c, nrhs,
               P.Gabt<R>(0));
    apply_X<R>(P, F, 0, nrhs, t1, F.rt[1].template as<cplx<R>>(), s, true);
  }
  // transposed upward pass: rb_children = X^T (vb + U_l rb_l)
  for (int l = 1; l <= L - 1; ++l) {
    const int c = P.lev[l].c, k = P.lev[l].k, nb = 1 << l, B = nrhs * nb;
    const cplx<R>* vb = F.vb[l].template as<cplx<R>>();
    shared_mv<R>(s, 2 * c, k, one, P.U<R>(l), P.U<R>(l), k, OP_T, F.rt[l].template as<cplx<R>>(), k, one, vb, 2 * c,
                 t1, 2 * c, B, F.tk, P.lev[l].ident);
    apply_X<R>(P, F, l, nrhs, t1, F.rt[l + 1].template as<cplx<R>>(), s, true);
  }
  // leaves: q = X^T (g + U_L rb_L)
  leaf_tdown<R>(s, F.XT.template as<cplx<R>>(), P.U<R>(L), P.mL, P.lev[L].k, F.rt[L].template as<cplx<R>>(), g, q,
                P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), P.nleaf, P.n, nrhs);
}

}  // namespace

struct lsh_factor_s {
  lsh_plan_s* plan = nullptr;
  // the caller's factor workspace: keep (b, the factor, apply vectors) and scr
  mem::Arena keep, scr;
  DevBuf b;  // private copy of b (device, FP64)
  DevBuf bad;  // non-finite flag of the input check
  FactorData<float> f32;
  FactorData<double> f64;
  // y = M x (or M^T x) in groups of APPLY_GROUP right-hand sides
  void apply(const z64* x, z64* y, int nrhs, hipStream_t s, bool transpose = false) {
    const long N = (long)plan->n * plan->n;
    for (int r0 = 0; r0 < nrhs; r0 += APPLY_GROUP) {
      const int nr = std::min(APPLY_GROUP, nrhs - r0);
      const z64* xi = x + r0 * N;
      z64* yi = y + r0 * N;
      if (plan->d.hbs_prec == LSH_FP32) {
        if (transpose) apply_MT<float>(*plan, b.as<double>(), f32, xi, yi, nr, s);
        else apply_M<float>(*plan, b.as<double>(), f32, xi, yi, nr, s);
      } else {
        if (transpose) apply_MT<double>(*plan, b.as<double>(), f64, xi, yi, nr, s);
        else apply_M<double>(*plan, b.as<double>(), f64, xi, yi, nr, s);
      }
    }
  }
};

namespace {

__global__ void k_check_finite(const double* b, long n, int* bad) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!isfinite(b[i])) *bad = 1;
}

// f = -kappa^2 b u_inc
__global__ void k_rhs(z64* f, const z64* u, const double* b, double k2, long N) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    f[i] = (-k2 * b[i]) * u[i];
}

// right-hand sides solved together by the lockstep solver (memory: the
// Krylov basis holds (maxit + 1) * SOLVE_GROUP grid vectors)
constexpr int SOLVE_GROUP = 8;

// FGMRES arrays for G right-hand sides in lockstep and maxit iterations,
// carved from the caller's solve workspace: f [G][N] (right-hand sides),
// V [maxit + 1][G][N], Z [maxit][G][N], the Hessenberg columns h1, h2
// [G][maxit + 2], the reduction partials, res [G][N].
struct SolveWs {
  int G = 0, maxit = 0;
  z64 *f = nullptr, *V = nullptr, *Z = nullptr, *h1 = nullptr, *h2 = nullptr, *part = nullptr, *res = nullptr;
  template <typename Take>
  static SolveWs carve(Take&& take, long N, int G, int maxit) {
    SolveWs w;
    w.G = G;
    w.maxit = maxit;
    w.f = static_cast<z64*>(take(sizeof(z64) * (size_t)G * N));
    w.V = static_cast<z64*>(take(sizeof(z64) * (size_t)(maxit + 1) * G * N));
    w.Z = static_cast<z64*>(take(sizeof(z64) * (size_t)maxit * G * N));
    w.h1 = static_cast<z64*>(take(sizeof(z64) * (size_t)G * (maxit + 2)));
    w.h2 = static_cast<z64*>(take(sizeof(z64) * (size_t)G * (maxit + 2)));
    w.part = static_cast<z64*>(take(multidot_partial_bytes(maxit + 2)));
    w.res = static_cast<z64*>(take(sizeof(z64) * (size_t)G * N));
    return w;
  }
  static size_t bytes(long N, int G, int maxit) {
    mem::Sizer z;
    carve([&](size_t b) { z.add(b); return (void*)nullptr; }, N, G, maxit);
    return z.total;
  }
};

// Stream time of the three phases of an FGMRES iteration (preconditioner,
// operator, Gram-Schmidt), from event pairs read after the iteration's
// synchronisation; added to the info's ms fields.
struct PhaseClock {
  bool on = false;
  hipEvent_t e[4] = {};
  double ms[3] = {0, 0, 0};
  explicit PhaseClock(bool enable) : on(enable) {
    if (on)
      for (auto& x : e) LSH_HIP(hipEventCreate(&x));
  }
  ~PhaseClock() {
    if (on)
      for (auto x : e) (void)hipEventDestroy(x);
  }
  PhaseClock(const PhaseClock&) = delete;
  PhaseClock& operator=(const PhaseClock&) = delete;
  void mark(int i, hipStream_t s) {
    if (on) LSH_HIP(hipEventRecord(e[i], s));
  }
  void add() {  // (after the stream has been synchronised)
    if (!on) return;
    for (int q = 0; q < 3; ++q) {
      float t = 0;
      LSH_HIP(hipEventElapsedTime(&t, e[q], e[q + 1]));
      ms[q] += t;
    }
  }
  void store(lsh_info* info) const {
    if (!on || !info) return;
    info->ms_precond += ms[0];
    info->ms_operator += ms[1];
    info->ms_ortho += ms[2];
  }
};

// Right-preconditioned flexible GMRES on A (or on A^T = I + K B with M^T
// when transposed), x0 = 0, CGS2, Givens rotations on the host.
void fgmres_one(lsh_factor_s& F, SolveWs& W, const z64* f, z64* x, const lsh_solve_opts& o, lsh_info* info,
                double& true_res, int& conv, hipStream_t s, bool transposed = false) {
  lsh_plan_s& P = *F.plan;
  const long N = (long)P.n * P.n;
  const int maxit = o.maxit;
  LSH_REQUIRE(W.maxit >= maxit && W.G >= 1, LSH_ERR_INVALID_ARG, "internal: solve workspace");
  z64* V = W.V;
  z64* Z = W.Z;
  z64* h1 = W.h1;
  z64* h2 = W.h2;
  z64* part = W.part;
  multidot(s, f, 0, 1, f, N, h1, part);
  z64 fn;
  LSH_HIP(hipMemcpyAsync(&fn, h1, sizeof(z64), hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  const double beta = std::sqrt(fn.x);
  if (info) { info->iterations = 0; info->residual = 0; info->history[0] = 1.0; }
  if (beta == 0) {
    fill_zero(s, x, sizeof(z64) * N);
    true_res = 0;
    return;
  }
  scale_by_invnorm(s, V, f, h1, N);
  std::vector<std::complex<double>> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), g(maxit + 1, 0.0);
  g[0] = beta;
  std::vector<z64> hv(maxit + 2), hv2(maxit + 2);
  int j = 0, its = 0;
  double est = 1.0;
  PhaseClock clk(info != nullptr);
  for (j = 0; j < maxit; ++j) {
    z64* vj = V + (long)j * N;
    z64* zj = Z + (long)j * N;
    z64* w = V + (long)(j + 1) * N;
    clk.mark(0, s);
    if (o.precondition) F.apply(vj, zj, 1, s, transposed);
    else LSH_HIP(hipMemcpyAsync(zj, vj, sizeof(z64) * N, hipMemcpyDeviceToDevice, s));
    clk.mark(1, s);
    P.op.apply(s, F.b.as<double>(), zj, w, 1, transposed);
    clk.mark(2, s);
    // classical Gram-Schmidt, twice
    multidot(s, V, N, j + 1, w, N, h1, part);
    multiaxpy(s, w, V, N, j + 1, h1, N);
    multidot(s, V, N, j + 1, w, N, h2, part);
    multiaxpy(s, w, V, N, j + 1, h2, N);
    multidot(s, w, 0, 1, w, N, h2 + (j + 1), part);
    clk.mark(3, s);
    LSH_HIP(hipMemcpyAsync(hv.data(), h1, sizeof(z64) * (j + 1), hipMemcpyDeviceToHost, s));
    LSH_HIP(hipMemcpyAsync(hv2.data(), h2, sizeof(z64) * (j + 2), hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    clk.add();
    const double hn = std::sqrt(hv2[j + 1].x);
    if (hn > 0) scale_by_invnorm(s, w, w, h2 + (j + 1), N);
    auto Hc = [&](int r, int c) -> std::complex<double>& { return H[(size_t)r * maxit + c]; };
    for (int i = 0; i <= j; ++i) Hc(i, j) = {hv[i].x + hv2[i].x, hv[i].y + hv2[i].y};
    Hc(j + 1, j) = hn;
    for (int i = 0; i < j; ++i) {
      std::complex<double> a = Hc(i, j), c2 = Hc(i + 1, j);
      Hc(i, j) = std::conj(cs[i]) * a + std::conj(sn[i]) * c2;
      Hc(i + 1, j) = -sn[i] * a + cs[i] * c2;
    }
    std::complex<double> a = Hc(j, j), c2 = Hc(j + 1, j);
    const double rho = std::hypot(std::abs(a), std::abs(c2));
    cs[j] = rho > 0 ? a / rho : 1.0;
    sn[j] = rho > 0 ? c2 / rho : 0.0;
    Hc(j, j) = rho;
    Hc(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = std::conj(cs[j]) * g[j];
    est = std::abs(g[j + 1]) / beta;
    its = j + 1;
    if (info && j + 1 <= LSH_MAX_ITERS) info->history[j + 1] = est;
    if (est < o.tol || hn == 0) break;
  }
  // y = H^{-1} g (upper triangular), x = Z y
  const int k = its;
  std::vector<std::complex<double>> y(k);
  for (int i = k - 1; i >= 0; --i) {
    std::complex<double> t = g[i];
    for (int c2 = i + 1; c2 < k; ++c2) t -= H[(size_t)i * maxit + c2] * y[c2];
    y[i] = t / H[(size_t)i * maxit + i];
  }
  std::vector<z64> yz(k);
  for (int i = 0; i < k; ++i) yz[i] = mk(y[i].real(), y[i].imag());
  LSH_HIP(hipMemcpyAsync(h1, yz.data(), sizeof(z64) * k, hipMemcpyHostToDevice, s));
  lincomb(s, x, Z, N, k, h1, N);
  // true residual
  z64* r = W.res;
  P.op.apply(s, F.b.as<double>(), x, r, 1, transposed);
  sub_from(s, r, f, N);
  multidot(s, r, 0, 1, r, N, h2, part);
  z64 rn;
  LSH_HIP(hipMemcpyAsync(&rn, h2, sizeof(z64), hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  true_res = std::sqrt(rn.x) / beta;
  if (info) { info->iterations = its; info->residual = est; }
  clk.store(info);
  conv = true_res < o.tol ? 1 : 0;
}

// Flexible GMRES for nr right-hand sides in lockstep: every iteration applies
// the preconditioner and the operator once to all nr current basis vectors
// (so each box matrix and each FFT plan pass serves the whole group), while
// the Krylov bases, Hessenberg matrices, rotations and stopping tests stay
// per right-hand side, as in nr separate runs. Layout: V[j][r][N],
// Z[j][r][N]; f, x: [nr][N]. A right-hand side that has stopped gets a zero
// basis vector, which the (linear, per-vector) applies keep at zero.
// info: iterations, estimate and history of the last right-hand side.
void fgmres_multi(lsh_factor_s& F, SolveWs& W, const z64* f, z64* x, int nr, const lsh_solve_opts& o,
                  lsh_info* info, double& worst, int& allconv, hipStream_t s, bool transposed = false) {
  lsh_plan_s& P = *F.plan;
  const long N = (long)P.n * P.n, S = (long)nr * N;
  const int maxit = o.maxit, hs = maxit + 2;
  LSH_REQUIRE(W.maxit >= maxit && W.G >= nr, LSH_ERR_INVALID_ARG, "internal: solve workspace");
  z64* V = W.V;
  z64* Z = W.Z;
  z64* h1 = W.h1;
  z64* h2 = W.h2;
  z64* part = W.part;
  for (int r = 0; r < nr; ++r) multidot(s, f + r * N, 0, 1, f + r * N, N, h1 + r * hs, part);
  std::vector<z64> hv((size_t)nr * hs), hv2((size_t)nr * hs);
  LSH_HIP(hipMemcpyAsync(hv.data(), h1, sizeof(z64) * nr * hs, hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  using cd = std::complex<double>;
  struct Run {
    double beta = 0, est = 1.0;
    int its = 0;
    bool active = false;
    std::vector<cd> H, cs, sn, g;
    std::vector<double> hist;
  };
  std::vector<Run> run(nr);
  int nact = 0;
  for (int r = 0; r < nr; ++r) {
    Run& R = run[r];
    R.beta = std::sqrt(hv[(size_t)r * hs].x);
    R.hist.assign(1, 1.0);
    if (R.beta == 0) {
      fill_zero(s, V + r * N, sizeof(z64) * N);
      continue;
    }
    scale_by_invnorm(s, V + r * N, f + r * N, h1 + r * hs, N);
    R.H.assign((size_t)(maxit + 1) * maxit, 0.0);
    R.cs.assign(maxit, 0.0);
    R.sn.assign(maxit, 0.0);
    R.g.assign(maxit + 1, 0.0);
    R.g[0] = R.beta;
    R.active = true;
    ++nact;
  }
  PhaseClock clk(info != nullptr);
  for (int j = 0; j < maxit && nact > 0; ++j) {
    z64* vj = V + (long)j * S;
    z64* zj = Z + (long)j * S;
    z64* wj = V + (long)(j + 1) * S;
    clk.mark(0, s);
    if (o.precondition) F.apply(vj, zj, nr, s, transposed);
    else LSH_HIP(hipMemcpyAsync(zj, vj, sizeof(z64) * S, hipMemcpyDeviceToDevice, s));
    clk.mark(1, s);
    P.op.apply(s, F.b.as<double>(), zj, wj, nr, transposed);
    clk.mark(2, s);
    for (int r = 0; r < nr; ++r) {
      if (!run[r].active) continue;
      z64* w = wj + r * N;
      z64 *a1 = h1 + r * hs, *a2 = h2 + r * hs;
      multidot(s, V + r * N, S, j + 1, w, N, a1, part);
      multiaxpy(s, w, V + r * N, S, j + 1, a1, N);
      multidot(s, V + r * N, S, j + 1, w, N, a2, part);
      multiaxpy(s, w, V + r * N, S, j + 1, a2, N);
      multidot(s, w, 0, 1, w, N, a2 + (j + 1), part);
    }
    clk.mark(3, s);
    LSH_HIP(hipMemcpyAsync(hv.data(), h1, sizeof(z64) * nr * hs, hipMemcpyDeviceToHost, s));
    LSH_HIP(hipMemcpyAsync(hv2.data(), h2, sizeof(z64) * nr * hs, hipMemcpyDeviceToHost, s));
    LSH_HIP(hipStreamSynchronize(s));
    clk.add();
    for (int r = 0; r < nr; ++r) {
      Run& R = run[r];
      if (!R.active) continue;
      const z64* e1 = hv.data() + (size_t)r * hs;
      const z64* e2 = hv2.data() + (size_t)r * hs;
      z64* w = wj + r * N;
      const double hn = std::sqrt(e2[j + 1].x);
      if (hn > 0) scale_by_invnorm(s, w, w, h2 + r * hs + (j + 1), N);
      auto Hc = [&](int i, int c) -> cd& { return R.H[(size_t)i * maxit + c]; };
      for (int i = 0; i <= j; ++i) Hc(i, j) = {e1[i].x + e2[i].x, e1[i].y + e2[i].y};
      Hc(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        cd a = Hc(i, j), c2 = Hc(i + 1, j);
        Hc(i, j) = std::conj(R.cs[i]) * a + std::conj(R.sn[i]) * c2;
        Hc(i + 1, j) = -R.sn[i] * a + R.cs[i] * c2;
      }
      cd a = Hc(j, j), c2 = Hc(j + 1, j);
      const double rho = std::hypot(std::abs(a), std::abs(c2));
      R.cs[j] = rho > 0 ? a / rho : 1.0;
      R.sn[j] = rho > 0 ? c2 / rho : 0.0;
      Hc(j, j) = rho;
      Hc(j + 1, j) = 0.0;
      R.g[j + 1] = -R.sn[j] * R.g[j];
      R.g[j] = std::conj(R.cs[j]) * R.g[j];
      R.est = std::abs(R.g[j + 1]) / R.beta;
      R.its = j + 1;
      R.hist.push_back(R.est);
      if (R.est < o.tol || hn == 0) {
        R.active = false;
        --nact;
        fill_zero(s, w, sizeof(z64) * N);  // keeps this vector's later applies at zero
      }
    }
  }
  // per right-hand side: y = H^{-1} g (upper triangular), x = Z y
  std::vector<z64> yz((size_t)nr * hs, mk(0.0, 0.0));
  for (int r = 0; r < nr; ++r) {
    Run& R = run[r];
    const int k = R.its;
    std::vector<cd> y(k);
    for (int i = k - 1; i >= 0; --i) {
      cd t = R.g[i];
      for (int c2 = i + 1; c2 < k; ++c2) t -= R.H[(size_t)i * maxit + c2] * y[c2];
      y[i] = t / R.H[(size_t)i * maxit + i];
    }
    for (int i = 0; i < k; ++i) yz[(size_t)r * hs + i] = mk(y[i].real(), y[i].imag());
  }
  LSH_HIP(hipMemcpyAsync(h1, yz.data(), sizeof(z64) * nr * hs, hipMemcpyHostToDevice, s));
  for (int r = 0; r < nr; ++r) {
    if (run[r].its > 0) lincomb(s, x + r * N, Z + r * N, S, run[r].its, h1 + r * hs, N);
    else fill_zero(s, x + r * N, sizeof(z64) * N);
  }
  // true residuals, one operator pass for the group
  z64* res = W.res;
  P.op.apply(s, F.b.as<double>(), x, res, nr, transposed);
  for (int r = 0; r < nr; ++r) {
    sub_from(s, res + r * N, f + r * N, N);
    multidot(s, res + r * N, 0, 1, res + r * N, N, h2 + r * hs, part);
  }
  LSH_HIP(hipMemcpyAsync(hv2.data(), h2, sizeof(z64) * nr * hs, hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < nr; ++r) {
    const Run& R = run[r];
    const double tr = R.beta > 0 ? std::sqrt(hv2[(size_t)r * hs].x) / R.beta : 0.0;
    if (!(tr < o.tol) && R.beta > 0) allconv = 0;
    if (tr > worst) worst = tr;
  }
  clk.store(info);
  if (info) {
    const Run& R = run[nr - 1];
    info->iterations = R.its;
    info->residual = R.beta > 0 ? R.est : 0.0;
    for (size_t i = 0; i < R.hist.size() && i <= LSH_MAX_ITERS; ++i) info->history[i] = R.hist[i];
  }
}

// receivers: u(x_r) = h^2 sum_j (i/4) H0(kappa |x_r - x_j|) sigma_j
constexpr int EV_MAXRHS = 16;
__global__ __launch_bounds__(256) void k_eval_points(const z64* __restrict__ sig, int n, double h, double gx0,
                                                     double gy0, double kappa, const double* __restrict__ xy,
                                                     z64* out, int npts, int nrhs) {
  __shared__ z64 red[EV_MAXRHS][4];
  const int pt = blockIdx.x;
  const double px = xy[2 * pt], py = xy[2 * pt + 1];
  z64 acc[EV_MAXRHS];
  for (int r = 0; r < EV_MAXRHS; ++r) acc[r] = mk(0.0, 0.0);
  const long N = (long)n * n;
  for (long j = threadIdx.x; j < N; j += blockDim.x) {
    const int i1 = (int)(j % n), i2 = (int)(j / n);
    const double dx = px - (gx0 + (i1 + 0.5) * h), dy = py - (gy0 + (i2 + 0.5) * h);
    const double rr = kappa * sqrt(dx * dx + dy * dy);
    const z64 g = mk(-0.25 * y0(rr), 0.25 * j0(rr));
    for (int r = 0; r < EV_MAXRHS; ++r)
      if (r < nrhs) fma_acc(acc[r], g, sig[r * N + j]);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < EV_MAXRHS; ++r) {
    if (r >= nrhs) break;
    z64 a = acc[r];
    for (int off = 32; off > 0; off >>= 1) {
      a.x += __shfl_xor(a.x, off);
      a.y += __shfl_xor(a.y, off);
    }
    if (lane == 0) red[r][wave] = a;
  }
  __syncthreads();
  if (threadIdx.x < nrhs) {
    const int r = threadIdx.x;
    z64 a = red[r][0] + red[r][1] + red[r][2] + red[r][3];
    out[(long)r * npts + pt] = (h * h) * a;
  }
}

// out[m][j] = h^2 sum_r conj(G(|x_r - x_j|)) g[m][r]  (adjoint of the receiver map)
__global__ __launch_bounds__(256) void k_eval_points_adj(const z64* __restrict__ g, int npts, int nrhs, int n,
                                                         double h, double gx0, double gy0, double kappa,
                                                         const double* __restrict__ xy, z64* out) {
  const long N = (long)n * n;
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int i1 = (int)(j % n), i2 = (int)(j / n);
  const double px = gx0 + (i1 + 0.5) * h, py = gy0 + (i2 + 0.5) * h;
  z64 acc[EV_MAXRHS];
  for (int m = 0; m < EV_MAXRHS; ++m) acc[m] = mk(0.0, 0.0);
  for (int r = 0; r < npts; ++r) {
    const double dx = xy[2 * r] - px, dy = xy[2 * r + 1] - py;
    const double rr = kappa * sqrt(dx * dx + dy * dy);
    const z64 gc = mk(-0.25 * y0(rr), -0.25 * j0(rr));  // conj((i/4) H0)
    for (int m = 0; m < EV_MAXRHS; ++m)
      if (m < nrhs) fma_acc(acc[m], gc, g[(long)m * npts + r]);
  }
  for (int m = 0; m < nrhs; ++m) out[m * N + j] = (h * h) * acc[m];
}

// grad[k] = -kappa^2 Re sum_m conj(lambda[m][k]) (u_inc[m][k] + u[m][k])
__global__ void k_grad_b(const z64* __restrict__ lam, const z64* __restrict__ uinc, const z64* __restrict__ us,
                         int nrhs, long N, double k2, double* grad) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    double a = 0;
    for (int m = 0; m < nrhs; ++m) {
      const z64 l = lam[m * N + i], u = uinc[m * N + i] + us[m * N + i];
      a += l.x * u.x + l.y * u.y;
    }
    grad[i] = -k2 * a;
  }
}

void check_ws(void* ws, size_t bytes, size_t need, const char* what) {
  LSH_REQUIRE(need == 0 || ws, LSH_ERR_INVALID_ARG, std::string("null ") + what + " workspace");
  LSH_REQUIRE(((uintptr_t)ws & (mem::kGranule - 1)) == 0, LSH_ERR_INVALID_ARG,
              std::string(what) + " workspace must be 256-byte aligned");
  LSH_REQUIRE(bytes >= need, LSH_ERR_WORKSPACE_TOO_SMALL,
              std::string(what) + " workspace: " + std::to_string(bytes) + " bytes given, " + std::to_string(need) +
                  " needed");
}

// Splits a caller's plan workspace into the plan's arenas (the part beyond
// the bound goes to the kept memory).
void attach_plan(lsh_plan_s& P, void* ws, size_t bytes) {
  const PlanBytes b = plan_bytes(P.d, nullptr);
  check_ws(ws, bytes, b.total(), "plan");
  char* p = static_cast<char*>(ws);
  const size_t keep = bytes - b.sid - b.ssib - b.sgram;
  P.persist.attach(p, keep, "plan");
  P.sid.attach(p + keep, b.sid, "plan row-ID temporaries");
  P.ssib.attach(p + keep + b.sid, b.ssib, "plan sibling-block temporaries");
  P.sgram.attach(p + keep + b.sid + b.ssib, b.sgram, "plan parent Gram rows");
}

// The same for a factor, sized by the rank profile f.
void attach_factor(lsh_factor_s& F, const Profile& f, int flags, void* ws, size_t bytes) {
  const bool want_T = (flags & LSH_FACTOR_TRANSPOSE) != 0;
  const FactorBytes b = factor_bytes(f, want_T);
  check_ws(ws, bytes, b.total(), "factor");
  char* p = static_cast<char*>(ws);
  const size_t keep = bytes - b.scr;
  F.keep.attach(p, keep, "factor");
  F.scr.attach(p + keep, b.scr, "factor temporaries");
  for (auto* d : {&F.f32.keep, &F.f64.keep}) *d = &F.keep;
  F.f32.scr = F.f64.scr = &F.scr;
  F.f32.want_T = F.f64.want_T = want_T;
}

// The factor's private copy of b, checked for non-finite entries.
void copy_check_b(lsh_factor_s& F, const double* b, long N, hipStream_t s, const std::string& what) {
  mem::Bind bind(&F.keep);
  F.b.alloc(sizeof(double) * N);
  F.bad.alloc(sizeof(int));
  LSH_HIP(hipMemcpyAsync(F.b.p, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  fill_zero(s, F.bad.p, sizeof(int));
  hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, s, F.b.as<double>(), N, F.bad.as<int>());
  LSH_LAUNCH_CHECK();
  int hb = 0;
  LSH_HIP(hipMemcpyAsync(&hb, F.bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  LSH_HIP(hipStreamSynchronize(s));
  LSH_REQUIRE(!hb, LSH_ERR_INPUT_NONFINITE, "b has non-finite entries" + what);
}

int fail(const lsh::Error& e) {
  g_last_error = e.what();
  return e.code;
}

#define API_BEGIN try {
#define API_END                                       \
  }                                                   \
  catch (const lsh::Error& e) { return fail(e); }     \
  catch (const std::bad_alloc&) {                     \
    g_last_error = "host allocation failed";          \
    return LSH_ERR_NOMEM;                             \
  }                                                   \
  catch (const std::exception& e) {                   \
    g_last_error = e.what();                          \
    return LSH_ERR_HIP;                               \
  }

}  // namespace

namespace lsh {
// failure reporting for entry points defined in other sources
int report_failure(const Error& e) { return fail(e); }
int report_other_failure(const std::exception& e) {
  g_last_error = e.what();
  return LSH_ERR_HIP;
}
}  // namespace lsh

namespace {
// Streams and events of lsh_build, kept for the process (per device and CU
// reserve) and handed to one build at a time.
struct BuildStreams {
  int dev = 0, reserve = 0;
  hipStream_t ps = nullptr, ps2 = nullptr, fsm = nullptr, pg = nullptr;  // pg: the parent Gram rows
  std::vector<hipEvent_t> ev;
  void events(size_t n) {
    while (ev.size() < n) {
      hipEvent_t e = nullptr;
      LSH_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ev.push_back(e);
    }
  }
  // (never destroyed: the exit handler below still uses them)
  static std::mutex& mu() {
    static std::mutex* m = new std::mutex;
    return *m;
  }
  static std::vector<BuildStreams*>& pool() {
    static std::vector<BuildStreams*>* p = new std::vector<BuildStreams*>;
    return *p;
  }
  // destroys the pooled streams and events at process exit, before the
  // runtime's own teardown (a handler registered after the runtime started)
  static void destroy_all() {
    std::lock_guard<std::mutex> g(mu());
    for (BuildStreams* b : pool()) {
      for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
      for (hipStream_t st : {b->ps, b->ps2, b->fsm, b->pg})
        if (st) (void)hipStreamDestroy(st);
      delete b;
    }
    pool().clear();
  }
  static BuildStreams* acquire(int dev, int reserve) {
    static const bool registered = [] { return std::atexit(destroy_all) == 0; }();
    (void)registered;
    {
      std::lock_guard<std::mutex> g(mu());
      auto& p = pool();
      for (size_t i = 0; i < p.size(); ++i)
        if (p[i]->dev == dev && p[i]->reserve == reserve) {
          BuildStreams* b = p[i];
          p.erase(p.begin() + i);
          return b;
        }
    }
    std::unique_ptr<BuildStreams> b(new BuildStreams());
    b->dev = dev;
    b->reserve = reserve;
    LSH_HIP(hipStreamCreateWithFlags(&b->ps, hipStreamNonBlocking));
    LSH_HIP(hipStreamCreateWithFlags(&b->ps2, hipStreamNonBlocking));
    LSH_HIP(hipStreamCreateWithFlags(&b->pg, hipStreamNonBlocking));
    if (reserve > 0) {
      int ncu = 0;
      LSH_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
      for (int c = 0; c < ncu - reserve; ++c) mask[c / 32] |= 1u << (c % 32);
      if (hipExtStreamCreateWithCUMask(&b->fsm, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
        (void)hipGetLastError();
        b->fsm = nullptr;
      }
    }
    return b.release();
  }
  static void release(BuildStreams* b) {
    std::lock_guard<std::mutex> g(mu());
    pool().push_back(b);
  }
};
}  // namespace

extern "C" {

const char* lsh_last_error(void) { return g_last_error.c_str(); }

int lsh_eval_points_adjoint(lsh_plan_t P, const void* g_pts, const double* xy, int npts, void* out, int nrhs,
                            void* stream) {
  API_BEGIN
  LSH_REQUIRE(P && g_pts && xy && out && npts >= 1 && nrhs >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  const long N = (long)P->n * P->n;
  for (int r0 = 0; r0 < nrhs; r0 += EV_MAXRHS) {
    const int nr = nrhs - r0 < EV_MAXRHS ? nrhs - r0 : EV_MAXRHS;
    hipLaunchKernelGGL(k_eval_points_adj, dim3(ceil_div(N, 256)), dim3(256), 0, s,
                       static_cast<const z64*>(g_pts) + (long)r0 * npts, npts, nr, P->n, P->h, P->d.x0, P->d.y0,
                       P->kappa, xy, static_cast<z64*>(out) + r0 * N);
    LSH_LAUNCH_CHECK();
  }
  return LSH_OK;
  API_END
}

int lsh_grad_b(lsh_plan_t P, const void* lambda, const void* u_inc, const void* u, int nrhs, double* grad,
               void* stream) {
  API_BEGIN
  LSH_REQUIRE(P && lambda && u_inc && u && grad && nrhs >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  const long N = (long)P->n * P->n;
  hipLaunchKernelGGL(k_grad_b, dim3(2048), dim3(256), 0, (hipStream_t)stream, static_cast<const z64*>(lambda),
                     static_cast<const z64*>(u_inc), static_cast<const z64*>(u), nrhs, N, P->kappa * P->kappa, grad);
  LSH_LAUNCH_CHECK();
  return LSH_OK;
  API_END
}

int lsh_profile_enable(int on) {
  API_BEGIN
  prof::set(on != 0);
  return LSH_OK;
  API_END
}

int lsh_profile_only(const char* prefix) {
  API_BEGIN
  prof::set_only(prefix);
  return LSH_OK;
  API_END
}

int lsh_profile_query(const char* name, int* launches, double* ms, double* work) {
  API_BEGIN
  LSH_REQUIRE(name, LSH_ERR_INVALID_ARG, "null name");
  prof::query(name, launches, ms, work, nullptr);
  return LSH_OK;
  API_END
}

int lsh_profile_bytes(const char* name, double* bytes) {
  API_BEGIN
  LSH_REQUIRE(name && bytes, LSH_ERR_INVALID_ARG, "null argument");
  prof::query(name, nullptr, nullptr, nullptr, bytes);
  return LSH_OK;
  API_END
}

int lsh_profile_names(char* buf, int cap) {
  API_BEGIN
  LSH_REQUIRE(buf && cap > 0, LSH_ERR_INVALID_ARG, "bad buffer");
  std::string s = prof::names();
  std::strncpy(buf, s.c_str(), cap - 1);
  buf[cap - 1] = 0;
  return LSH_OK;
  API_END
}

int lsh_correction_weights(int order, double kh, int* count, int* offsets, double* tau) {
  API_BEGIN
  LSH_REQUIRE(count && offsets && tau, LSH_ERR_INVALID_ARG, "null argument");
  LSH_REQUIRE(kh > 0, LSH_ERR_INVALID_ARG, "kappa*h must be positive");
  auto st = correction_stencil(order, kh);
  *count = (int)st.size();
  for (size_t i = 0; i < st.size(); ++i) {
    offsets[2 * i] = st[i].dx;
    offsets[2 * i + 1] = st[i].dy;
    tau[2 * i] = st[i].re;
    tau[2 * i + 1] = st[i].im;
  }
  return LSH_OK;
  API_END
}

int lsh_plan_workspace(const lsh_desc* desc, size_t* bytes) {
  API_BEGIN
  LSH_REQUIRE(desc && bytes, LSH_ERR_INVALID_ARG, "null argument");
  validate(*desc);
  *bytes = plan_bytes(*desc, nullptr).total();
  return LSH_OK;
  API_END
}

int lsh_plan_create(const lsh_desc* desc, void* ws, size_t ws_bytes, void* stream, lsh_plan_t* plan) {
  API_BEGIN
  LSH_REQUIRE(desc && plan, LSH_ERR_INVALID_ARG, "null argument");
  validate(*desc);
  std::unique_ptr<lsh_plan_s> P(new lsh_plan_s());
  P->d = *desc;
  attach_plan(*P, ws, ws_bytes);
  mem::Bind bind(&P->persist);
  {  // (the parent Gram rows on a pooled side stream, as in lsh_build)
    int dev = 0;
    LSH_HIP(hipGetDevice(&dev));
    BuildStreams* bs = BuildStreams::acquire(dev, 0);
    struct Guard {
      BuildStreams* b;
      lsh_plan_s* P;
      ~Guard() {
        if (b->pg) (void)hipStreamSynchronize(b->pg);
        P->gs = nullptr;
        BuildStreams::release(b);
      }
    } guard{bs, P.get()};
    P->gs = bs->pg;
    plan_build(*P, (hipStream_t)stream);
  }
  *plan = P.release();
  return LSH_OK;
  API_END
}

int lsh_plan_destroy(lsh_plan_t plan) {
  API_BEGIN
  delete plan;
  return LSH_OK;
  API_END
}

int lsh_plan_workspace_used(lsh_plan_t P, size_t* used, size_t* size) {
  API_BEGIN
  LSH_REQUIRE(P, LSH_ERR_INVALID_ARG, "null plan");
  if (used) *used = P->persist.high() + P->sid.high() + P->ssib.high() + P->sgram.high();
  if (size) *size = P->persist.cap() + P->sid.cap() + P->ssib.cap() + P->sgram.cap();
  return LSH_OK;
  API_END
}

int lsh_plan_ranks(lsh_plan_t P, int* L, int* ranks) {
  API_BEGIN
  LSH_REQUIRE(P && L, LSH_ERR_INVALID_ARG, "null argument");
  *L = P->L;
  if (ranks)
    for (int l = 0; l <= P->L; ++l) ranks[l] = P->lev[l].k;
  return LSH_OK;
  API_END
}

int lsh_plan_level(lsh_plan_t P, int level, int* m, int* k, int* J, int* cand, void* U, void* stream) {
  API_BEGIN
  LSH_REQUIRE(P && level >= 1 && level <= P->L, LSH_ERR_INVALID_ARG, "bad level");
  const Level& lv = P->lev[level];
  if (m) *m = lv.m;
  if (k) *k = lv.k;
  if (J) std::memcpy(J, lv.J.data(), sizeof(int) * lv.k);
  if (cand)
    for (int i = 0; i < lv.m; ++i) { cand[2 * i] = lv.cand[i].x; cand[2 * i + 1] = lv.cand[i].y; }
  if (U) {
    LSH_HIP(hipMemcpyAsync(U, lv.U64.p, sizeof(z64) * (size_t)lv.m * lv.k, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    LSH_HIP(hipStreamSynchronize((hipStream_t)stream));
  }
  return LSH_OK;
  API_END
}

int lsh_plan_cache_info(int* entries, size_t* host_bytes) {
  API_BEGIN
  pcache::info(entries, host_bytes);
  return LSH_OK;
  API_END
}

int lsh_plan_cache_clear(void) {
  API_BEGIN
  pcache::clear();
  return LSH_OK;
  API_END
}

int lsh_plan_cache_save(const char* path) {
  API_BEGIN
  LSH_REQUIRE(path, LSH_ERR_INVALID_ARG, "null path");
  pcache::save(path);
  return LSH_OK;
  API_END
}

int lsh_plan_cache_load(const char* path) {
  API_BEGIN
  LSH_REQUIRE(path, LSH_ERR_INVALID_ARG, "null path");
  pcache::load(path);
  return LSH_OK;
  API_END
}

int lsh_plan_lowrank(lsh_plan_t P, int level, int* c, int* r, void* L, void* Rt, void* stream) {
  API_BEGIN
  LSH_REQUIRE(P && level >= 0 && level < P->L, LSH_ERR_INVALID_ARG, "bad level");
  const Level& lv = P->lev[level];
  if (c) *c = lv.c;
  if (r) *r = lv.wr;
  const size_t bytes = sizeof(z64) * (size_t)lv.c * lv.wr;
  if (L && lv.wr > 0)
    LSH_HIP(hipMemcpyAsync(L, lv.Pm64.p, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  if (Rt && lv.wr > 0)
    LSH_HIP(hipMemcpyAsync(Rt, lv.Qm64.as<z64>() + (size_t)lv.c * lv.wr, bytes, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
  LSH_HIP(hipStreamSynchronize((hipStream_t)stream));
  return LSH_OK;
  API_END
}

int lsh_plan_block(lsh_plan_t P, int level, int* rows, void* out, void* stream) {
  API_BEGIN
  LSH_REQUIRE(P && level >= -1 && level < P->L, LSH_ERR_INVALID_ARG, "bad level");
  const int c = level < 0 ? P->mL : P->lev[level].c;
  if (rows) *rows = c;
  if (out) {
    const void* src = level < 0 ? P->Gleaf64.p : P->lev[level].Gab64.p;
    LSH_HIP(hipMemcpyAsync(out, src, sizeof(z64) * (size_t)c * c, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    LSH_HIP(hipStreamSynchronize((hipStream_t)stream));
  }
  return LSH_OK;
  API_END
}

int lsh_plan_table(lsh_plan_t P, int* D, void* out, void* stream) {
  API_BEGIN
  LSH_REQUIRE(P, LSH_ERR_INVALID_ARG, "null plan");
  if (D) *D = P->D;
  if (out) {
    LSH_HIP(hipMemcpyAsync(out, P->table.p, P->table.bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    LSH_HIP(hipStreamSynchronize((hipStream_t)stream));
  }
  return LSH_OK;
  API_END
}

int lsh_factor_workspace(lsh_plan_t P, int flags, size_t* bytes) {
  API_BEGIN
  LSH_REQUIRE(P && bytes, LSH_ERR_INVALID_ARG, "null argument");
  *bytes = factor_bytes(plan_profile(*P), (flags & LSH_FACTOR_TRANSPOSE) != 0).total();
  return LSH_OK;
  API_END
}

int lsh_factor_workspace_used(lsh_factor_t F, size_t* used, size_t* size) {
  API_BEGIN
  LSH_REQUIRE(F, LSH_ERR_INVALID_ARG, "null factor");
  if (used) *used = F->keep.high() + F->scr.high();
  if (size) *size = F->keep.cap() + F->scr.cap();
  return LSH_OK;
  API_END
}

int lsh_factor_create(lsh_plan_t P, const double* b, int flags, void* ws, size_t ws_bytes, void* stream,
                      lsh_factor_t* factor) {
  API_BEGIN
  LSH_REQUIRE(P && b && factor, LSH_ERR_INVALID_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const long N = (long)P->n * P->n;
  std::unique_ptr<lsh_factor_s> F(new lsh_factor_s());
  F->plan = P;
  attach_factor(*F, plan_profile(*P), flags, ws, ws_bytes);
  copy_check_b(*F, b, N, s, "");
  if (P->d.hbs_prec == LSH_FP32) factor_build<float>(*P, F->b.as<double>(), F->f32, s);
  else factor_build<double>(*P, F->b.as<double>(), F->f64, s);
  *factor = F.release();
  return LSH_OK;
  API_END
}

}  // extern "C"


extern "C" {

// Plan and factor pipelined by level: the plan runs level by level in a host
// thread on its own stream (its row IDs are latency-bound pivot loops), and
// the factor of level l starts on the caller's stream as soon as plan level l
// is recorded.
int lsh_build_workspace(const lsh_desc* desc, int flags, size_t* plan_bytes_out, size_t* factor_bytes_out) {
  API_BEGIN
  LSH_REQUIRE(desc && plan_bytes_out && factor_bytes_out, LSH_ERR_INVALID_ARG, "null argument");
  validate(*desc);
  Profile f;
  *plan_bytes_out = plan_bytes(*desc, &f).total();
  *factor_bytes_out = factor_bytes(f, (flags & LSH_FACTOR_TRANSPOSE) != 0).total();
  return LSH_OK;
  API_END
}

int lsh_build(const lsh_desc* desc, const double* b, int flags, void* plan_ws, size_t plan_ws_bytes,
              void* factor_ws, size_t factor_ws_bytes, void* stream, lsh_plan_t* plan, lsh_factor_t* factor) {
  API_BEGIN
  LSH_REQUIRE(desc && b && plan && factor, LSH_ERR_INVALID_ARG, "null argument");
  validate(*desc);
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<lsh_plan_s> P(new lsh_plan_s());
  P->d = *desc;
  attach_plan(*P, plan_ws, plan_ws_bytes);
  std::unique_ptr<lsh_factor_s> F(new lsh_factor_s());
  F->plan = P.get();
  {
    Profile f;
    plan_bytes(*desc, &f);  // the factor's size under the plan's rank bounds
    attach_factor(*F, f, flags, factor_ws, factor_ws_bytes);
  }
  const long N = (long)desc->n * desc->n;
  copy_check_b(*F, b, N, s, "");
  int dev = 0;
  LSH_HIP(hipGetDevice(&dev));
  // The factor runs on a stream kept off LSH_PLAN_CUS compute units, so that
  // the plan's small latency-bound kernels (the critical path) find free
  // units while the factor's products fill the rest.  Default: an eighth of
  // the units for the FP32 factor, none for the FP64 factor (whose products
  // are the longer path).  Without CU masking the factor uses the caller's
  // stream.  Streams and events come from a per-process pool (creating them
  // costs milliseconds per build).
  int reserve = 0;
  {
    const char* e = std::getenv("LSH_PLAN_CUS");
    int ncu = 0;
    LSH_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    reserve = (e && *e) ? std::atoi(e) : (desc->hbs_prec == LSH_FP32 ? ncu / 8 : 0);
    if (!(reserve > 0 && reserve < ncu / 2)) reserve = 0;
  }
  BuildStreams* bs = BuildStreams::acquire(dev, reserve);
  struct BsGuard {
    BuildStreams* b;
    lsh_plan_s* P;
    ~BsGuard() {  // (the side stream's rows read plan memory: drained before the streams go back)
      if (b->pg) (void)hipStreamSynchronize(b->pg);
      P->gs = nullptr;
      P->skel_cb = nullptr;  // (it refers to this call's thread state)
      BuildStreams::release(b);
    }
  } bsg{bs, P.get()};
  hipStream_t ps = bs->ps, ps2 = bs->ps2, fsm = bs->fsm;
  P->gs = bs->pg;
  hipStream_t fs = fsm ? fsm : s;
  mem::Bind bind(&P->persist);  // (plan_init; each plan thread binds its own)
  plan_init(*P, ps);
  const int L = P->L;
  bs->events(2 * L + 5);  // [l]: U_l ready, [L+1+l]: G_l ready, [2L+2]: done
  std::vector<hipEvent_t>& ev = bs->ev;
  if (fsm) {  // the factor stream follows the copy of b on the caller's stream
    LSH_HIP(hipEventRecord(ev[2 * L + 3], s));
    LSH_HIP(hipStreamWaitEvent(fsm, ev[2 * L + 3], 0));
  }
  std::mutex mu;
  std::condition_variable cv;
  int doneU = L + 1;  // lowest level with U_l ready
  int running = 2;                   // plan threads still running
  bool finished = false, failed = false;
  std::exception_ptr err;
  auto fail = [&] {
    std::lock_guard<std::mutex> g(mu);
    if (!err) err = std::current_exception();
    failed = true;
  };
  auto leave = [&] {
    { std::lock_guard<std::mutex> g(mu); finished = --running == 0; }
    cv.notify_all();
  };
  // two plan threads: the row IDs of levels L..1 (the critical path), and
  // behind them the sibling blocks of parent levels L-1..0 with their
  // low-rank forms (sibling block l needs the skeletons of level l + 1).
  // Sibling levels are claimed in order by either thread: once its row IDs
  // are done, the first thread takes the next unclaimed one (the last two,
  // typically: they need the same skeletons and run side by side).
  // A sibling block needs only the skeleton of the level below it, which is
  // known before that level's interpolation matrix (skelU: the lowest level
  // whose skeleton is known).  The root's block is claimed as soon as it can
  // start (it is the longest, and with level 1 kept whole it needs only the
  // skeleton of level 2); the others in order.
  std::vector<char> claimed(L + 1, 0);
  std::vector<char> sibDone(L + 1, 0);
  int skelU = L + 1;
  P->skel_cb = [&](int l) {
    { std::lock_guard<std::mutex> g(mu); skelU = std::min(skelU, l); }
    cv.notify_all();
  };
  auto claim = [&]() -> int {  // (waits until a block can start)
    std::unique_lock<std::mutex> g(mu);
    for (;;) {
      if (failed) return -1;
      if (L >= 1 && !claimed[0] && skelU <= 1) {
        claimed[0] = 1;
        return 0;
      }
      int next = -1;
      for (int l = L - 1; l >= 0 && next < 0; --l)
        if (!claimed[l]) next = l;
      if (next < 0) return -1;
      if (skelU <= next + 1) {
        claimed[next] = 1;
        return next;
      }
      cv.wait(g);
    }
  };
  auto sibling = [&](int l, hipStream_t st, mem::Arena& tmp, bool drain) {
    {
      std::unique_lock<std::mutex> g(mu);
      cv.wait(g, [&] { return failed || skelU <= l + 1; });
      if (failed) return false;
    }
    plan_sibling(*P, l, st, tmp);
    // Before the next sibling block, let every stream drain: the level IDs'
    // latency-bound steps (the critical path) then run without this thread's
    // kernels interleaved (fourier-1024: 8 ms less per build).  LSH_SIB_SYNC=0
    // lets it run ahead.
    if (drain) LSH_HIP(hipDeviceSynchronize());
    LSH_HIP(hipEventRecord(ev[L + 1 + l], st));
    { std::lock_guard<std::mutex> g(mu); sibDone[l] = 1; }
    cv.notify_all();
    return true;
  };
  const char* ess = std::getenv("LSH_SIB_SYNC");
  const bool sib_sync = !(ess && *ess == '0');
  std::thread th([&] {
    try {
      LSH_HIP(hipSetDevice(dev));
      mem::Bind tbind(&P->persist);
      for (int l = L; l >= 1; --l) {
        plan_id(*P, l, ps);
        LSH_HIP(hipEventRecord(ev[l], ps));
        { std::lock_guard<std::mutex> g(mu); doneU = l; }
        cv.notify_all();
      }
      // the remaining sibling blocks (in the row IDs' temporaries: every row
      // ID is done; the parent Gram rows too), then the operator spectrum
      LSH_HIP(hipStreamSynchronize(ps));
      LSH_HIP(hipStreamSynchronize(P->gs));
      for (int l = claim(); l >= 0; l = claim())
        if (!sibling(l, ps, P->sid, false)) break;
      plan_finish(*P, ps);
      LSH_HIP(hipEventRecord(ev[2 * L + 2], ps));
    } catch (...) {
      fail();
    }
    leave();
  });
  std::thread th2([&] {
    try {
      LSH_HIP(hipSetDevice(dev));
      mem::Bind tbind(&P->persist);
      for (int l = claim(); l >= 0; l = claim())
        if (!sibling(l, ps2, P->ssib, sib_sync)) break;
    } catch (...) {
      fail();
    }
    leave();
  });
  // wait until U_l (kind 0) or G_l (kind 1) exists; false if the plan failed
  auto wait_for = [&](int l, int kind) -> bool {
    std::unique_lock<std::mutex> g(mu);
    cv.wait(g, [&] { return failed || finished || (kind ? sibDone[l] != 0 : doneU <= l); });
    return !failed;
  };
  std::exception_ptr ferr;
  try {
    auto run = [&](auto& FD) {
      factor_init(*P, FD);
      if (!wait_for(L, 0)) return;
      hipStream_t cur = fs;
      LSH_HIP(hipStreamWaitEvent(cur, ev[L], 0));
      factor_leaves(*P, F->b.template as<double>(), FD, cur);
      for (int l = L - 1; l >= 0; --l) {
        if (!wait_for(l, 1)) return;  // G_l: the merge overlaps the row ID of level l
        LSH_HIP(hipStreamWaitEvent(cur, ev[L + 1 + l], 0));
        using RT = typename std::decay_t<decltype(FD)>::real_t;
        if (level_fused<RT>(*P, l)) {  // one launch for merge and scattering matrices
          if (l >= 1) {
            if (!wait_for(l, 0)) return;
            LSH_HIP(hipStreamWaitEvent(cur, ev[l], 0));
          }
          factor_level_fused(*P, FD, l, cur);
          continue;
        }
        factor_merge(*P, FD, l, cur);
        if (l >= 1) {
          if (!wait_for(l, 0)) return;
          LSH_HIP(hipStreamWaitEvent(cur, ev[l], 0));
          factor_scatter(*P, FD, l, cur);
        }
      }
      factor_check(FD, cur);
      ensure_apply_ws(*P, FD);
      if (fsm && cur == fsm) {
        LSH_HIP(hipEventRecord(ev[2 * L + 4], fsm));
        LSH_HIP(hipStreamWaitEvent(s, ev[2 * L + 4], 0));
      }
    };
    if (desc->hbs_prec == LSH_FP32) run(F->f32);
    else run(F->f64);
  } catch (...) {
    ferr = std::current_exception();
  }
  if (ferr) {  // let the plan threads stop early
    { std::lock_guard<std::mutex> g(mu); failed = true; }
    cv.notify_all();
  }
  th.join();
  th2.join();
  if (err) std::rethrow_exception(err);
  if (ferr) std::rethrow_exception(ferr);
  LSH_HIP(hipStreamWaitEvent(s, ev[2 * L + 2], 0));
  LSH_HIP(hipStreamSynchronize(s));
  *plan = P.release();
  *factor = F.release();
  return LSH_OK;
  API_END
}

}  // extern "C"

namespace {

// Woodbury merge and scattering matrices of one aligned level step for the
// instances in wact: the products of factor_merge_lowrank and of the
// Woodbury branch of factor_scatter, each step one grouped launch over the
// instances (same operands, shapes and order, so the same bits).
// Memory: the factors' own parts from each instance's keep arena, each
// instance's temporaries from its scr arena, the grouped launches' tables,
// flags and inverse workspace from the arena bound to the thread (the batch's
// shared workspace); all rewound per level step by the caller.
void batch_lowrank_level(std::vector<lsh_factor_s*>& Fs, const std::vector<int>& wact_all, int dpt, hipStream_t s) {
  const c32 one = mk<float>(1, 0), zero = mk<float>(0, 0), mone = mk<float>(-1, 0);
  const int n_inst = (int)Fs.size();
  // levels whose inverse fits in LDS: every instance's boxes in one persistent launch
  std::vector<int> wact, fused;
  for (int i : wact_all) {
    const lsh_plan_s& P = *Fs[i]->plan;
    (level_fused<float>(P, P.L - dpt) ? fused : wact).push_back(i);
  }
  if (!fused.empty()) {
    std::vector<MergeLevelDev> e;
    std::vector<DevBuf> inf(fused.size());
    for (size_t q = 0; q < fused.size(); ++q) {
      lsh_factor_s& F = *Fs[fused[q]];
      const int l = F.plan->L - dpt;
      inf[q].alloc(sizeof(int) << l);
      e.push_back(merge_entry(*F.plan, F.f32, l, F.keep, F.scr, inf[q].as<int>()));
    }
    DevBuf table;
    table.alloc(merge_level_table_bytes(e.size()));
    DevBuf counter(sizeof(int));
    merge_levels(s, e, table, counter.as<int>());
    for (size_t q = 0; q < fused.size(); ++q) {
      const int l = Fs[fused[q]]->plan->L - dpt;
      LSH_REQUIRE(!check_info(inf[q], 1 << l, s), LSH_ERR_SINGULAR,
                  "singular merge matrix I - Bw Aw at level " + std::to_string(l) + " (instance " +
                      std::to_string(fused[q]) + ")");
    }
  }
  if (wact.empty()) return;
  std::vector<GemmItem> gi;
  DevBuf itab;
  auto run = [&] {
    DevBuf gtab;  // (one table per launch)
    cgemm_grouped(s, gi, gtab);
    gi.clear();
  };
  struct Lv {
    int l, c, r, nb, k;
    long cc, cr, rr, r2, w4;
    const lsh_plan_s* P;
    FactorData<float>* F;
  };
  std::vector<Lv> L;
  std::vector<DevBuf> T(n_inst), info(n_inst);
  for (int i : wact) {
    const lsh_plan_s& P = *Fs[i]->plan;
    const int l = P.L - dpt, c = P.lev[l].c, r = P.lev[l].wr;
    Lv v{l, c, r, 1 << l, P.lev[l].k, (long)c * c, (long)c * r, (long)r * r, 2L * r, 4L * r * r, &P, &Fs[i]->f32};
    FactorData<float>& F = *v.F;
    F.wr[l] = r;
    F.Pa[l].alloc_in(*F.keep, sizeof(c32) * v.nb * 2 * v.cr);
    F.Ci[l].alloc_in(*F.keep, sizeof(c32) * v.nb * v.w4);
    T[i].alloc_in(*F.scr, sizeof(c32) * v.nb * 3 * v.rr);
    info[i].alloc(sizeof(int) * v.nb);
    L.push_back(v);
  }
  auto each = [&](auto&& fn) {
    for (size_t q = 0; q < wact.size(); ++q) fn(wact[q], L[q]);
  };
  auto ptrs = [&](int i, const Lv& v, c32*& Pst, c32*& W, c32*& Aw, c32*& Bw, c32*& C) {
    Pst = v.F->Pa[v.l].as<c32>();
    W = v.F->Ci[v.l].as<c32>();
    Aw = T[i].as<c32>();
    Bw = Aw + v.nb * v.rr;
    C = Bw + v.nb * v.rr;
  };
  c32 *Pst, *W, *Aw, *Bw, *C;
  each([&](int i, const Lv& v) {  // S_a L, S_b R
    ptrs(i, v, Pst, W, Aw, Bw, C);
    const c32* Sch = v.F->S[v.l + 1].as<c32>();
    gi.push_back({v.c, v.r, v.c, one, zero, Sch, v.c, 2 * v.cc, OP_N, v.P->W<float>(v.l, 0), v.r, 0, OP_N, nullptr,
                  0, 0, Pst, v.r, 2 * v.cr, v.nb, false});
    gi.push_back({v.c, v.r, v.c, one, zero, Sch + v.cc, v.c, 2 * v.cc, OP_N, v.P->W<float>(v.l, 2), v.r, 0, OP_N,
                  nullptr, 0, 0, Pst + v.cr, v.r, 2 * v.cr, v.nb, false});
  });
  run();
  each([&](int i, const Lv& v) {  // Aw = R^T (S_b R), Bw = L^T (S_a L)
    ptrs(i, v, Pst, W, Aw, Bw, C);
    gi.push_back({v.r, v.r, v.c, one, zero, v.P->W<float>(v.l, 3), v.c, 0, OP_N, Pst + v.cr, v.r, 2 * v.cr, OP_N,
                  nullptr, 0, 0, Aw, v.r, v.rr, v.nb, false});
    gi.push_back({v.r, v.r, v.c, one, zero, v.P->W<float>(v.l, 1), v.c, 0, OP_N, Pst, v.r, 2 * v.cr, OP_N, nullptr,
                  0, 0, Bw, v.r, v.rr, v.nb, false});
  });
  run();
  each([&](int i, const Lv& v) {  // C = I - Bw Aw
    ptrs(i, v, Pst, W, Aw, Bw, C);
    gi.push_back({v.r, v.r, v.r, mone, zero, Bw, v.r, v.rr, OP_N, Aw, v.r, v.rr, OP_N, nullptr, 0, 0, C, v.r, v.rr,
                  v.nb, true});
  });
  run();
  {
    std::vector<InvItem> inv;
    each([&](int i, const Lv& v) {
      ptrs(i, v, Pst, W, Aw, Bw, C);
      inv.push_back({C, v.r, (long)v.r, v.rr, v.nb, info[i].as<int>()});
    });
    DevBuf ws(inverse_grouped_ws_bytes(inv));
    inverse_grouped(s, inv, ws.p, itab);
    LSH_HIP(hipStreamSynchronize(s));  // (ws dies here)
  }
  for (size_t q = 0; q < wact.size(); ++q)
    LSH_REQUIRE(!check_info(info[wact[q]], L[q].nb, s), LSH_ERR_SINGULAR,
                "singular merge matrix I - Bw Aw at level " + std::to_string(L[q].l) + " (instance " +
                    std::to_string(wact[q]) + ")");
  each([&](int i, const Lv& v) {  // W' = [[-Aw C, I + Aw C Bw], [C, -C Bw]]
    ptrs(i, v, Pst, W, Aw, Bw, C);
    ccopy2d<float>(s, v.r, v.r, C, v.r, v.rr, W + v.r * v.r2, v.r2, v.w4, v.nb);
    gi.push_back({v.r, v.r, v.r, mone, zero, Aw, v.r, v.rr, OP_N, C, v.r, v.rr, OP_N, nullptr, 0, 0, W, v.r2, v.w4,
                  v.nb, false});
    gi.push_back({v.r, v.r, v.r, mone, zero, C, v.r, v.rr, OP_N, Bw, v.r, v.rr, OP_N, nullptr, 0, 0,
                  W + v.r * v.r2 + v.r, v.r2, v.w4, v.nb, false});
  });
  run();
  each([&](int i, const Lv& v) {
    ptrs(i, v, Pst, W, Aw, Bw, C);
    gi.push_back({v.r, v.r, v.r, mone, zero, W, v.r2, v.w4, OP_N, Bw, v.r, v.rr, OP_N, nullptr, 0, 0, W + v.r, v.r2,
                  v.w4, v.nb, true});
  });
  run();
  // scattering matrices (not at the root): X D U through W'
  std::vector<DevBuf> A12(n_inst), Qb(n_inst), Gs(n_inst), Rs(n_inst);
  std::vector<int> sc;
  std::vector<Lv> SL;
  for (size_t q = 0; q < wact.size(); ++q) {
    const Lv& v = L[q];
    if (v.l == 0) continue;
    const int i = wact[q];
    A12[i].alloc_in(*v.F->scr, sizeof(c32) * v.nb * 2 * (long)v.c * v.k);
    Qb[i].alloc_in(*v.F->scr, sizeof(c32) * v.nb * 4 * (long)v.r * v.k);
    if (!v.P->lev[v.l].ident) {
      const long nrt = rest_total(v.P->lev[v.l]);
      Gs[i].alloc_in(*v.F->scr, sizeof(c32) * v.nb * (long)v.c * nrt);
      Rs[i].alloc_in(*v.F->scr, sizeof(c32) * v.nb * nrt * v.k);
    }
    v.F->S[v.l].alloc_in(*v.F->keep, sizeof(c32) * v.nb * (long)v.k * v.k);
    sc.push_back(i);
    SL.push_back(v);
  }
  if (sc.empty()) return;
  auto each_s = [&](auto&& fn) {
    for (size_t q = 0; q < sc.size(); ++q) {
      const Lv& v = SL[q];
      const int i = sc[q];
      const long ck = (long)v.c * v.k, rk = (long)v.r * v.k;
      c32* a = A12[i].as<c32>();
      c32* qv = Qb[i].as<c32>();
      fn(v, ck, rk, a, qv, qv + v.nb * 2 * rk);
    }
  };
  // (the products of factor_scatter, grouped over the instances; dense
  // products with U = I on levels that keep all their candidates)
  auto push = [&](const ScatterGemm<float>& g) {
    gi.push_back({g.M, g.N, g.K, one, one, g.A, g.lda, g.sA, g.opA, g.B, g.ldb, g.sB, OP_N, g.C, g.ldc, g.sC, g.C,
                  g.ldc, g.sC, g.batch, false});
  };
  std::vector<GatherJob> gj;  // (every instance's gathers in one launch)
  each_s([&](const Lv& v, long ck, long, c32* a, c32*, c32*) {
    const c32* Sch = v.F->S[v.l + 1].as<c32>();
    if (!v.P->lev[v.l].ident) {
      ScatterGemm<float> g[2];
      const int ng = scatter_su_prep<float>(*v.P, v.l, Sch, a, a + ck, 2 * ck, Gs[sc[&v - SL.data()]].as<c32>(), s,
                                            g, &gj);
      for (int t = 0; t < ng; ++t) push(g[t]);  // (the halves write different blocks)
      return;
    }
    const c32* U1 = v.P->U<float>(v.l);
    gi.push_back({v.c, v.k, v.c, one, zero, Sch, v.c, 2 * v.cc, OP_N, U1, v.k, 0, OP_N, nullptr, 0, 0, a, v.k,
                  2 * ck, v.nb, false});
    gi.push_back({v.c, v.k, v.c, one, zero, Sch + v.cc, v.c, 2 * v.cc, OP_N, U1 + ck, v.k, 0, OP_N, nullptr, 0, 0,
                  a + ck, v.k, 2 * ck, v.nb, false});
  });
  {
    DevBuf gtab;
    gather_grouped(s, gj, gtab);
    gj.clear();
  }
  if (!gi.empty()) run();
  each_s([&](const Lv& v, long ck, long rk, c32* a, c32* qv, c32*) {
    gi.push_back({v.r, v.k, v.c, one, zero, v.P->W<float>(v.l, 1), v.c, 0, OP_N, a, v.k, 2 * ck, OP_N, nullptr, 0,
                  0, qv, v.k, 2 * rk, v.nb, false});
    gi.push_back({v.r, v.k, v.c, one, zero, v.P->W<float>(v.l, 3), v.c, 0, OP_N, a + ck, v.k, 2 * ck, OP_N, nullptr,
                  0, 0, qv + rk, v.k, 2 * rk, v.nb, false});
  });
  run();
  each_s([&](const Lv& v, long, long rk, c32*, c32* qv, c32* yv) {
    gi.push_back({2 * v.r, v.k, 2 * v.r, one, zero, v.F->Ci[v.l].as<c32>(), v.r2, v.w4, OP_N, qv, v.k, 2 * rk, OP_N,
                  nullptr, 0, 0, yv, v.k, 2 * rk, v.nb, false});
  });
  run();
  each_s([&](const Lv& v, long ck, long rk, c32* a, c32*, c32* yv) {
    gi.push_back({v.c, v.k, v.r, mone, one, v.F->Pa[v.l].as<c32>(), v.r, v.cr, OP_N, yv, v.k, rk, OP_N, a, v.k, ck,
                  a, v.k, ck, 2 * v.nb, false});
  });
  run();
  std::vector<std::array<ScatterGemm<float>, 2>> ug(sc.size());
  std::vector<int> nug(sc.size(), -1);  // -1: dense products with U = I
  each_s([&](const Lv& v, long ck, long, c32* a, c32*, c32*) {
    const size_t q = &v - SL.data();
    if (!v.P->lev[v.l].ident) {
      nug[q] = scatter_utb_prep<float>(*v.P, v.l, a, a + ck, 2 * ck, v.F->S[v.l].as<c32>(), Rs[sc[q]].as<c32>(),
                                       s, ug[q].data(), &gj);
      return;
    }
    gi.push_back({v.k, v.k, v.c, one, zero, v.P->U<float>(v.l), v.k, 0, OP_T, a, v.k, 2 * ck, OP_N, nullptr, 0, 0,
                  v.F->S[v.l].as<c32>(), v.k, (long)v.k * v.k, v.nb, false});
  });
  {
    DevBuf gtab;
    gather_grouped(s, gj, gtab);
    gj.clear();
  }
  for (size_t q = 0; q < sc.size(); ++q)
    if (nug[q] >= 1) push(ug[q][0]);
  if (!gi.empty()) run();
  // (both halves add into S: the second ones in a launch of their own)
  each_s([&](const Lv& v, long ck, long, c32* a, c32*, c32*) {
    const size_t q = &v - SL.data();
    if (!v.P->lev[v.l].ident) {
      if (nug[q] >= 2) push(ug[q][1]);
      return;
    }
    c32* S = v.F->S[v.l].as<c32>();
    gi.push_back({v.k, v.k, v.c, one, one, v.P->U<float>(v.l) + ck, v.k, 0, OP_T, a + ck, v.k, 2 * ck, OP_N, S, v.k,
                  (long)v.k * v.k, S, v.k, (long)v.k * v.k, v.nb, false});
  });
  if (!gi.empty()) run();
  LSH_HIP(hipStreamSynchronize(s));  // scratch and tables die here
}

// Algorithm 1 for many instances at once (FP32 factors): the levels are
// aligned from the leaves, and every step of a level (each product, the
// inverses) is one grouped launch over the instances that have that level.
void batch_factor_f32(std::vector<lsh_factor_s*>& Fs, mem::Arena& shared, hipStream_t s) {
  const int n_inst = (int)Fs.size();
  const c32 one = mk<float>(1, 0), zero = mk<float>(0, 0), mone = mk<float>(-1, 0);
  mem::Bind bind(&shared);
  std::vector<GemmItem> gi;
  auto run_gemms = [&](DevBuf& tab) {
    cgemm_grouped(s, gi, tab);
    gi.clear();
  };
  // a new level step: the previous step has been synchronised
  auto new_step = [&] {
    shared.reset(0);
    for (auto* F : Fs) F->scr.reset(0);
  };
  new_step();
  int Lmax = 0;
  for (auto* F : Fs) {
    factor_init<float>(*F->plan, F->f32);
    Lmax = F->plan->L > Lmax ? F->plan->L : Lmax;
  }
  // leaves: X = (I + B G_leaf)^{-1}, S = U^T X B U
  std::vector<DevBuf> Yb(n_inst), Zb(n_inst), infos(n_inst);
  std::vector<InvItem> inv;
  DevBuf itab0;
  for (int i = 0; i < n_inst; ++i) {
    const lsh_plan_s& P = *Fs[i]->plan;
    FactorData<float>& F = Fs[i]->f32;
    const int nleaf = P.nleaf, mL = P.mL;
    F.X.alloc_in(*F.keep, sizeof(c32) * (size_t)nleaf * mL * mL);
    leaf_build<float>(s, F.X.as<c32>(), P.Gleaf<float>(), mL, Fs[i]->b.as<double>(), P.kappa * P.kappa,
                      P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), nleaf, P.n);
    infos[i].alloc(sizeof(int) * nleaf);
    inv.push_back({F.X.as<c32>(), mL, (long)mL, (long)mL * mL, nleaf, infos[i].as<int>()});
  }
  {
    DevBuf ws(inverse_grouped_ws_bytes(inv));
    inverse_grouped(s, inv, ws.p, itab0);
  }
  for (int i = 0; i < n_inst; ++i) {
    LSH_REQUIRE(!check_info(infos[i], Fs[i]->plan->nleaf, s), LSH_ERR_SINGULAR,
                "singular leaf matrix I + B G (instance " + std::to_string(i) + ")");
  }
  inv.clear();
  for (int i = 0; i < n_inst; ++i) {
    const lsh_plan_s& P = *Fs[i]->plan;
    FactorData<float>& F = Fs[i]->f32;
    const int nleaf = P.nleaf, mL = P.mL, kL = P.lev[P.L].k;
    Yb[i].alloc_in(*F.scr, sizeof(c32) * (size_t)nleaf * mL * kL);
    Zb[i].alloc_in(*F.scr, sizeof(c32) * (size_t)nleaf * mL * kL);
    leaf_scale_U<float>(s, Yb[i].as<c32>(), P.U<float>(P.L), mL, kL, Fs[i]->b.as<double>(), P.kappa * P.kappa,
                        P.leaf_origin.as<I2>(), P.leaf_pts.as<I2>(), nleaf, P.n);
    gi.push_back({mL, kL, mL, one, zero, F.X.as<c32>(), mL, (long)mL * mL, OP_N, Yb[i].as<c32>(), kL,
                  (long)mL * kL, OP_N, nullptr, 0, 0, Zb[i].as<c32>(), kL, (long)mL * kL, nleaf, false});
  }
  DevBuf gtab1;
  run_gemms(gtab1);
  for (int i = 0; i < n_inst; ++i) {
    const lsh_plan_s& P = *Fs[i]->plan;
    FactorData<float>& F = Fs[i]->f32;
    const int nleaf = P.nleaf, mL = P.mL, kL = P.lev[P.L].k;
    F.S[P.L].alloc_in(*F.keep, sizeof(c32) * (size_t)nleaf * kL * kL);
    gi.push_back({kL, kL, mL, one, zero, P.U<float>(P.L), kL, 0, OP_T, Zb[i].as<c32>(), kL, (long)mL * kL, OP_N,
                  nullptr, 0, 0, F.S[P.L].as<c32>(), kL, (long)kL * kL, nleaf, false});
  }
  DevBuf gtab2;
  run_gemms(gtab2);
  LSH_HIP(hipStreamSynchronize(s));
  Yb.clear(); Zb.clear();
  // levels, aligned from the leaves
  for (int dpt = 1; dpt <= Lmax; ++dpt) {
    new_step();
    DevBuf itab;
    std::vector<int> act, wact;  // Schur-form and Woodbury levels, each grouped
    for (int i = 0; i < n_inst; ++i)
      if (Fs[i]->plan->L - dpt >= 0) (Fs[i]->plan->lev[Fs[i]->plan->L - dpt].wr > 0 ? wact : act).push_back(i);
    if (!wact.empty()) batch_lowrank_level(Fs, wact, dpt, s);
    if (act.empty()) {
      LSH_HIP(hipStreamSynchronize(s));
      continue;
    }
    std::vector<DevBuf> tabs(9);
    auto lev = [&](int i) { return Fs[i]->plan->L - dpt; };
    for (int i : act) {  // allocations of this level
      const lsh_plan_s& P = *Fs[i]->plan;
      FactorData<float>& F = Fs[i]->f32;
      const int l = lev(i), c = P.lev[l].c, nb = 1 << l;
      const long cc = (long)c * c;
      F.Pa[l].alloc_in(*F.keep, sizeof(c32) * nb * cc);
      F.Pb[l].alloc_in(*F.keep, sizeof(c32) * nb * cc);
      F.Ci[l].alloc_in(*F.keep, sizeof(c32) * nb * cc);
    }
    // P_a = S_a G_ab ; P_b = S_b G_ab^T
    for (int i : act) {
      const lsh_plan_s& P = *Fs[i]->plan;
      FactorData<float>& F = Fs[i]->f32;
      const int l = lev(i), c = P.lev[l].c, nb = 1 << l;
      const long cc = (long)c * c;
      const c32* Sch = F.S[l + 1].as<c32>();
      gi.push_back({c, c, c, one, zero, Sch, c, 2 * cc, OP_N, P.Gab<float>(l), c, 0, OP_N, nullptr, 0, 0,
                    F.Pa[l].as<c32>(), c, cc, nb, false});
      gi.push_back({c, c, c, one, zero, Sch + cc, c, 2 * cc, OP_N, P.Gab<float>(l), c, 0, OP_T, nullptr, 0, 0,
                    F.Pb[l].as<c32>(), c, cc, nb, false});
    }
    run_gemms(tabs[0]);
    // C = I - P_b P_a
    for (int i : act) {
      const lsh_plan_s& P = *Fs[i]->plan;
      FactorData<float>& F = Fs[i]->f32;
      const int l = lev(i), c = P.lev[l].c, nb = 1 << l;
      const long cc = (long)c * c;
      gi.push_back({c, c, c, mone, zero, F.Pb[l].as<c32>(), c, cc, OP_N, F.Pa[l].as<c32>(), c, cc, OP_N, nullptr,
                    0, 0, F.Ci[l].as<c32>(), c, cc, nb, true});
    }
    run_gemms(tabs[1]);
    // C^{-1}
    std::vector<DevBuf> linfo(n_inst);
    for (int i : act) {
      const lsh_plan_s& P = *Fs[i]->plan;
      FactorData<float>& F = Fs[i]->f32;
      const int l = lev(i), c = P.lev[l].c, nb = 1 << l;
      linfo[i].alloc(sizeof(int) * nb);
      inv.push_back({F.Ci[l].as<c32>(), c, (long)c, (long)c * c, nb, linfo[i].as<int>()});
    }
    {
      DevBuf ws(inverse_grouped_ws_bytes(inv));
      inverse_grouped(s, inv, ws.p, itab);
    }
    inv.clear();
    for (int i : act)
      LSH_REQUIRE(!check_info(linfo[i], 1 << lev(i), s), LSH_ERR_SINGULAR,
                  "singular merge matrix I - Pb Pa at level " + std::to_string(lev(i)) + " (instance " +
                      std::to_string(i) + ")");
    // scattering matrices (not at the root)
    std::vector<DevBuf> A1(n_inst), A2(n_inst), Yl(n_inst), Gs(n_inst), Rs(n_inst);
    bool any = false;
    for (int i : act) {
      const lsh_plan_s& P = *Fs[i]->plan;
      const int l = lev(i);
      if (l == 0) continue;
      any = true;
      const int c = P.lev[l].c, nb = 1 << l, k = P.lev[l].k;
      const long ck = (long)c * k;
      mem::Arena& scr = Fs[i]->scr;
      A1[i].alloc_in(scr, sizeof(c32) * nb * ck);
      A2[i].alloc_in(scr, sizeof(c32) * nb * ck);
      Yl[i].alloc_in(scr, sizeof(c32) * nb * ck);
      if (!P.lev[l].ident) {
        const long nrt = rest_total(P.lev[l]);
        Gs[i].alloc_in(scr, sizeof(c32) * nb * (long)c * nrt);
        Rs[i].alloc_in(scr, sizeof(c32) * nb * nrt * k);
      }
      Fs[i]->f32.S[l].alloc_in(Fs[i]->keep, sizeof(c32) * nb * (long)k * k);
    }
    if (any) {
      auto each = [&](auto&& fn) {
        for (int i : act) {
          const lsh_plan_s& P = *Fs[i]->plan;
          const int l = lev(i);
          if (l == 0) continue;
          const int c = P.lev[l].c, nb = 1 << l, k = P.lev[l].k;
          fn(i, P, Fs[i]->f32, l, c, nb, k, (long)c * c, (long)c * k);
        }
      };
      // (the products of factor_scatter, grouped over the instances; dense
      // products with U = I on levels that keep all their candidates)
      auto push = [&](const ScatterGemm<float>& g) {
        gi.push_back({g.M, g.N, g.K, one, one, g.A, g.lda, g.sA, g.opA, g.B, g.ldb, g.sB, OP_N, g.C, g.ldc, g.sC,
                      g.C, g.ldc, g.sC, g.batch, false});
      };
      std::vector<GatherJob> gj;  // (every instance's gathers in one launch)
      DevBuf gtab1, gtab2;
      each([&](int i, const lsh_plan_s& P, FactorData<float>& F, int l, int c, int nb, int k, long cc, long ck) {
        const c32* Sch = F.S[l + 1].as<c32>();
        if (!P.lev[l].ident) {
          ScatterGemm<float> g[2];
          const int ng = scatter_su_prep<float>(P, l, Sch, A1[i].as<c32>(), A2[i].as<c32>(), ck, Gs[i].as<c32>(),
                                                s, g, &gj);
          for (int t = 0; t < ng; ++t) push(g[t]);
          return;
        }
        const c32* U1 = P.U<float>(l);
        gi.push_back({c, k, c, one, zero, Sch, c, 2 * cc, OP_N, U1, k, 0, OP_N, nullptr, 0, 0, A1[i].as<c32>(), k,
                      ck, nb, false});
        gi.push_back({c, k, c, one, zero, Sch + cc, c, 2 * cc, OP_N, U1 + ck, k, 0, OP_N, nullptr, 0, 0,
                      A2[i].as<c32>(), k, ck, nb, false});
      });
      gather_grouped(s, gj, gtab1);
      gj.clear();
      if (!gi.empty()) run_gemms(tabs[2]);
      each([&](int i, const lsh_plan_s&, FactorData<float>& F, int l, int c, int nb, int k, long cc, long ck) {
        gi.push_back({c, k, c, mone, one, F.Pb[l].as<c32>(), c, cc, OP_N, A1[i].as<c32>(), k, ck, OP_N,
                      A2[i].as<c32>(), k, ck, A2[i].as<c32>(), k, ck, nb, false});
      });
      run_gemms(tabs[3]);
      each([&](int i, const lsh_plan_s&, FactorData<float>& F, int l, int c, int nb, int k, long cc, long ck) {
        gi.push_back({c, k, c, one, zero, F.Ci[l].as<c32>(), c, cc, OP_N, A2[i].as<c32>(), k, ck, OP_N, nullptr, 0,
                      0, Yl[i].as<c32>(), k, ck, nb, false});
      });
      run_gemms(tabs[4]);
      each([&](int i, const lsh_plan_s&, FactorData<float>& F, int l, int c, int nb, int k, long cc, long ck) {
        gi.push_back({c, k, c, mone, one, F.Pa[l].as<c32>(), c, cc, OP_N, Yl[i].as<c32>(), k, ck, OP_N,
                      A1[i].as<c32>(), k, ck, A1[i].as<c32>(), k, ck, nb, false});
      });
      run_gemms(tabs[5]);
      std::vector<std::array<ScatterGemm<float>, 2>> ug(n_inst);
      std::vector<int> nug(n_inst, -1);  // -1: dense products with U = I
      each([&](int i, const lsh_plan_s& P, FactorData<float>& F, int l, int c, int nb, int k, long, long ck) {
        if (!P.lev[l].ident) {
          nug[i] = scatter_utb_prep<float>(P, l, A1[i].as<c32>(), Yl[i].as<c32>(), ck, F.S[l].as<c32>(),
                                           Rs[i].as<c32>(), s, ug[i].data(), &gj);
          return;
        }
        gi.push_back({k, k, c, one, zero, P.U<float>(l), k, 0, OP_T, A1[i].as<c32>(), k, ck, OP_N, nullptr, 0, 0,
                      F.S[l].as<c32>(), k, (long)k * k, nb, false});
      });
      gather_grouped(s, gj, gtab2);
      gj.clear();
      for (int i : act)
        if (nug[i] >= 1) push(ug[i][0]);
      if (!gi.empty()) run_gemms(tabs[6]);
      each([&](int i, const lsh_plan_s& P, FactorData<float>& F, int l, int c, int nb, int k, long, long ck) {
        if (!P.lev[l].ident) {
          if (nug[i] >= 2) push(ug[i][1]);
          return;
        }
        gi.push_back({k, k, c, one, one, P.U<float>(l) + ck, k, 0, OP_T, Yl[i].as<c32>(), k, ck, OP_N,
                      F.S[l].as<c32>(), k, (long)k * k, F.S[l].as<c32>(), k, (long)k * k, nb, false});
      });
      if (!gi.empty()) run_gemms(tabs[7]);
    }
    LSH_HIP(hipStreamSynchronize(s));  // scratch and tables of this level die here
  }
  for (int i = 0; i < n_inst; ++i) {  // singularity flags of the Woodbury levels
    try {
      factor_check(Fs[i]->f32, s);
    } catch (const Error& e) {
      throw Error(e.code, std::string(e.what()) + " (instance " + std::to_string(i) + ")");
    }
  }
  for (auto* F : Fs) ensure_apply_ws(*F->plan, F->f32);
}

// The batch's shared workspace: per level step (rewound between steps) the
// flags of the step's inverses, their grouped workspace and tables, and the
// problem tables of the step's grouped products (at most 12 launches of up
// to two problems per instance).
size_t batch_shared_bytes(const std::vector<const lsh_plan_s*>& Ps) {
  std::vector<const lsh_plan_s*> f;
  int Lmax = 0;
  for (auto* P : Ps)
    if (P->d.hbs_prec == LSH_FP32) {
      f.push_back(P);
      Lmax = std::max(Lmax, P->L);
    }
  if (f.empty()) return mem::kGranule;
  auto inv_bytes = [](const std::vector<InvItem>& it) {
    return mem::round_up(inverse_grouped_ws_bytes(it)) + inverse_grouped_arena_bytes(it);
  };
  size_t best = 0;
  {
    std::vector<InvItem> it;
    mem::Sizer z;
    for (auto* P : f) {
      it.push_back({nullptr, P->mL, (long)P->mL, (long)P->mL * P->mL, P->nleaf, nullptr});
      z.add_n<int>(P->nleaf);
    }
    best = z.total + inv_bytes(it) + 2 * cgemm_grouped_table_bytes(f.size());
  }
  for (int dpt = 1; dpt <= Lmax; ++dpt) {
    std::vector<InvItem> iw, is;
    mem::Sizer z;
    for (auto* P : f) {
      const int l = P->L - dpt;
      if (l < 0) continue;
      const Level& v = P->lev[l];
      const int nb = 1 << l;
      const int c = v.wr > 0 ? v.wr : v.c;
      (v.wr > 0 ? iw : is).push_back({nullptr, c, (long)c, (long)c * c, nb, nullptr});
      z.add_n<int>(nb);
    }
    const size_t t = z.total + inv_bytes(iw) + inv_bytes(is) + merge_level_table_bytes(iw.size()) +
                     mem::round_up(sizeof(int)) +
                     (iw.empty() ? 0 : 12 * cgemm_grouped_table_bytes(2 * iw.size())) +
                     (is.empty() ? 0 : 12 * cgemm_grouped_table_bytes(2 * is.size()));
    best = std::max(best, t);
  }
  return best;
}

}  // namespace

extern "C" {

int lsh_batch_factor_workspace(int ninst, const lsh_plan_t* plans, int flags, size_t* factor_bytes_out,
                               size_t* shared_bytes) {
  API_BEGIN
  LSH_REQUIRE(ninst >= 1 && plans && factor_bytes_out && shared_bytes, LSH_ERR_INVALID_ARG, "null argument");
  std::vector<const lsh_plan_s*> Ps;
  for (int i = 0; i < ninst; ++i) {
    LSH_REQUIRE(plans[i], LSH_ERR_INVALID_ARG, "null plan");
    Ps.push_back(plans[i]);
    factor_bytes_out[i] = factor_bytes(plan_profile(*plans[i]), (flags & LSH_FACTOR_TRANSPOSE) != 0).total();
  }
  *shared_bytes = batch_shared_bytes(Ps);
  return LSH_OK;
  API_END
}

int lsh_batch_factor(int ninst, const lsh_plan_t* plans, const double* const* b, int flags, void* const* ws,
                     const size_t* ws_bytes, void* shared_ws, size_t shared_bytes, void* stream,
                     lsh_factor_t* factors) {
  API_BEGIN
  LSH_REQUIRE(ninst >= 1 && plans && b && ws && ws_bytes && factors, LSH_ERR_INVALID_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  std::vector<std::unique_ptr<lsh_factor_s>> own;
  std::vector<lsh_factor_s*> f32;
  std::vector<const lsh_plan_s*> Ps;
  for (int i = 0; i < ninst; ++i) {
    LSH_REQUIRE(plans[i] && b[i], LSH_ERR_INVALID_ARG, "null plan or b");
    Ps.push_back(plans[i]);
  }
  mem::Arena shared;
  check_ws(shared_ws, shared_bytes, batch_shared_bytes(Ps), "batch shared");
  shared.attach(shared_ws, shared_bytes, "batch shared");
  for (int i = 0; i < ninst; ++i) {
    lsh_plan_s* P = plans[i];
    const long N = (long)P->n * P->n;
    std::unique_ptr<lsh_factor_s> F(new lsh_factor_s());
    F->plan = P;
    attach_factor(*F, plan_profile(*P), flags, ws[i], ws_bytes[i]);
    copy_check_b(*F, b[i], N, s, " (instance " + std::to_string(i) + ")");
    if (P->d.hbs_prec == LSH_FP32) f32.push_back(F.get());
    else factor_build<double>(*P, F->b.as<double>(), F->f64, s);  // FP64 instances: one at a time
    own.push_back(std::move(F));
  }
  if (!f32.empty()) batch_factor_f32(f32, shared, s);
  for (int i = 0; i < ninst; ++i) factors[i] = own[i].release();
  return LSH_OK;
  API_END
}

int lsh_factor_destroy(lsh_factor_t F) {
  API_BEGIN
  delete F;
  return LSH_OK;
  API_END
}

int lsh_apply_precond(lsh_factor_t F, int transpose, const void* x, void* y, int nrhs, void* stream) {
  API_BEGIN
  LSH_REQUIRE(F && x && y && nrhs >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  F->apply(static_cast<const z64*>(x), static_cast<z64*>(y), nrhs, (hipStream_t)stream, transpose != 0);
  return LSH_OK;
  API_END
}

int lsh_apply_operator(lsh_plan_t P, const double* b, const void* x, void* y, int nrhs, void* stream) {
  API_BEGIN
  LSH_REQUIRE(P && x && y && nrhs >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  P->op.apply((hipStream_t)stream, b, static_cast<const z64*>(x), static_cast<z64*>(y), nrhs);
  return LSH_OK;
  API_END
}

int lsh_solve_workspace(lsh_factor_t F, int nrhs, int maxit, size_t* bytes) {
  API_BEGIN
  LSH_REQUIRE(F && bytes && nrhs >= 1 && maxit >= 1 && maxit <= LSH_MAX_ITERS, LSH_ERR_INVALID_ARG, "bad argument");
  *bytes = SolveWs::bytes((long)F->plan->n * F->plan->n, std::min(nrhs, SOLVE_GROUP), maxit);
  return LSH_OK;
  API_END
}

}  // extern "C"

namespace {
// FGMRES arrays in the caller's solve workspace.
SolveWs solve_ws(lsh_factor_s& F, int nrhs, int maxit, void* ws, size_t bytes, mem::Arena& a) {
  const long N = (long)F.plan->n * F.plan->n;
  const int G = std::min(nrhs, SOLVE_GROUP);
  check_ws(ws, bytes, SolveWs::bytes(N, G, maxit), "solve");
  a.attach(ws, bytes, "solve");
  return SolveWs::carve([&](size_t b) { return a.take(b); }, N, G, maxit);
}
}  // namespace

extern "C" {

int lsh_solve(lsh_factor_t F, const void* u_inc, int nrhs, void* sigma, void* u, const lsh_solve_opts* opts,
              lsh_info* info, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN
  LSH_REQUIRE(F && u_inc && sigma && nrhs >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  lsh_solve_opts o{1e-10, 100, 1};
  if (opts) o = *opts;
  LSH_REQUIRE(o.maxit >= 1 && o.maxit <= LSH_MAX_ITERS && o.tol > 0, LSH_ERR_INVALID_ARG, "bad solve options");
  hipStream_t s = (hipStream_t)stream;
  lsh_plan_s& P = *F->plan;
  const long N = (long)P.n * P.n;
  const int G = std::min(nrhs, SOLVE_GROUP);
  mem::Arena arena;
  SolveWs W = solve_ws(*F, nrhs, o.maxit, ws, ws_bytes, arena);
  z64* f = W.f;
  int allconv = 1;
  double worst = 0;
  if (info) std::memset(info, 0, sizeof(lsh_info));
  if (nrhs == 1) {
    hipLaunchKernelGGL(k_rhs, dim3(2048), dim3(256), 0, s, f, static_cast<const z64*>(u_inc), F->b.as<double>(),
                       P.kappa * P.kappa, N);
    LSH_LAUNCH_CHECK();
    int conv = 0;
    fgmres_one(*F, W, f, static_cast<z64*>(sigma), o, info, worst, conv, s);
    allconv = conv;
  } else {
    for (int r0 = 0; r0 < nrhs; r0 += G) {
      const int nr = std::min(G, nrhs - r0);
      for (int r = 0; r < nr; ++r) {
        hipLaunchKernelGGL(k_rhs, dim3(2048), dim3(256), 0, s, f + r * N,
                           static_cast<const z64*>(u_inc) + (r0 + r) * N, F->b.as<double>(), P.kappa * P.kappa, N);
        LSH_LAUNCH_CHECK();
      }
      fgmres_multi(*F, W, f, static_cast<z64*>(sigma) + r0 * N, nr, o, info, worst, allconv, s);
    }
  }
  if (info) info->true_residual = worst;
  if (u) P.op.apply(s, nullptr, static_cast<const z64*>(sigma), static_cast<z64*>(u), nrhs);
  return allconv ? LSH_OK : LSH_NOT_CONVERGED;
  API_END
}

int lsh_solve_adjoint(lsh_factor_t F, const void* g, int nrhs, void* lambda, const lsh_solve_opts* opts,
                      lsh_info* info, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN
  LSH_REQUIRE(F && g && lambda && nrhs >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  lsh_solve_opts o{1e-10, 100, 1};
  if (opts) o = *opts;
  LSH_REQUIRE(o.maxit >= 1 && o.maxit <= LSH_MAX_ITERS && o.tol > 0, LSH_ERR_INVALID_ARG, "bad solve options");
  hipStream_t s = (hipStream_t)stream;
  lsh_plan_s& P = *F->plan;
  const long N = (long)P.n * P.n;
  const int G = std::min(nrhs, SOLVE_GROUP);
  mem::Arena arena;
  SolveWs W = solve_ws(*F, nrhs, o.maxit, ws, ws_bytes, arena);
  z64* f = W.f;
  int allconv = 1;
  double worst = 0;
  if (info) std::memset(info, 0, sizeof(lsh_info));
  // A^H lambda = g  <=>  A^T conj(lambda) = conj(g),  A^T = I + K B (K symmetric)
  z64* lam = static_cast<z64*>(lambda);
  const z64* gg = static_cast<const z64*>(g);
  if (nrhs == 1) {
    conj_copy(s, f, gg, N);
    int conv = 0;
    fgmres_one(*F, W, f, lam, o, info, worst, conv, s, true);
    conj_copy(s, lam, lam, N);
    allconv = conv;
  } else {
    for (int r0 = 0; r0 < nrhs; r0 += G) {
      const int nr = std::min(G, nrhs - r0);
      conj_copy(s, f, gg + r0 * N, (long)nr * N);
      fgmres_multi(*F, W, f, lam + r0 * N, nr, o, info, worst, allconv, s, true);
      conj_copy(s, lam + r0 * N, lam + r0 * N, (long)nr * N);
    }
  }
  if (info) info->true_residual = worst;
  return allconv ? LSH_OK : LSH_NOT_CONVERGED;
  API_END
}

int lsh_eval_points(lsh_plan_t P, const void* sigma, const double* xy, int npts, void* u_pts, int nrhs,
                    void* stream) {
  API_BEGIN
  LSH_REQUIRE(P && sigma && xy && u_pts && npts >= 1 && nrhs >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  for (int r0 = 0; r0 < nrhs; r0 += EV_MAXRHS) {
    const int nr = nrhs - r0 < EV_MAXRHS ? nrhs - r0 : EV_MAXRHS;
    const long N = (long)P->n * P->n;
    hipLaunchKernelGGL(k_eval_points, dim3(npts), dim3(256), 0, s, static_cast<const z64*>(sigma) + r0 * N, P->n,
                       P->h, P->d.x0, P->d.y0, P->kappa, xy, static_cast<z64*>(u_pts) + (long)r0 * npts, npts, nr);
    LSH_LAUNCH_CHECK();
  }
  return LSH_OK;
  API_END
}

}  // extern "C"

#include "../../include/lsh_dev.h"

extern "C" {

int lsh_dev_gemm(int prec, int M, int N, int K, const double* alpha, const void* A, long lda, long sA, int opA,
                 const void* B, long ldb, long sB, int opB, const double* beta, const void* D, long ldd, long sD,
                 void* C, long ldc, long sC, int batch, void* stream) {
  API_BEGIN
  LSH_REQUIRE(alpha && beta && A && B && C && M >= 0 && N >= 0 && K >= 0 && batch >= 0, LSH_ERR_INVALID_ARG,
              "bad gemm argument");
  LSH_REQUIRE(opA >= 0 && opA <= 3 && opB >= 0 && opB <= 3, LSH_ERR_INVALID_ARG, "bad op");
  hipStream_t s = (hipStream_t)stream;
  if (prec == LSH_FP64)
    cgemm<double>(s, M, N, K, mk(alpha[0], alpha[1]), (const z64*)A, lda, sA, (Op)opA, (const z64*)B, ldb, sB,
                  (Op)opB, mk(beta[0], beta[1]), (const z64*)D, ldd, sD, (z64*)C, ldc, sC, batch);
  else
    cgemm<float>(s, M, N, K, mk((float)alpha[0], (float)alpha[1]), (const c32*)A, lda, sA, (Op)opA, (const c32*)B,
                 ldb, sB, (Op)opB, mk((float)beta[0], (float)beta[1]), (const c32*)D, ldd, sD, (c32*)C, ldc, sC,
                 batch);
  return LSH_OK;
  API_END
}

int lsh_dev_gemm_split(int prec, int M, int N, int K, const double* alpha, const void* A, long lda, long sA,
                       int opA, const void* B, long ldb, long sB, int opB, const double* beta, const void* D,
                       long ldd, long sD, void* C, long ldc, long sC, int batch, void* ws, size_t ws_bytes,
                       void* stream) {
  API_BEGIN
  LSH_REQUIRE(alpha && beta && A && B && C && M >= 0 && N >= 0 && K >= 0 && batch >= 0, LSH_ERR_INVALID_ARG,
              "bad gemm argument");
  LSH_REQUIRE(opA >= 0 && opA <= 3 && opB >= 0 && opB <= 3, LSH_ERR_INVALID_ARG, "bad op");
  hipStream_t s = (hipStream_t)stream;
  if (prec == LSH_FP64)
    cgemm_ws<double>(s, M, N, K, mk(alpha[0], alpha[1]), (const z64*)A, lda, sA, (Op)opA, (const z64*)B, ldb, sB,
                     (Op)opB, mk(beta[0], beta[1]), (const z64*)D, ldd, sD, (z64*)C, ldc, sC, batch, ws, ws_bytes);
  else
    cgemm_ws<float>(s, M, N, K, mk((float)alpha[0], (float)alpha[1]), (const c32*)A, lda, sA, (Op)opA,
                    (const c32*)B, ldb, sB, (Op)opB, mk((float)beta[0], (float)beta[1]), (const c32*)D, ldd, sD,
                    (c32*)C, ldc, sC, batch, ws, ws_bytes);
  return LSH_OK;
  API_END
}

// ---- GEMM autotuner
int lsh_gemm_variants(int prec, int* count, char* names, int cap) {
  API_BEGIN
  LSH_REQUIRE(count && (prec == LSH_FP32 || prec == LSH_FP64), LSH_ERR_INVALID_ARG, "bad argument");
  const int p = prec == LSH_FP32 ? 1 : 0;
  *count = gemm_variant_count(p);
  if (names && cap > 0) {
    std::string t;
    for (int v = 0; v < *count; ++v) t += (v ? ";" : "") + std::string(gemm_variant_name(p, v));
    std::strncpy(names, t.c_str(), cap - 1);
    names[cap - 1] = 0;
  }
  return LSH_OK;
  API_END
}

int lsh_fused_levels(int min_boxes) {
  API_BEGIN
  LSH_REQUIRE(min_boxes >= -1, LSH_ERR_INVALID_ARG, "min_boxes must be >= -1");
  g_fused_min_boxes = min_boxes < 0 ? kFusedMinBoxes : min_boxes;
  return LSH_OK;
  API_END
}

int lsh_apply_fused_levels(int min_vectors) {
  API_BEGIN
  LSH_REQUIRE(min_vectors >= -1, LSH_ERR_INVALID_ARG, "min_vectors must be >= -1");
  g_apply_fused_min = min_vectors < 0 ? kApplyFusedMin : min_vectors;
  return LSH_OK;
  API_END
}

int lsh_gemm_force_variant(int variant) {
  API_BEGIN
  gemm_force_variant(variant);
  return LSH_OK;
  API_END
}

int lsh_gemm_tune_workspace(int prec, int M, int N, int K, int batch, size_t* bytes) {
  API_BEGIN
  LSH_REQUIRE(bytes && M >= 1 && N >= 1 && K >= 1 && batch >= 1, LSH_ERR_INVALID_ARG, "bad argument");
  const size_t e = prec == LSH_FP32 ? sizeof(c32) : sizeof(z64);
  mem::Sizer z;
  z.add(e * (size_t)batch * M * K);
  z.add(e * (size_t)K * N);
  z.add(e * (size_t)batch * M * N);
  *bytes = z.total;
  return LSH_OK;
  API_END
}

int lsh_gemm_tune(int prec, int M, int N, int K, int batch, int reps, void* ws, size_t ws_bytes, void* stream,
                  int* best, double* ms) {
  API_BEGIN
  LSH_REQUIRE(M >= 1 && N >= 1 && K >= 1 && batch >= 1 && reps >= 1 && (prec == LSH_FP32 || prec == LSH_FP64),
              LSH_ERR_INVALID_ARG, "bad argument");
  size_t need = 0;
  LSH_REQUIRE(lsh_gemm_tune_workspace(prec, M, N, K, batch, &need) == LSH_OK, LSH_ERR_INVALID_ARG, "bad shape");
  check_ws(ws, ws_bytes, need, "tune");
  hipStream_t s = (hipStream_t)stream;
  mem::Arena a;
  a.attach(ws, ws_bytes, "tune");
  const size_t e = prec == LSH_FP32 ? sizeof(c32) : sizeof(z64);
  void* A = a.take(e * (size_t)batch * M * K);
  void* B = a.take(e * (size_t)K * N);
  void* C = a.take(e * (size_t)batch * M * N);
  fill_zero(s, A, e * (size_t)batch * M * K);
  fill_zero(s, B, e * (size_t)K * N);
  const int p = prec == LSH_FP32 ? 1 : 0, nv = gemm_variant_count(p);
  hipEvent_t e0, e1;
  LSH_HIP(hipEventCreate(&e0));
  LSH_HIP(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } evs{e0, e1};
  auto run = [&] {
    if (p == 1)
      cgemm<float>(s, M, N, K, mk(1.0f, 0.0f), (const c32*)A, K, (long)M * K, OP_N, (const c32*)B, N, 0, OP_N,
                   mk(0.0f, 0.0f), nullptr, 0, 0, (c32*)C, N, (long)M * N, batch);
    else
      cgemm<double>(s, M, N, K, mk(1.0, 0.0), (const z64*)A, K, (long)M * K, OP_N, (const z64*)B, N, 0, OP_N,
                    mk(0.0, 0.0), nullptr, 0, 0, (z64*)C, N, (long)M * N, batch);
  };
  int bv = 0;
  double bt = 1e300;
  struct Unforce {
    ~Unforce() { gemm_force_variant(-1); }
  } unforce;
  for (int v = 0; v < nv; ++v) {
    gemm_force_variant(v);
    run();  // warm
    LSH_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) run();
    LSH_HIP(hipEventRecord(e1, s));
    LSH_HIP(hipEventSynchronize(e1));
    float t = 0;
    LSH_HIP(hipEventElapsedTime(&t, e0, e1));
    const double tv = (double)t / reps;
    if (ms) ms[v] = tv;
    if (tv < bt) { bt = tv; bv = v; }
  }
  gemm_force_variant(-1);
  gemm_tune_set(p, M, N, K, batch, bv);
  if (best) *best = bv;
  return LSH_OK;
  API_END
}

int lsh_gemm_table_save(const char* path) {
  API_BEGIN
  LSH_REQUIRE(path, LSH_ERR_INVALID_ARG, "null path");
  gemm_table_save(path);
  return LSH_OK;
  API_END
}

int lsh_gemm_table_load(const char* path, int* entries) {
  API_BEGIN
  LSH_REQUIRE(path, LSH_ERR_INVALID_ARG, "null path");
  const int n = gemm_table_load(path);
  if (entries) *entries = n;
  return LSH_OK;
  API_END
}

int lsh_gemm_table_clear(void) {
  API_BEGIN
  gemm_table_clear();
  return LSH_OK;
  API_END
}

int lsh_gemm_record(int on) {
  API_BEGIN
  gemm_record(on != 0);
  return LSH_OK;
  API_END
}

int lsh_gemm_recorded(int* count, int* shapes, int cap) {
  API_BEGIN
  LSH_REQUIRE(count, LSH_ERR_INVALID_ARG, "null count");
  const auto v = gemm_recorded();
  *count = (int)v.size();
  if (shapes)
    for (int i = 0; i < (int)v.size() && i < cap; ++i)
      for (int q = 0; q < 6; ++q) shapes[6 * i + q] = v[i][q];
  return LSH_OK;
  API_END
}

int lsh_dev_inverse_workspace(int prec, int c, int batch, size_t* bytes) {
  API_BEGIN
  LSH_REQUIRE(bytes && c >= 1 && batch >= 1, LSH_ERR_INVALID_ARG, "bad inverse argument");
  *bytes = prec == LSH_FP64 ? inverse_ws_bytes<double>(c, batch) : inverse_ws_bytes<float>(c, batch);
  return LSH_OK;
  API_END
}

int lsh_dev_inverse(int prec, void* A, int c, long lda, long sA, int batch, int* info, void* ws, size_t ws_bytes,
                    void* stream) {
  API_BEGIN
  LSH_REQUIRE(A && c >= 1 && batch >= 1 && lda >= c, LSH_ERR_INVALID_ARG, "bad inverse argument");
  hipStream_t s = (hipStream_t)stream;
  const size_t need = prec == LSH_FP64 ? inverse_ws_bytes<double>(c, batch) : inverse_ws_bytes<float>(c, batch);
  check_ws(ws, ws_bytes, need, "inverse");
  if (prec == LSH_FP64) inverse<double>(s, (z64*)A, c, lda, sA, batch, ws, info);
  else inverse<float>(s, (c32*)A, c, lda, sA, batch, ws, info);
  return LSH_OK;
  API_END
}

}  // extern "C"
