// Corrected-trapezoidal weights for the 2-D Helmholtz kernel (host, FP64).
//
// Paper Sec. 2.2, eq. (corrected), Fig. 2: the punctured trapezoidal rule is
// corrected on 1/5/13/25-point stencils (orders 4/6/8/10); the weights depend
// only on kappa*h.  Construction used here: split
//   (i/4) H0(kappa r) = -(1/2 pi) J0(kappa r) ln r + R(r),  R smooth,
//   R(0) = i/4 - (ln(kappa/2) + gamma) / (2 pi);
// the smooth part only needs the missing centre node h^2 R(0); the log part
// is corrected through the lattice zeta function Z_p(s) = sum' p(j)|j|^-2s:
// a stencil weight set tau' with sum_d tau'_d d^a = Z'_{x^a}(0)/2 for every
// D4-invariant monomial moment up to degree 2m removes the error terms
// through h^{2m+2}.  The zeta derivatives are evaluated from their theta
// function (Mellin) representations by Gauss-Legendre quadrature:
//   pi^-s Gamma(s) Z(s) = int_1^inf (t^{s-1} + t^{-s})(theta(t) - 1) dt - 1/s - 1/(1-s),
//   theta(t) = sum_j exp(-pi t |j|^2),
// and for the degree-4 harmonic polynomial P = Re (x+iy)^4 (theta_P(t) =
// t^-5 theta_P(1/t)):  pi^-s Gamma(s) Z_P(s) = int_1^inf (t^{s-1} + t^{4-s}) theta_P(t) dt.
#include <cmath>
#include <vector>

#include "weights.hpp"

namespace lsh {
namespace {

typedef long double ld;
const ld PI_L = 3.141592653589793238462643383279502884L;
const ld EULER_L = 0.577215664901532860606512090082402431L;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<ld>& x, std::vector<ld>& w) {
  x.assign(n, 0);
  w.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    ld z = std::cos(PI_L * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      ld dp = n * (z * p1 - p0) / (z * z - 1);
      ld dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    ld p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    ld dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

// theta(t) - 1 and theta_P(t), summed over |j_i| <= 8 (t >= 1: tail < 1e-80)
void thetas(ld t, ld& th1, ld& thp) {
  th1 = 0;
  thp = 0;
  for (int a = -8; a <= 8; ++a)
    for (int b = -8; b <= 8; ++b) {
      if (!a && !b) continue;
      ld r2 = (ld)a * a + (ld)b * b;
      ld e = std::exp(-PI_L * t * r2);
      th1 += e;
      ld p = (ld)a * a * a * a - 6.0L * a * a * b * b + (ld)b * b * b * b;
      thp += p * e;
    }
}

struct ZetaData {
  ld dZ[4];   // Z'(0), Z'(-1), Z'(-2), Z'(-3)
  ld dH[2];   // Z_P'(0), Z_P'(-1)
};

ZetaData compute_zeta() {
  std::vector<ld> gx, gw;
  gauss_legendre(24, gx, gw);
  // integrals over [1, 41] in 40 unit panels
  ld F[4] = {0, 0, 0, 0};   // F(0), F(-1), F(-2), F(-3)
  ld LP[2] = {0, 0};        // Lambda_P(0), Lambda_P(-1)
  for (int pnl = 0; pnl < 40; ++pnl) {
    ld a = 1 + pnl, b = a + 1;
    for (size_t q = 0; q < gx.size(); ++q) {
      ld t = 0.5L * (a + b) + 0.5L * (b - a) * gx[q];
      ld wt = 0.5L * (b - a) * gw[q];
      ld th1, thp;
      thetas(t, th1, thp);
      for (int n = 0; n < 4; ++n) {
        ld s = -n;
        F[n] += wt * (std::pow(t, s - 1) + std::pow(t, -s)) * th1;
      }
      for (int n = 0; n < 2; ++n) {
        ld s = -n;
        LP[n] += wt * (std::pow(t, s - 1) + std::pow(t, 4 - s)) * thp;
      }
    }
  }
  ZetaData z;
  z.dZ[0] = F[0] - EULER_L - 1 - std::log(PI_L);
  ld fact = 1;
  for (int n = 1; n <= 3; ++n) {
    fact *= n;
    ld lam = F[n] + 1.0L / n - 1.0L / (n + 1);
    z.dZ[n] = std::pow(PI_L, -(ld)n) * lam * fact * ((n & 1) ? -1 : 1);
  }
  z.dH[0] = LP[0];
  z.dH[1] = -LP[1] / PI_L;
  return z;
}

const int ORB[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {3, 0}};

int orbit_points(int o, int pts[8][2]) {
  int a = ORB[o][0], b = ORB[o][1], n = 0;
  for (int sw = 0; sw < 2; ++sw)
    for (int sx = -1; sx <= 1; sx += 2)
      for (int sy = -1; sy <= 1; sy += 2) {
        int x = sx * (sw ? b : a), y = sy * (sw ? a : b);
        bool dup = false;
        for (int k = 0; k < n; ++k)
          if (pts[k][0] == x && pts[k][1] == y) dup = true;
        if (!dup) { pts[n][0] = x; pts[n][1] = y; ++n; }
      }
  return n;
}

ld moment(int r, ld x, ld y) {
  switch (r) {
    case 0: return 1;
    case 1: return x * x + y * y;
    case 2: return x * x * x * x + y * y * y * y;
    case 3: return x * x * y * y;
    case 4: return std::pow(x, 6) + std::pow(y, 6);
    default: return x * x * x * x * y * y + x * x * y * y * y * y;
  }
}

}  // namespace

std::vector<double> orbit_weights(int order) {
  static ZetaData z = compute_zeta();
  int m = order == 4 ? 1 : order == 6 ? 2 : order == 8 ? 4 : order == 10 ? 6 : 0;
  if (!m) throw Error(-1, "correction order must be 4, 6, 8 or 10");
  // half derivatives of the six moment zeta functions (radial + harmonic split)
  ld c[6] = {z.dZ[0] / 2,
             z.dZ[1] / 2,
             (0.75L * z.dZ[2] + 0.25L * z.dH[0]) / 2,
             (0.125L * z.dZ[2] - 0.125L * z.dH[0]) / 2,
             (0.625L * z.dZ[3] + 0.375L * z.dH[1]) / 2,
             (0.125L * z.dZ[3] - 0.125L * z.dH[1]) / 2};
  ld A[6][7];
  for (int r = 0; r < m; ++r) {
    for (int o = 0; o < m; ++o) {
      int pts[8][2];
      int np = orbit_points(o, pts);
      ld s = 0;
      for (int k = 0; k < np; ++k) s += moment(r, pts[k][0], pts[k][1]);
      A[r][o] = s;
    }
    A[r][m] = c[r];
  }
  for (int col = 0; col < m; ++col) {  // Gaussian elimination, partial pivoting
    int p = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(A[r][col]) > std::fabs(A[p][col])) p = r;
    for (int k = 0; k <= m; ++k) std::swap(A[col][k], A[p][k]);
    for (int r = 0; r < m; ++r) {
      if (r == col) continue;
      ld f = A[r][col] / A[col][col];
      for (int k = col; k <= m; ++k) A[r][k] -= f * A[col][k];
    }
  }
  std::vector<double> out(m);
  for (int r = 0; r < m; ++r) out[r] = (double)(A[r][m] / A[r][r]);
  return out;
}

std::vector<StencilEntry> correction_stencil(int order, double kh) {
  std::vector<double> tw = orbit_weights(order);
  std::vector<StencilEntry> st;
  for (size_t o = 0; o < tw.size(); ++o) {
    int pts[8][2];
    int np = orbit_points((int)o, pts);
    for (int k = 0; k < np; ++k) {
      StencilEntry e;
      e.dx = pts[k][0];
      e.dy = pts[k][1];
      double r = std::sqrt((double)e.dx * e.dx + (double)e.dy * e.dy);
      e.re = -tw[o] / (2 * M_PI) * ::j0(kh * r);
      e.im = 0;
      if (!e.dx && !e.dy) {
        e.re += -(std::log(kh / 2) + (double)EULER_L) / (2 * M_PI);
        e.im += 0.25;
      }
      st.push_back(e);
    }
  }
  return st;
}

}  // namespace lsh
