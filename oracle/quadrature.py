"""Corrected trapezoidal weights for the 2-D Helmholtz kernel (oracle side).

Paper, Sec. 2.2, eq. (corrected) and Fig. 2: the punctured trapezoidal rule
is corrected on a 1/5/13/25-point stencil to reach orders 4/6/8/10; the
weights depend only on kappa*h and the order.  The paper does not print the
weights (it refers to Duan & Rokhlin), so this module constructs them from
first principles:

1. Split the kernel G(r) = (i/4) H0(kappa r) = -(1/2pi) J0(kappa r) ln r + R(r)
   with R smooth (even, entire in r^2) and
   R(0) = i/4 - (1/2pi) (ln(kappa/2) + gamma_E)   (series of Y0).
2. The smooth part is integrated spectrally by the full trapezoidal rule; the
   punctured rule only misses the centre node, worth h^2 R(0) sigma_i.
3. For the log part the generalised Euler-Maclaurin formula for the punctured
   lattice sum of ln|x| phi(x) (phi = J0(kappa|x|) sigma(x_i + x)) has the
   error expansion
      h^2 sum' ln|hj| phi(hj) - int ln|x| phi
          = -h^2 ln h phi(0) - sum_a h^{2+|a|} (d^a phi(0)/a!) * (1/2) Z'_{x^a}(0)
   with the lattice zeta function Z_p(s) = sum'_{j in Z^2} p(j) |j|^{-2s}.
   A stencil sum h^2 sum_d tau'_d phi(hd) reproduces the last term through
   degree 2m when sum_d tau'_d d^a = (1/2) Z'_{x^a}(0) for |a| <= 2m.  By the
   square-lattice symmetry only the D4-invariant moments
   {1, x^2+y^2, x^4+y^4, x^2 y^2, x^6+y^6, x^4 y^2 + x^2 y^4} matter, which
   gives 1/2/4/6 equations for orders 4/6/8/10 on the orbits of Fig. 2.
4. The weight applied to sigma at offset d from the target (in units of h^2):
      tau_d = -(1/2pi) tau'_{orbit(d)} J0(kappa h |d|)
              + [d = 0] (i/4 - (1/2pi)(ln(kappa h / 2) + gamma_E)).

The zeta derivatives come from closed forms for the radial moments,
Z(s) = 4 zeta(s) beta(s) on the square lattice, and from the theta-function
(Hecke) integral for the degree-4 harmonic moment Re((x+iy)^4); both are
evaluated here with mpmath at 30 digits.
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np
from scipy import special

EULER_GAMMA = float(mpmath.euler)

# Orbits of the correction stencil under the symmetry group of the square
# lattice (Fig. 2): a representative and the full list of offsets.
ORBIT_REPS = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (3, 0)]


def _orbit(rep):
    a, b = rep
    pts = set()
    for (x, y) in [(a, b), (b, a)]:
        for sx in (1, -1):
            for sy in (1, -1):
                pts.add((sx * x, sy * y))
    return sorted(pts)


ORBITS = [_orbit(r) for r in ORBIT_REPS]
# number of orbits used by each order (Fig. 2: 1, 5, 13, 25 points)
N_ORBITS = {4: 1, 6: 2, 8: 4, 10: 6}

# The D4-invariant moment polynomials, in the order of the equations.
MOMENTS = [
    lambda x, y: 1.0 + 0 * x,
    lambda x, y: x * x + y * y,
    lambda x, y: x ** 4 + y ** 4,
    lambda x, y: x * x * y * y,
    lambda x, y: x ** 6 + y ** 6,
    lambda x, y: x ** 4 * y * y + x * x * y ** 4,
]


@functools.lru_cache(maxsize=None)
def radial_zeta_derivs():
    """Z'(0), Z'(-1), Z'(-2), Z'(-3) for Z(s) = sum'_{j in Z^2} |j|^{-2s}.

    Square lattice: Z(s) = 4 zeta(s) beta(s) (Dirichlet beta).  With
    zeta(0) = -1/2, zeta'(0) = -ln(2pi)/2, beta(0) = 1/2,
    beta'(0) = ln(Gamma(1/4)^2 / (2 pi sqrt 2)), beta(-n) = E_n / 2, and the
    functional equation of beta for beta'(-1), beta'(-3):
      Z'(0)  = ln(4 pi) - 4 ln Gamma(1/4)
      Z'(-1) = -2 G / (3 pi)            (G = Catalan's constant)
      Z'(-2) = zeta(3) / (2 pi^2)
      Z'(-3) = -(8/5) beta(4) / pi^3
    Z_{|x|^{2m}}(s) = Z(s - m) gives the radial moments.
    """
    with mpmath.workdps(30):
        pi = mpmath.pi
        return (
            float(mpmath.log(4 * pi) - 4 * mpmath.loggamma(mpmath.mpf(1) / 4)),
            float(-2 * mpmath.catalan / (3 * pi)),
            float(mpmath.zeta(3) / (2 * pi ** 2)),
            float(-mpmath.mpf(8) / 5 * mpmath.dirichlet(4, [0, 1, 0, -1]) / pi ** 3),
        )


def _theta_harmonic4(t):
    """sum_j Re((j1 + i j2)^4) exp(-pi t |j|^2) (mpmath, t >= 1)."""
    s = mpmath.mpf(0)
    J = 7  # exp(-49 pi) < 1e-66: far below 30 digits
    for j1 in range(-J, J + 1):
        for j2 in range(-J, J + 1):
            p = j1 ** 4 - 6 * j1 * j1 * j2 * j2 + j2 ** 4
            if p:
                s += p * mpmath.exp(-mpmath.pi * t * (j1 * j1 + j2 * j2))
    return s


@functools.lru_cache(maxsize=None)
def harmonic4_zeta_derivs():
    """H'(0), H'(-1) for H(s) = sum'_j Re((j1+ij2)^4) |j|^{-2s}.

    Hecke: the lattice theta series of a degree-4 harmonic polynomial obeys
    theta_P(t) = t^{-5} theta_P(1/t), so
      pi^{-s} Gamma(s) H(s) = int_1^inf (t^{s-1} + t^{4-s}) theta_P(t) dt
    is entire; with 1/Gamma(s) ~ s near 0 and ~ -(s+1) near -1:
      H'(0) = Lambda(0),  H'(-1) = -Lambda(-1)/pi.
    """
    with mpmath.workdps(30):
        lam = lambda s: mpmath.quad(
            lambda t: (t ** (s - 1) + t ** (4 - s)) * _theta_harmonic4(t),
            [1, 2, 4, 8, 16, 40])
        return float(lam(0)), float(-lam(-1) / mpmath.pi)


@functools.lru_cache(maxsize=None)
def moment_constants():
    """c_p = (1/2) Z'_p(0) for the six D4-invariant moment polynomials.

    Decomposition into radial and harmonic parts (z = x + iy):
      x^4+y^4       = (3|z|^4 + Re z^4)/4
      x^2 y^2       = (|z|^4 - Re z^4)/8
      x^6+y^6       = (5|z|^6 + 3|z|^2 Re z^4)/8
      x^4y^2+x^2y^4 = (|z|^6 - |z|^2 Re z^4)/8
    (Re z^6 terms vanish on the square lattice by the 90-degree symmetry.)
    """
    z0, z1, z2, z3 = radial_zeta_derivs()
    h0, h1 = harmonic4_zeta_derivs()
    dz = [
        z0,
        z1,
        0.75 * z2 + 0.25 * h0,
        0.125 * z2 - 0.125 * h0,
        0.625 * z3 + 0.375 * h1,
        0.125 * z3 - 0.125 * h1,
    ]
    return tuple(0.5 * v for v in dz)


@functools.lru_cache(maxsize=None)
def orbit_weights(order: int):
    """tau' per orbit (kappa-independent) from the moment equations."""
    if order not in N_ORBITS:
        raise ValueError("order must be one of 4, 6, 8, 10")
    m = N_ORBITS[order]
    A = np.zeros((m, m))
    for r in range(m):
        for o in range(m):
            A[r, o] = sum(MOMENTS[r](float(x), float(y)) for (x, y) in ORBITS[o])
    c = np.array(moment_constants()[:m])
    return tuple(np.linalg.solve(A, c))


def correction_weights(order: int, kh: float):
    """{(dx, dy): tau_d} -- the correction added to h^2 G at offset d.

    The matrix entry coupling target x_i to source x_i + h d is
    h^2 (G(h|d|) [d != 0] + tau_d) (paper eq. (corrected), (Gmat)).
    """
    tw = orbit_weights(order)
    out = {}
    for o, w in enumerate(tw):
        for (dx, dy) in ORBITS[o]:
            r = np.hypot(dx, dy)
            out[(dx, dy)] = complex(-w / (2 * np.pi) * special.j0(kh * r))
    out[(0, 0)] += 0.25j - (np.log(kh / 2) + EULER_GAMMA) / (2 * np.pi)
    return out


def green(kappa: float, r):
    """(i/4) H0^(1)(kappa r), paper eq. (kernel)."""
    return 0.25j * special.hankel1(0, kappa * np.asarray(r, dtype=float))
