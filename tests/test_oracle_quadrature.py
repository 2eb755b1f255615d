"""Pins for the oracle's corrected quadrature (paper Sec. 2.2, eq. (corrected), Fig. 2).

* The radial lattice-zeta derivatives (closed forms in the oracle) are checked
  against an independent numerical route: the theta-function (Ewald) split
  of the Epstein zeta function integrated in double precision.
* The whole weight construction -- moment constants, the harmonic part, the
  J0 factor, the R(0) centre term -- is pinned by the convergence orders the
  paper states (2 uncorrected, then 4/6/8/10) on a smooth compactly
  supported density whose integral against the kernel is known in closed
  form up to a 1-D integral (Bessel-I0 angular average), evaluated with
  mpmath.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

from oracle import quadrature as quad


def _theta_m1(t):
    j = np.arange(-8, 9)
    J1, J2 = np.meshgrid(j, j)
    r2 = (J1 ** 2 + J2 ** 2).ravel()
    r2 = r2[r2 > 0]
    return float(np.sum(np.exp(-np.pi * t * r2)))


def _epstein_deriv_theta(n):
    """Z'(-n) of Z(s) = sum' |j|^{-2s} from pi^-s Gamma(s) Z(s) = F(s) - 1/s - 1/(1-s)."""
    F = lambda s: integrate.quad(lambda t: (t ** (s - 1) + t ** (-s)) * _theta_m1(t), 1, 40,
                                 epsabs=1e-16, epsrel=1e-14, limit=200)[0]
    if n == 0:
        return F(0) - np.euler_gamma - 1 - np.log(np.pi)
    lam = F(-n) + 1.0 / n - 1.0 / (1 + n)
    return np.pi ** (-n) * lam * math.factorial(n) * (-1) ** n


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_radial_zeta_closed_forms_match_theta_split(n):
    assert quad.radial_zeta_derivs()[n] == pytest.approx(_epstein_deriv_theta(n), rel=1e-12, abs=1e-14)


def test_stencil_sizes_fig2():
    sizes = {o: sum(len(quad.ORBITS[i]) for i in range(quad.N_ORBITS[o])) for o in (4, 6, 8, 10)}
    assert sizes == {4: 1, 6: 5, 8: 13, 10: 25}


def test_weights_depend_on_kh_only_and_are_symmetric():
    w = quad.correction_weights(10, 0.3)
    for (dx, dy), v in w.items():
        assert w[(dy, dx)] == v and w[(-dx, dy)] == v


# --- convergence orders -------------------------------------------------------

KAPPA, S, C = 20.0, 0.1, np.array([0.03, 0.02])


@pytest.fixture(scope="module")
def exact_integral():
    """int G(|y|) exp(-|y - c|^2 / s^2) dy by polar coordinates about the target 0."""
    d = float(np.hypot(*C))
    with mpmath.workdps(20):
        f = lambda r: (mpmath.mpc(0, 0.25) * (mpmath.besselj(0, KAPPA * r) + 1j * mpmath.bessely(0, KAPPA * r))
                       * r * mpmath.exp(-(r * r + d * d) / S ** 2) * mpmath.besseli(0, 2 * r * d / S ** 2))
        return complex(2 * mpmath.pi * mpmath.quad(f, [0, d, d + 2 * S, d + 4 * S, d + 8 * S, d + 12 * S]))


def _rule(h, order):
    J = int(np.ceil((np.hypot(*C) + 12 * S) / h))
    j = np.arange(-J, J + 1)
    X, Y = np.meshgrid(j, j, indexing="ij")
    r = h * np.hypot(X, Y)
    phi = np.exp(-((h * X - C[0]) ** 2 + (h * Y - C[1]) ** 2) / S ** 2)
    G = np.where(r > 0, quad.green(KAPPA, np.where(r > 0, r, 1.0)), 0)
    val = h * h * np.sum(G * phi)
    if order:
        for (dx, dy), t in quad.correction_weights(order, KAPPA * h).items():
            val += h * h * t * np.exp(-((h * dx - C[0]) ** 2 + (h * dy - C[1]) ** 2) / S ** 2)
    return val


@pytest.mark.parametrize("order,lo,hi", [(0, 1.5, 2.5), (4, 3.7, 4.4), (6, 5.7, 6.4), (8, 7.6, 8.5), (10, 9.4, 10.7)])
def test_convergence_order(exact_integral, order, lo, hi):
    e1 = abs(_rule(S / 16, order) - exact_integral)
    e2 = abs(_rule(S / 24, order) - exact_integral)
    p = np.log(e1 / e2) / np.log(24 / 16)
    assert lo < p < hi, (order, p, e1, e2)
    if order == 10:
        assert e2 / abs(exact_integral) < 1e-13
