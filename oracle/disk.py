"""Transmission by a constant-b disk: textbook separation of variables.

TEST INFRASTRUCTURE (a pin for the dense oracle).  Remark 1.1 of the paper:
the Lippmann-Schwinger solution is the solution of
  -Lap u_tot - kappa^2 (1 - b) u_tot = 0,
u_tot = u_inc + u, u outgoing.  For b = b0 inside a disk of radius a centred
at the origin (0 outside) and u_inc = exp(i kappa x1), with
k_in = kappa sqrt(1 - b0):
  inside  u_tot = sum_m c_m J_m(k_in r) e^{i m t}
  outside u_tot = sum_m (i^m J_m(kappa r) + d_m H_m(kappa r)) e^{i m t}
with continuity of u_tot and its radial derivative at r = a.  The density is
sigma = -kappa^2 b u_tot (eq. (ls) rearranged).
"""
from __future__ import annotations

import numpy as np
from scipy import special


def coefficients(kappa, b0, a, mmax):
    kin = kappa * np.sqrt(1.0 - b0)
    m = np.arange(-mmax, mmax + 1)
    Jm_in = special.jv(m, kin * a)
    dJm_in = kin * special.jvp(m, kin * a)
    Jm = special.jv(m, kappa * a)
    dJm = kappa * special.jvp(m, kappa * a)
    Hm = special.hankel1(m, kappa * a)
    dHm = kappa * special.h1vp(m, kappa * a)
    inc = (1j) ** m
    # c J_in - d H = inc J ; c J_in' - d H' = inc J'
    det = -Jm_in * dHm + dJm_in * Hm
    c = inc * (-Jm * dHm + dJm * Hm) / det
    d = inc * (Jm_in * dJm - dJm_in * Jm) / det
    return m, kin, c, d


def total_field(kappa, b0, a, x1, x2, mmax=None):
    x1 = np.asarray(x1, dtype=float)
    x2 = np.asarray(x2, dtype=float)
    if mmax is None:
        mmax = int(kappa * max(a, float(np.max(np.hypot(x1, x2)))) + 30)
    m, kin, c, d = coefficients(kappa, b0, a, mmax)
    r = np.hypot(x1, x2)[..., None]
    t = np.arctan2(x2, x1)[..., None]
    e = np.exp(1j * m * t)
    inside = np.sum(c * special.jv(m, kin * r) * e, axis=-1)
    outside = np.sum(((1j) ** m * special.jv(m, kappa * r) + d * special.hankel1(m, kappa * r)) * e, axis=-1)
    return np.where(r[..., 0] < a, inside, outside)
