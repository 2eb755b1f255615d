"""Seeded synthetic workloads (shared by the tests, the oracle checks and the benchmark).

This module only produces inputs -- grids sizes, wavenumbers, scattering
potentials b, incident fields, receiver points -- and holds none of the
solver's arithmetic.  RNG: numpy PCG64 (``default_rng(seed)``) with draws in
the order written.  Nodes are cell centred on [-0.5, 0.5]^2 with h = 1/n,
arrays in C order [i2][i1] (x1 fastest).

Workload shapes follow the paper's experiments (unit square, smooth bumps and
cavity-like strong scatterers, about 10 points per wavelength as in its
Table 10); the paper's own potentials (lens, random bumps, photonic crystal)
and their reference solutions are not available, and these stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def nodes(n: int):
    h = 1.0 / n
    t = -0.5 + (np.arange(n) + 0.5) * h
    X2, X1 = np.meshgrid(t, t, indexing="ij")
    return X1, X2


def gaussian_b(n: int, amp=0.5, width=0.15):
    X1, X2 = nodes(n)
    return amp * np.exp(-(X1 ** 2 + X2 ** 2) / (2 * width ** 2))


def bumps(n: int, rng, nb=10, clip=0.95, smooth_beta=None):
    """Sum of nb Gaussian bumps: centres U[-.4,.4]^2, widths U[.03,.1], amplitudes U[-1.5,.9]."""
    X1, X2 = nodes(n)
    s = np.zeros((n, n))
    c = rng.uniform(-0.4, 0.4, size=(nb, 2))
    w = rng.uniform(0.03, 0.1, size=nb)
    a = rng.uniform(-1.5, 0.9, size=nb)
    for i in range(nb):
        s += a[i] * np.exp(-((X1 - c[i, 0]) ** 2 + (X2 - c[i, 1]) ** 2) / (2 * w[i] ** 2))
    if smooth_beta is None:
        return np.minimum(s, clip)
    return smooth_clip(s, clip, smooth_beta)


def smooth_clip(s, clip, beta):
    """clip - softplus_beta(clip - s): a smooth min(s, clip)."""
    z = beta * (clip - s)
    return clip - (np.logaddexp(0.0, z)) / beta


def fourier_field(n: int, rng, kmax_cycles=20.0, lo=-1.0, hi=0.9):
    """Random real field with Fourier modes |k| <= kmax cycles per unit, scaled to [lo, hi]."""
    K = int(math.ceil(kmax_cycles))
    k = np.arange(-K, K + 1)
    KY, KX = np.meshgrid(k, k, indexing="ij")
    mask = np.hypot(KX, KY) <= kmax_cycles
    coef = (rng.standard_normal(KX.shape) + 1j * rng.standard_normal(KX.shape)) * mask
    coef = 0.5 * (coef + np.conj(coef[::-1, ::-1]))  # Hermitian symmetry -> real field
    X1, X2 = nodes(n)
    f = np.zeros((n, n))
    ph1 = np.exp(2j * np.pi * np.outer(X1[0], k))          # [i1, kx]
    ph2 = np.exp(2j * np.pi * np.outer(X2[:, 0], k))       # [i2, ky]
    f = np.real(ph2 @ coef @ ph1.T)
    f = (f - f.min()) / (f.max() - f.min())
    return lo + (hi - lo) * f


def plane_wave(n: int, kappa: float, theta: float = 0.0):
    X1, X2 = nodes(n)
    return np.exp(1j * kappa * (np.cos(theta) * X1 + np.sin(theta) * X2))


def receivers(m=64, radius=0.7):
    t = 2 * np.pi * np.arange(m) / m
    return np.stack([radius * np.cos(t), radius * np.sin(t)], axis=1)


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    kappa: float
    b: np.ndarray
    u_inc: np.ndarray          # (nrhs, n, n) complex
    op_order: int
    pc_order: int = 4
    leaf: int = 8
    tol: float = 1e-4
    proxy_width: int = 2
    gmres_tol: float = 1e-10
    extra: dict = dataclasses.field(default_factory=dict)


def small(n=32):
    """N = 1024, kappa = 8 pi, b = 0.5 exp(-|x|^2 / (2 0.15^2)), 4th order, tol 1e-10."""
    kappa = 8 * np.pi
    return Workload("small-32", n, kappa, gaussian_b(n), plane_wave(n, kappa)[None],
                    op_order=4, tol=1e-10, proxy_width=3)


def bumps20(n=256, seed=2, kappa=40 * np.pi):
    """N = 65536, kappa = 40 pi, 10 seeded bumps clipped at 0.95, 6th-order operator."""
    rng = np.random.default_rng(seed)
    return Workload(f"bumps-{n}", n, kappa, bumps(n, rng), plane_wave(n, kappa)[None],
                    op_order=6, tol=1e-4)


def batched(count=64, seed0=3000):
    """Instances with sides from {64, 96, 128, 192, 256} and 5-20 wavelengths."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.choice([64, 96, 128, 192, 256]))
        kappa = 2 * np.pi * rng.uniform(5, 20)
        b = bumps(n, rng)
        leaf = 8 if n in (64, 128, 256) else 6
        out.append(Workload(f"inst{i}-{n}", n, kappa, b, plane_wave(n, kappa)[None],
                            op_order=6, leaf=leaf, tol=1e-4))
    return out


def differentiation(n=512, seed=4, kappa=80 * np.pi, nwaves=8, nrec=64):
    """30 smooth bumps (smooth clip 0.9), 8 plane waves, 64 receivers at radius 0.7."""
    rng = np.random.default_rng(seed)
    b = bumps(n, rng, nb=30, clip=0.9, smooth_beta=50.0)
    rng2 = np.random.default_rng(seed * 10)
    X1, X2 = nodes(n)
    pert = np.zeros((n, n))
    for _ in range(5):
        c = rng2.uniform(-0.4, 0.4, size=2)
        w = rng2.uniform(0.03, 0.1)
        pert += np.exp(-((X1 - c[0]) ** 2 + (X2 - c[1]) ** 2) / (2 * w * w))
    b_target = smooth_clip(b + 0.1 * pert, 0.9, 50.0)
    u = np.stack([plane_wave(n, kappa, 2 * np.pi * m / nwaves) for m in range(nwaves)])
    return Workload(f"diff-{n}", n, kappa, b, u, op_order=10, tol=1e-4,
                    extra={"receivers": receivers(nrec), "b_target": b_target})


def largest(n=1024, seed=5, kappa=200 * np.pi):
    """N = 1048576, kappa = 200 pi, random Fourier field (|k| <= 20 cycles) in [-1, 0.9], 10th order."""
    rng = np.random.default_rng(seed)
    return Workload(f"fourier-{n}", n, kappa, fourier_field(n, rng), plane_wave(n, kappa)[None],
                    op_order=10, tol=1e-4)
