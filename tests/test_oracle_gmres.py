"""Pins for the oracle's flexible GMRES (paper Sec. 5)."""
import numpy as np
import pytest
from scipy import special

from oracle import dense, fftop, gmres, hbs
import synth


def test_exact_preconditioner_one_iteration():
    n, kappa = 12, 9.0
    b = synth.gaussian_b(n)
    D = dense.DenseSolver(n, kappa, 6, b)
    f = dense.rhs(b, synth.plane_wave(n, kappa), kappa)
    x, it, hist = gmres.fgmres(lambda v: D.A @ v, lambda v: np.linalg.solve(D.A, v), f, 1e-12, 10)
    assert it == 1
    assert np.linalg.norm(D.A @ x - f) <= 1e-12 * np.linalg.norm(f)


def test_unpreconditioned_matches_lu_and_true_residual():
    n, kappa = 16, 14.0
    b = synth.bumps(n, np.random.default_rng(4))
    D = dense.DenseSolver(n, kappa, 10, b)
    f = dense.rhs(b, synth.plane_wave(n, kappa), kappa)
    x, it, hist = gmres.fgmres(lambda v: D.A @ v, lambda v: v, f, 1e-13, 256)
    sig, _ = D.solve(synth.plane_wave(n, kappa)[None])
    true_res = np.linalg.norm(D.A @ x - f) / np.linalg.norm(f)
    assert hist[-1] < 1e-13 and true_res < 1e-12
    assert np.linalg.norm(x - sig[0]) <= 1e-10 * np.linalg.norm(sig[0])


def test_spectra_example_iteration_counts():
    """Paper Sec. 5: N = 1600, kappa = 8 pi, lens b, 10th-order operator, HBS at
    tol 1e-2 with 4th order: 3 / 6 preconditioned iterations to 1e-5 / 1e-10
    (62 / 80 without).  Soft check (this build measures 5-6 / 11 and 51 / 68 with
    the lens placed on [-0.5, 0.5]^2 and leaf 5 x 5): a handful of iterations,
    several times fewer than unpreconditioned."""
    n, kappa = 40, 8 * np.pi
    X1, X2 = synth.nodes(n)
    b = 4 * (X2 - 0.1) * (1 - special.erf(25 * (np.hypot(X1, X2) - 0.3)))
    F = fftop.FFTOperator(n, kappa, 10)
    A = lambda v: F.apply(b, v).reshape(-1)
    f = dense.rhs(b, synth.plane_wave(n, kappa), kappa)
    M = hbs.Inverse(hbs.Compression(n, kappa, 5, 1e-2, 2), b)
    _, itp, hp = gmres.fgmres(A, M.apply, f, 1e-10, 100)
    _, itu, hu = gmres.fgmres(A, lambda v: v, f, 1e-10, 200)
    it5 = next(i for i, r in enumerate(hp) if r < 1e-5)
    assert it5 <= 6 and itp <= 12
    assert itu >= 5 * itp and itu >= 50
