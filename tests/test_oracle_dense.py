"""Pins for the dense Nystrom oracle (paper eqs. (ls), (linsys), (Gmat); Sec. 5 FFT operator).

Pinned against things the oracle does not compute itself: the exact
complex symmetry of the kernel, the textbook transmission series for a
constant-b disk (Remark 1.1), the Born limit, discrete reciprocity of the
far field, a 30-digit mpmath solve on a tiny grid, and finite differences of
the misfit for the dense adjoint gradient.
"""
import mpmath
import numpy as np
import pytest

from oracle import dense, disk, fftop
from oracle import quadrature as quad
import synth


def test_kernel_matrix_complex_symmetric():
    K = dense.dense_K(12, 9.0, 10)
    assert np.array_equal(K, K.T)
    assert not np.allclose(K, K.conj().T)


@pytest.mark.parametrize("order", [4, 6, 10])
def test_fft_operator_matches_dense(order):
    n, kappa = 20, 14.0
    rng = np.random.default_rng(1)
    b = rng.uniform(-1, 0.9, (n, n))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = dense.dense_A(b, dense.dense_K(n, kappa, order), kappa)
    y = fftop.FFTOperator(n, kappa, order).apply(b, x).reshape(-1)
    ref = A @ x.reshape(-1)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_direct_sum_rows_match_dense_matrix():
    """The row-by-row direct sum (used for spot checks at full size) against
    the dense matrix, on every row of a non-square-friendly grid."""
    n, kappa = 11, 13.0
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 0.9, (n, n))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = dense.dense_A(b, dense.dense_K(n, kappa, 10), kappa)
    rows = np.arange(n * n)
    y = dense.apply_rows(dense.kernel_offsets(n, kappa, 10), b, x, kappa, rows)
    assert np.max(np.abs(y - A @ x.reshape(-1))) <= 1e-13 * np.max(np.abs(A @ x.reshape(-1)))


def test_disk_transmission_series():
    """Constant b0 = 0.5 in a disk of radius 0.3 (discontinuous b: low order)."""
    kappa, b0, a = 4 * np.pi, 0.5, 0.3
    errs = []
    for n in (24, 72):
        X1, X2, h = dense.grid(n)
        r = np.hypot(X1, X2)
        b = np.where(r < a, b0, 0.0)
        uinc = np.exp(1j * kappa * X1)
        sig, u = dense.DenseSolver(n, kappa, 4, b).solve(uinc[None])
        utot = uinc.reshape(-1) + u[0]
        ex = disk.total_field(kappa, b0, a, X1, X2).reshape(-1)
        m = (np.abs(r - a) > 2 * h).reshape(-1)
        errs.append(np.linalg.norm((utot - ex)[m]) / np.linalg.norm(ex[m]))
        # eq. (ls) rearranged: sigma = -kappa^2 b u_tot
        assert np.allclose(sig[0], -kappa ** 2 * b.reshape(-1) * utot, atol=1e-10 * np.abs(sig).max())
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 4, errs


def test_born_limit():
    n, kappa = 16, 10.0
    b = synth.gaussian_b(n)
    uinc = synth.plane_wave(n, kappa)
    r = []
    for eps in (1e-3, 1e-4):
        sig, _ = dense.DenseSolver(n, kappa, 6, eps * b).solve(uinc[None])
        born = -kappa ** 2 * eps * b.reshape(-1) * uinc.reshape(-1)
        r.append(np.linalg.norm(sig[0] - born) / np.linalg.norm(born))
    assert r[0] / r[1] == pytest.approx(10, rel=0.05)


def test_far_field_reciprocity():
    n, kappa = 16, 12.0
    X1, X2, h = dense.grid(n)
    b = synth.bumps(n, np.random.default_rng(7))
    S = dense.DenseSolver(n, kappa, 8, b)
    ff = lambda xh, d: np.sum(np.exp(-1j * kappa * (xh[0] * X1 + xh[1] * X2)).reshape(-1)
                              * S.solve(np.exp(1j * kappa * (d[0] * X1 + d[1] * X2))[None])[0][0])
    for (t1, t2) in [(0.3, 2.1), (1.7, -0.4)]:
        xh, d = np.array([np.cos(t1), np.sin(t1)]), np.array([np.cos(t2), np.sin(t2)])
        assert ff(xh, d) == pytest.approx(ff(-d, -xh), rel=1e-12)


def test_tiny_grid_30_digit_solve():
    n, kappa, order = 4, 7.0, 6
    h = 1.0 / n
    b = np.linspace(0.2, 0.9, n * n)
    tw = quad.correction_weights(order, kappa * h)
    with mpmath.workdps(30):
        N = n * n
        A = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                dx, dy = j % n - i % n, j // n - i // n
                r = mpmath.sqrt(dx * dx + dy * dy) * h
                g = mpmath.mpc(0, 0.25) * mpmath.hankel1(0, kappa * r) if (dx or dy) else 0
                g += tw.get((dx, dy), 0)
                A[i, j] = (1 if i == j else 0) + kappa ** 2 * b[i] * h * h * g
        f = mpmath.matrix([-kappa ** 2 * b[i] for i in range(N)])
        x = mpmath.lu_solve(A, f)
        ref = np.array([complex(v) for v in x])
    sig, _ = dense.DenseSolver(n, kappa, order, b).solve(np.ones((1, n * n)))
    assert np.abs(sig[0] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_adjoint_gradient_matches_finite_differences():
    n, kappa, order = 8, 9.0, 6
    rng = np.random.default_rng(3)
    b = 0.5 * synth.gaussian_b(n, width=0.3)
    U = np.stack([synth.plane_wave(n, kappa, t) for t in (0.0, 1.3)])
    pts = synth.receivers(6, 0.7)
    tgt = rng.standard_normal((2, 6)) * 1e-3
    L0, g = dense.misfit_loss_and_grad(n, kappa, order, b, U, pts, tgt)
    eps = 1e-6
    for k in (5, 27, 40):
        bp, bm = b.copy().reshape(-1), b.copy().reshape(-1)
        bp[k] += eps
        bm[k] -= eps
        fd = (dense.misfit_loss_and_grad(n, kappa, order, bp, U, pts, tgt)[0]
              - dense.misfit_loss_and_grad(n, kappa, order, bm, U, pts, tgt)[0]) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-6)


def test_receiver_sum_matches_disk_series_off_grid():
    """The off-grid receiver sum u(x) = h^2 sum_j (i/4) H0(kappa |x - x_j|) sigma_j
    (eq. (ansatz), trapezoidal) against the transmission series of a constant-b
    disk (Remark 1.1) at 16 points off the grid: 8 outside the domain (radius
    0.7) and 8 inside it but outside the disk (radius 0.42), at angles with no
    symmetry in x1 <-> x2 or x -> -x.  b is discontinuous, so the error falls
    like O(h); a dropped h^2, a missing i/4, swapped coordinates or a flipped
    offset would leave an O(1) error."""
    kappa, b0, a = 4 * np.pi, 0.5, 0.3
    th = np.linspace(0, 2 * np.pi, 8, endpoint=False) + 0.37
    pts = np.concatenate([np.stack([0.7 * np.cos(th), 0.7 * np.sin(th)], 1),
                          np.stack([0.42 * np.cos(th + 0.2), 0.42 * np.sin(th + 0.2)], 1)])
    exact = disk.total_field(kappa, b0, a, pts[:, 0], pts[:, 1]) - np.exp(1j * kappa * pts[:, 0])
    errs = []
    for n in (24, 72):
        X1, X2, h = dense.grid(n)
        b = np.where(np.hypot(X1, X2) < a, b0, 0.0)
        sig, _ = dense.DenseSolver(n, kappa, 4, b).solve(np.exp(1j * kappa * X1)[None])
        up = dense.receiver_matrix(n, kappa, pts) @ sig[0]
        errs.append(np.abs(up - exact).max() / np.abs(exact).max())
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 4, errs
