"""Dense Nystrom discretisation and direct solve (oracle side; test infrastructure).

Paper eqs. (ls), (corrected), (linsys), (Gmat):
  sigma_i + kappa^2 b_i sum_j K_ij sigma_j = -kappa^2 b_i u_inc_i,
  K_ij = h^2 [ G(x_i, x_j) [i != j] + tau_{x_j - x_i} ],
with tau the order-p correction of ``quadrature.correction_weights``.
Grid: n x n cell-centred nodes on [-0.5, 0.5]^2, h = 1/n, C-order index
i2 * n + i1 (x1 fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import quadrature as quad


def grid(n: int):
    """Node coordinates (x1, x2), each (n, n) in [i2, i1] order, and h."""
    h = 1.0 / n
    t = -0.5 + (np.arange(n) + 0.5) * h
    X2, X1 = np.meshgrid(t, t, indexing="ij")
    return X1, X2, h


def kernel_offsets(n: int, kappa: float, order: int):
    """Koff[dy + n - 1, dx + n - 1] = K entry for source - target offset (dx, dy).

    Offsets span (-n, n) in each direction (all pairs of nodes of the grid).
    """
    h = 1.0 / n
    d = np.arange(-(n - 1), n)
    DY, DX = np.meshgrid(d, d, indexing="ij")
    r = h * np.hypot(DX, DY)
    K = np.zeros(r.shape, dtype=complex)
    nz = r > 0
    K[nz] = quad.green(kappa, r[nz])
    for (dx, dy), t in quad.correction_weights(order, kappa * h).items():
        if abs(dx) < n and abs(dy) < n:
            K[dy + n - 1, dx + n - 1] += t
    return h * h * K


def dense_K(n: int, kappa: float, order: int):
    """N x N matrix K (N = n^2), K[i, j] couples target i to source j."""
    Koff = kernel_offsets(n, kappa, order)
    i1 = np.tile(np.arange(n), n)
    i2 = np.repeat(np.arange(n), n)
    DX = i1[None, :] - i1[:, None]
    DY = i2[None, :] - i2[:, None]
    return Koff[DY + n - 1, DX + n - 1]


def dense_A(b, K, kappa: float):
    """A = I + diag(kappa^2 b) K  (paper eq. (linsys))."""
    b = np.asarray(b, dtype=float).reshape(-1)
    return np.eye(K.shape[0], dtype=complex) + (kappa ** 2 * b)[:, None] * K


def apply_rows(Koff, b, x, kappa: float, rows):
    """(A x)_i for the flat target indices in ``rows``, each by the direct sum
    over all n^2 sources (eqs. (linsys), (Gmat)).

    ``Koff`` is ``kernel_offsets(n, kappa, order)``; target (t1, t2) meets
    source (j1, j2) at offset (j1 - t1, j2 - t2), so its row of K is the n x n
    window of the offset table that starts at (n - 1 - t2, n - 1 - t1).
    O(n^2) work per row: spot checks at sizes where A cannot be formed.
    """
    n = Koff.shape[0] // 2 + 1
    b = np.asarray(b, dtype=float).reshape(n, n)
    x = np.asarray(x, dtype=complex).reshape(n, n)
    out = np.empty(len(rows), dtype=complex)
    for k, i in enumerate(rows):
        t2, t1 = divmod(int(i), n)
        win = Koff[n - 1 - t2:2 * n - 1 - t2, n - 1 - t1:2 * n - 1 - t1]
        out[k] = x[t2, t1] + kappa ** 2 * b[t2, t1] * np.sum(win * x)
    return out


def rhs(b, u_inc, kappa: float):
    """f = -kappa^2 b u_inc (paper eq. (linsys))."""
    return -kappa ** 2 * np.asarray(b, dtype=float).reshape(-1) * np.asarray(u_inc).reshape(-1)


class DenseSolver:
    """LU of A = I + diag(kappa^2 b) K with LAPACK (zgetrf/zgetrs)."""

    def __init__(self, n: int, kappa: float, order: int, b):
        self.n, self.kappa, self.order = n, kappa, order
        self.b = np.asarray(b, dtype=float).reshape(-1)
        self.K = dense_K(n, kappa, order)
        self.A = dense_A(self.b, self.K, kappa)
        self.lu = sla.lu_factor(self.A, check_finite=False)

    def solve(self, u_inc):
        """sigma and the grid scattered field u = K sigma for each column of u_inc."""
        U = np.asarray(u_inc).reshape(-1, self.n * self.n).T
        F = -self.kappa ** 2 * self.b[:, None] * U
        sig = sla.lu_solve(self.lu, F, check_finite=False)
        return sig.T, (self.K @ sig).T

    def solve_adjoint(self, g):
        """lambda = A^{-H} g."""
        G = np.asarray(g).reshape(-1, self.n * self.n).T
        return sla.lu_solve(self.lu, G, trans=2, check_finite=False).T


def receiver_matrix(n: int, kappa: float, pts):
    """E[r, j] = h^2 G(|x_r - x_j|): scattered field at off-grid points (eq. (ansatz))."""
    X1, X2, h = grid(n)
    pts = np.asarray(pts, dtype=float).reshape(-1, 2)
    dx = pts[:, 0:1] - X1.reshape(1, -1)
    dy = pts[:, 1:2] - X2.reshape(1, -1)
    return h * h * quad.green(kappa, np.hypot(dx, dy))


def misfit_loss_and_grad(n, kappa, order, b, u_inc, pts, target):
    """L = sum_m ||E sigma_m - t_m||^2 and dL/db by the dense adjoint.

    A sigma_m = f_m with f_m = -kappa^2 b u_inc_m; differentiating,
    d sigma = -kappa^2 A^{-1} (db * u_tot) with u_tot = u_inc + K sigma, so
    dL/db_k = -2 kappa^2 Re sum_m conj(lambda_mk) u_tot_mk,
    lambda_m = A^{-H} E^H (E sigma_m - t_m).
    """
    S = DenseSolver(n, kappa, order, b)
    U = np.asarray(u_inc).reshape(-1, n * n)
    sig, u = S.solve(U)
    E = receiver_matrix(n, kappa, pts)
    res = sig @ E.T - np.asarray(target).reshape(U.shape[0], -1)
    L = float(np.sum(np.abs(res) ** 2))
    lam = S.solve_adjoint(res @ E.conj())
    utot = U + u
    grad = -2 * kappa ** 2 * np.real(np.sum(np.conj(lam) * utot, axis=0))
    return L, grad
